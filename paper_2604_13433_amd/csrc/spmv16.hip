// Products of 16-bit-word PackSELL matrices (E5MY and FIX16 values), the
// loop of sec. 4.4 over words of W = 16.
//
// Layout: every 32-bit slot holds two consecutive words of one row (word 2i
// in the low half, 2i + 1 in the high half), slots column-major per slice of
// C = 64 rows, so a lane reads a dword per two words and a wave a 256-byte
// line per slot index, as with 32-bit words.  A wave walks S consecutive
// slices together (S = 2 for narrow slices), G slots (2G words) in flight
// per slice; each word is decoded in registers (flag, delta of D
// or 15 bits, value field), the running column gathers x (flag-0 words
// gather past the buffer resource: 0, no request), and the products are
// summed in float32 in word order.  FIX16 rows are scaled by 2^(e - D - 1)
// once at the end.
#include <algorithm>

#include "rowdot.hpp"

namespace pksell {

namespace {

constexpr int kB16 = 128;  // threads per workgroup

struct Spmv16Args {
  const uint32_t *pack;
  const int64_t *offset;  // in words
  const void *perm;
  const int16_t *row_exp;
  const float *x;
  float *y;
  uint32_t n, m, n_slices;
  int32_t perm_bytes, D;
  RowGeo geo;
  uint32_t dmask;  // 2^D - 1: the flag-1 delta after >> 1
  uint32_t vmask;  // 0xFFFF & ~(2^(D+1) - 1): the value field
};

// A value field as float32: E5MY is a binary16 pattern; FIX16 the signed
// field as stored, q * 2^(D+1).
template <int FMT>
__device__ inline float value16(uint32_t bits) {
  if constexpr (FMT == PKSELL_E5MY) return __half2float(__ushort_as_half((unsigned short)bits));
  else return (float)(int32_t)(int16_t)(uint16_t)bits;
}

// G slots (2G words) per group and slice, sized on the host to the
// matrix's slice width: every slot of a group issues a load and both of its
// words a gather, so a group wider than the slices issues instructions for
// padding (each a full 64-lane instruction, however few bytes it moves).
template <int FMT, bool IMPL, int S, int G>
__global__ __launch_bounds__(kB16) void k_spmv16(Spmv16Args a) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(b * (kB16 / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t k0 = wave * S;
  if (k0 >= a.n_slices) return;
  constexpr bool kFix = FMT == PKSELL_FIX16;
  RowOut ro[S];  // destinations (and FIX16 exponents) read up front
  if constexpr (IMPL || kFix) {
#pragma unroll
    for (int i = 0; i < S; ++i)
      ro[i] = row_out<FMT>(IMPL ? a.perm : nullptr, a.perm_bytes, a.row_exp,
                           (k0 + i) * kWave + lane, a.n, a.geo);
  }
  int64_t off[S + 1];
#pragma unroll
  for (int i = 0; i <= S; ++i) off[i] = a.offset[min(k0 + i, a.n_slices)];
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * 4u);
  const uint32_t oob = a.m * 4u;
  uint32_t w[S], c[S], wm = 0;  // w: slots per lane
  float acc[S];
  __amdgpu_buffer_rsrc_t rs[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    w[i] = (uint32_t)((off[i + 1] - off[i]) >> 7);
    wm = max(wm, w[i]);
    c[i] = left_offset32((k0 + i) * kWave + lane, a.geo);
    acc[i] = 0.0f;
    rs[i] = slice_words(a.pack + (off[i] >> 1), w[i]);
  }
  for (uint32_t j = 0; j < wm; j += G) {
    uint32_t p[S][G];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int q = 0; q < G; ++q) p[i][q] = j + q < w[i] ? stream_word(rs[i], lane, j + q) : 0u;
    uint32_t o[S][2 * G];
    float v[S][2 * G];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int h = 0; h < 2 * G; ++h) {
        const uint32_t wd = (h & 1) ? p[i][h >> 1] >> 16 : p[i][h >> 1] & 0xFFFFu;
        const bool flag = wd & 1u;
        c[i] += flag ? (wd >> 1) & a.dmask : (wd >> 1);
        o[i][h] = flag ? c[i] << 2 : oob;
        v[i][h] = value16<FMT>(flag ? wd & a.vmask : 0u);
      }
    float xv[S][2 * G];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int h = 0; h < 2 * G; ++h) xv[i][h] = buffer_load_f32(rx, o[i][h]);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int h = 0; h < 2 * G; ++h) acc[i] = fmaf(v[i][h], xv[i][h], acc[i]);
  }
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const uint32_t t = (k0 + i) * kWave + lane;
    if (k0 + i >= a.n_slices || t >= a.n) continue;
    float r = acc[i];
    if constexpr (kFix) r = ldexpf(r, ro[i].shift(Codec{0u, 0u, a.D}));
    a.y[IMPL ? ro[i].row() : t] = r;
  }
}

__global__ void k_zero16(float *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0f;
}

// Two slices per wave with G < 8 (narrow slices), one with G = 8.
template <int FMT, bool IMPL, int G>
void launch16g(const Spmv16Args &a, hipStream_t st) {
  if constexpr (G < 8)
    k_spmv16<FMT, IMPL, 2, G><<<cdiv(cdiv(a.n_slices, 2), kB16 / kWave), kB16, 0, st>>>(a);
  else
    k_spmv16<FMT, IMPL, 1, G><<<cdiv(a.n_slices, kB16 / kWave), kB16, 0, st>>>(a);
}

template <int FMT, bool IMPL>
void launch16(const Spmv16Args &a, int G, hipStream_t st) {
  switch (G) {
    case 1: launch16g<FMT, IMPL, 1>(a, st); break;
    case 2: launch16g<FMT, IMPL, 2>(a, st); break;
    case 3: launch16g<FMT, IMPL, 3>(a, st); break;
    case 4: launch16g<FMT, IMPL, 4>(a, st); break;
    case 5: launch16g<FMT, IMPL, 5>(a, st); break;
    case 6: launch16g<FMT, IMPL, 6>(a, st); break;
    case 7: launch16g<FMT, IMPL, 7>(a, st); break;
    default: launch16g<FMT, IMPL, 8>(a, st); break;
  }
}

}  // namespace

// y = A_q x for 16-bit words, k = 1 (called by pksell_spmv).
int spmv16(const pksell_matrix *A, const float *x, float *y, int64_t k, hipStream_t st) {
  PKS_CHECK(A->C == kWave, PKSELL_EINVAL, "16-bit words need C = 64");
  PKS_CHECK(k == 1, PKSELL_EINVAL, "16-bit words: k must be 1");
  PKS_CHECK(A->n == 0 || (A->offset && (A->n_words == 0 || A->pack)), PKSELL_EINVAL,
            "matrix arrays not set");
  PKS_CHECK(A->perm_mode != PKSELL_IMPLICIT || A->n == 0 || A->perm, PKSELL_EINVAL,
            "implicit mode needs perm");
  PKS_CHECK(A->fmt != PKSELL_FIX16 || A->n == 0 || A->row_exp, PKSELL_EINVAL,
            "FIX16 needs row_exp");
  PKS_CHECK(A->n_words < (int64_t(1) << 31), PKSELL_ERANGE,
            "16-bit words: n_words must be below 2^31 (32-bit slot offsets)");
  PKS_CHECK(A->n == 0 || y, PKSELL_EINVAL, "null y");
  if (A->n == 0) return PKSELL_OK;
  if (A->m == 0) {
    k_zero16<<<cdiv(A->n, 256), 256, 0, st>>>(y, A->n);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  PKS_CHECK(x, PKSELL_EINVAL, "null x");
  Spmv16Args a;
  a.pack = A->pack;
  a.offset = A->offset;
  a.perm = A->perm;
  a.row_exp = A->row_exp;
  a.x = x;
  a.y = y;
  a.n = (uint32_t)A->n;
  a.m = (uint32_t)A->m;
  a.n_slices = (uint32_t)A->n_slices;
  a.perm_bytes = A->perm_bytes;
  a.D = A->D;
  a.geo = make_geo(A->sigma, A->k_left, A->C);
  a.dmask = (1u << A->D) - 1u;
  a.vmask = 0xFFFFu & ~((2u << A->D) - 1u);
  // slots per group: the average slots per lane, rounded up, at most 8
  const int64_t slots = A->n_words / 2, lanes = (int64_t)kWave * A->n_slices;
  const int G = (int)std::min<int64_t>(8, std::max<int64_t>(1, cdiv(slots, lanes)));
  const bool impl = A->perm_mode == PKSELL_IMPLICIT;
  if (A->fmt == PKSELL_E5MY) {
    if (impl) launch16<PKSELL_E5MY, true>(a, G, st);
    else launch16<PKSELL_E5MY, false>(a, G, st);
  } else {
    if (impl) launch16<PKSELL_FIX16, true>(a, G, st);
    else launch16<PKSELL_FIX16, false>(a, G, st);
  }
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // namespace pksell
