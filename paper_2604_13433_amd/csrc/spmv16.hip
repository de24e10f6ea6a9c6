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
// once at the end.  Several right-hand sides (x and y row-major) run in
// passes of up to eight columns, one slice per wave.
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

// k right-hand sides (x m x k and y n x k, row-major): columns r0 .. r0 +
// KB - 1 per launch, one slice per wave, four slots (eight words) per
// group.  V4 (k and r0 multiples of 4, x and y 16-byte aligned): four
// columns per 16-byte gather and store.  Each column's products are summed
// in word order, as for k = 1.
template <int FMT, bool IMPL, int KB, bool V4>
__global__ __launch_bounds__(kB16) void k_spmv16_k(Spmv16Args a, uint32_t k, uint32_t r0) {
  constexpr int G = 4;
  constexpr bool kFix = FMT == PKSELL_FIX16;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t ks = __builtin_amdgcn_readfirstlane(b * (kB16 / kWave) + threadIdx.x / kWave);
  if (ks >= a.n_slices) return;
  const uint32_t lane = threadIdx.x & (kWave - 1), t = ks * kWave + lane;
  RowOut ro{t, 0u, 0u};
  if constexpr (IMPL || kFix)
    ro = row_out<FMT>(IMPL ? a.perm : nullptr, a.perm_bytes, a.row_exp, t, a.n, a.geo);
  const int64_t s = a.offset[ks];
  const uint32_t w = (uint32_t)((a.offset[ks + 1] - s) >> 7);  // slots per lane
  const __amdgpu_buffer_rsrc_t rs = slice_words(a.pack + (s >> 1), w);
  const uint32_t kx = k * 4u, x0 = r0 * 4u;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * kx);
  const uint32_t oob = a.m * kx;  // past the resource: 0, no request
  uint32_t c = left_offset32(t, a.geo);
  float acc[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) acc[r] = 0.0f;
  for (uint32_t j = 0; j < w; j += G) {
    uint32_t p[G];
#pragma unroll
    for (int q = 0; q < G; ++q) p[q] = j + q < w ? stream_word(rs, lane, j + q) : 0u;
    uint32_t o[2 * G];
    float v[2 * G];
#pragma unroll
    for (int h = 0; h < 2 * G; ++h) {
      const uint32_t wd = (h & 1) ? p[h >> 1] >> 16 : p[h >> 1] & 0xFFFFu;
      const bool flag = wd & 1u;
      c += flag ? (wd >> 1) & a.dmask : (wd >> 1);
      o[h] = flag ? c * kx + x0 : oob;
      v[h] = value16<FMT>(flag ? wd & a.vmask : 0u);
    }
#pragma unroll
    for (int h = 0; h < 2 * G; ++h) {
      if constexpr (V4) {
#pragma unroll
        for (int g = 0; g < KB / 4; ++g) {
          const f32x4 xv = buffer_load_f32x4(rx, o[h] == oob ? oob : o[h] + 16u * g);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[4 * g + e] = fmaf(v[h], xv[e], acc[4 * g + e]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < KB; ++r)
          acc[r] = fmaf(v[h], buffer_load_f32(rx, o[h] == oob ? oob : o[h] + 4u * r), acc[r]);
      }
    }
  }
  if (t >= a.n) return;
  if constexpr (kFix) {
    const int sh = ro.shift(Codec{0u, 0u, a.D});
#pragma unroll
    for (int r = 0; r < KB; ++r) acc[r] = ldexpf(acc[r], sh);
  }
  float *yo = a.y + (int64_t)(IMPL ? ro.row() : t) * k + r0;
  if constexpr (V4) {
#pragma unroll
    for (int g = 0; g < KB / 4; ++g)
      reinterpret_cast<f32x4 *>(yo)[g] = f32x4{acc[4 * g], acc[4 * g + 1], acc[4 * g + 2],
                                               acc[4 * g + 3]};
  } else {
#pragma unroll
    for (int r = 0; r < KB; ++r) yo[r] = acc[r];
  }
}

// k > 1: passes of 8 columns (then 4, 2, 1) over the words.
template <int FMT, bool IMPL>
int launch16_k(const Spmv16Args &a, int64_t k, bool v4, hipStream_t st) {
  const int64_t grid = cdiv(a.n_slices, kB16 / kWave);
  const uint32_t kk = (uint32_t)k;
  for (int64_t r0 = 0; r0 < k;) {
    const int64_t left = k - r0;
    const uint32_t r = (uint32_t)r0;
    if (v4 && left >= 8) {
      k_spmv16_k<FMT, IMPL, 8, true><<<grid, kB16, 0, st>>>(a, kk, r);
      r0 += 8;
    } else if (v4) {
      k_spmv16_k<FMT, IMPL, 4, true><<<grid, kB16, 0, st>>>(a, kk, r);
      r0 += 4;
    } else if (left >= 8) {
      k_spmv16_k<FMT, IMPL, 8, false><<<grid, kB16, 0, st>>>(a, kk, r);
      r0 += 8;
    } else if (left >= 4) {
      k_spmv16_k<FMT, IMPL, 4, false><<<grid, kB16, 0, st>>>(a, kk, r);
      r0 += 4;
    } else if (left >= 2) {
      k_spmv16_k<FMT, IMPL, 2, false><<<grid, kB16, 0, st>>>(a, kk, r);
      r0 += 2;
    } else {
      k_spmv16_k<FMT, IMPL, 1, false><<<grid, kB16, 0, st>>>(a, kk, r);
      r0 += 1;
    }
    PKS_LAUNCHED();
  }
  return PKSELL_OK;
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

// y = A_q x for 16-bit words, k right-hand sides (called by pksell_spmv).
int spmv16(const pksell_matrix *A, const float *x, float *y, int64_t k, hipStream_t st) {
  PKS_CHECK(A->C == kWave, PKSELL_EINVAL, "16-bit words need C = 64");
  PKS_CHECK(k >= 1 && k <= 64, PKSELL_EINVAL, "k must be in [1, 64]");
  PKS_CHECK(A->m * k * 4 < (int64_t(1) << 32), PKSELL_ERANGE, "m * k * 4 must be below 2^32");
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
    k_zero16<<<cdiv(A->n * k, 256), 256, 0, st>>>(y, A->n * k);
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
  if (k > 1) {
    const bool v4 = k % 4 == 0 && (((uintptr_t)x | (uintptr_t)y) & 15) == 0;
    if (A->fmt == PKSELL_E5MY)
      return impl ? launch16_k<PKSELL_E5MY, true>(a, k, v4, st)
                  : launch16_k<PKSELL_E5MY, false>(a, k, v4, st);
    return impl ? launch16_k<PKSELL_FIX16, true>(a, k, v4, st)
                : launch16_k<PKSELL_FIX16, false>(a, k, v4, st);
  }
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
