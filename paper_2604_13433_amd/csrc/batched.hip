// Batched PackSELL products: many matrices of uneven size, k right-hand
// sides each, in one persistent launch.
//
// The plan flattens every (matrix, slice) pair into one list of work units
// (slice counts prefix-summed per matrix) and stores one descriptor per
// matrix in device memory.  Each wave of a fixed, chip-filling grid takes a
// contiguous run of units, finds the matrix of its first unit once and
// walks on; each unit is one slice (C = 64, a wave) processed like the
// single-matrix product, with k right-hand sides in passes of up to KB.
// The transposed product scatters with float32 atomics after zeroing its
// outputs in a separate launch.  Launches read only the device table, so
// they can be captured into a graph and replayed.
#include <algorithm>
#include <vector>

#include "rowdot.hpp"

namespace pksell {

namespace {

constexpr int kB = kRowBlock;

struct Item {
  const uint32_t *pack;
  const int64_t *offset;
  const void *perm;
  const int16_t *row_exp;
  const float *in;
  float *out;
  uint32_t n, m, n_slices, perm_bytes;
  RowGeo geo;
  Codec cd;
};

// Finds the matrix holding unit u (unit_start is the prefix sum of slice
// counts, count + 1 entries); scalar loop, once per wave.
__device__ inline uint32_t find_item(const uint32_t *unit_start, uint32_t count, uint32_t u) {
  uint32_t lo = 0, hi = count;  // unit_start[lo] <= u < unit_start[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (unit_start[mid] <= u) lo = mid; else hi = mid;
  }
  return lo;
}

template <int FMT, int KB, bool TRANS, bool V4>
__device__ inline void do_unit(const Item &it, uint32_t k_slice, uint32_t lane, int k, int r0) {
  const uint32_t t = k_slice * kWave + lane;
  const int64_t s = it.offset[k_slice];
  const uint32_t w = (uint32_t)((it.offset[k_slice + 1] - s) >> 6);
  const uint32_t *P = it.pack + s + lane;
  uint32_t c = left_offset32(t, it.geo);
  int sh = 0;  // FIX: the row scale 2^(e - D - 1), applied with ldexp
  if constexpr (FMT == PKSELL_FIX)
    if (t < it.n) sh = (int)it.row_exp[t] - (it.cd.D + 1);
  if constexpr (!TRANS) {
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(it.in, it.m * (uint32_t)k * 4u);
    const uint32_t kx = (uint32_t)k * 4u, x0 = (uint32_t)r0 * 4u;
    float acc[KB];
#pragma unroll
    for (int r = 0; r < KB; ++r) acc[r] = 0.0f;
    if constexpr (V4) {
      packsell_row_v4<FMT, KB>(P, kWave, w, c, it.cd,
                               [&](uint32_t cc, int g) {
                                 return buffer_load_f32x4(rx, cc * kx + x0 + 16u * g);
                               },
                               acc);
    } else {
      packsell_row<FMT, KB>(P, kWave, w, c, it.cd,
                            [&](uint32_t cc, int r) { return buffer_load_f32(rx, cc * kx + x0 + 4u * r); },
                            acc);
    }
    if (t < it.n) {
      const int64_t o = (int64_t)out_row(it.perm, it.perm_bytes, t, it.geo) * k + r0;
#pragma unroll
      for (int r = 0; r < KB; ++r)
        if constexpr (FMT == PKSELL_FIX) acc[r] = ldexpf(acc[r], sh);
      if constexpr (V4) {
        f32x4 *yo = reinterpret_cast<f32x4 *>(it.out + o);
#pragma unroll
        for (int g = 0; g < KB / 4; ++g)
          yo[g] = f32x4{acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]};
      } else {
#pragma unroll
        for (int r = 0; r < KB; ++r) it.out[o + r] = acc[r];
      }
    }
  } else {
    if (t >= it.n) return;
    const float *g = it.in + (int64_t)out_row(it.perm, it.perm_bytes, t, it.geo) * k + r0;
    float gr[KB];
#pragma unroll
    for (int r = 0; r < KB; ++r) gr[r] = FMT == PKSELL_FIX ? ldexpf(g[r], sh) : g[r];
    for (uint32_t j = 0; j < w; ++j) {
      const uint32_t p = __builtin_nontemporal_load(P + j * kWave);
      const Unpacked u = unpack(p, it.cd);
      c += u.delta;
      if (p & 1u) {
        const float v = decode_value<FMT>(u.vbits);
        float *o = it.out + (int64_t)c * k + r0;
#pragma unroll
        for (int r = 0; r < KB; ++r) unsafeAtomicAdd(o + r, v * gr[r]);
      }
    }
  }
}

template <int FMT, int KB, bool TRANS, bool V4>
__global__ __launch_bounds__(kB) void k_batched(const Item *__restrict__ items,
                                               const uint32_t *__restrict__ unit_start,
                                               uint32_t count, uint32_t total, uint32_t per_wave,
                                               int k, int r0) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(b * (kB / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t u = wave * per_wave;
  const uint32_t u1 = min(u + per_wave, total);
  if (u >= u1) return;
  uint32_t it = find_item(unit_start, count, u);
  for (; u < u1; ++u) {
    while (u >= unit_start[it + 1]) ++it;
    do_unit<FMT, KB, TRANS, V4>(items[it], u - unit_start[it], lane, k, r0);
  }
}

template <typename T>
__global__ void k_zero_batched(const Item *__restrict__ items, uint32_t count, int k) {
  for (uint32_t i = 0; i < count; ++i) {
    const uint64_t len = (uint64_t)items[i].m * k;
    for (uint64_t e = (uint64_t)blockIdx.x * kB + threadIdx.x; e < len; e += (uint64_t)gridDim.x * kB)
      items[i].out[e] = T(0);
  }
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_batch_plan_bytes(int32_t count, size_t *bytes) {
  PKS_CHECK(count >= 1 && bytes, PKSELL_EINVAL, "count must be >= 1");
  Carver cv(nullptr);
  cv.take<Item>((size_t)count);
  cv.take<uint32_t>((size_t)count + 1);
  *bytes = cv.used;
  return PKSELL_OK;
}

int pksell_batch_plan(const pksell_batch_item *items, int32_t count, int64_t k,
                      int32_t transpose, pksell_batch *plan, void *ws, size_t ws_bytes,
                      void *stream) {
  PKS_CHECK(items && plan && count >= 1, PKSELL_EINVAL, "null argument");
  PKS_CHECK(k >= 1 && k <= 64, PKSELL_EINVAL, "k must be in [1, 64]");
  size_t need = 0;
  pksell_batch_plan_bytes(count, &need);
  PKS_CHECK(ws && ws_bytes >= need, PKSELL_EWORKSPACE, "plan workspace: need %zu bytes", need);
  std::vector<Item> host((size_t)count);
  std::vector<uint32_t> start((size_t)count + 1, 0);
  int fmt = -1;
  for (int32_t i = 0; i < count; ++i) {
    const pksell_matrix *A = items[i].A;
    PKS_CHECK(A, PKSELL_EINVAL, "item %d: null matrix", i);
    PKS_CHECK(A->C == kWave, PKSELL_EINVAL, "item %d: batched products need C = 64", i);
    PKS_CHECK(fmt < 0 || A->fmt == fmt, PKSELL_EINVAL, "item %d: all matrices need one format", i);
    fmt = A->fmt;
    PKS_CHECK(A->perm_mode != PKSELL_IMPLICIT || A->perm, PKSELL_EINVAL, "item %d: no perm", i);
    PKS_CHECK(A->fmt != PKSELL_FIX || A->row_exp, PKSELL_EINVAL, "item %d: no row_exp", i);
    PKS_CHECK(A->n == 0 || (A->offset && A->pack), PKSELL_EINVAL, "item %d: arrays not set", i);
    PKS_CHECK(A->m * k * 4 < (int64_t(1) << 32), PKSELL_ERANGE, "item %d: m * k too large", i);
    PKS_CHECK((A->n == 0 || items[i].in) && (A->n == 0 || items[i].out), PKSELL_EINVAL,
              "item %d: null in/out", i);
    Item &h = host[(size_t)i];
    h.pack = A->pack;
    h.offset = A->offset;
    h.perm = A->perm_mode == PKSELL_IMPLICIT ? A->perm : nullptr;
    h.row_exp = A->row_exp;
    h.in = items[i].in;
    h.out = items[i].out;
    h.n = (uint32_t)A->n;
    h.m = (uint32_t)A->m;
    h.n_slices = (uint32_t)A->n_slices;
    h.perm_bytes = (uint32_t)A->perm_bytes;
    h.geo = make_geo(A->sigma, A->k_left, A->C);
    h.cd = make_codec(A->D);
    start[(size_t)i + 1] = start[(size_t)i] + (uint32_t)A->n_slices;
    PKS_CHECK(start[(size_t)i + 1] >= start[(size_t)i], PKSELL_ERANGE, "too many slices");
  }
  Carver cv(ws);
  Item *dev_items = cv.take<Item>((size_t)count);
  uint32_t *dev_start = cv.take<uint32_t>((size_t)count + 1);
  hipStream_t st = as_stream(stream);
  PKS_HIP(hipMemcpyAsync(dev_items, host.data(), sizeof(Item) * (size_t)count,
                         hipMemcpyHostToDevice, st));
  PKS_HIP(hipMemcpyAsync(dev_start, start.data(), sizeof(uint32_t) * ((size_t)count + 1),
                         hipMemcpyHostToDevice, st));
  PKS_HIP(hipStreamSynchronize(st));
  int dev = 0, cus = 256;
  PKS_HIP(hipGetDevice(&dev));
  PKS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  std::memset(plan, 0, sizeof(*plan));
  plan->count = count;
  plan->fmt = fmt;
  plan->k = (int32_t)k;
  plan->transpose = transpose ? 1 : 0;
  // 16-byte gathers and stores need k % 4 == 0 and 16-byte aligned blocks
  bool aligned = k % 4 == 0;
  for (int32_t i = 0; i < count; ++i)
    aligned &= ((reinterpret_cast<uintptr_t>(items[i].in) |
                 reinterpret_cast<uintptr_t>(items[i].out)) & 15) == 0;
  plan->vec4 = aligned ? 1 : 0;
  plan->total_units = start[(size_t)count];
  // a chip-filling grid: 8 waves per SIMD, 4 SIMDs per CU
  const int64_t max_waves = (int64_t)cus * 32;
  const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(plan->total_units, max_waves));
  plan->units_per_wave = (int32_t)cdiv(std::max<int64_t>(1, plan->total_units), waves);
  plan->waves = (int32_t)cdiv(std::max<int64_t>(1, plan->total_units), plan->units_per_wave);
  plan->items = dev_items;
  plan->unit_start = dev_start;
  return PKSELL_OK;
}

int pksell_spmv_batched(const pksell_batch *plan, void *stream) {
  PKS_CHECK(plan && plan->items && plan->unit_start, PKSELL_EINVAL, "plan not set");
  hipStream_t st = as_stream(stream);
  const Item *items = static_cast<const Item *>(plan->items);
  const uint32_t *start = static_cast<const uint32_t *>(plan->unit_start);
  const int k = plan->k;
  if (plan->transpose) {
    k_zero_batched<float><<<1024, kB, 0, st>>>(items, (uint32_t)plan->count, k);
    PKS_LAUNCHED();
  }
  if (plan->total_units == 0) return PKSELL_OK;
  const int64_t grid = cdiv(plan->waves, kB / kWave);
  const uint32_t cnt = (uint32_t)plan->count, tot = (uint32_t)plan->total_units,
                 pw = (uint32_t)plan->units_per_wave;
  // 16-byte gathers and stores when every x / y row group is aligned
  const bool v4 = plan->vec4 && !plan->transpose;
  for (int r0 = 0; r0 < k;) {
    const int left = k - r0;
    const int kb = left >= 32 ? 32 : left >= 8 ? 8 : 1;
#define PKS_B(F, KB, T, V) \
  k_batched<F, KB, T, V><<<grid, kB, 0, st>>>(items, start, cnt, tot, pw, k, r0)
#define PKS_BK(F, T)                                  \
  do {                                                \
    if (kb == 32) {                                   \
      if (v4) PKS_B(F, 32, T, true);                  \
      else PKS_B(F, 32, T, false);                    \
    } else if (kb == 8) {                             \
      if (v4) PKS_B(F, 8, T, true);                   \
      else PKS_B(F, 8, T, false);                     \
    } else {                                          \
      PKS_B(F, 1, T, false);                          \
    }                                                 \
  } while (0)
#define PKS_BT(F) do { if (plan->transpose) PKS_BK(F, true); else PKS_BK(F, false); } while (0)
    switch (plan->fmt) {
      case PKSELL_FP16: PKS_BT(PKSELL_FP16); break;
      case PKSELL_E8MY: PKS_BT(PKSELL_E8MY); break;
      default: PKS_BT(PKSELL_FIX); break;
    }
#undef PKS_BT
#undef PKS_BK
#undef PKS_B
    PKS_LAUNCHED();
    r0 += kb;
  }
  return PKSELL_OK;
}

}  // extern "C"
