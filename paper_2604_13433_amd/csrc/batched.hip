// Batched PackSELL products: many matrices of uneven size, k right-hand
// sides each, in one persistent launch.
//
// The plan flattens every (matrix, slice) pair into one list of work units
// (slice counts prefix-summed per matrix) and stores one descriptor per
// matrix in device memory.  Each wave of a fixed, chip-filling grid takes
// every W-th unit (W = the grid's wave count), so at any moment the
// resident waves work on one contiguous window of units and share the x
// rows it touches in L2; a wave finds the matrix of its first unit once and
// walks on; each unit is one slice (C = 64, a wave) processed like the
// single-matrix product, with k right-hand sides in passes of up to KB --
// or, for forward products with k a multiple of 4 and k >= 8, a 64 / L-row
// part of a slice in lane groups of L lanes per row (all k in one pass).
// The transposed product scatters with float32 atomics after zeroing its
// outputs in a separate launch.  Forward products with k = 1 instead run
// the single-matrix two-slice kernel over the batch: one wave per pair of
// consecutive slices of one matrix (pairs prefix-summed per matrix), on a
// grid of all pairs.  Launches read only the device table, so they can be
// captured into a graph and replayed.
#include <algorithm>
#include <vector>

#include "pair.hpp"

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
    const uint32_t oob = it.m * kx;  // flag-0 words: past the resource, no request
    if constexpr (V4) {
      packsell_row_v4<FMT, KB>(P, kWave, w, c, it.cd,
                               [&](uint32_t cc, int g, bool live) {
                                 return buffer_load_f32x4(rx, live ? cc * kx + x0 + 16u * g : oob);
                               },
                               acc);
    } else {
      packsell_row<FMT, KB>(P, kWave, w, c, it.cd,
                            [&](uint32_t cc, int r, bool live) {
                              return buffer_load_f32(rx, live ? cc * kx + x0 + 4u * r : oob);
                            },
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
                                               uint32_t count, uint32_t total, int k, int r0) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(b * (kB / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t stride = gridDim.x * (kB / kWave);
  uint32_t u = wave;
  if (u >= total) return;
  uint32_t it = find_item(unit_start, count, u);
  for (; u < total; u += stride) {
    while (u >= unit_start[it + 1]) ++it;
    do_unit<FMT, KB, TRANS, V4>(items[it], u - unit_start[it], lane, k, r0);
  }
}

// Software-pipelined persistent loop for k = 1 (L = 1: one lane per row)
// and for lane groups (L >= 2, k a multiple of 4, aligned): while the
// gathers of unit u are in flight, the slice bounds and the first eight
// words of unit u + 1 are already loading, so a wave pays about one memory
// round trip per unit instead of two.  Same arithmetic, in the same word
// order, as the single-matrix kernels.
struct Unit {
  uint32_t item, ks, l, q, w;
  bool live;
  int64_t s;
};

template <int L>
__device__ inline Unit unit_at(const Item *items, const uint32_t *unit_start, uint32_t item,
                               uint32_t u, uint32_t lane, uint32_t k4) {
  Unit x;
  x.item = item;
  const uint32_t ul = u - unit_start[item];
  if constexpr (L == 1) {
    x.ks = ul;
    x.l = lane;
    x.q = 0;
    x.live = true;
  } else {
    x.ks = ul / L;
    const GroupLane g = group_lane<L>(ul % L, lane, k4);
    x.l = g.l;
    x.q = g.q;
    x.live = g.live;
  }
  const Item &I = items[item];
  x.s = I.offset[x.ks];
  x.w = (uint32_t)((I.offset[x.ks + 1] - x.s) >> 6);
  return x;
}

// Words j .. j+G-1 of lane l of the slice starting at word s (w is
// wave-uniform; words past w are padding).  Nontemporal when one wave reads
// each word (L = 1), plain when lane groups share them.  (Streamed buffer
// loads, faster in the single-matrix kernels, made this pipelined loop 20 %
// slower.)
template <bool NT, int G>
__device__ inline void load_words(const Item &it, int64_t s, uint32_t l, uint32_t w, uint32_t j,
                                  uint32_t (&p)[G]) {
  const uint32_t *P = it.pack + s + l;
#pragma unroll
  for (int q = 0; q < G; ++q) {
    uint32_t v = 0u;
    if (j + q < w) v = load_word<NT>(P + (j + q) * kWave);
    p[q] = v;
  }
}

// Decode G words and accumulate; flag-0 words gather at ``oob`` (past
// the resource: 0, no memory request).
template <int FMT, int L, int NA, int G>
__device__ inline void fma_words(const uint32_t (&p)[G], uint32_t &c, const Codec &cd,
                                 __amdgpu_buffer_rsrc_t rx, uint32_t kx, uint32_t xq,
                                 uint32_t oob, float (&acc)[NA]) {
  uint32_t cq[G];
  float v[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const Unpacked u = unpack(p[q], cd);
    c += u.delta;
    cq[q] = c;
    v[q] = decode_value<FMT>(u.vbits);
  }
  if constexpr (L == 1) {
    float xv[G];
#pragma unroll
    for (int q = 0; q < G; ++q) xv[q] = buffer_load_f32(rx, (p[q] & 1u) ? cq[q] << 2 : oob);
#pragma unroll
    for (int q = 0; q < G; ++q) acc[0] = fmaf(v[q], xv[q], acc[0]);
  } else {
    f32x4 xv[G];
#pragma unroll
    for (int q = 0; q < G; ++q)
      xv[q] = buffer_load_f32x4(rx, (p[q] & 1u) ? cq[q] * kx + xq : oob);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      acc[0] = fmaf(v[q], xv[q].x, acc[0]);
      acc[1] = fmaf(v[q], xv[q].y, acc[1]);
      acc[2] = fmaf(v[q], xv[q].z, acc[2]);
      acc[3] = fmaf(v[q], xv[q].w, acc[3]);
    }
  }
}

template <int FMT, int L, int G = kUnroll>
__global__ __launch_bounds__(kB) void k_batched_pipe(const Item *__restrict__ items,
                                                    const uint32_t *__restrict__ unit_start,
                                                    uint32_t count, uint32_t total, int k) {
  constexpr int NA = L == 1 ? 1 : 4;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(b * (kB / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t stride = gridDim.x * (kB / kWave);
  uint32_t u = wave;
  if (u >= total) return;
  const uint32_t k4 = (uint32_t)k >> 2, kx = (uint32_t)k * 4u;
  Unit cur = unit_at<L>(items, unit_start, find_item(unit_start, count, u), u, lane, k4);
  constexpr bool NT = L == 1;
  uint32_t p[G];
  load_words<NT, G>(items[cur.item], cur.s, cur.l, cur.w, 0, p);
  for (;;) {
    const bool more = u + stride < total;
    Unit nx;
    uint32_t pn[G];
    if (more) {  // the next unit's bounds and first words, before this unit's gathers
      uint32_t itn = cur.item;
      while (u + stride >= unit_start[itn + 1]) ++itn;
      nx = unit_at<L>(items, unit_start, itn, u + stride, lane, k4);
      load_words<NT, G>(items[itn], nx.s, nx.l, nx.w, 0, pn);
    }
    const Item &I = items[cur.item];
    const uint32_t t = cur.ks * kWave + cur.l;
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(I.in, I.m * kx);
    const uint32_t xq = 16u * cur.q;
    uint32_t c = left_offset32(t, I.geo);
    float acc[NA];
#pragma unroll
    for (int r = 0; r < NA; ++r) acc[r] = 0.0f;
    const uint32_t oob = I.m * kx;
    fma_words<FMT, L, NA, G>(p, c, I.cd, rx, kx, xq, oob, acc);
    for (uint32_t j = G; j < cur.w; j += G) {  // slices wider than one group
      uint32_t pr[G];
      load_words<NT, G>(I, cur.s, cur.l, cur.w, j, pr);
      fma_words<FMT, L, NA, G>(pr, c, I.cd, rx, kx, xq, oob, acc);
    }
    if (t < I.n && cur.live) {
      if constexpr (FMT == PKSELL_FIX) {
        const int sh = (int)I.row_exp[t] - (I.cd.D + 1);
#pragma unroll
        for (int r = 0; r < NA; ++r) acc[r] = ldexpf(acc[r], sh);
      }
      const uint32_t row = out_row(I.perm, I.perm_bytes, t, I.geo);
      if constexpr (L == 1) {  // streaming (nontemporal) stores
        __builtin_nontemporal_store(acc[0], I.out + row);
      } else {
        __builtin_nontemporal_store(f32x4{acc[0], acc[1], acc[2], acc[3]},
                                    reinterpret_cast<f32x4 *>(I.out + (int64_t)row * k + 4 * cur.q));
      }
    }
    if (!more) break;
    cur = nx;
#pragma unroll
    for (int q = 0; q < G; ++q) p[q] = pn[q];
    u += stride;
  }
}

typedef void (*PipeKernel)(const Item *, const uint32_t *, uint32_t, uint32_t, int);

template <int FMT>
PipeKernel k_batched_pipe_for(int L, int G) {
  switch (L) {
    case 1:
      switch (G) {
        case 4: return k_batched_pipe<FMT, 1, 4>;
        case 5: return k_batched_pipe<FMT, 1, 5>;
        case 6: return k_batched_pipe<FMT, 1, 6>;
        case 7: return k_batched_pipe<FMT, 1, 7>;
        default: return k_batched_pipe<FMT, 1, 8>;
      }
    case 2: return k_batched_pipe<FMT, 2>;
    case 4: return k_batched_pipe<FMT, 4>;
    case 8: return k_batched_pipe<FMT, 8>;
    default: return k_batched_pipe<FMT, 16>;
  }
}

// k = 1, forward: the two-slice product of the single-matrix kernels, one
// wave per slice pair u (pair_start: pairs prefix-summed per matrix), on a
// grid of every pair (workgroups remapped so each XCD walks one contiguous
// range of pairs).  The matrix of a pair is found by a scalar binary search
// of the prefix table.
template <int FMT, int G>
__global__ __launch_bounds__(kPairBlock) void k_batched_pair(const Item *__restrict__ items,
                                                           const uint32_t *__restrict__ pair_start,
                                                           uint32_t count, uint32_t total) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t u =
      __builtin_amdgcn_readfirstlane(b * (kPairBlock / kWave) + threadIdx.x / kWave);
  if (u >= total) return;
  const uint32_t it = find_item(pair_start, count, u);
  const Item &I = items[it];
  SpmvArgs a;
  a.pack = I.pack;
  a.offset = I.offset;
  a.perm = I.perm;
  a.row_exp = I.row_exp;
  a.x = I.in;
  a.y = I.out;
  a.n = I.n;
  a.m = I.m;
  a.n_slices = I.n_slices;
  a.C = kWave;
  a.perm_bytes = (int32_t)I.perm_bytes;
  a.k = 1;
  a.r0 = 0;
  a.geo = I.geo;
  a.cd = I.cd;
  const uint32_t k0 = (u - pair_start[it]) * 2;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  if (I.perm != nullptr)
    pair_product<FMT, true, true, G, false>(a, k0, lane);
  else
    pair_product<FMT, true, false, G, false>(a, k0, lane);
}

typedef void (*PairKernel)(const Item *, const uint32_t *, uint32_t, uint32_t);

template <int FMT>
PairKernel k_batched_pair_for(int G) {
  switch (G) {
    case 4: return k_batched_pair<FMT, 4>;
    case 5: return k_batched_pair<FMT, 5>;
    case 6: return k_batched_pair<FMT, 6>;
    case 7: return k_batched_pair<FMT, 7>;
    default: return k_batched_pair<FMT, 8>;
  }
}

// Forward products with k = 1 run the two-slice kernel when the plan has
// pairs (every matrix's words addressable through 32-bit byte offsets);
// lane groups (and k = 1 without pairs) the pipelined loop; transposed
// products and other k run k_batched in passes.
bool uses_pairs(const pksell_batch &p) { return !p.transpose && p.k == 1 && p.pair_units > 0; }
bool uses_pipe(const pksell_batch &p) { return !p.transpose && (p.k == 1 || p.group > 1); }

// Workgroups of the batched kernel that fit on one CU at once.
int resident_blocks(const pksell_batch &p) {
  const void *fn = nullptr;
  if (uses_pipe(p)) {
    fn = p.fmt == PKSELL_FP16   ? (const void *)k_batched_pipe_for<PKSELL_FP16>(p.group, p.words_per_group)
         : p.fmt == PKSELL_E8MY ? (const void *)k_batched_pipe_for<PKSELL_E8MY>(p.group, p.words_per_group)
                                : (const void *)k_batched_pipe_for<PKSELL_FIX>(p.group, p.words_per_group);
  } else {
    fn = (const void *)k_batched<PKSELL_E8MY, 8, false, false>;  // the largest pass kernel
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kB, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
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
  cv.take<uint32_t>(2 * ((size_t)count + 1));  // unit prefix, then slice-pair prefix
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
  std::vector<uint32_t> start(2 * ((size_t)count + 1), 0);  // units, then slice pairs
  uint32_t *pstart = start.data() + count + 1;
  bool pairs_ok = true;  // every matrix's words addressable by 32-bit byte offsets
  int fmt = -1;
  // 16-byte gathers and stores need k % 4 == 0 and 16-byte aligned blocks;
  // forward products with k >= 8 then use lane groups of L lanes per row
  bool aligned = k % 4 == 0;
  for (int32_t i = 0; i < count; ++i)
    aligned &= ((reinterpret_cast<uintptr_t>(items[i].in) |
                 reinterpret_cast<uintptr_t>(items[i].out)) & 15) == 0;
  const int L = (aligned && !transpose && k >= 8) ? group_size(k) : 1;  // lanes per row
  int64_t all_words = 0, all_slices = 0;
  for (int32_t i = 0; i < count; ++i) {
    const pksell_matrix *A = items[i].A;
    PKS_CHECK(A, PKSELL_EINVAL, "item %d: null matrix", i);
    PKS_CHECK(A->C == kWave, PKSELL_EINVAL, "item %d: batched products need C = 64", i);
    PKS_CHECK(A->fmt >= PKSELL_FP16 && A->fmt <= PKSELL_FIX, PKSELL_EINVAL,
              "item %d: batched products take FP16, E8MY or FIX words", i);
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
    all_words += A->n_words;
    all_slices += A->n_slices;
    const int64_t next = (int64_t)start[(size_t)i] + A->n_slices * L;
    PKS_CHECK(next < (int64_t(1) << 32), PKSELL_ERANGE, "too many work units");
    start[(size_t)i + 1] = (uint32_t)next;
    pstart[i + 1] = pstart[i] + (uint32_t)cdiv(A->n_slices, 2);
    pairs_ok &= A->n_words < (int64_t(1) << 30);
  }
  Carver cv(ws);
  Item *dev_items = cv.take<Item>((size_t)count);
  uint32_t *dev_start = cv.take<uint32_t>(2 * ((size_t)count + 1));
  hipStream_t st = as_stream(stream);
  PKS_HIP(hipMemcpyAsync(dev_items, host.data(), sizeof(Item) * (size_t)count,
                         hipMemcpyHostToDevice, st));
  PKS_HIP(hipMemcpyAsync(dev_start, start.data(), sizeof(uint32_t) * 2 * ((size_t)count + 1),
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
  plan->vec4 = aligned ? 1 : 0;
  plan->group = L;
  // k = 1: the batch's average words per lane spread evenly over the fewest
  // groups of at most 8 (at least 4); lane groups keep 8
  const int64_t wl = std::max<int64_t>(1, cdiv(all_words, (int64_t)kWave * std::max<int64_t>(1, all_slices)));
  plan->words_per_group = L == 1 ? (int32_t)std::max<int64_t>(4, cdiv(wl, cdiv(wl, 8))) : kUnroll;
  plan->total_units = start[(size_t)count];
  // a chip-filling grid: as many workgroups as fit on every CU at once
  const int64_t max_waves = (int64_t)cus * resident_blocks(*plan) * (kB / kWave);
  const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(plan->total_units, max_waves));
  plan->units_per_wave = (int32_t)cdiv(std::max<int64_t>(1, plan->total_units), waves);
  plan->waves = (int32_t)waves;
  PKS_CHECK(plan->total_units + 4 * waves < (int64_t(1) << 32), PKSELL_ERANGE, "too many work units");
  plan->items = dev_items;
  plan->unit_start = dev_start;
  // k = 1 forward: the two-slice kernel's work units (slice pairs)
  plan->pair_units = (L == 1 && k == 1 && !transpose && pairs_ok) ? (int32_t)pstart[count] : 0;
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
  const uint32_t cnt = (uint32_t)plan->count, tot = (uint32_t)plan->total_units;
  // 16-byte gathers and stores when every x / y row group is aligned
  const bool v4 = plan->vec4 && !plan->transpose;
  if (uses_pairs(*plan)) {
    const uint32_t pairs = (uint32_t)plan->pair_units;
    const int64_t pg = cdiv(pairs, kPairBlock / kWave);
    const uint32_t *pstart = start + plan->count + 1;
    const int G = plan->words_per_group;
    switch (plan->fmt) {
      case PKSELL_FP16: k_batched_pair_for<PKSELL_FP16>(G)<<<pg, kPairBlock, 0, st>>>(items, pstart, cnt, pairs); break;
      case PKSELL_E8MY: k_batched_pair_for<PKSELL_E8MY>(G)<<<pg, kPairBlock, 0, st>>>(items, pstart, cnt, pairs); break;
      default: k_batched_pair_for<PKSELL_FIX>(G)<<<pg, kPairBlock, 0, st>>>(items, pstart, cnt, pairs); break;
    }
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  if (uses_pipe(*plan)) {
    PKS_CHECK(plan->group == 1 || (v4 && k >= 8 && plan->group == group_size(k)), PKSELL_EINVAL,
              "bad plan");
    switch (plan->fmt) {
      case PKSELL_FP16: k_batched_pipe_for<PKSELL_FP16>(plan->group, plan->words_per_group)<<<grid, kB, 0, st>>>(items, start, cnt, tot, k); break;
      case PKSELL_E8MY: k_batched_pipe_for<PKSELL_E8MY>(plan->group, plan->words_per_group)<<<grid, kB, 0, st>>>(items, start, cnt, tot, k); break;
      default: k_batched_pipe_for<PKSELL_FIX>(plan->group, plan->words_per_group)<<<grid, kB, 0, st>>>(items, start, cnt, tot, k); break;
    }
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  for (int r0 = 0; r0 < k;) {
    const int left = k - r0;
    const int kb = left >= 32 ? 32 : left >= 8 ? 8 : 1;
#define PKS_B(F, KB, T, V) \
  k_batched<F, KB, T, V><<<grid, kB, 0, st>>>(items, start, cnt, tot, k, r0)
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
