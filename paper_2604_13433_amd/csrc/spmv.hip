// PackSELL SpMV y = A_q x (sec. 4.4) and the plain SELL-C-sigma SpMV
// (sec. 3) on gfx950.
//
// One lane per stored row: thread t of the grid owns stored row t, i.e.
// slice t / C, lane t mod C, so a wave64 reads 64 consecutive words of the
// column-major slice per step (fully coalesced; with C = 64 the wave is one
// slice and its loop bounds are scalar).  Each word is unpacked in
// registers, the column is the running sum of deltas from the eq. 4 offset,
// and x is gathered through a buffer resource whose range check returns 0
// past the end (padding of empty rows can point past m).  Accumulation is
// float32, in word order.  Workgroups are remapped so each XCD walks one
// contiguous range of slices and its L2 serves the x window they share.
#include <algorithm>
#include <type_traits>

#include "pair.hpp"

namespace pksell {

namespace {

constexpr int kBlock = kRowBlock;

// KB right-hand sides (columns r0 .. r0+KB-1 of the row-major x / y blocks;
// K1: k == 1, so the x offset is a shift; V4: k and r0 are multiples of 4,
// so x is gathered and y stored four columns at a time; RES: streamed words
// loaded with the default policy, for cache_hint RESIDENT).
template <int FMT, bool CWAVE, int KB, bool K1, bool V4 = false, bool BUF = false,
          bool RES = false>
__global__ __launch_bounds__(kBlock) void k_spmv(SpmvArgs a) {
  Lane ln;
  if (!lane_slice<CWAVE>(a.offset, a.n_slices, a.geo, ln)) return;
  const uint32_t t = ln.t;
  const RowOut ro = row_out<FMT>(a.perm, a.perm_bytes, a.row_exp, t, a.n, a.geo);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, (uint32_t)a.m * (uint32_t)a.k * 4u);
  const uint32_t kx = (uint32_t)a.k * 4u, x0 = (uint32_t)a.r0 * 4u;
  const uint32_t oob = (uint32_t)a.m * kx;  // past the resource: returns 0, no request
  float acc[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) acc[r] = 0.0f;
  const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)a.C;
  if constexpr (V4) {
    packsell_row_v4<FMT, KB>(a.pack + ln.s + ln.l, stride, ln.w, left_offset32(t, a.geo), a.cd,
                             [&](uint32_t c, int g, bool live) {
                               return buffer_load_f32x4(rx, live ? c * kx + x0 + 16u * g : oob);
                             },
                             acc);
  } else if constexpr (BUF) {  // C = 64: streamed words (slice start is wave-uniform)
    static_assert(CWAVE, "streamed words need C = 64");
    const __amdgpu_buffer_rsrc_t rs = slice_words(a.pack + ln.s, ln.w);
    packsell_row_f<FMT, KB>(
        [&](uint32_t j) { return stream_word<word_policy<RES>()>(rs, ln.l, j); }, ln.w,
                            left_offset32(t, a.geo), a.cd,
                            [&](uint32_t c, int r, bool live) {
                              const uint32_t xo = K1 ? (c << 2) : (c * kx + x0 + 4u * r);
                              return buffer_load_f32(rx, live ? xo : oob);
                            },
                            acc);
  } else {
    packsell_row<FMT, KB>(a.pack + ln.s + ln.l, stride, ln.w, left_offset32(t, a.geo), a.cd,
                          [&](uint32_t c, int r, bool live) {
                            const uint32_t xo = K1 ? (c << 2) : (c * kx + x0 + 4u * r);
                            return buffer_load_f32(rx, live ? xo : oob);
                          },
                          acc);
  }
  if (t >= a.n) return;
  if constexpr (FMT == PKSELL_FIX) {
#pragma unroll
    for (int r = 0; r < KB; ++r) acc[r] = ldexpf(acc[r], ro.shift(a.cd));
  }
  const int64_t o = (int64_t)ro.row() * a.k + a.r0;
  if constexpr (V4) {
    f32x4 *yo = reinterpret_cast<f32x4 *>(a.y + o);
#pragma unroll
    for (int g = 0; g < KB / 4; ++g)
      yo[g] = f32x4{acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]};
  } else {
#pragma unroll
    for (int r = 0; r < KB; ++r) a.y[o + r] = acc[r];
  }
}

// C = 64, k a multiple of 4 and >= 8, 16-byte aligned x and y: lane groups
// of L lanes per row (group_lane), one wave per (slice, h) with h < L.
template <int FMT, int L>
__global__ __launch_bounds__(kBlock) void k_spmv_group(SpmvArgs a) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wv = __builtin_amdgcn_readfirstlane(b * (kBlock / kWave) + threadIdx.x / kWave);
  const uint32_t ks = wv / L, h = wv % L;
  if (ks >= a.n_slices) return;
  const GroupLane g = group_lane<L>(h, threadIdx.x & (kWave - 1), (uint32_t)a.k >> 2);
  const uint32_t t = ks * kWave + g.l;
  const RowOut ro = row_out<FMT>(a.perm, a.perm_bytes, a.row_exp, g.live ? t : a.n, a.n, a.geo);
  const int64_t s = a.offset[ks];
  const uint32_t w = (uint32_t)((a.offset[ks + 1] - s) >> 6);
  const uint32_t kx = (uint32_t)a.k * 4u, xq = 16u * g.q;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * kx);
  const uint32_t oob = a.m * kx;
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  // the L waves of a slice share its words: plain (not nontemporal) loads
  packsell_row_v4<FMT, 4, false>(a.pack + s + g.l, kWave, w, left_offset32(t, a.geo), a.cd,
                                 [&](uint32_t c, int, bool live) {
                                   return buffer_load_f32x4(rx, live ? c * kx + xq : oob);
                                 },
                                 acc);
  if (t >= a.n || !g.live) return;
  if constexpr (FMT == PKSELL_FIX) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = ldexpf(acc[r], ro.shift(a.cd));
  }
  const int64_t o = (int64_t)ro.row() * a.k + 4 * g.q;
  // streaming (nontemporal) store, as for the single-vector results
  __builtin_nontemporal_store(f32x4{acc[0], acc[1], acc[2], acc[3]},
                              reinterpret_cast<f32x4 *>(a.y + o));
}

// C = 64, k = 1: each wave walks two consecutive slices together, so the
// words (and then the gathers) of both are in flight at once -- more bytes
// per wave between its dependent loads (offsets, words, x) than one slice
// gives.  Same arithmetic, in the same word order per row, as k_spmv.
// Words per group for the two-slice kernels: the average words per lane w
// (rounded up) spread evenly over the fewest groups of at most 8, i.e.
// ceil(w / ceil(w / 8)), at least 2.
inline int pair_group(int64_t words, int64_t n_slices) {
  const int64_t w = std::max<int64_t>(1, cdiv(words, (int64_t)kWave * (n_slices > 0 ? n_slices : 1)));
  return (int)std::max<int64_t>(2, cdiv(w, cdiv(w, 8)));
}

template <int FMT, bool BUF, bool IMPL, int G = kUnroll, bool RES = false>
__global__ __launch_bounds__(kPairBlock) void k_spmv_pair(SpmvArgs a) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(b * (kPairBlock / kWave) + threadIdx.x / kWave);
  const uint32_t k0 = wave * 2;
  if (k0 >= a.n_slices) return;
  pair_product<FMT, BUF, IMPL, G, RES>(a, k0, threadIdx.x & (kWave - 1));
}

// Wide-slice splitting (C = 64, k = 1): one wave per work unit {slice,
// chunk, chunks, base}.  A unit of an unsplit slice (chunks == 1) is the
// whole slice and stores y; a chunk of a split slice starts from the column
// recorded by the encoder for that chunk and stores its float32 sum in
// ``partial``.  k_combine_chunks then adds each split slice's chunk sums in
// chunk order, so the result is deterministic; it differs from the unsplit
// sum only in rounding order.
struct UnitArgs {
  const uint32_t *units;
  const uint32_t *splits;
  const uint32_t *ckpt;
  float *partial;
  uint32_t n_units, n_split_slices, J;
};

template <int FMT, bool BUF>
__global__ __launch_bounds__(kBlock) void k_spmv_units(SpmvArgs a, UnitArgs u) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t unit = __builtin_amdgcn_readfirstlane(b * (kBlock / kWave) + threadIdx.x / kWave);
  if (unit >= u.n_units) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t k = u.units[4 * unit], c = u.units[4 * unit + 1];
  const uint32_t chunks = u.units[4 * unit + 2], base = u.units[4 * unit + 3];
  const int64_t s = a.offset[k];
  const uint32_t w = (uint32_t)((a.offset[k + 1] - s) >> 6);
  const uint32_t j0 = c * u.J;
  const uint32_t wl = chunks == 1 ? w : min(u.J, w - j0);
  const uint32_t t = k * kWave + lane;
  const RowOut ro = row_out<FMT>(a.perm, a.perm_bytes, a.row_exp, chunks == 1 ? t : a.n, a.n,
                                 a.geo);
  const uint32_t c0 = chunks == 1 ? left_offset32(t, a.geo) : u.ckpt[(base + c) * kWave + lane];
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * 4u);
  float acc[1] = {0.0f};
  const uint32_t *first = a.pack + s + (int64_t)j0 * kWave;
  const __amdgpu_buffer_rsrc_t rs = slice_words(first, wl);
  packsell_row_f<FMT, 1>(
      [&](uint32_t j) {
        return BUF ? stream_word(rs, lane, j) : __builtin_nontemporal_load(first + lane + j * kWave);
      },
      wl, c0, a.cd,
      [&](uint32_t col, int, bool live) { return buffer_load_f32(rx, live ? col << 2 : a.m * 4u); },
      acc);
  if (chunks > 1) {
    u.partial[(base + c) * kWave + lane] = acc[0];
    return;
  }
  if (t >= a.n) return;
  float r = acc[0];
  if constexpr (FMT == PKSELL_FIX) r = ldexpf(r, ro.shift(a.cd));
  a.y[ro.row()] = r;
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_combine_chunks(SpmvArgs a, UnitArgs u) {
  const uint32_t sp = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);
  if (sp >= u.n_split_slices) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t k = u.splits[4 * sp], base = u.splits[4 * sp + 1], chunks = u.splits[4 * sp + 2];
  const uint32_t t = k * kWave + lane;
  if (t >= a.n) return;
  const RowOut ro = row_out<FMT>(a.perm, a.perm_bytes, a.row_exp, t, a.n, a.geo);
  // eight chunk sums in flight at a time, added in chunk order
  float r = 0.0f;
  for (uint32_t c0 = 0; c0 < chunks; c0 += 8) {
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = c0 + i < chunks ? u.partial[(base + c0 + i) * kWave + lane] : 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (c0 + i < chunks) r += v[i];
  }
  if constexpr (FMT == PKSELL_FIX) r = ldexpf(r, ro.shift(a.cd));
  a.y[ro.row()] = r;
}

// Word-by-word decode: the column reached at each word position and the
// decoded value (0 for flag-0 words, FIX times the row scale).
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_decode(SpmvArgs a, int32_t *cols, float *vals) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= a.n) return;
  const uint32_t k = t >> a.geo.c_log2, l = t - (k << a.geo.c_log2);
  const int64_t s = a.offset[k];
  const int64_t w = (a.offset[k + 1] - s) >> a.geo.c_log2;
  uint32_t c = left_offset32(t, a.geo);
  for (int64_t j = 0; j < w; ++j) {
    const int64_t p = s + j * a.C + l;
    Unpacked u = unpack(a.pack[p], a.cd);
    c += u.delta;
    cols[p] = (int32_t)c;
    float v = decode_value<FMT>(u.vbits);
    if constexpr (FMT == PKSELL_FIX) v = ldexpf(v, (int)a.row_exp[t] - (a.cd.D + 1));
    vals[p] = v;
  }
}

__global__ void k_fill_zero_f32(float *p, int64_t len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = 0.0f;
}

template <typename T>
__global__ void k_fill_zero(T *p, int64_t len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = T(0);
}

// Value type tag of paired SELL slots: one uint64 per slot, the column in
// the low 4 bytes and the float32 value bits in the high 4.
struct Paired {
  uint64_t u;
};
template <typename VT>
constexpr bool kPairedVT = std::is_same<VT, Paired>::value;

// One fused multiply-add in the vector type: SELL sums products exactly as
// the PackSELL kernels do (fmaf in slot order), so half-value SELL and FP16
// words give bit-identical results on the same values.
__device__ inline float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return fma(a, b, c); }

// Plain SELL-C-sigma SpMV (sec. 3): the float32 / float64 / half-value
// comparator, with the same lane mapping and batched loads as the PackSELL
// kernel.  Values are VT (T, or half with T = float), vectors and sums T.
// BUF (C = 64 and arrays below 4 GiB): columns and values are streamed
// through per-slice buffer resources, as the PackSELL words are (RES: with
// the default policy, for cache_hint RESIDENT).
template <typename T, bool CWAVE, bool BUF = false, typename VT = T, int G = kUnroll,
          bool RES = false>
__global__ __launch_bounds__(kBlock) void k_sell_spmv(const int64_t *__restrict__ offset,
                                                      const int32_t *__restrict__ scol,
                                                      const VT *__restrict__ sval, const void *perm,
                                                      int32_t perm_bytes, const T *__restrict__ x,
                                                      T *__restrict__ y, uint32_t n, uint32_t m,
                                                      uint32_t n_slices, int32_t C, RowGeo g) {
  Lane ln;
  if (!lane_slice<CWAVE>(offset, n_slices, g, ln)) return;
  const uint32_t t = ln.t, w = ln.w;
  const RowOut dst = row_out(perm, perm_bytes, t, n, g);
  const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)C;
  T acc = 0;
  if constexpr (BUF) {
    // Branch-free, as the two-slice kernel: slots past the slice's width
    // read 0 from its resources (no request), their gathers point past x
    // (0, no request) and their products add 0 exactly, so each gather
    // goes out as soon as its slot has arrived.
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(scol + ln.s, kPairedVT<VT> ? 0u : w * 256u);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc(sval + ln.s, w * kWave * (uint32_t)sizeof(VT));
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(x, m * (uint32_t)sizeof(T));
    const uint32_t oob = m * (uint32_t)sizeof(T);
    constexpr int P = word_policy<RES>();
    for (uint32_t j = 0; j < w; j += G) {
      T vv[G], xv[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        int32_t cc;
        if constexpr (kPairedVT<VT>) {  // one 8-byte load per slot
          const uint64_t u = stream_elem<uint64_t, P>(rv, ln.l, j + q);
          cc = (int32_t)(uint32_t)u;
          vv[q] = __uint_as_float((uint32_t)(u >> 32));
        } else {
          cc = stream_elem<int32_t, P>(rc, ln.l, j + q);
          vv[q] = (T)stream_elem<VT, P>(rv, ln.l, j + q);
        }
        const uint32_t o = j + q < w ? (uint32_t)cc * (uint32_t)sizeof(T) : oob;
        if constexpr (sizeof(T) == 8)
          xv[q] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rx, o, 0, 0));
        else
          xv[q] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rx, o, 0, 0));
      }
#pragma unroll
      for (int q = 0; q < G; ++q) acc = fma_t(vv[q], xv[q], acc);
    }
    if (t < n) y[dst.row()] = acc;
    return;
  }
  const int32_t *pc = kPairedVT<VT> ? nullptr : scol + ln.s + ln.l;
  const VT *pv = sval + ln.s + ln.l;
  for (uint32_t j = 0; j < w; j += G) {
    int32_t cc[G];
    T vv[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const bool in = j + q < w;
      if constexpr (kPairedVT<VT>) {  // one 8-byte load per slot
        uint64_t u = 0;
        if (in) u = __builtin_nontemporal_load(&pv[(j + q) * stride].u);
        cc[q] = (int32_t)(uint32_t)u;
        vv[q] = __uint_as_float((uint32_t)(u >> 32));
      } else {
        cc[q] = in ? __builtin_nontemporal_load(pc + (j + q) * stride) : 0;
        vv[q] = in ? (T)__builtin_nontemporal_load(pv + (j + q) * stride) : T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (j + q < w) acc = fma_t(vv[q], x[cc[q]], acc);
  }
  if (t >= n) return;
  y[dst.row()] = acc;
}

// SELL with C = 64 and streamed slots, two slices per wave in 128-thread
// workgroups: the comparator gets the same structure as k_spmv_pair.
template <typename T, bool IMPL, typename VT = T, int G = kUnroll, bool RES = false>
__global__ __launch_bounds__(kPairBlock) void k_sell_pair(const int64_t *__restrict__ offset,
                                                         const int32_t *__restrict__ scol,
                                                         const VT *__restrict__ sval,
                                                         const void *perm, int32_t perm_bytes,
                                                         const T *__restrict__ x,
                                                         T *__restrict__ y, uint32_t n,
                                                         uint32_t m, uint32_t n_slices,
                                                         RowGeo g) {
  static_assert(sizeof(T) == 4, "the two-slice SELL kernel serves float32 vectors");
  constexpr int S = 2;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(b * (kPairBlock / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t k0 = wave * S;
  if (k0 >= n_slices) return;
  RowOut dst[S];  // implicit order: destinations read up front
  if constexpr (IMPL) {
#pragma unroll
    for (int i = 0; i < S; ++i) dst[i] = row_out(perm, perm_bytes, (k0 + i) * kWave + lane, n, g);
  }
  int64_t off[S + 1];
#pragma unroll
  for (int i = 0; i <= S; ++i) off[i] = offset[min(k0 + i, n_slices)];
  uint32_t w[S], wm = 0;
  __amdgpu_buffer_rsrc_t rc[S], rv[S];
  T acc[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    w[i] = (uint32_t)((off[i + 1] - off[i]) >> 6);
    wm = max(wm, w[i]);
    rc[i] = kPairedVT<VT> ? make_rsrc(scol, 0u) : make_rsrc(scol + off[i], w[i] * 256u);
    rv[i] = make_rsrc(sval + off[i], w[i] * kWave * (uint32_t)sizeof(VT));
    acc[i] = T(0);
  }
  // Same structure as k_spmv_pair: branch-free streamed loads (slots past
  // a slice's width read 0), gathers through a range-checked resource
  // (padding points past x: 0, no request; its product adds 0 exactly), and
  // in the last group each slice's sum stored before the next slice's
  // products wait on their gathers.
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(x, m * 4u);
  const uint32_t oob = m * 4u;
  auto group = [&](uint32_t j, T (&vv)[S][G], T (&xv)[S][G]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int q = 0; q < G; ++q) {
        int32_t cc;
        if constexpr (kPairedVT<VT>) {  // one 8-byte load per slot
          const uint64_t u = stream_elem<uint64_t, word_policy<RES>()>(rv[i], lane, j + q);
          cc = (int32_t)(uint32_t)u;
          vv[i][q] = __uint_as_float((uint32_t)(u >> 32));
        } else {
          cc = stream_elem<int32_t, word_policy<RES>()>(rc[i], lane, j + q);
          vv[i][q] = (T)stream_elem<VT, word_policy<RES>()>(rv[i], lane, j + q);
        }
        const uint32_t o = j + q < w[i] ? (uint32_t)cc * 4u : oob;
        xv[i][q] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rx, o, 0, 0));
      }
  };
  uint32_t j = 0;
  for (; j + G < wm; j += G) {
    T vv[S][G], xv[S][G];
    group(j, vv, xv);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int q = 0; q < G; ++q) acc[i] = fma_t(vv[i][q], xv[i][q], acc[i]);
  }
  T vv[S][G], xv[S][G];
  group(j, vv, xv);
#pragma unroll
  for (int i = 0; i < S; ++i) {
#pragma unroll
    for (int q = 0; q < G; ++q) acc[i] = fma_t(vv[i][q], xv[i][q], acc[i]);
    const uint32_t t = (k0 + i) * kWave + lane;
    const uint32_t row = (k0 + i < n_slices && t < n) ? (IMPL ? dst[i].row() : t) : n;
    store_result(y, n, row, acc[i]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---- 64-bit words (E11MY) in float64 -------------------------------------------

struct Spmv64Args {
  const uint64_t *pack;
  const int64_t *offset;
  const void *perm;
  const double *x;
  double *y;
  uint32_t n, m, n_slices;
  int32_t C, perm_bytes;
  RowGeo geo;
  uint32_t dmask;  // the flag-1 delta after >> 1 (columns < 2^30, so at most 31 bits)
  uint64_t vmask;  // ~(2^(D+1) - 1): the value field
};

// The sec. 4.4 loop for 64-bit words: groups of eight words in flight, the
// delta from the low half (every delta is below 2^30), the value field as a
// float64, gathers of x in float64 (flag-0 words past the resource), float64
// FMA in word order.  BUF (C = 64, words below 4 GiB): words streamed
// through a buffer resource on the slice, as in the 32-bit kernels.
template <bool CWAVE, bool BUF, int G = kUnroll>
__global__ __launch_bounds__(kBlock) void k_spmv64(Spmv64Args a) {
  Lane ln;
  if (!lane_slice<CWAVE>(a.offset, a.n_slices, a.geo, ln)) return;
  const uint32_t t = ln.t, w = ln.w;
  const RowOut dst = row_out(a.perm, a.perm_bytes, t, a.n, a.geo);
  const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)a.C;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * 8u);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(BUF ? a.pack + ln.s : a.pack, BUF ? w * 512u : 0u);
  const uint64_t *P = a.pack + ln.s + ln.l;
  uint32_t c = left_offset32(t, a.geo);
  double acc = 0.0;
  for (uint32_t j = 0; j < w; j += G) {
    uint64_t p[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      uint64_t v = 0ull;
      if (j + q < w) {
        if constexpr (BUF)
          v = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(
                                               rs, (ln.l + (j + q) * kWave) * 8u, 0, kStreamPolicy));
        else
          v = __builtin_nontemporal_load(P + (j + q) * stride);
      }
      p[q] = v;
    }
    uint32_t off[G];
    double val[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const uint32_t lo = (uint32_t)p[q];
      const bool flag = lo & 1u;
      c += flag ? ((lo >> 1) & a.dmask) : (uint32_t)(p[q] >> 1);
      off[q] = flag ? c * 8u : a.m * 8u;
      val[q] = flag ? __builtin_bit_cast(double, p[q] & a.vmask) : 0.0;
    }
    double xv[G];
#pragma unroll
    for (int q = 0; q < G; ++q)
      xv[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, off[q], 0, 0));
#pragma unroll
    for (int q = 0; q < G; ++q) acc = fma(val[q], xv[q], acc);
  }
  if (t >= a.n) return;
  a.y[dst.row()] = acc;
}

// k right-hand sides in float64 (x m x k and y n x k, row-major): columns
// r0 .. r0 + KB - 1 per launch, four words per group, each column's
// products summed in word order as for k = 1.
template <bool CWAVE, int KB>
__global__ __launch_bounds__(kBlock) void k_spmv64k(Spmv64Args a, uint32_t k, uint32_t r0) {
  constexpr int G = 4;
  Lane ln;
  if (!lane_slice<CWAVE>(a.offset, a.n_slices, a.geo, ln)) return;
  const uint32_t t = ln.t, w = ln.w;
  const RowOut dst = row_out(a.perm, a.perm_bytes, t, a.n, a.geo);
  const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)a.C;
  const uint32_t kx = k * 8u, x0 = r0 * 8u;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * kx);
  const uint32_t oob = a.m * kx;  // past the resource: 0, no request
  const uint64_t *P = a.pack + ln.s + ln.l;
  uint32_t c = left_offset32(t, a.geo);
  double acc[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) acc[r] = 0.0;
  for (uint32_t j = 0; j < w; j += G) {
    uint64_t p[G];
#pragma unroll
    for (int q = 0; q < G; ++q) p[q] = j + q < w ? __builtin_nontemporal_load(P + (j + q) * stride) : 0ull;
    uint32_t off[G];
    double val[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const uint32_t lo = (uint32_t)p[q];
      const bool flag = lo & 1u;
      c += flag ? ((lo >> 1) & a.dmask) : (uint32_t)(p[q] >> 1);
      off[q] = flag ? c * kx + x0 : oob;
      val[q] = flag ? __builtin_bit_cast(double, p[q] & a.vmask) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < G; ++q)
#pragma unroll
      for (int r = 0; r < KB; ++r)
        acc[r] = fma(val[q],
                     __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                    rx, off[q] == oob ? oob : off[q] + 8u * r, 0, 0)),
                     acc[r]);
  }
  if (t >= a.n) return;
  double *yo = a.y + (int64_t)dst.row() * k + r0;
#pragma unroll
  for (int r = 0; r < KB; ++r) yo[r] = acc[r];
}

SpmvArgs make_args(const pksell_matrix *A, const float *x, float *y, int64_t k) {
  SpmvArgs a;
  a.pack = A->pack;
  a.offset = A->offset;
  a.perm = A->perm_mode == PKSELL_IMPLICIT ? A->perm : nullptr;
  a.row_exp = A->row_exp;
  a.x = x;
  a.y = y;
  a.n = (uint32_t)A->n;
  a.m = (uint32_t)A->m;
  a.n_slices = (uint32_t)A->n_slices;
  a.C = A->C;
  a.geo = make_geo(A->sigma, A->k_left, A->C);
  a.perm_bytes = A->perm_bytes;
  a.k = (int32_t)k;
  a.r0 = 0;
  a.cd = make_codec(A->D);
  a.group = pair_group(A->n_words, A->n_slices);
  a.resident = A->cache_hint == PKSELL_CACHE_RESIDENT;
  return a;
}

// The streamed word loads address a slice through 32-bit byte offsets.
bool stream_words_ok(const pksell_matrix *A) { return A->n_words < (int64_t(1) << 30); }

int check_matrix(const pksell_matrix *A) {
  PKS_CHECK(A, PKSELL_EINVAL, "null matrix");
  PKS_CHECK(A->fmt != PKSELL_E11MY, PKSELL_EINVAL,
            "64-bit words (E11MY): use pksell_spmv_f64, the only entry point for them");
  PKS_CHECK(!is_w16(A->fmt), PKSELL_EINVAL,
            "16-bit words (E5MY, FIX16): pksell_spmv with k = 1 is their only product");
  PKS_CHECK(A->n == 0 || (A->offset && (A->n_words == 0 || A->pack)), PKSELL_EINVAL,
            "matrix arrays not set");
  PKS_CHECK(A->perm_mode != PKSELL_IMPLICIT || A->n == 0 || A->perm, PKSELL_EINVAL,
            "implicit mode needs perm");
  PKS_CHECK(A->fmt != PKSELL_FIX || A->n == 0 || A->row_exp, PKSELL_EINVAL, "FIX needs row_exp");
  PKS_CHECK(A->fmt >= PKSELL_FP16 && A->fmt <= PKSELL_FIX, PKSELL_EINVAL, "bad fmt");
  return PKSELL_OK;
}

// Two slices per wave pay off for narrow slices (the stencils: 7 words per
// lane on the 128^3 and 256^3 Laplacians); for wide ones (81 on the block
// stencil, thousands on power-law rows) one slice per wave ran faster, for
// PackSELL and SELL alike.
inline bool pair_slices(int64_t words, int64_t n_slices) {
  return n_slices > 0 && words <= 16 * (int64_t)kWave * n_slices;
}

// The same rule for the one-slice-per-wave kernels, at least 4 words.
inline int slice_group(int64_t words, int64_t n_slices) {
  return std::max(4, pair_group(words, n_slices));
}

// Runs the launch statement given after G (which names the group size GG)
// with GG = G in [4, 8].
#define PKS_GROUP(G, ...)                                  \
  switch (G) {                                             \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;  \
    case 5: { constexpr int GG = 5; __VA_ARGS__; } break;  \
    case 6: { constexpr int GG = 6; __VA_ARGS__; } break;  \
    case 7: { constexpr int GG = 7; __VA_ARGS__; } break;  \
    default: { constexpr int GG = 8; __VA_ARGS__; } break; \
  }

template <int FMT, bool IMPL, bool RES>
void launch_pair_res(const SpmvArgs &a, int G, int64_t pg, hipStream_t st) {
  switch (G) {
    case 2: k_spmv_pair<FMT, true, IMPL, 2, RES><<<pg, kPairBlock, 0, st>>>(a); break;
    case 3: k_spmv_pair<FMT, true, IMPL, 3, RES><<<pg, kPairBlock, 0, st>>>(a); break;
    case 4: k_spmv_pair<FMT, true, IMPL, 4, RES><<<pg, kPairBlock, 0, st>>>(a); break;
    case 5: k_spmv_pair<FMT, true, IMPL, 5, RES><<<pg, kPairBlock, 0, st>>>(a); break;
    case 6: k_spmv_pair<FMT, true, IMPL, 6, RES><<<pg, kPairBlock, 0, st>>>(a); break;
    case 7: k_spmv_pair<FMT, true, IMPL, 7, RES><<<pg, kPairBlock, 0, st>>>(a); break;
    default: k_spmv_pair<FMT, true, IMPL, 8, RES><<<pg, kPairBlock, 0, st>>>(a); break;
  }
}

template <int FMT, bool IMPL>
void launch_pair(const SpmvArgs &a, int G, int64_t pg, hipStream_t st) {
  if (a.resident)
    launch_pair_res<FMT, IMPL, true>(a, G, pg, st);
  else
    launch_pair_res<FMT, IMPL, false>(a, G, pg, st);
}

template <int FMT, bool CW>
int launch_fmt_cw(const SpmvArgs &base, int64_t grid, int64_t k, bool buf, bool pair,
                  hipStream_t st) {
  if (k == 1) {
    if constexpr (CW) {
      if (!pair) {
        if (buf && base.resident)
          k_spmv<FMT, CW, 1, true, false, true, true><<<grid, kBlock, 0, st>>>(base);
        else if (buf)
          k_spmv<FMT, CW, 1, true, false, true><<<grid, kBlock, 0, st>>>(base);
        else
          k_spmv<FMT, CW, 1, true><<<grid, kBlock, 0, st>>>(base);
        PKS_LAUNCHED();
        return PKSELL_OK;
      }
      const int64_t pg = cdiv(cdiv(base.n_slices, 2), kPairBlock / kWave);
      const bool impl = base.perm != nullptr;
      const int G = base.group;
      if (buf && impl) launch_pair<FMT, true>(base, G, pg, st);
      else if (buf) launch_pair<FMT, false>(base, G, pg, st);
      else if (impl) k_spmv_pair<FMT, false, true><<<pg, kPairBlock, 0, st>>>(base);
      else k_spmv_pair<FMT, false, false><<<pg, kPairBlock, 0, st>>>(base);
    } else {
      k_spmv<FMT, CW, 1, true><<<grid, kBlock, 0, st>>>(base);
    }
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  int64_t r0 = 0;
  const bool aligned = ((reinterpret_cast<uintptr_t>(base.x) | reinterpret_cast<uintptr_t>(base.y)) & 15) == 0;
  if constexpr (CW) {
    if (k % 4 == 0 && k >= 8 && aligned) {  // lane groups: one pass for every k
      const int L = group_size(k);
      const int64_t g = cdiv((int64_t)base.n_slices * L, kBlock / kWave);
      switch (L) {
        case 2: k_spmv_group<FMT, 2><<<g, kBlock, 0, st>>>(base); break;
        case 4: k_spmv_group<FMT, 4><<<g, kBlock, 0, st>>>(base); break;
        case 8: k_spmv_group<FMT, 8><<<g, kBlock, 0, st>>>(base); break;
        default: k_spmv_group<FMT, 16><<<g, kBlock, 0, st>>>(base); break;
      }
      PKS_LAUNCHED();
      return PKSELL_OK;
    }
  }
  if (k % 4 == 0 && aligned) {  // 16-byte gathers and stores
    while (r0 < k) {
      SpmvArgs a = base;
      a.r0 = (int32_t)r0;
      if (k - r0 >= 8) {
        k_spmv<FMT, CW, 8, false, true><<<grid, kBlock, 0, st>>>(a);
        r0 += 8;
      } else {
        k_spmv<FMT, CW, 4, false, true><<<grid, kBlock, 0, st>>>(a);
        r0 += 4;
      }
      PKS_LAUNCHED();
    }
    return PKSELL_OK;
  }
  while (r0 < k) {
    SpmvArgs a = base;
    a.r0 = (int32_t)r0;
    int64_t left = k - r0;
    if (left >= 8) {
      k_spmv<FMT, CW, 8, false><<<grid, kBlock, 0, st>>>(a);
      r0 += 8;
    } else if (left >= 4) {
      k_spmv<FMT, CW, 4, false><<<grid, kBlock, 0, st>>>(a);
      r0 += 4;
    } else if (left >= 2) {
      k_spmv<FMT, CW, 2, false><<<grid, kBlock, 0, st>>>(a);
      r0 += 2;
    } else {
      k_spmv<FMT, CW, 1, false><<<grid, kBlock, 0, st>>>(a);
      r0 += 1;
    }
    PKS_LAUNCHED();
  }
  return PKSELL_OK;
}

template <int FMT>
int launch_fmt(const SpmvArgs &a, int64_t grid, int64_t k, int32_t C, bool buf, bool pair,
               hipStream_t st) {
  return C == kWave ? launch_fmt_cw<FMT, true>(a, grid, k, buf, pair, st)
                    : launch_fmt_cw<FMT, false>(a, grid, k, buf, pair, st);
}

template <int FMT>
int launch_units(const SpmvArgs &a, const UnitArgs &u, bool buf, hipStream_t st) {
  constexpr int wpb = kBlock / kWave;
  if (buf)
    k_spmv_units<FMT, true><<<cdiv(u.n_units, wpb), kBlock, 0, st>>>(a, u);
  else
    k_spmv_units<FMT, false><<<cdiv(u.n_units, wpb), kBlock, 0, st>>>(a, u);
  PKS_LAUNCHED();
  k_combine_chunks<FMT><<<cdiv(u.n_split_slices, wpb), kBlock, 0, st>>>(a, u);
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // namespace

// Zero-fills float32 device memory with a kernel (safe inside captured graphs).
int zero_f32(float *p, int64_t len, hipStream_t st) {
  if (len <= 0) return PKSELL_OK;
  k_fill_zero_f32<<<cdiv(len, kBlock), kBlock, 0, st>>>(p, len);
  PKS_LAUNCHED();
  return PKSELL_OK;
}

int check_matrix_public(const pksell_matrix *A) { return check_matrix(A); }

// The two-slice SELL comparator with G slots per group, as k_spmv_pair.
template <bool IMPL, typename VT>
void launch_sell_pair(const pksell_sell *S, const void *x, void *y, const void *perm, int G,
                      int64_t pg, hipStream_t st) {
  const VT *val = static_cast<const VT *>(S->val);
  const float *xf = static_cast<const float *>(x);
  float *yf = static_cast<float *>(y);
  const RowGeo g = make_geo(S->sigma, 0, S->C);
  const uint32_t n = (uint32_t)S->n, ns = (uint32_t)S->n_slices;
  const bool res = S->cache_hint == PKSELL_CACHE_RESIDENT;
#define PKS_SP1(GG, RES)                                                                       \
  k_sell_pair<float, IMPL, VT, GG, RES><<<pg, kPairBlock, 0, st>>>(S->offset, S->col, val, perm, \
                                                                   S->perm_bytes, xf, yf, n,     \
                                                                   (uint32_t)S->m, ns, g)
#define PKS_SP(GG) (res ? PKS_SP1(GG, true) : PKS_SP1(GG, false))
  switch (G) {
    case 2: PKS_SP(2); break;
    case 3: PKS_SP(3); break;
    case 4: PKS_SP(4); break;
    case 5: PKS_SP(5); break;
    case 6: PKS_SP(6); break;
    case 7: PKS_SP(7); break;
    default: PKS_SP(8); break;
  }
#undef PKS_SP
#undef PKS_SP1
}

// 16-bit words (spmv16.hip).
int spmv16(const pksell_matrix *A, const float *x, float *y, int64_t k, hipStream_t st);
int spmv_chunks(const pksell_matrix *A, const float *x, float *y, int64_t k, hipStream_t st);

// The chunk plan of a CSR-packed matrix serves k = 1, 2 and 4; its k = 4
// form gathers 16-byte x rows, so a misaligned x takes the one-row-slice
// product instead.
bool chunk_path(const pksell_matrix *A, const float *x, int64_t k) {
  const bool x16 = ((uintptr_t)x & 15) == 0;
  return (k == 1 || k == 2 || (k == 4 && x16)) && A->C == 1 && A->split_words > 0;
}

// Split wide slices run one work unit per wave for single-vector products.
bool split_path(const pksell_matrix *A, int64_t k) {
  return k == 1 && A->C == kWave && A->split_words > 0 && A->n_split_units > 0;
}

// Floats of A->partial that pksell_spmv(A, x, ., k) uses as scratch: the
// pieces of rows that cross chunk edges (chunk plan) or the per-chunk sums
// of split slices; 0 when the product needs none.
int64_t spmv_partial_floats(const pksell_matrix *A, const float *x, int64_t k) {
  if (!A || is_w16(A->fmt) || A->n == 0 || A->m == 0) return 0;
  if (chunk_path(A, x, k)) return (2 * k + 1) * A->n_units;
  if (split_path(A, k)) return kWave * A->n_split_units;
  return 0;
}

}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_spmv(const pksell_matrix *A, const float *x, float *y, int64_t k, void *stream) {
  if (A && is_w16(A->fmt)) return spmv16(A, x, y, k, as_stream(stream));
  int rc = check_matrix(A);
  if (rc) return rc;
  PKS_CHECK(k >= 1 && k <= 64, PKSELL_EINVAL, "k must be in [1, 64]");
  PKS_CHECK(A->m * k * 4 < (int64_t(1) << 32), PKSELL_ERANGE, "m * k * 4 must be below 2^32");
  PKS_CHECK(A->n == 0 || y, PKSELL_EINVAL, "null y");
  hipStream_t st = as_stream(stream);
  if (A->n == 0) return PKSELL_OK;
  if (A->m == 0) return zero_f32(y, A->n * k, st);
  PKS_CHECK(x, PKSELL_EINVAL, "null x");
  if (chunk_path(A, x, k)) return spmv_chunks(A, x, y, k, st);
  SpmvArgs a = make_args(A, x, y, k);
  if (split_path(A, k)) {
    PKS_CHECK(A->units && A->splits && A->ckpt && A->partial, PKSELL_EINVAL,
              "split slices need units, splits, ckpt and partial");
    PKS_CHECK(A->n_units < (int64_t(1) << 31) && A->n_split_units * kWave < (int64_t(1) << 32),
              PKSELL_ERANGE, "too many work units");
    UnitArgs u{A->units, A->splits, A->ckpt, A->partial, (uint32_t)A->n_units,
               (uint32_t)A->n_split_slices, (uint32_t)A->split_words};
    const bool buf = stream_words_ok(A);
    switch (A->fmt) {
      case PKSELL_FP16: return launch_units<PKSELL_FP16>(a, u, buf, st);
      case PKSELL_E8MY: return launch_units<PKSELL_E8MY>(a, u, buf, st);
      default: return launch_units<PKSELL_FIX>(a, u, buf, st);
    }
  }
  const int64_t grid = cdiv(A->n_slices * A->C, kBlock);
  const bool buf = stream_words_ok(A);
  const bool pair = pair_slices(A->n_words, A->n_slices);
  switch (A->fmt) {
    case PKSELL_FP16: return launch_fmt<PKSELL_FP16>(a, grid, k, A->C, buf, pair, st);
    case PKSELL_E8MY: return launch_fmt<PKSELL_E8MY>(a, grid, k, A->C, buf, pair, st);
    default: return launch_fmt<PKSELL_FIX>(a, grid, k, A->C, buf, pair, st);
  }
}

int pksell_spmv_f64(const pksell_matrix *A, const double *x, double *y, int64_t k,
                    void *stream) {
  PKS_CHECK(A, PKSELL_EINVAL, "null matrix");
  PKS_CHECK(A->fmt == PKSELL_E11MY, PKSELL_EINVAL, "pksell_spmv_f64 needs fmt E11MY");
  PKS_CHECK(A->n == 0 || (A->offset && (A->n_words == 0 || A->pack)), PKSELL_EINVAL,
            "matrix arrays not set");
  PKS_CHECK(A->perm_mode != PKSELL_IMPLICIT || A->n == 0 || A->perm, PKSELL_EINVAL,
            "implicit mode needs perm");
  PKS_CHECK(k >= 1 && k <= 64, PKSELL_EINVAL, "k must be in [1, 64]");
  PKS_CHECK(A->m * k < (int64_t(1) << 29), PKSELL_ERANGE, "m * k must be below 2^29 (8-byte x)");
  PKS_CHECK(A->n == 0 || y, PKSELL_EINVAL, "null y");
  hipStream_t st = as_stream(stream);
  if (A->n == 0) return PKSELL_OK;
  if (A->m == 0) {
    k_fill_zero<double><<<cdiv(A->n * k, kBlock), kBlock, 0, st>>>(y, A->n * k);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  PKS_CHECK(x, PKSELL_EINVAL, "null x");
  Spmv64Args a;
  a.pack = reinterpret_cast<const uint64_t *>(A->pack);
  a.offset = A->offset;
  a.perm = A->perm_mode == PKSELL_IMPLICIT ? A->perm : nullptr;
  a.x = x;
  a.y = y;
  a.n = (uint32_t)A->n;
  a.m = (uint32_t)A->m;
  a.n_slices = (uint32_t)A->n_slices;
  a.C = A->C;
  a.perm_bytes = A->perm_bytes;
  a.geo = make_geo(A->sigma, A->k_left, A->C);
  a.dmask = A->D >= 31 ? 0x7FFFFFFFu : (1u << A->D) - 1u;
  a.vmask = ~((2ull << A->D) - 1ull);
  const int64_t grid = cdiv(A->n_slices * A->C, kBlock);
  if (k > 1) {  // passes of four columns (then two, one)
    const bool cw = A->C == kWave;
    for (int64_t r0 = 0; r0 < k;) {
      const int64_t left = k - r0;
      const uint32_t kk = (uint32_t)k, r = (uint32_t)r0;
      if (left >= 4) {
        if (cw) k_spmv64k<true, 4><<<grid, kBlock, 0, st>>>(a, kk, r);
        else k_spmv64k<false, 4><<<grid, kBlock, 0, st>>>(a, kk, r);
        r0 += 4;
      } else if (left >= 2) {
        if (cw) k_spmv64k<true, 2><<<grid, kBlock, 0, st>>>(a, kk, r);
        else k_spmv64k<false, 2><<<grid, kBlock, 0, st>>>(a, kk, r);
        r0 += 2;
      } else {
        if (cw) k_spmv64k<true, 1><<<grid, kBlock, 0, st>>>(a, kk, r);
        else k_spmv64k<false, 1><<<grid, kBlock, 0, st>>>(a, kk, r);
        r0 += 1;
      }
      PKS_LAUNCHED();
    }
    return PKSELL_OK;
  }
  const bool buf = A->C == kWave && A->n_words < (int64_t(1) << 29);
  if (buf) {
    PKS_GROUP(slice_group(A->n_words, A->n_slices),
              k_spmv64<true, true, GG><<<grid, kBlock, 0, st>>>(a));
  } else if (A->C == kWave) k_spmv64<true, false><<<grid, kBlock, 0, st>>>(a);
  else k_spmv64<false, false><<<grid, kBlock, 0, st>>>(a);
  PKS_LAUNCHED();
  return PKSELL_OK;
}

int pksell_decode(const pksell_matrix *A, int32_t *cols, float *vals, void *stream) {
  int rc = check_matrix(A);
  if (rc) return rc;
  PKS_CHECK(A->n_words == 0 || (cols && vals), PKSELL_EINVAL, "null output");
  hipStream_t st = as_stream(stream);
  if (A->n == 0) return PKSELL_OK;
  SpmvArgs a = make_args(A, nullptr, nullptr, 1);
  const int64_t grid = cdiv(A->n, kBlock);
  switch (A->fmt) {
    case PKSELL_FP16: k_decode<PKSELL_FP16><<<grid, kBlock, 0, st>>>(a, cols, vals); break;
    case PKSELL_E8MY: k_decode<PKSELL_E8MY><<<grid, kBlock, 0, st>>>(a, cols, vals); break;
    default: k_decode<PKSELL_FIX><<<grid, kBlock, 0, st>>>(a, cols, vals); break;
  }
  PKS_LAUNCHED();
  return PKSELL_OK;
}

int pksell_sell_spmv(const pksell_sell *S, const void *x, void *y, void *stream) {
  PKS_CHECK(S, PKSELL_EINVAL, "null matrix");
  PKS_CHECK(S->n == 0 || (S->offset && y), PKSELL_EINVAL, "arrays not set");
  PKS_CHECK(S->n_slots == 0 || ((S->col || S->dtype == PKSELL_F32_PAIRED) && S->val),
            PKSELL_EINVAL, "arrays not set");
  PKS_CHECK(S->perm_mode != PKSELL_IMPLICIT || S->n == 0 || S->perm, PKSELL_EINVAL,
            "implicit mode needs perm");
  hipStream_t st = as_stream(stream);
  if (S->n == 0) return PKSELL_OK;
  const void *perm = S->perm_mode == PKSELL_IMPLICIT ? S->perm : nullptr;
  if (S->m == 0) {
    if (S->dtype != PKSELL_F64) return zero_f32(static_cast<float *>(y), S->n, st);
    k_fill_zero<double><<<cdiv(S->n, kBlock), kBlock, 0, st>>>(static_cast<double *>(y), S->n);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  PKS_CHECK(x, PKSELL_EINVAL, "null x");
  const int64_t grid = cdiv(S->n_slices * S->C, kBlock);
#define PKS_SELL_R(T, CW, BF, VT, RES)                                                      \
  k_sell_spmv<T, CW, BF, VT, kUnroll, RES><<<grid, kBlock, 0, st>>>(                         \
      S->offset, S->col, static_cast<const VT *>(S->val), perm, S->perm_bytes,               \
      static_cast<const T *>(x), static_cast<T *>(y), (uint32_t)S->n, (uint32_t)S->m,        \
      (uint32_t)S->n_slices, S->C, make_geo(S->sigma, 0, S->C))
#define PKS_SELL(T, CW, BF, VT) PKS_SELL_R(T, CW, BF, VT, false)
  const bool res = S->cache_hint == PKSELL_CACHE_RESIDENT;
  // streamed slots and range-checked gathers: 32-bit byte offsets
  const bool buf = S->C == kWave && S->n_slots < (int64_t(1) << 29) && S->m < (int64_t(1) << 29);
  // two slices per wave for narrow float32-vector slices (float64 ran
  // slower paired)
  if (buf && S->dtype != PKSELL_F64 && pair_slices(S->n_slots, S->n_slices)) {
    const int64_t pg = cdiv(cdiv(S->n_slices, 2), kPairBlock / kWave);
    const int G = pair_group(S->n_slots, S->n_slices);
    if (S->dtype == PKSELL_F16) {
      if (perm) launch_sell_pair<true, _Float16>(S, x, y, perm, G, pg, st);
      else launch_sell_pair<false, _Float16>(S, x, y, perm, G, pg, st);
    } else if (S->dtype == PKSELL_F32_PAIRED) {
      if (perm) launch_sell_pair<true, Paired>(S, x, y, perm, G, pg, st);
      else launch_sell_pair<false, Paired>(S, x, y, perm, G, pg, st);
    } else {
      if (perm) launch_sell_pair<true, float>(S, x, y, perm, G, pg, st);
      else launch_sell_pair<false, float>(S, x, y, perm, G, pg, st);
    }
  } else if (S->dtype == PKSELL_F32_PAIRED) {
    if (buf && res) PKS_SELL_R(float, true, true, Paired, true);
    else if (buf) PKS_SELL(float, true, true, Paired);
    else if (S->C == kWave) PKS_SELL(float, true, false, Paired);
    else PKS_SELL(float, false, false, Paired);
  } else if (S->dtype == PKSELL_F16) {
    if (buf && res) PKS_SELL_R(float, true, true, _Float16, true);
    else if (buf) PKS_SELL(float, true, true, _Float16);
    else if (S->C == kWave) PKS_SELL(float, true, false, _Float16);
    else PKS_SELL(float, false, false, _Float16);
  } else if (S->dtype == PKSELL_F32) {
    if (buf && res) PKS_SELL_R(float, true, true, float, true);
    else if (buf) PKS_SELL(float, true, true, float);
    else if (S->C == kWave) PKS_SELL(float, true, false, float);
    else PKS_SELL(float, false, false, float);
  } else {
    if (buf) {
      PKS_GROUP(slice_group(S->n_slots, S->n_slices),
                k_sell_spmv<double, true, true, double, GG><<<grid, kBlock, 0, st>>>(
                    S->offset, S->col, static_cast<const double *>(S->val), perm, S->perm_bytes,
                    static_cast<const double *>(x), static_cast<double *>(y), (uint32_t)S->n,
                    (uint32_t)S->m, (uint32_t)S->n_slices, S->C, make_geo(S->sigma, 0, S->C)));
    } else if (S->C == kWave) PKS_SELL(double, true, false, double);
    else PKS_SELL(double, false, false, double);
  }
#undef PKS_SELL
#undef PKS_SELL_R
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // extern "C"
