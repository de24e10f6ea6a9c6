// Solvers on the device (sec. 5.2): float64 conjugate gradients on a SELL
// matrix, and the inner-outer CG of sec. 5.2.2 -- a flexible CG outer
// iteration in float64 whose preconditioner is m_in float32 CG iterations
// on the PackSELL matrix.  Dot products, alpha/beta and the convergence test
// are float64 on the device; the host polls a few device scalars once per
// captured graph replay.
//
// One CG iteration is two kernels: (A) the product q = A p, where p is
// formed on the fly as r + beta * p_old at every gathered column and
// written once by its row's lane (two p buffers alternate), writing the
// workgroup partial sums of p.q; (B) the vector updates, writing the
// partial sums of r.r.  In float64 CG, r and p_old sit side by side as one
// pair per row (two pair buffers alternate: (B) writes the next one), so a
// gathered column is one 16-byte load, not two.  There is no communication between workgroups inside
// a kernel: every workgroup of the next kernel sums the previous kernel's
// partials itself, in one fixed order, so all of them reach the same alpha,
// beta and stopping decision (deterministically), and workgroup 0 records
// the scalars for the next kernels and the host.  Partial buffers alternate
// so a kernel never overwrites the partials its own workgroups are still
// reading, and no kernel reads a state field it writes (workgroups start at
// different times) unless every workgroup would reach the same outcome
// either way.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "rowdot.hpp"

namespace pksell {

namespace {

constexpr int kB = kRowBlock;
constexpr uint32_t kVecBlocks = 512;

struct State {
  double rr;        // r.r of the outer residual (host-visible)
  double rr0;       // r.r at a (re)start: read by the first CG step
  double rr_cur;    // r.r the current CG step works with (written by step A)
  double rr_used;   // r.r of the last CG update (alpha's numerator, beta's denominator)
  double bnorm2, tol2, alpha, beta;
  double pq_prev, beta_o, nr;                  // flexible CG
  double in_rr_cur, in_rr_used, in_alpha, in_beta;  // inner CG
  int32_t done, breakdown, inner_stop, iters, inner_iters, max_iters;
  int32_t first, in_first;     // the next step starts a fresh direction
  int32_t step_ok, in_step_ok;  // step A ran, so step B must run
};

// A set of per-workgroup partial sums: slot q of workgroup b at q * count + b.
struct Parts {
  double *p;
  uint32_t count;
};

// ---- reductions -----------------------------------------------------------------

template <int NV, int BS = kB>
__device__ inline void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][BS / kWave];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][w] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int i = 0; i < BS / kWave; ++i) s += sh[q][i];
    v[q] = s;  // every thread holds the total
  }
  __syncthreads();
}

// Writes this workgroup's partial sums (BS threads per workgroup).
template <int NV, int BS = kB>
__device__ inline void put_partials(double (&v)[NV], Parts out) {
  block_sum<NV, BS>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) out.p[q * out.count + blockIdx.x] = v[q];
}

// Elements of one thread in flight at once in the grid-stride loops: each
// loop loads kVecUnroll elements (stride apart) before computing on any of
// them, then computes them in index order, so every sum is accumulated in
// the same order as a plain one-element-at-a-time loop.
constexpr int kVecUnroll = 8;

// Sums a previous kernel's partials; every thread of every workgroup gets the
// same totals (same order of additions everywhere).
// Every thread sums the partials t, t + BS, t + 2 BS, ... in that order,
// U loads per batch (U = 16 with 256 threads takes the 3907 partials of a
// product kernel over a 10^6-row matrix in one memory round trip, at the
// cost of 16 more registers).
template <int NV, int BS = kB, int U = kVecUnroll>
__device__ inline void get_totals(Parts in, double (&tot)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) tot[q] = 0.0;
  for (uint32_t i0 = threadIdx.x; i0 < in.count; i0 += U * BS) {
    double v[NV][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = i0 + u * BS;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q][u] = i < in.count ? in.p[q * in.count + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * BS < in.count)
#pragma unroll
        for (int q = 0; q < NV; ++q) tot[q] += v[q][u];
  }
  block_sum<NV, BS>(tot);
}

__device__ inline bool outer_stopped(const State *st) {
  return st->done || st->iters >= st->max_iters;
}

// ---- matrix views ---------------------------------------------------------------

struct PackView {
  const uint32_t *pack;
  const int64_t *offset;
  const void *perm;
  const int16_t *row_exp;
  uint32_t n, n_slices;
  int32_t C, perm_bytes;
  RowGeo geo;
  Codec cd;
};

// The float64 operator of the outer iteration and of FP64 CG: SELL slots
// (kind 0: col + val) or 64-bit-word PackSELL (kind 1: E11MY words).
struct SellView {
  const int64_t *offset;
  const int32_t *col;
  const double *val;
  const void *perm;
  uint32_t n, n_slices;
  int32_t C, perm_bytes;
  RowGeo geo;
  uint32_t stream;  // C = 64 and arrays below 4 GiB: stream through buffer resources
  uint32_t kind;    // 0: SELL, 1: 64-bit PackSELL words
  const uint64_t *words;
  uint32_t dmask;   // 64-bit words: the flag-1 delta after >> 1 (columns < 2^30)
  uint64_t vmask;   // 64-bit words: the value field
  int32_t group;    // slots per group of the product loops (host side)
};

// Slots per group for a loop over w slots per lane on average: w spread
// evenly over the fewest groups of at most 8, at least 4.
inline int32_t group_for(int64_t slots, int64_t lanes) {
  const int64_t w = std::max<int64_t>(1, cdiv(slots, lanes > 0 ? lanes : 1));
  return (int32_t)std::max<int64_t>(4, cdiv(w, cdiv(w, 8)));
}

// Row dot product of a 64-bit-word PackSELL lane (sec. 4.4 with W = 64):
// columns from the eq. 4 offset plus the deltas, value * gather(column) for
// flag-1 words; flag-0 words add 0 * gather(column) (a valid column of the
// square operator), which keeps the loop branch-free.
template <bool CWAVE, int G, typename Gather>
__device__ inline double words64_row(const SellView &S, const Lane &ln, uint32_t stride,
                                     Gather gather) {
  const uint64_t *P = S.words + ln.s + ln.l;
  const bool buf = CWAVE && S.stream;
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc(CWAVE ? S.words + ln.s : S.words, buf ? ln.w * 512u : 0u);
  uint32_t c = left_offset32(ln.t, S.geo);
  double acc = 0.0;
  for (uint32_t j = 0; j < ln.w; j += G) {
    uint64_t p[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      uint64_t v = 0ull;
      if (j + q < ln.w)
        v = buf ? __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(
                                                   rs, (ln.l + (j + q) * kWave) * 8u, 0,
                                                   kStreamPolicy))
                : __builtin_nontemporal_load(P + (j + q) * stride);
      p[q] = v;
    }
    uint32_t cq[G];
    double vv[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const uint32_t lo = (uint32_t)p[q];
      const bool flag = lo & 1u;
      c += flag ? ((lo >> 1) & S.dmask) : (uint32_t)(p[q] >> 1);
      cq[q] = c;
      vv[q] = flag ? __builtin_bit_cast(double, p[q] & S.vmask) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < G; ++q) acc = fma(vv[q], gather((int32_t)cq[q]), acc);
  }
  return acc;
}

// Row dot product of a lane of the float64 operator: sum over its w slots
// of val * gather(col).
// G slots (or words) per group, sized on the host to the operator's slice
// width (each slot of a group issues its loads and a gather, padding or not).
template <bool CWAVE, int G, typename Gather>
__device__ inline double sell_row(const SellView &S, const Lane &ln, uint32_t stride,
                                  Gather gather) {
  if (S.kind == 1) return words64_row<CWAVE, G>(S, ln, stride, gather);
  const int32_t *pc = S.col + ln.s + ln.l;
  const double *pv = S.val + ln.s + ln.l;
  // streamed slots need a wave-uniform slice start (C = 64)
  const bool buf = CWAVE && S.stream;
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(CWAVE ? S.col + ln.s : S.col, buf ? ln.w * 256u : 0u);
  const __amdgpu_buffer_rsrc_t rv =
      make_rsrc(CWAVE ? S.val + ln.s : S.val, buf ? ln.w * 512u : 0u);
  double acc = 0.0;
  for (uint32_t j = 0; j < ln.w; j += G) {
    int32_t cc[G];
    double vv[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const uint32_t jj = min(j + q, ln.w - 1);
      if (buf) {
        cc[q] = stream_elem<int32_t>(rc, ln.l, jj);
        vv[q] = j + q < ln.w ? stream_elem<double>(rv, ln.l, jj) : 0.0;
      } else {
        cc[q] = __builtin_nontemporal_load(pc + jj * stride);
        vv[q] = j + q < ln.w ? __builtin_nontemporal_load(pv + jj * stride) : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) acc = fma(vv[q], gather(cc[q]), acc);
  }
  return acc;
}

// ---- CG kernels -----------------------------------------------------------------

// (A) float32 inner step on PackSELL.  Totals of the previous r.r give
// beta (0 on the first inner step); then p_new = r + beta p_old, q = A_q
// p_new, and the partials of p_new . q.
template <int FMT, bool CWAVE>
__global__ __launch_bounds__(kB) void k_inner_a(PackView A, const float *__restrict__ r,
                                               const float *__restrict__ p_old,
                                               float *__restrict__ p_new, float *__restrict__ q,
                                               State *st, Parts rr_in, Parts pq_out) {
  const bool stop = outer_stopped(st) || st->inner_stop;
  const bool first = st->in_first;
  double rr[1] = {0.0};
  if (!stop) get_totals(rr_in, rr);
  const double beta_d = first ? 0.0 : rr[0] / st->in_rr_used;
  const bool quit = !stop && !(rr[0] > 0.0 && isfinite(beta_d));  // inner residual vanished
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->in_step_ok = !(stop || quit);
    if (quit) st->inner_stop = 1;
    st->in_rr_cur = rr[0];
    st->in_beta = beta_d;
  }
  if (stop || quit) return;
  const float beta = (float)beta_d;
  Lane ln;
  const bool live = lane_slice<CWAVE>(A.offset, A.n_slices, A.geo, ln);
  const RowOut ro =
      row_out<FMT>(A.perm, A.perm_bytes, A.row_exp, live ? ln.t : A.n, A.n, A.geo);
  double part = 0.0;
  if (live) {
    const __amdgpu_buffer_rsrc_t rr_r = make_rsrc(r, A.n * 4u);
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(p_old, A.n * 4u);
    float acc[1] = {0.0f};
    const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)A.C;
    packsell_row<FMT, 1>(A.pack + ln.s + ln.l, stride, ln.w, left_offset32(ln.t, A.geo), A.cd,
                         [&](uint32_t c, int, bool live) {
                           const uint32_t o = live ? c << 2 : A.n * 4u;  // flag 0: no request
                           return fmaf(beta, buffer_load_f32(rp, o), buffer_load_f32(rr_r, o));
                         },
                         acc);
    if (ln.t < A.n) {
      float qi = acc[0];
      if constexpr (FMT == PKSELL_FIX) qi = ldexpf(qi, ro.shift(A.cd));
      const uint32_t i = ro.row();
      const float pn = fmaf(beta, p_old[i], r[i]);
      p_new[i] = pn;
      q[i] = qi;
      part = (double)pn * (double)qi;
    }
  }
  double v[1] = {part};
  put_partials(v, pq_out);
}

// Word loads of the inner products.  The inner operator is read once per
// inner iteration, m_in times in a row.  When its words (with the inner
// vectors) fit in the 256 MB last-level cache, loads with the default
// policy (RES) let the later iterations find them there: the inner-outer
// CG with E8M8 words on the 27-point 100^3 system took 14.7 ms against
// 17.7 ms with the streaming policy.  When they do not fit, the streaming
// policy (read once, not kept) is the faster one.
template <bool RES>
__device__ inline uint32_t inner_word(__amdgpu_buffer_rsrc_t rs, uint32_t lane, uint32_t j) {
  return __builtin_amdgcn_raw_buffer_load_b32(rs, (lane + j * kWave) * 4u, 0,
                                              RES ? 0 : kStreamPolicy);
}

// One float32 element stored through a buffer resource on [v, v + n) with
// the default policy (the next kernels read p and q again); rows at or past
// n fall outside the resource and are dropped.
__device__ inline void store_row(float *v, uint32_t n, uint32_t row, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), make_rsrc(v, n * 4u),
                                        row * 4u, 0, 0);
}

// (A) for C = 64: the same step with two slices per wave and 128-thread
// workgroups (four slices per workgroup, as in k_inner_a), so the grid runs
// in about one round of waves.  The first group of words of both slices,
// and r and p_old at the lane's own rows, are requested before the previous
// partials are summed, so their latency overlaps the beta prologue.  With
// streamed words the loads need no branch (words past a slice's width read
// 0 from its resource, with no request), so each gather goes out as soon as
// its word has arrived; the last group finishes and stores one slice before
// the next slice's products wait on their gathers.  Same arithmetic per row
// as k_inner_a.
constexpr int kPairB = 128;

// G words per group and slice, sized on the host to the matrix's slice
// width (each word of a group issues a load and a gather, padding or not).
// RES: words loaded with the default policy (see inner_word).
template <int FMT, bool BUF, int G = kUnroll, bool RES = false>
__global__ __launch_bounds__(kPairB) void k_inner_a2(PackView A, const float *__restrict__ r,
                                                    const float *__restrict__ p_old,
                                                    float *__restrict__ p_new,
                                                    float *__restrict__ q, State *st,
                                                    Parts rr_in, Parts pq_out) {
  constexpr int S = 2;
  const bool stop = outer_stopped(st) || st->inner_stop;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(b * (kPairB / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t k0 = wave * S;
  int64_t off[S + 1];
  uint32_t w[S], p[S][G];
  __amdgpu_buffer_rsrc_t rs[S];
#pragma unroll
  for (int i = 0; i <= S; ++i) off[i] = A.offset[min(k0 + i, A.n_slices)];
  RowOut ro[S];
#pragma unroll
  for (int i = 0; i < S; ++i)
    ro[i] = row_out<FMT>(A.perm, A.perm_bytes, A.row_exp, stop ? A.n : (k0 + i) * kWave + lane,
                         A.n, A.geo);
#pragma unroll
  for (int i = 0; i < S; ++i) {
    w[i] = stop ? 0u : (uint32_t)((off[i + 1] - off[i]) >> 6);
    rs[i] = slice_words(A.pack + off[i], w[i]);
  }
  auto load_group = [&](uint32_t j) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int u = 0; u < G; ++u) {
        uint32_t v = 0u;  // past the slice's width: a padding word
        if (BUF)
          v = inner_word<RES>(rs[i], lane, j + u);
        else if (j + u < w[i])
          v = __builtin_nontemporal_load(A.pack + off[i] + lane + (j + u) * kWave);
        p[i][u] = v;
      }
  };
  load_group(0);
  // The lane's own rows (row n, past every resource, for phantom rows and
  // slices past the end: their loads read 0 and their stores are dropped).
  const __amdgpu_buffer_rsrc_t rr_r = make_rsrc(r, A.n * 4u);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(p_old, A.n * 4u);
  uint32_t dst[S];
  float r_row[S], p_row[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const uint32_t t = (k0 + i) * kWave + lane;
    dst[i] = (!stop && k0 + i < A.n_slices && t < A.n) ? ro[i].row() : A.n;
  }
  const bool first = st->in_first;
  double rr[1] = {0.0};
  if (!stop) get_totals<1, kPairB>(rr_in, rr);
  const double beta_d = first ? 0.0 : rr[0] / st->in_rr_used;
  const bool quit = !stop && !(rr[0] > 0.0 && isfinite(beta_d));  // inner residual vanished
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->in_step_ok = !(stop || quit);
    if (quit) st->inner_stop = 1;
    st->in_rr_cur = rr[0];
    st->in_beta = beta_d;
  }
  if (stop || quit) return;
  const float beta = (float)beta_d;
  const uint32_t oob = A.n * 4u;  // flag-0 words: past the resources, no request
  uint32_t c[S];
  float acc[S];
  uint32_t wm = 0;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    c[i] = left_offset32((k0 + i) * kWave + lane, A.geo);
    acc[i] = 0.0f;
    wm = max(wm, w[i]);
  }
  // columns, values and gathers of the loaded group
  auto gather_group = [&](float (&v)[S][G], float (&xv)[S][G]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const Unpacked d = unpack(p[i][u], A.cd);
        c[i] += d.delta;
        const uint32_t o = (p[i][u] & 1u) ? c[i] << 2 : oob;
        v[i][u] = decode_value<FMT>(d.vbits);
        xv[i][u] = fmaf(beta, buffer_load_f32(rp, o), buffer_load_f32(rr_r, o));
      }
  };
  uint32_t j = 0;
  for (; j + G < wm; j += G) {  // every group but the last
    float v[S][G], xv[S][G];
    gather_group(v, xv);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int u = 0; u < G; ++u) acc[i] = fmaf(v[i][u], xv[i][u], acc[i]);
    load_group(j + G);
  }
#pragma unroll
  for (int i = 0; i < S; ++i) {
    r_row[i] = buffer_load_f32(rr_r, dst[i] * 4u);
    p_row[i] = buffer_load_f32(rp, dst[i] * 4u);
  }
  float v[S][G], xv[S][G];
  gather_group(v, xv);
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < S; ++i) {
#pragma unroll
    for (int u = 0; u < G; ++u) acc[i] = fmaf(v[i][u], xv[i][u], acc[i]);
    float qi = acc[i];
    if constexpr (FMT == PKSELL_FIX) qi = ldexpf(qi, ro[i].shift(A.cd));
    const float pn = fmaf(beta, p_row[i], r_row[i]);  // 0 for rows past n
    store_row(p_new, A.n, dst[i], pn);
    store_row(q, A.n, dst[i], qi);
    part += (double)pn * (double)qi;
    __builtin_amdgcn_sched_barrier(0);  // keep the next slice's products after these stores
  }
  double vv[1] = {part};
  put_partials<1, kPairB>(vv, pq_out);
}

// (A) for 16-bit words (E5MY, FIX16; C = 64): the step of k_inner_a2 with
// every 32-bit slot holding two consecutive words of a row (low half
// first), G slots (2G words) per group.  Same grid and partial layout as
// k_inner_a2 (two slices per wave, 128-thread workgroups), and the same
// order of work: the first slots and the own rows' r and p_old requested
// before the previous partials are summed, branch-free slot loads, the
// first slice stored before the second waits on its gathers.
template <int FMT, int G, bool RES = false>
__global__ __launch_bounds__(kPairB) void k_inner16(PackView A, const float *__restrict__ r,
                                                   const float *__restrict__ p_old,
                                                   float *__restrict__ p_new,
                                                   float *__restrict__ q, State *st,
                                                   Parts rr_in, Parts pq_out) {
  constexpr int S = 2;
  const bool stop = outer_stopped(st) || st->inner_stop;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(b * (kPairB / kWave) + threadIdx.x / kWave);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t k0 = wave * S;
  int64_t off[S + 1];
  uint32_t w[S], p[S][G];  // w: slots per lane
  __amdgpu_buffer_rsrc_t rs[S];
#pragma unroll
  for (int i = 0; i <= S; ++i) off[i] = A.offset[min(k0 + i, A.n_slices)];
  RowOut ro[S];
#pragma unroll
  for (int i = 0; i < S; ++i)
    ro[i] = row_out<FMT>(A.perm, A.perm_bytes, A.row_exp, stop ? A.n : (k0 + i) * kWave + lane,
                         A.n, A.geo);
#pragma unroll
  for (int i = 0; i < S; ++i) {
    w[i] = stop ? 0u : (uint32_t)((off[i + 1] - off[i]) >> 7);
    rs[i] = slice_words(A.pack + (off[i] >> 1), w[i]);
  }
  // slots past a slice's width read 0 from its resource, with no request
  auto load_group = [&](uint32_t j) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int u = 0; u < G; ++u) p[i][u] = inner_word<RES>(rs[i], lane, j + u);
  };
  load_group(0);
  uint32_t dst[S];  // row n (past every resource) for phantom rows
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const uint32_t t = (k0 + i) * kWave + lane;
    dst[i] = (!stop && k0 + i < A.n_slices && t < A.n) ? ro[i].row() : A.n;
  }
  const bool first = st->in_first;
  double rr[1] = {0.0};
  if (!stop) get_totals<1, kPairB>(rr_in, rr);
  const double beta_d = first ? 0.0 : rr[0] / st->in_rr_used;
  const bool quit = !stop && !(rr[0] > 0.0 && isfinite(beta_d));  // inner residual vanished
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->in_step_ok = !(stop || quit);
    if (quit) st->inner_stop = 1;
    st->in_rr_cur = rr[0];
    st->in_beta = beta_d;
  }
  if (stop || quit) return;
  const float beta = (float)beta_d;
  const __amdgpu_buffer_rsrc_t rr_r = make_rsrc(r, A.n * 4u);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(p_old, A.n * 4u);
  const uint32_t oob = A.n * 4u;  // flag-0 words: past the resources, no request
  const uint32_t dmask = A.cd.dmask, vmask = A.cd.vmask & 0xFFFFu;
  uint32_t c[S];
  float acc[S];
  uint32_t wm = 0;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    c[i] = left_offset32((k0 + i) * kWave + lane, A.geo);
    acc[i] = 0.0f;
    wm = max(wm, w[i]);
  }
  // columns, values and gathers of the loaded group (two words per slot)
  auto gather_group = [&](float (&v)[S][2 * G], float (&xv)[S][2 * G]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int h = 0; h < 2 * G; ++h) {
        const uint32_t wd = (h & 1) ? p[i][h >> 1] >> 16 : p[i][h >> 1] & 0xFFFFu;
        const bool flag = wd & 1u;
        c[i] += flag ? (wd >> 1) & dmask : (wd >> 1);
        const uint32_t o = flag ? c[i] << 2 : oob;
        const uint32_t bits = flag ? wd & vmask : 0u;
        if constexpr (FMT == PKSELL_E5MY)
          v[i][h] = __half2float(__ushort_as_half((unsigned short)bits));
        else
          v[i][h] = (float)(int32_t)(int16_t)(uint16_t)bits;  // FIX16: q * 2^(D+1)
        xv[i][h] = fmaf(beta, buffer_load_f32(rp, o), buffer_load_f32(rr_r, o));
      }
  };
  uint32_t j = 0;
  for (; j + G < wm; j += G) {  // every group but the last
    float v[S][2 * G], xv[S][2 * G];
    gather_group(v, xv);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int h = 0; h < 2 * G; ++h) acc[i] = fmaf(v[i][h], xv[i][h], acc[i]);
    load_group(j + G);
  }
  float r_row[S], p_row[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    r_row[i] = buffer_load_f32(rr_r, dst[i] * 4u);
    p_row[i] = buffer_load_f32(rp, dst[i] * 4u);
  }
  float v[S][2 * G], xv[S][2 * G];
  gather_group(v, xv);
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < S; ++i) {
#pragma unroll
    for (int h = 0; h < 2 * G; ++h) acc[i] = fmaf(v[i][h], xv[i][h], acc[i]);
    float qi = acc[i];
    if constexpr (FMT == PKSELL_FIX16) qi = ldexpf(qi, ro[i].shift(A.cd));
    const float pn = fmaf(beta, p_row[i], r_row[i]);  // 0 for rows past n
    store_row(p_new, A.n, dst[i], pn);
    store_row(q, A.n, dst[i], qi);
    part += (double)pn * (double)qi;
    __builtin_amdgcn_sched_barrier(0);  // keep the next slice's products after these stores
  }
  double vv[1] = {part};
  put_partials<1, kPairB>(vv, pq_out);
}

// (B) float32 inner update: alpha = rr / pq; z += alpha p, r -= alpha q;
// partials of the new r.r.  The first elements' loads are issued before
// the product's partials are summed, so their latency overlaps that sum.
__global__ __launch_bounds__(kB) void k_inner_b(uint32_t n, float *__restrict__ z,
                                               float *__restrict__ r, const float *__restrict__ p,
                                               const float *__restrict__ q, State *st,
                                               Parts pq_in, Parts rr_out) {
  if (!st->in_step_ok) return;
  const uint32_t S = gridDim.x * kB;
  float zz[kVecUnroll], pp[kVecUnroll], qq[kVecUnroll], rv[kVecUnroll];
  auto load = [&](uint32_t i0) {
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      const bool in = i < n;
      zz[u] = in ? z[i] : 0.0f;
      pp[u] = in ? p[i] : 0.0f;
      qq[u] = in ? q[i] : 0.0f;
      rv[u] = in ? r[i] : 0.0f;
    }
  };
  const uint32_t first_i = blockIdx.x * kB + threadIdx.x;
  if (first_i < n) load(first_i);
  double pq[1];
  get_totals<1, kB, 16>(pq_in, pq);
  if (!(pq[0] > 0.0 && isfinite(pq[0]))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->inner_stop = 1;
    return;
  }
  const double rr = st->in_rr_cur;
  const double alpha_d = rr / pq[0];
  const float alpha = (float)alpha_d;
  double part = 0.0;
  for (uint32_t i0 = first_i; i0 < n; i0 += kVecUnroll * S) {
    if (i0 != first_i) load(i0);
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      if (i < n) {
        z[i] = fmaf(alpha, pp[u], zz[u]);
        const float ri = fmaf(-alpha, qq[u], rv[u]);
        r[i] = ri;
        part += (double)ri * (double)ri;
      }
    }
  }
  double v[1] = {part};
  put_partials(v, rr_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->in_rr_used = rr;
    st->in_alpha = alpha_d;
    st->inner_iters += 1;
    st->in_first = 0;
  }
}

// (A) float64 CG step on SELL.  The current r.r (st->rr0 on a fresh start,
// else the totals of the previous update's partials) gives the stopping
// test and beta; then p_new = r + beta p_old, q = A p_new, partials of
// p_new . q.  r and p_old are read as one interleaved pair (r_i, p_i) per
// row: one 16-byte load per gathered column.
template <bool CWAVE, int G = kUnroll>
__global__ __launch_bounds__(kB) void k_cg_a(SellView S, const double2 *__restrict__ rp_cur,
                                            double *__restrict__ p_new, double *__restrict__ q,
                                            State *st, Parts rr_in, Parts pq_out) {
  const bool stop = outer_stopped(st);
  const bool first = st->first;
  double rr[1] = {st->rr0};
  if (!stop && !first) get_totals(rr_in, rr);
  const bool conv = !stop && !(rr[0] >= st->tol2);  // converged (or NaN)
  const double beta = first ? 0.0 : rr[0] / st->rr_used;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->step_ok = !(stop || conv);
    st->rr_cur = rr[0];
    st->beta = beta;
    if (conv) {
      st->rr = rr[0];
      st->done = 1;  // every workgroup takes the same exit
    }
  }
  if (stop || conv) return;
  Lane ln;
  const bool live = lane_slice<CWAVE>(S.offset, S.n_slices, S.geo, ln);
  const RowOut ri = row_out(S.perm, S.perm_bytes, live ? ln.t : S.n, S.n, S.geo);
  double part = 0.0;
  if (live) {
    const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)S.C;
    // p_new at the row's own index: from the gathers when that column is
    // among them (the same fma of the same values), else loaded
    double own = 0.0;
    bool found = false;
    const double qi = sell_row<CWAVE, G>(S, ln, stride, [&](int32_t c) {
      const double2 pr = rp_cur[c];
      const double g = fma(beta, pr.y, pr.x);
      if ((uint32_t)c - ri.base == ri.p) {  // column c is the row's own index
        own = g;
        found = true;
      }
      return g;
    });
    if (ln.t < S.n) {
      const uint32_t i = ri.row();
      double pn = own;
      if (!found) {
        const double2 pr = rp_cur[i];
        pn = fma(beta, pr.y, pr.x);
      }
      p_new[i] = pn;
      q[i] = qi;
      part = pn * qi;
    }
  }
  double v[1] = {part};
  put_partials(v, pq_out);
}

// (B) float64 CG update: alpha = rr / pq, x += alpha p, r -= alpha q; the
// next (r, p) pairs; partials of the new r.r.  The first elements' loads
// are issued before the product's partials are summed.
__global__ __launch_bounds__(kB) void k_cg_b(uint32_t n, double *__restrict__ x,
                                            const double2 *__restrict__ rp_cur,
                                            double2 *__restrict__ rp_next,
                                            const double *__restrict__ p,
                                            const double *__restrict__ q, State *st, Parts pq_in,
                                            Parts rr_out) {
  if (!st->step_ok) return;
  const uint32_t S = gridDim.x * kB;
  double xx[kVecUnroll], pp[kVecUnroll], qq[kVecUnroll], rv[kVecUnroll];
  auto load = [&](uint32_t i0) {
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      const bool in = i < n;
      xx[u] = in ? x[i] : 0.0;
      pp[u] = in ? p[i] : 0.0;
      qq[u] = in ? q[i] : 0.0;
      rv[u] = in ? rp_cur[i].x : 0.0;
    }
  };
  const uint32_t first_i = blockIdx.x * kB + threadIdx.x;
  if (first_i < n) load(first_i);
  double pq[1];
  get_totals(pq_in, pq);
  if (!(pq[0] > 0.0 && isfinite(pq[0]))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->breakdown = 1;
      st->done = 1;
    }
    return;
  }
  const double rr = st->rr_cur;
  const double alpha = rr / pq[0];
  double part = 0.0;
  for (uint32_t i0 = first_i; i0 < n; i0 += kVecUnroll * S) {
    if (i0 != first_i) load(i0);
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      if (i < n) {
        x[i] = fma(alpha, pp[u], xx[u]);
        const double ri = fma(-alpha, qq[u], rv[u]);
        rp_next[i] = make_double2(ri, pp[u]);
        part += ri * ri;
      }
    }
  }
  double v[1] = {part};
  put_partials(v, rr_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rr_used = rr;
    st->alpha = alpha;
    st->iters += 1;
    st->first = 0;
  }
}

// The pairs (r, p) = (r, 0) that start a plain CG run.
__global__ __launch_bounds__(kB) void k_pair_init(uint32_t n, const double *__restrict__ r,
                                                 double2 *__restrict__ rp0) {
  for (uint32_t i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB)
    rp0[i] = make_double2(r[i], 0.0);
}

// ---- flexible-CG outer kernels (sec. 5.2.2) -----------------------------------

// Inner start: nr = ||r|| (from st->rr), r_in = r / nr (float32), z = 0,
// p_old = 0, partials of r_in . r_in.
__global__ __launch_bounds__(kB) void k_inner_init(uint32_t n, const double *__restrict__ r,
                                                  float *__restrict__ rin, float *__restrict__ zin,
                                                  float *__restrict__ p0, State *st,
                                                  Parts rr_out) {
  if (outer_stopped(st)) return;
  const double nr = sqrt(st->rr);
  const bool stop = !(nr > 0.0 && isfinite(nr));
  const double inv = stop ? 0.0 : 1.0 / nr;
  double part = 0.0;
  const uint32_t S = gridDim.x * kB;
  for (uint32_t i0 = blockIdx.x * kB + threadIdx.x; i0 < n; i0 += kVecUnroll * S) {
    double rv[kVecUnroll];
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) rv[u] = i0 + u * S < n ? r[i0 + u * S] : 0.0;
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      if (i < n) {
        const float v = (float)(rv[u] * inv);
        rin[i] = v;
        zin[i] = 0.0f;
        p0[i] = 0.0f;
        part += (double)v * (double)v;
      }
    }
  }
  double v[1] = {part};
  put_partials(v, rr_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->nr = stop ? 0.0 : nr;
    st->inner_stop = stop;
    st->in_first = 1;
  }
}

// Partials of (z, q_prev) with z = nr * z_in (skipped on a fresh start,
// when pq_prev = 0).
__global__ __launch_bounds__(kB) void k_outer_zq(uint32_t n, const float *__restrict__ zin,
                                                const double *__restrict__ q, State *st,
                                                Parts zq_out) {
  if (outer_stopped(st) || st->pq_prev == 0.0) return;
  const double nr = st->nr;
  double part = 0.0;
  for (uint32_t i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB)
    part += (double)zin[i] * nr * q[i];
  double v[1] = {part};
  put_partials(v, zq_out);
}

// beta_o = (z, q_prev) / (p_prev, q_prev); p = z - beta_o p (in place).
__global__ __launch_bounds__(kB) void k_outer_p(uint32_t n, const float *__restrict__ zin,
                                               double *__restrict__ p, State *st, Parts zq_in) {
  if (outer_stopped(st)) return;
  double zq[1] = {0.0};
  const bool fresh = st->pq_prev == 0.0;
  if (!fresh) get_totals(zq_in, zq);
  const double bo = fresh ? 0.0 : zq[0] / st->pq_prev;
  const double nr = st->nr;
  for (uint32_t i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB)
    p[i] = (double)zin[i] * nr - bo * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->beta_o = bo;
}

// q = A p (float64 SELL) with partials of p.q and p.r.
template <bool CWAVE, int G = kUnroll>
__global__ __launch_bounds__(kB) void k_outer_aq(SellView S, const double *__restrict__ p,
                                                const double *__restrict__ r,
                                                double *__restrict__ q, State *st,
                                                Parts out) {
  if (outer_stopped(st)) return;
  Lane ln;
  const bool live = lane_slice<CWAVE>(S.offset, S.n_slices, S.geo, ln);
  const RowOut ri = row_out(S.perm, S.perm_bytes, live ? ln.t : S.n, S.n, S.geo);
  double pq = 0.0, pr = 0.0;
  if (live) {
    const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)S.C;
    double own = 0.0;  // p at the row's own index, from the gathers when possible
    bool found = false;
    const double qi = sell_row<CWAVE, G>(S, ln, stride, [&](int32_t c) {
      const double g = p[c];
      if ((uint32_t)c - ri.base == ri.p) {  // column c is the row's own index
        own = g;
        found = true;
      }
      return g;
    });
    if (ln.t < S.n) {
      const uint32_t i = ri.row();
      const double pi = found ? own : p[i];
      q[i] = qi;
      pq = pi * qi;
      pr = pi * r[i];
    }
  }
  double v[2] = {pq, pr};
  put_partials(v, out);
}

// alpha = (p, r) / (p, q); x += alpha p, r -= alpha q; partials of r.r.
// The first elements' loads are issued before the partials are summed.
__global__ __launch_bounds__(kB) void k_outer_update(uint32_t n, double *__restrict__ x,
                                                    double *__restrict__ r,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ q, State *st,
                                                    Parts pq_pr_in, Parts rr_out) {
  if (outer_stopped(st)) return;
  const uint32_t S = gridDim.x * kB;
  double xx[kVecUnroll], pp[kVecUnroll], qq[kVecUnroll], rv[kVecUnroll];
  auto load = [&](uint32_t i0) {
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      const bool in = i < n;
      xx[u] = in ? x[i] : 0.0;
      pp[u] = in ? p[i] : 0.0;
      qq[u] = in ? q[i] : 0.0;
      rv[u] = in ? r[i] : 0.0;
    }
  };
  const uint32_t first_i = blockIdx.x * kB + threadIdx.x;
  if (first_i < n) load(first_i);
  double t[2];
  get_totals(pq_pr_in, t);
  if (!(t[0] > 0.0 && isfinite(t[0]))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->breakdown = 1;
      st->done = 1;
    }
    return;
  }
  const double alpha = t[1] / t[0];
  double part = 0.0;
  for (uint32_t i0 = first_i; i0 < n; i0 += kVecUnroll * S) {
    if (i0 != first_i) load(i0);
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const uint32_t i = i0 + u * S;
      if (i < n) {
        x[i] = fma(alpha, pp[u], xx[u]);
        const double ri = fma(-alpha, qq[u], rv[u]);
        r[i] = ri;
        part += ri * ri;
      }
    }
  }
  double v[1] = {part};
  put_partials(v, rr_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->alpha = alpha;
    st->pq_prev = t[0];
  }
}

// One workgroup: the new r.r, the outer iteration count and the stopping
// test of a flexible-CG step.
__global__ __launch_bounds__(kB) void k_outer_check(State *st, Parts rr_in) {
  if (outer_stopped(st)) return;
  double rr[1];
  get_totals(rr_in, rr);
  if (threadIdx.x == 0) {
    st->rr = rr[0];
    st->iters += 1;
    if (!(rr[0] >= st->tol2)) st->done = 1;
  }
}

// True residual r = b - A x with partials of r.r and b.b (float64 SELL).
template <bool CWAVE, int G = kUnroll>
__global__ __launch_bounds__(kB) void k_residual(SellView S, const double *__restrict__ b,
                                                const double *__restrict__ x,
                                                double *__restrict__ r, Parts out) {
  Lane ln;
  const bool live = lane_slice<CWAVE>(S.offset, S.n_slices, S.geo, ln);
  const RowOut dst = row_out(S.perm, S.perm_bytes, live ? ln.t : S.n, S.n, S.geo);
  double rr = 0.0, bb = 0.0;
  if (live) {
    const uint32_t stride = CWAVE ? (uint32_t)kWave : (uint32_t)S.C;
    const double ax = sell_row<CWAVE, G>(S, ln, stride, [&](int32_t c) { return x[c]; });
    if (ln.t < S.n) {
      const uint32_t i = dst.row();
      const double ri = b[i] - ax;
      r[i] = ri;
      rr = ri * ri;
      bb = b[i] * b[i];
    }
  }
  double v[2] = {rr, bb};
  put_partials(v, out);
}

// One workgroup: totals of the residual kernel into the state.
__global__ __launch_bounds__(kB) void k_residual_totals(State *st, Parts in) {
  double t[2];
  get_totals(in, t);
  if (threadIdx.x == 0) {
    st->rr = t[0];
    st->rr0 = t[0];
    st->bnorm2 = t[1];
  }
}

template <typename T>
__global__ void k_zero(T *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB) p[i] = T(0);
}

// ---- host side ------------------------------------------------------------------

struct Work {
  State *st;
  Parts pa, pb0, pb1;  // product-grid partials; two alternating vector-grid sets
  double *r, *q, *p0, *p1;
  double2 *dp0, *dp1;  // plain CG: (r, p) pairs, alternating
  float *rin, *zin, *f0, *f1, *qin;
  size_t bytes;
};

Work carve_work(void *ws, int64_t n, int64_t max_blocks, bool plain) {
  Carver cv(ws);
  Work w;
  const size_t nn = n > 0 ? (size_t)n : 1;
  w.st = cv.take<State>(1);
  w.pa = {cv.take<double>(2 * (size_t)max_blocks), 0};
  w.pb0 = {cv.take<double>(2 * (size_t)kVecBlocks), 0};
  w.pb1 = {cv.take<double>(2 * (size_t)kVecBlocks), 0};
  w.r = cv.take<double>(nn);
  w.q = cv.take<double>(nn);
  w.p0 = cv.take<double>(nn);
  w.p1 = cv.take<double>(nn);
  w.dp0 = plain ? cv.take<double2>(nn) : nullptr;
  w.dp1 = plain ? cv.take<double2>(nn) : nullptr;
  w.rin = cv.take<float>(nn);
  w.zin = cv.take<float>(nn);
  w.f0 = cv.take<float>(nn);
  w.f1 = cv.take<float>(nn);
  w.qin = cv.take<float>(nn);
  w.bytes = cv.used;
  return w;
}

int64_t max_blocks_of(const SellView &S, const pksell_matrix *A) {
  int64_t mb = cdiv((int64_t)S.n_slices * S.C, kB);
  if (A) mb = std::max<int64_t>(mb, cdiv(A->n_slices * A->C, kB));
  return std::max<int64_t>(mb, 1);
}

SellView sell_view(const pksell_sell *S) {
  SellView v;
  v.offset = S->offset;
  v.col = S->col;
  v.val = static_cast<const double *>(S->val);
  v.perm = S->perm;
  v.n = (uint32_t)S->n;
  v.n_slices = (uint32_t)S->n_slices;
  v.C = S->C;
  v.perm_bytes = S->perm_bytes;
  v.geo = make_geo(S->sigma, 0, S->C);
  v.stream = S->C == kWave && S->n_slots < (int64_t(1) << 29) ? 1u : 0u;
  v.kind = 0;
  v.words = nullptr;
  v.dmask = 0;
  v.vmask = 0;
  v.group = group_for(S->n_slots, S->n_slices * S->C);
  return v;
}

// The float64 operator from a 64-bit-word (E11MY) PackSELL matrix.
SellView words64_view(const pksell_matrix *A) {
  SellView v;
  v.offset = A->offset;
  v.col = nullptr;
  v.val = nullptr;
  v.perm = A->perm;
  v.n = (uint32_t)A->n;
  v.n_slices = (uint32_t)A->n_slices;
  v.C = A->C;
  v.perm_bytes = A->perm_bytes;
  v.geo = make_geo(A->sigma, A->k_left, A->C);
  v.stream = A->C == kWave && A->n_words < (int64_t(1) << 29) ? 1u : 0u;
  v.kind = 1;
  v.words = reinterpret_cast<const uint64_t *>(A->pack);
  v.dmask = A->D >= 31 ? 0x7FFFFFFFu : (1u << A->D) - 1u;
  v.vmask = ~((2ull << A->D) - 1ull);
  v.group = group_for(A->n_words, A->n_slices * A->C);
  return v;
}

PackView pack_view(const pksell_matrix *A) {
  PackView v;
  v.pack = A->pack;
  v.offset = A->offset;
  v.perm = A->perm;
  v.row_exp = A->row_exp;
  v.n = (uint32_t)A->n;
  v.n_slices = (uint32_t)A->n_slices;
  v.C = A->C;
  v.perm_bytes = A->perm_bytes;
  v.geo = make_geo(A->sigma, A->k_left, A->C);
  v.cd = make_codec(A->D);
  return v;
}

// Runs the launch statement given after G (which names the group size GG)
// with GG = G in [4, 8].
#define PKS_G(G, ...)                                      \
  switch (G) {                                             \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;  \
    case 5: { constexpr int GG = 5; __VA_ARGS__; } break;  \
    case 6: { constexpr int GG = 6; __VA_ARGS__; } break;  \
    case 7: { constexpr int GG = 7; __VA_ARGS__; } break;  \
    default: { constexpr int GG = 8; __VA_ARGS__; } break; \
  }

struct Solve {
  const pksell_matrix *lo;
  SellView hv;  // the float64 operator
  const double *b;
  double *x;
  Work w;
  hipStream_t s;
  uint32_t n, vb;
  uint32_t gs, gp;  // grids of the SELL and PackSELL product kernels
  bool stream_ok;   // the inner words are addressable by 32-bit byte offsets
  int g_in;         // inner product: words per group (4..8)
  int g16;          // 16-bit inner words: slots per group (2..4)
  bool resident;    // inner words loaded so that they stay in the last-level cache

  Parts pa_for(uint32_t grid) const { return {w.pa.p, grid}; }
  Parts vec(const Parts &p) const { return {p.p, vb}; }

  // r = b - A x, then rr and bnorm2 into the state (two launches).
  int residual() {
    const SellView &S = hv;
    const Parts out = pa_for(gs);
    if (hv.C == kWave) {
      PKS_G(hv.group, k_residual<true, GG><<<gs, kB, 0, s>>>(S, b, x, w.r, out));
    } else
      k_residual<false><<<gs, kB, 0, s>>>(S, b, x, w.r, out);
    PKS_LAUNCHED();
    k_residual_totals<<<1, kB, 0, s>>>(w.st, out);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }

  // Enqueues ``count`` float64 CG iterations (count even: the p buffers and
  // the r.r partial sets alternate, so a replay starts where the last ended).
  int cg_iterations(int count) {
    const SellView &S = hv;
    for (int it = 0; it < count; ++it) {
      const double2 *rp = (it & 1) ? w.dp1 : w.dp0;
      double2 *rp_next = (it & 1) ? w.dp0 : w.dp1;
      const Parts rr_in = vec((it & 1) ? w.pb0 : w.pb1);
      const Parts rr_out = vec((it & 1) ? w.pb1 : w.pb0);
      const Parts pq = pa_for(gs);
      if (hv.C == kWave) {
        PKS_G(hv.group, k_cg_a<true, GG><<<gs, kB, 0, s>>>(S, rp, w.p1, w.q, w.st, rr_in, pq));
      } else
        k_cg_a<false><<<gs, kB, 0, s>>>(S, rp, w.p1, w.q, w.st, rr_in, pq);
      PKS_LAUNCHED();
      k_cg_b<<<vb, kB, 0, s>>>(n, x, rp, rp_next, w.p1, w.q, w.st, pq, rr_out);
      PKS_LAUNCHED();
    }
    return PKSELL_OK;
  }

  template <int FMT, bool CW>
  void inner_a(const PackView &A, const float *po, float *pn, Parts rr_in, Parts pq_out) {
    // gp workgroups either way: 4 slices each (256 threads x 1 slice per
    // wave, or 128 threads x 2 slices per wave), so the partial count agrees
    if constexpr (CW) {
      if (stream_ok) {
#define PKS_IA2(GG)                                                                      \
  (resident ? k_inner_a2<FMT, true, GG, true><<<gp, kPairB, 0, s>>>(A, w.rin, po, pn, w.qin,  \
                                                                   w.st, rr_in, pq_out)      \
            : k_inner_a2<FMT, true, GG, false><<<gp, kPairB, 0, s>>>(A, w.rin, po, pn, w.qin, \
                                                                    w.st, rr_in, pq_out))
        switch (g_in) {
          case 4: PKS_IA2(4); break;
          case 5: PKS_IA2(5); break;
          case 6: PKS_IA2(6); break;
          case 7: PKS_IA2(7); break;
          default: PKS_IA2(8); break;
        }
#undef PKS_IA2
      } else {
        k_inner_a2<FMT, false><<<gp, kPairB, 0, s>>>(A, w.rin, po, pn, w.qin, w.st, rr_in, pq_out);
      }
    } else
      k_inner_a<FMT, CW><<<gp, kB, 0, s>>>(A, w.rin, po, pn, w.qin, w.st, rr_in, pq_out);
  }

  // 16-bit inner words (C = 64): g16 slots per group.
  template <int FMT>
  void inner16(const PackView &A, const float *po, float *pn, Parts rr_in, Parts pq_out) {
#define PKS_I16(GG)                                                                         \
  (resident                                                                                     \
       ? k_inner16<FMT, GG, true><<<gp, kPairB, 0, s>>>(A, w.rin, po, pn, w.qin, w.st, rr_in,   \
                                                        pq_out)                                 \
       : k_inner16<FMT, GG, false><<<gp, kPairB, 0, s>>>(A, w.rin, po, pn, w.qin, w.st, rr_in,  \
                                                         pq_out))
    switch (g16) {
      case 2: PKS_I16(2); break;
      case 3: PKS_I16(3); break;
      default: PKS_I16(4); break;
    }
#undef PKS_I16
  }

  // Enqueues one flexible-CG outer iteration with m_in inner iterations.
  int outer_iteration(int m_in) {
    const SellView &S = hv;
    const PackView A = pack_view(lo);
    const Parts ppq = pa_for(gp);
    k_inner_init<<<vb, kB, 0, s>>>(n, w.r, w.rin, w.zin, w.f0, w.st, vec(w.pb0));
    PKS_LAUNCHED();
    for (int it = 0; it < m_in; ++it) {
      const float *po = (it & 1) ? w.f1 : w.f0;
      float *pn = (it & 1) ? w.f0 : w.f1;
      const Parts rr_in = vec((it & 1) ? w.pb1 : w.pb0);
      const Parts rr_out = vec((it & 1) ? w.pb0 : w.pb1);
      const bool cw = lo->C == kWave;
      switch (lo->fmt) {
        case PKSELL_FP16: cw ? inner_a<PKSELL_FP16, true>(A, po, pn, rr_in, ppq) : inner_a<PKSELL_FP16, false>(A, po, pn, rr_in, ppq); break;
        case PKSELL_E8MY: cw ? inner_a<PKSELL_E8MY, true>(A, po, pn, rr_in, ppq) : inner_a<PKSELL_E8MY, false>(A, po, pn, rr_in, ppq); break;
        case PKSELL_E5MY: inner16<PKSELL_E5MY>(A, po, pn, rr_in, ppq); break;
        case PKSELL_FIX16: inner16<PKSELL_FIX16>(A, po, pn, rr_in, ppq); break;
        default: cw ? inner_a<PKSELL_FIX, true>(A, po, pn, rr_in, ppq) : inner_a<PKSELL_FIX, false>(A, po, pn, rr_in, ppq); break;
      }
      PKS_LAUNCHED();
      k_inner_b<<<vb, kB, 0, s>>>(n, w.zin, w.rin, pn, w.qin, w.st, ppq, rr_out);
      PKS_LAUNCHED();
    }
    k_outer_zq<<<vb, kB, 0, s>>>(n, w.zin, w.q, w.st, vec(w.pb0));
    PKS_LAUNCHED();
    k_outer_p<<<vb, kB, 0, s>>>(n, w.zin, w.p0, w.st, vec(w.pb0));
    PKS_LAUNCHED();
    const Parts paq = pa_for(gs);
    if (hv.C == kWave) {
      PKS_G(hv.group, k_outer_aq<true, GG><<<gs, kB, 0, s>>>(S, w.p0, w.r, w.q, w.st, paq));
    } else
      k_outer_aq<false><<<gs, kB, 0, s>>>(S, w.p0, w.r, w.q, w.st, paq);
    PKS_LAUNCHED();
    k_outer_update<<<vb, kB, 0, s>>>(n, x, w.r, w.p0, w.q, w.st, paq, vec(w.pb1));
    PKS_LAUNCHED();
    k_outer_check<<<1, kB, 0, s>>>(w.st, vec(w.pb1));
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
};

int read_state(const Work &w, State &h, hipStream_t s) {
  PKS_HIP(hipMemcpyAsync(&h, w.st, sizeof(State), hipMemcpyDeviceToHost, s));
  PKS_HIP(hipStreamSynchronize(s));
  return PKSELL_OK;
}

int write_state(const Work &w, const State &h, hipStream_t s) {
  PKS_HIP(hipMemcpyAsync(w.st, &h, sizeof(State), hipMemcpyHostToDevice, s));
  PKS_HIP(hipStreamSynchronize(s));
  return PKSELL_OK;
}

// Captures the work ``enqueue`` puts on stream s into an executable graph.
template <typename F>
int capture(hipStream_t s, F enqueue, hipGraphExec_t *exec) {
  hipGraph_t g = nullptr;
  PKS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = enqueue();
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  PKS_CHECK(e == hipSuccess, PKSELL_EHIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  PKS_CHECK(e == hipSuccess, PKSELL_EHIP, "graph instantiate: %s", hipGetErrorString(e));
  return PKSELL_OK;
}

// A fresh start from the current residual: plain CG takes p = r, flexible
// CG forgets its previous direction.
int restart(Solve &sv, State &h) {
  h.done = 0;
  h.first = 1;
  h.beta = 0.0;
  h.pq_prev = 0.0;
  k_zero<double><<<sv.vb, kB, 0, sv.s>>>(sv.w.p0, sv.n);
  k_zero<double><<<sv.vb, kB, 0, sv.s>>>(sv.w.p1, sv.n);
  PKS_LAUNCHED();
  if (sv.lo == nullptr) {  // plain CG starts from the pairs (r, 0)
    k_pair_init<<<sv.vb, kB, 0, sv.s>>>(sv.n, sv.w.r, sv.w.dp0);
    PKS_LAUNCHED();
  }
  return write_state(sv.w, h, sv.s);
}

int solve(Solve &sv, double tol, int32_t m_in, int32_t max_outer, pksell_pcg_info *info) {
  hipStream_t s = sv.s;
  const uint32_t n = sv.n;
  const Work &w = sv.w;
  k_zero<double><<<sv.vb, kB, 0, s>>>(w.q, n);
  PKS_LAUNCHED();
  State h{};
  h.max_iters = max_outer;
  int rc = write_state(w, h, s);
  if (rc) return rc;
  if ((rc = sv.residual()) || (rc = read_state(w, h, s))) return rc;
  if (h.bnorm2 == 0.0) {  // b = 0: x = 0 solves it
    k_zero<double><<<sv.vb, kB, 0, s>>>(sv.x, n);
    PKS_LAUNCHED();
    PKS_HIP(hipStreamSynchronize(s));
    info->rel_residual = 0.0;
    return PKSELL_OK;
  }
  h.tol2 = tol * tol * h.bnorm2;
  if (!(h.rr >= h.tol2)) {  // the initial guess already satisfies the test
    info->rel_residual = std::sqrt(h.rr / h.bnorm2);
    return PKSELL_OK;
  }
  if ((rc = restart(sv, h))) return rc;

  const bool plain = sv.lo == nullptr;
  // Iterations per graph replay: the host reads the state once per replay,
  // and the steps enqueued after convergence (or the iteration limit) find
  // the solver stopped and exit at once.  Two outer steps per replay halve
  // the host round trips (about 40 us each) for at most one idle step.
  constexpr int kCgPerGraph = 16, kOuterPerGraph = 2;
  hipGraphExec_t exec = nullptr;
  rc = plain ? capture(s, [&] { return sv.cg_iterations(kCgPerGraph); }, &exec)
             : capture(s,
                       [&] {
                         int r = PKSELL_OK;
                         for (int i = 0; i < kOuterPerGraph && r == PKSELL_OK; ++i)
                           r = sv.outer_iteration(m_in);
                         return r;
                       },
                       &exec);
  if (rc) return rc;
  int status = PKSELL_OK;
  for (;;) {
    hipError_t e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) {
      set_error("graph launch: %s", hipGetErrorString(e));
      status = PKSELL_EHIP;
      break;
    }
    if ((status = read_state(w, h, s))) break;
    if (h.breakdown) {
      set_error("breakdown after %d iterations (p^T A p <= 0 or not finite)", h.iters);
      status = PKSELL_EBREAKDOWN;
      break;
    }
    if (h.done) {
      // confirm on the true residual b - A x; otherwise restart from it
      if ((status = sv.residual()) || (status = read_state(w, h, s))) break;
      if (h.rr < h.tol2) break;
      if ((status = restart(sv, h))) break;
    }
    if (h.iters >= max_outer) {
      set_error("no convergence in %d iterations (relative residual %.3e)", h.iters,
                std::sqrt(h.rr / h.bnorm2));
      status = PKSELL_ENOTCONV;
      break;
    }
  }
  (void)hipGraphExecDestroy(exec);
  info->outer_iterations = h.iters;
  info->inner_iterations = h.inner_iters;
  if (status == PKSELL_ENOTCONV) {
    int rc2 = sv.residual();
    if (rc2 == PKSELL_OK) rc2 = read_state(w, h, s);
    if (rc2) return rc2;
  }
  info->rel_residual = std::sqrt(h.rr / h.bnorm2);
  return status;
}

// The shared body of pksell_pcg and pksell_pcg64 once the outer operator's
// own checks passed: inner-matrix checks, the workspace, a private stream.
int run_pcg(const pksell_matrix *A_lo, const SellView &hv, int64_t n, const double *b, double *x,
            double tol, int32_t m_in, int32_t max_outer, pksell_pcg_info *info, void *ws,
            size_t ws_bytes, void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (A_lo) {
    PKS_CHECK(A_lo->n == n && A_lo->m == n, PKSELL_EINVAL, "shape mismatch");
    PKS_CHECK(A_lo->perm_mode == PKSELL_IMPLICIT && A_lo->perm && A_lo->pack && A_lo->offset,
              PKSELL_EINVAL, "inner PackSELL matrix must be implicit with arrays set");
    PKS_CHECK((A_lo->fmt >= PKSELL_FP16 && A_lo->fmt <= PKSELL_FIX) || is_w16(A_lo->fmt),
              PKSELL_EINVAL, "the inner matrix takes FP16, E8MY, FIX, E5MY or FIX16 words");
    PKS_CHECK((A_lo->fmt != PKSELL_FIX && A_lo->fmt != PKSELL_FIX16) || A_lo->row_exp,
              PKSELL_EINVAL, "FIX needs row_exp");
    PKS_CHECK(!is_w16(A_lo->fmt) || (A_lo->C == kWave && A_lo->n_words < (int64_t(1) << 31)),
              PKSELL_EINVAL, "16-bit inner words need C = 64 and fewer than 2^31 words");
    PKS_CHECK(m_in >= 1 && m_in <= 10000, PKSELL_EINVAL, "m_in must be in [1, 10000]");
  }
  PKS_CHECK(tol > 0.0 && max_outer >= 1, PKSELL_EINVAL, "tol must be > 0, max_outer >= 1");
  Solve sv;
  sv.lo = A_lo;
  sv.hv = hv;
  sv.b = b;
  sv.x = x;
  sv.n = (uint32_t)n;
  sv.vb = (uint32_t)std::min<int64_t>(kVecBlocks, cdiv(n, kB));
  sv.gs = (uint32_t)cdiv((int64_t)hv.n_slices * hv.C, kB);
  sv.gp = A_lo ? (uint32_t)cdiv(A_lo->n_slices * A_lo->C, kB) : 0u;
  sv.stream_ok = A_lo && A_lo->n_words < (int64_t(1) << 30);
  // The inner words and the five float32 inner vectors, read m_in times in
  // a row, stay in the 256 MB last-level cache when they take at most
  // 192 MiB of it (a margin for the rest of the traffic).
  if (A_lo) {
    const int64_t word_bytes = is_w16(A_lo->fmt) ? 2 : 4;
    sv.resident = A_lo->n_words * word_bytes + 20 * (int64_t)n <= (int64_t(192) << 20);
  } else {
    sv.resident = false;
  }
  sv.g_in = A_lo ? group_for(A_lo->n_words, A_lo->n_slices * A_lo->C) : 8;
  sv.g16 = 4;
  if (A_lo && is_w16(A_lo->fmt) && A_lo->n_slices > 0) {
    // slots per lane spread evenly over the fewest groups of at most 4
    const int64_t ws = std::max<int64_t>(1, cdiv(A_lo->n_words / 2, (int64_t)kWave * A_lo->n_slices));
    sv.g16 = (int)std::max<int64_t>(2, cdiv(ws, cdiv(ws, 4)));
  }
  sv.w = carve_work(ws, n, max_blocks_of(hv, A_lo), A_lo == nullptr);
  PKS_CHECK(ws && ws_bytes >= sv.w.bytes, PKSELL_EWORKSPACE, "workspace: need %zu bytes",
            sv.w.bytes);
  // The solve runs on a private stream (graph capture needs a non-default
  // stream), ordered after the caller's prior work and finished on return.
  PKS_HIP(hipStreamSynchronize(as_stream(stream)));
  PKS_HIP(hipStreamCreateWithFlags(&sv.s, hipStreamNonBlocking));
  int rc = solve(sv, tol, m_in, max_outer, info);
  hipError_t e = hipStreamSynchronize(sv.s);
  (void)hipStreamDestroy(sv.s);
  if (rc == PKSELL_OK && e != hipSuccess) {
    set_error("solver: %s", hipGetErrorString(e));
    rc = PKSELL_EHIP;
  }
  info->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_pcg_workspace(const pksell_matrix *A_lo, const pksell_sell *A_hi, size_t *ws_bytes) {
  PKS_CHECK(A_hi && ws_bytes, PKSELL_EINVAL, "null argument");
  *ws_bytes =
      carve_work(nullptr, A_hi->n, max_blocks_of(sell_view(A_hi), A_lo), A_lo == nullptr).bytes;
  return PKSELL_OK;
}

int pksell_pcg64_workspace(const pksell_matrix *A_lo, const pksell_matrix *A_hi,
                           size_t *ws_bytes) {
  PKS_CHECK(A_hi && ws_bytes, PKSELL_EINVAL, "null argument");
  PKS_CHECK(A_hi->fmt == PKSELL_E11MY, PKSELL_EINVAL, "the outer matrix must have 64-bit words");
  *ws_bytes = carve_work(nullptr, A_hi->n, max_blocks_of(words64_view(A_hi), A_lo),
                         A_lo == nullptr)
                  .bytes;
  return PKSELL_OK;
}

int pksell_pcg(const pksell_matrix *A_lo, const pksell_sell *A_hi, const double *b, double *x,
               double tol, int32_t m_in, int32_t max_outer, pksell_pcg_info *info, void *ws,
               size_t ws_bytes, void *stream) {
  PKS_CHECK(A_hi && b && x && info, PKSELL_EINVAL, "null argument");
  std::memset(info, 0, sizeof(*info));
  PKS_CHECK(A_hi->n == A_hi->m, PKSELL_EINVAL, "the matrix must be square");
  PKS_CHECK(A_hi->dtype == PKSELL_F64, PKSELL_EINVAL, "the outer matrix must be float64 SELL");
  PKS_CHECK(A_hi->perm_mode == PKSELL_IMPLICIT, PKSELL_EINVAL,
            "the solver needs implicit row order (original ordering)");
  PKS_CHECK(A_hi->n > 0 && A_hi->offset && A_hi->col && A_hi->val && A_hi->perm, PKSELL_EINVAL,
            "outer matrix arrays not set");
  return run_pcg(A_lo, sell_view(A_hi), A_hi->n, b, x, tol, m_in, max_outer, info, ws, ws_bytes,
                 stream);
}

int pksell_pcg64(const pksell_matrix *A_lo, const pksell_matrix *A_hi, const double *b, double *x,
                 double tol, int32_t m_in, int32_t max_outer, pksell_pcg_info *info, void *ws,
                 size_t ws_bytes, void *stream) {
  PKS_CHECK(A_hi && b && x && info, PKSELL_EINVAL, "null argument");
  std::memset(info, 0, sizeof(*info));
  PKS_CHECK(A_hi->fmt == PKSELL_E11MY, PKSELL_EINVAL, "the outer matrix must have 64-bit words");
  PKS_CHECK(A_hi->n == A_hi->m, PKSELL_EINVAL, "the matrix must be square");
  PKS_CHECK(A_hi->perm_mode == PKSELL_IMPLICIT, PKSELL_EINVAL,
            "the solver needs implicit row order (original ordering)");
  PKS_CHECK(A_hi->n > 0 && A_hi->offset && A_hi->pack && A_hi->perm, PKSELL_EINVAL,
            "outer matrix arrays not set");
  return run_pcg(A_lo, words64_view(A_hi), A_hi->n, b, x, tol, m_in, max_outer, info, ws,
                 ws_bytes, stream);
}

}  // extern "C"
