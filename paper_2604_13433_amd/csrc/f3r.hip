// F3R, the nested Krylov solver of sec. 5.2.1, on the device: an outer
// flexible GMRES(m1) in float64, restarted until the true relative residual
// passes the tolerance, preconditioned by one FGMRES(m2) cycle, itself
// preconditioned by one FGMRES(m3) cycle, itself preconditioned by m4
// Richardson iterations.  Layers 2-4 run from zero with no convergence
// test.  Mixed precision (the paper's FP16-F3R and PackSELL-F3R): layers
// 2-4 keep float32 vectors, layer 2 multiplies with float32 SELL and layers
// 3-4 with FP16 values (half-value SELL or PackSELL FP16 words); all-float64
// (FP64-F3R): every layer uses the float64 operator and float64 vectors.
//
// Arnoldi uses classical Gram-Schmidt with one reorthogonalisation (two
// passes of "all dot products, then one combined update"), which needs two
// grid-wide reductions per pass instead of one per basis vector.  Dot
// products, the Hessenberg matrices, Givens rotations and the small
// triangular solves are float64.  Every reduction has one fixed order, so a
// solve repeats bit for bit, and the only difference between the half-value
// SELL and PackSELL forms is the product kernel of layers 3-4, which gives
// bit-identical results on the same values.
//
// One outer step (its whole preconditioner included) is a fixed sequence of
// kernels: it is captured once into a HIP graph and replayed per step.  The
// step index lives in device memory, so the same graph serves every step;
// the host reads the residual estimate after each replay.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.hpp"

namespace pksell {
namespace {

constexpr int kFB = 256;          // threads per block of the vector kernels
constexpr uint32_t kFBlocks = 512;  // at most this many vector blocks
constexpr int kDotChunk = 8;      // basis vectors per pass of the dot kernel
// Rows per thread whose loads are in flight together: 8 for float32
// vectors, 4 for float64 (registers).
template <typename T>
constexpr int rows_of() {
  return sizeof(T) == 4 ? 8 : 4;
}
constexpr int kMaxM = 200;        // longest FGMRES cycle

// Small float64 state of one FGMRES layer: the Hessenberg matrix
// (column-major, ld = m + 1) after the rotations so far, the rotations and
// the rotated right-hand side g.
struct Hess {
  double *H, *cs, *sn, *g;
  int32_t ld;
};

// What the host polls after each outer step.
struct Poll {
  double est;   // |g[j + 1]|: the outer residual norm estimate
  double beta;  // ||r|| at the last (re)start
  int32_t j;    // outer steps of the current cycle
  int32_t pad;
};

__device__ inline double block_sum1(double v) {
  __shared__ double sh[kFB / kWave];
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kFB / kWave; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// block_sum1 of NV values at once (one exchange through LDS for all of
// them); each sum in the same order as block_sum1's.
template <int NV>
__device__ inline void block_sum_n(double (&v)[NV]) {
  __shared__ double sh[NV][kFB / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double t = wave_sum(v[q]);
    if (lane == 0) sh[q][w] = t;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int i = 0; i < kFB / kWave; ++i) s += sh[q][i];
    v[q] = s;
  }
  __syncthreads();
}

// Sum of the nblk partials of slot q, the same order in every block.
// (Each thread adds its partials t, t + kFB, t + 2 kFB, ... in that order,
// two requested at once: a grid of kFBlocks blocks is one round trip.)
__device__ inline double sum_parts(const double *part, uint32_t nblk, int q) {
  const double *pq = part + (size_t)q * nblk;
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < nblk; i += 2 * kFB) {
    const bool two = i + kFB < nblk;
    const double a = pq[i], b = two ? pq[i + kFB] : 0.0;
    s += a;
    if (two) s += b;
  }
  return block_sum1(s);
}

// sum_parts of slots q0 .. q0 + kDotChunk - 1 (those below nv) into h, with
// all their partials loaded at once; the same sums in the same order.
__device__ inline void sum_parts_chunk(const double *part, uint32_t nblk, int q0, int nv,
                                       double *h) {
  double v[kDotChunk];
#pragma unroll
  for (int u = 0; u < kDotChunk; ++u) v[u] = 0.0;
  for (uint32_t i = threadIdx.x; i < nblk; i += 2 * kFB) {
    const bool two = i + kFB < nblk;
    double a[2][kDotChunk];
#pragma unroll
    for (int u = 0; u < kDotChunk; ++u) {
      const double *pu = part + (size_t)(q0 + u) * nblk;
      a[0][u] = q0 + u < nv ? pu[i] : 0.0;
      a[1][u] = q0 + u < nv && two ? pu[i + kFB] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDotChunk; ++u)
      if (q0 + u < nv) {
        v[u] += a[0][u];
        if (two) v[u] += a[1][u];
      }
  }
  block_sum_n<kDotChunk>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int u = 0; u < kDotChunk; ++u)
      if (q0 + u < nv) h[q0 + u] = v[u];
}

__device__ inline uint32_t rows_lo(uint32_t n) {
  const uint32_t tile = (n + gridDim.x - 1) / gridDim.x;
  return min(n, blockIdx.x * tile);
}
__device__ inline uint32_t rows_hi(uint32_t n) {
  const uint32_t tile = (n + gridDim.x - 1) / gridDim.x;
  return min(n, (blockIdx.x + 1) * tile);
}

__device__ inline int count_of(int fixed, const int32_t *jdev, int plus) {
  return jdev ? *jdev + plus : fixed;
}

// part[q * nblk + b] = sum over this block's rows of V_q[r] * w[r], for the
// nv basis vectors (nv = *jdev + 1 when jdev is set, else nv_fixed).
template <typename T>
__global__ __launch_bounds__(kFB) void k_mdot(const T *__restrict__ V, int64_t ld, int nv_fixed,
                                               const int32_t *jdev, const T *__restrict__ w,
                                               uint32_t n, double *__restrict__ part) {
  constexpr int kRows = rows_of<T>();
  const int nv = count_of(nv_fixed, jdev, 1);
  const uint32_t lo = rows_lo(n), hi = rows_hi(n);
  for (int q0 = 0; q0 < nv; q0 += kDotChunk) {
    double acc[kDotChunk];
#pragma unroll
    for (int u = 0; u < kDotChunk; ++u) acc[u] = 0.0;
    // kRows rows per thread in flight; each sum still runs over the rows in
    // order
    for (uint32_t r0 = lo + threadIdx.x; r0 < hi; r0 += kRows * kFB) {
      T wv[kRows], vv[kRows][kDotChunk];
#pragma unroll
      for (int e = 0; e < kRows; ++e) {
        const uint32_t r = r0 + e * kFB;
        const bool in = r < hi;
        wv[e] = in ? w[r] : T(0);
#pragma unroll
        for (int u = 0; u < kDotChunk; ++u)
          vv[e][u] = in && q0 + u < nv ? V[(int64_t)(q0 + u) * ld + r] : T(0);
      }
#pragma unroll
      for (int e = 0; e < kRows; ++e)
        if (r0 + e * kFB < hi)
#pragma unroll
          for (int u = 0; u < kDotChunk; ++u)
            if (q0 + u < nv) acc[u] += (double)vv[e][u] * (double)wv[e];
    }
    block_sum_n<kDotChunk>(acc);
    if (threadIdx.x == 0)
#pragma unroll
      for (int u = 0; u < kDotChunk; ++u)
        if (q0 + u < nv) part[(size_t)(q0 + u) * gridDim.x + blockIdx.x] = acc[u];
  }
}

// One Gram-Schmidt update: h_q = the reduced dots; w -= sum_q h_q V_q.
// Block 0 stores h into column j of H (pass 1) or adds it (pass 2).  With
// norm_part set, also leaves this block's partial of ||w||^2.
template <typename T>
__global__ __launch_bounds__(kFB) void k_maxpy(const T *__restrict__ V, int64_t ld, int nv_fixed,
                                                const int32_t *jdev, const double *__restrict__ part,
                                                T *__restrict__ w, uint32_t n, Hess hs, int j_fixed,
                                                int accumulate, double *__restrict__ norm_part) {
  constexpr int kRows = rows_of<T>();
  __shared__ double h[kMaxM + 1];
  const int nv = count_of(nv_fixed, jdev, 1);
  const int j = count_of(j_fixed, jdev, 0);
  for (int q0 = 0; q0 < nv; q0 += kDotChunk) sum_parts_chunk(part, gridDim.x, q0, nv, h);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int q = 0; q < nv; ++q) {
      double *hq = hs.H + (int64_t)j * hs.ld + q;
      *hq = accumulate ? *hq + h[q] : h[q];
    }
  }
  const uint32_t lo = rows_lo(n), hi = rows_hi(n);
  double nrm = 0.0;
  for (uint32_t r0 = lo + threadIdx.x; r0 < hi; r0 += kRows * kFB) {
    double s[kRows];
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = r0 + e * kFB;
      s[e] = r < hi ? (double)w[r] : 0.0;
    }
    for (int q = 0; q < nv; ++q) {
      T vq[kRows];
#pragma unroll
      for (int e = 0; e < kRows; ++e) {
        const uint32_t r = r0 + e * kFB;
        vq[e] = r < hi ? V[(int64_t)q * ld + r] : T(0);
      }
#pragma unroll
      for (int e = 0; e < kRows; ++e) s[e] -= h[q] * (double)vq[e];
    }
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = r0 + e * kFB;
      if (r < hi) {
        const T t = (T)s[e];
        w[r] = t;
        nrm += (double)t * (double)t;
      }
    }
  }
  if (norm_part) {
    nrm = block_sum1(nrm);
    if (threadIdx.x == 0) norm_part[blockIdx.x] = nrm;
  }
}

// k_mdot and k_maxpy for a basis of NC <= kDotChunk vectors, a count known
// when the launch is recorded (the inner layers): the same sums in the same
// order, with the loads of kRows rows of every vector in flight together
// and no per-vector test.  Rows past the tile read its last row again and
// add nothing.
template <typename T, int NC>
__global__ __launch_bounds__(kFB) void k_mdot_n(const T *__restrict__ V, int64_t ld,
                                                 const T *__restrict__ w, uint32_t n,
                                                 double *__restrict__ part) {
  constexpr int kRows = rows_of<T>();
  const uint32_t lo = rows_lo(n), hi = rows_hi(n);
  double acc[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) acc[u] = 0.0;
  for (uint32_t r0 = lo + threadIdx.x; r0 < hi; r0 += kRows * kFB) {
    T wv[kRows], vv[kRows][NC];
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = min(r0 + e * kFB, hi - 1);
      wv[e] = w[r];
#pragma unroll
      for (int u = 0; u < NC; ++u) vv[e][u] = V[(int64_t)u * ld + r];
    }
#pragma unroll
    for (int e = 0; e < kRows; ++e)
      if (r0 + e * kFB < hi)
#pragma unroll
        for (int u = 0; u < NC; ++u) acc[u] += (double)vv[e][u] * (double)wv[e];
  }
  block_sum_n<NC>(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int u = 0; u < NC; ++u) part[(size_t)u * gridDim.x + blockIdx.x] = acc[u];
}

template <typename T, int NC>
__global__ __launch_bounds__(kFB) void k_maxpy_n(const T *__restrict__ V, int64_t ld,
                                                  const double *__restrict__ part,
                                                  T *__restrict__ w, uint32_t n, Hess hs, int j,
                                                  int accumulate, double *__restrict__ norm_part) {
  constexpr int kRows = rows_of<T>();
  __shared__ double h[kDotChunk];
  const uint32_t lo = rows_lo(n), hi = rows_hi(n), first = lo + threadIdx.x;
  T sv[kRows], vv[kRows][NC];
  auto load = [&](uint32_t r0) {  // r0 < hi
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = min(r0 + e * kFB, hi - 1);
      sv[e] = w[r];
#pragma unroll
      for (int q = 0; q < NC; ++q) vv[e][q] = V[(int64_t)q * ld + r];
    }
  };
  // the first batch is requested before the dot products' partials are
  // summed, so the two memory round trips overlap
  if (first < hi) load(first);
  sum_parts_chunk(part, gridDim.x, 0, NC, h);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int q = 0; q < NC; ++q) {
      double *hq = hs.H + (int64_t)j * hs.ld + q;
      *hq = accumulate ? *hq + h[q] : h[q];
    }
  }
  double hq[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) hq[q] = h[q];
  double nrm = 0.0;
  for (uint32_t r0 = first; r0 < hi; r0 += kRows * kFB) {
    if (r0 != first) load(r0);
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      if (r0 + e * kFB >= hi) continue;
      double t = (double)sv[e];
#pragma unroll
      for (int q = 0; q < NC; ++q) t -= hq[q] * (double)vv[e][q];
      const T tt = (T)t;
      w[r0 + e * kFB] = tt;
      nrm += (double)tt * (double)tt;
    }
  }
  if (norm_part) {
    nrm = block_sum1(nrm);
    if (threadIdx.x == 0) norm_part[blockIdx.x] = nrm;
  }
}

// dst = src / h with h = sqrt(sum of norm_part) (0 where h is 0).
//  - start (j < 0): h is the right-hand side's norm beta: g = beta e1.
//  - step j: h = H[j+1, j]; block 0 rotates column j by the previous
//    rotations, makes the rotation that clears H[j+1, j], updates g and
//    leaves |g[j+1]| in poll->est (when poll is set).
// src and dst: fixed pointers, or (with jdev) base + (*jdev + 1) * ld for
// dst (the next basis vector of the outer layer).
template <typename T>
__global__ __launch_bounds__(kFB) void k_scale_rotate(const T *src, T *dst, int64_t dst_ld,
                                                       const int32_t *jdev, uint32_t n,
                                                       const double *__restrict__ norm_part,
                                                       uint32_t nblk, Hess hs, int j_fixed,
                                                       Poll *poll) {
  constexpr int kRows = rows_of<T>();
  const uint32_t S = gridDim.x * kFB, first = blockIdx.x * kFB + threadIdx.x;
  T v[kRows];  // all loads of a batch first (src and d may be the same vector)
  auto load = [&](uint32_t r0) {
#pragma unroll
    for (int e = 0; e < kRows; ++e) v[e] = r0 + e * S < n ? src[r0 + e * S] : T(0);
  };
  // the first batch is requested before the norm's partials are summed, so
  // the two memory round trips overlap
  if (first < n) load(first);
  const double h = sqrt(sum_parts(norm_part, nblk, 0));
  const int j = jdev ? (j_fixed < 0 ? -1 : *jdev) : j_fixed;
  T *d = jdev && j >= 0 ? dst + (int64_t)(j + 1) * dst_ld : dst;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  for (uint32_t r0 = first; r0 < n; r0 += kRows * S) {
    if (r0 != first) load(r0);
#pragma unroll
    for (int e = 0; e < kRows; ++e)
      if (r0 + e * S < n) d[r0 + e * S] = (T)((double)v[e] * inv);
  }
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (j < 0) {
    hs.g[0] = h;
    for (int i = 1; i < hs.ld; ++i) hs.g[i] = 0.0;
    if (poll) {
      poll->beta = h;
      poll->est = h;
      poll->j = 0;
    }
    return;
  }
  double *col = hs.H + (int64_t)j * hs.ld;
  col[j + 1] = h;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = hs.cs[i] * a + hs.sn[i] * b;
    col[i + 1] = -hs.sn[i] * a + hs.cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double dd = hypot(a, b);
  const double c = dd > 0.0 ? a / dd : 1.0, s = dd > 0.0 ? b / dd : 0.0;
  hs.cs[j] = c;
  hs.sn[j] = s;
  col[j] = dd;
  col[j + 1] = 0.0;
  hs.g[j + 1] = -s * hs.g[j];
  hs.g[j] = c * hs.g[j];
  if (poll) {
    poll->est = fabs(hs.g[j + 1]);
    poll->j = j + 1;
  }
}

// x (+)= sum_q y_q Z_q over the k steps taken, y solving R y = g (R the
// rotated Hessenberg matrix; a vanished diagonal gives y_q = 0).  Every
// block solves the small triangle itself.  The result goes to x, and also
// to x2 when set; with xjdev, x is base + (*xjdev) * x_ld.
template <typename TZ, typename TX>
__global__ __launch_bounds__(kFB) void k_combine(const TZ *__restrict__ Z, int64_t ld, int k_fixed,
                                                  const int32_t *jdev, Hess hs, TX *x,
                                                  int64_t x_ld, const int32_t *xjdev, TX *x2,
                                                  uint32_t n, int add) {
  __shared__ double y[kMaxM];
  const int k = count_of(k_fixed, jdev, 0);
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s = hs.g[i];
      for (int q = i + 1; q < k; ++q) s -= hs.H[(int64_t)q * hs.ld + i] * y[q];
      const double d = hs.H[(int64_t)i * hs.ld + i];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
  }
  __syncthreads();
  TX *xo = xjdev ? x + (int64_t)(*xjdev) * x_ld : x;
  for (uint32_t r = blockIdx.x * kFB + threadIdx.x; r < n; r += gridDim.x * kFB) {
    double s = add ? (double)xo[r] : 0.0;
    for (int q = 0; q < k; ++q) s += y[q] * (double)Z[(int64_t)q * ld + r];
    const TX t = (TX)s;
    xo[r] = t;
    if (x2) x2[r] = t;
  }
}

// k_combine for a cycle length K known when the step is recorded (the inner
// layers): the first rows of every Z_q are requested before the triangle is
// solved, the triangle and g are read into LDS by all threads at once, and
// each thread keeps kRows rows of every Z_q in flight.  Same operations in
// the same order as k_combine.
template <typename TZ, typename TX, int K>
__global__ __launch_bounds__(kFB) void k_combine_n(const TZ *__restrict__ Z, int64_t ld, Hess hs,
                                                    TX *x, int64_t x_ld, const int32_t *xjdev,
                                                    TX *x2, uint32_t n, int add) {
  constexpr int kRows = rows_of<TZ>();
  __shared__ double rs[K][K], gs[K], y[K];
  const uint32_t S = gridDim.x * kFB, first = blockIdx.x * kFB + threadIdx.x;
  TZ zv[kRows][K];
  auto load = [&](uint32_t r0) {
#pragma unroll
    for (int e = 0; e < kRows; ++e)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const uint32_t r = r0 + e * S;
        zv[e][q] = r < n ? Z[(int64_t)q * ld + r] : TZ(0);
      }
  };
  if (first < n) load(first);
  for (int t = threadIdx.x; t < K * K; t += kFB) {  // column q, rows i <= q
    const int q = t / K, i = t % K;
    if (i <= q) rs[q][i] = hs.H[(int64_t)q * hs.ld + i];
  }
  if (threadIdx.x < K) gs[threadIdx.x] = hs.g[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = K - 1; i >= 0; --i) {
      double sum = gs[i];
      for (int q = i + 1; q < K; ++q) sum -= rs[q][i] * y[q];
      const double d = rs[i][i];
      y[i] = d != 0.0 ? sum / d : 0.0;
    }
  }
  __syncthreads();
  double yq[K];
#pragma unroll
  for (int q = 0; q < K; ++q) yq[q] = y[q];
  TX *xo = xjdev ? x + (int64_t)(*xjdev) * x_ld : x;
  for (uint32_t r0 = first; r0 < n; r0 += kRows * S) {
    if (r0 != first) load(r0);
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = r0 + e * S;
      if (r >= n) continue;
      double sum = add ? (double)xo[r] : 0.0;
#pragma unroll
      for (int q = 0; q < K; ++q) sum += yq[q] * (double)zv[e][q];
      const TX t = (TX)sum;
      xo[r] = t;
      if (x2) x2[r] = t;
    }
  }
}

// k_combine over k_fixed steps, through k_combine_n when k_fixed <= 8.
template <typename TZ, typename TX>
void launch_combine(uint32_t nb, hipStream_t s, const TZ *Z, int64_t ld, int k_fixed, Hess hs,
                    TX *x, int64_t x_ld, const int32_t *xjdev, TX *x2, uint32_t n, int add) {
  switch (k_fixed) {
#define PKS_CB(K)                                                                          \
  case K:                                                                                  \
    k_combine_n<TZ, TX, K><<<nb, kFB, 0, s>>>(Z, ld, hs, x, x_ld, xjdev, x2, n, add);      \
    return;
    PKS_CB(1) PKS_CB(2) PKS_CB(3) PKS_CB(4) PKS_CB(5) PKS_CB(6) PKS_CB(7) PKS_CB(8)
#undef PKS_CB
    default:
      k_combine<TZ, TX><<<nb, kFB, 0, s>>>(Z, ld, k_fixed, nullptr, hs, x, x_ld, xjdev, x2, n,
                                           add);
  }
}

// dst = (TD) src, with src = base + (*jdev) * ld when jdev is set; leaves
// the partials of ||dst||^2 (the start of an inner cycle).
template <typename TS, typename TD>
__global__ __launch_bounds__(kFB) void k_load_rhs(const TS *src, int64_t ld, const int32_t *jdev,
                                                   TD *__restrict__ dst, uint32_t n,
                                                   double *__restrict__ norm_part) {
  constexpr int kRows = rows_of<TS>();
  const TS *s = jdev ? src + (int64_t)(*jdev) * ld : src;
  const uint32_t lo = rows_lo(n), hi = rows_hi(n);
  double nrm = 0.0;
  for (uint32_t r0 = lo + threadIdx.x; r0 < hi; r0 += kRows * kFB) {
    TS v[kRows];
#pragma unroll
    for (int e = 0; e < kRows; ++e) v[e] = r0 + e * kFB < hi ? s[r0 + e * kFB] : TS(0);
#pragma unroll
    for (int e = 0; e < kRows; ++e)
      if (r0 + e * kFB < hi) {
        const TD t = (TD)v[e];
        dst[r0 + e * kFB] = t;
        nrm += (double)t * (double)t;
      }
  }
  nrm = block_sum1(nrm);
  if (threadIdx.x == 0) norm_part[blockIdx.x] = nrm;
}

// r = b - Ax (Ax in r on entry) and the partials of ||r||^2.
__global__ __launch_bounds__(kFB) void k_residual(const double *__restrict__ b, double *r,
                                                   uint32_t n, double *__restrict__ norm_part) {
  constexpr int kRows = rows_of<double>();
  const uint32_t lo = rows_lo(n), hi = rows_hi(n);
  double nrm = 0.0;
  for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += kRows * kFB) {
    double bv[kRows], rv[kRows];
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t i = i0 + e * kFB;
      bv[e] = i < hi ? b[i] : 0.0;
      rv[e] = i < hi ? r[i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kRows; ++e)
      if (i0 + e * kFB < hi) {
        const double v = bv[e] - rv[e];
        r[i0 + e * kFB] = v;
        nrm += v * v;
      }
  }
  nrm = block_sum1(nrm);
  if (threadIdx.x == 0) norm_part[blockIdx.x] = nrm;
}

// Richardson with the identity preconditioner: the first two iterations
// from z = 0 in one pass, z = w v + w (v - w t) with t = A v; then
// z += w (v - t) with t = A z; one iteration alone is z = w v.
template <typename T>
__global__ __launch_bounds__(kFB) void k_rich(const T *__restrict__ v, const T *__restrict__ t,
                                               T *__restrict__ z, uint32_t n, double omega,
                                               int mode) {
  constexpr int kRows = rows_of<T>();
  const T w = (T)omega;
  const uint32_t S = gridDim.x * kFB;
  for (uint32_t r0 = blockIdx.x * kFB + threadIdx.x; r0 < n; r0 += kRows * S) {
    T vr[kRows], tr[kRows], zr[kRows];
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = r0 + e * S;
      const bool in = r < n;
      vr[e] = in ? v[r] : T(0);
      tr[e] = in && mode != 0 ? t[r] : T(0);
      zr[e] = in && mode == 2 ? z[r] : T(0);
    }
#pragma unroll
    for (int e = 0; e < kRows; ++e) {
      const uint32_t r = r0 + e * S;
      if (r >= n) continue;
      if (mode == 0) z[r] = w * vr[e];
      else if (mode == 1) z[r] = w * vr[e] + w * (vr[e] - w * tr[e]);
      else z[r] = zr[e] + w * (vr[e] - tr[e]);
    }
  }
}

__global__ void k_next_step(int32_t *j) { *j += 1; }
__global__ void k_set_step(int32_t *j, int32_t v) { *j = v; }

// ---- host side --------------------------------------------------------------------

// A product y = A x of one layer: float64 or float32 SELL (also half values)
// or 32-bit PackSELL words.
struct Op {
  const pksell_sell *sell = nullptr;
  const pksell_matrix *pack = nullptr;
  int run(const void *x, void *y, hipStream_t s) const {
    return pack ? pksell_spmv(pack, static_cast<const float *>(x), static_cast<float *>(y), 1, s)
                : pksell_sell_spmv(sell, x, y, s);
  }
};

struct F3RWork {
  double *V1, *Z1, *zbuf, *wbuf;  // outer layer (float64)
  void *V2, *Z2, *V3, *Z3, *t4;   // inner layers (float32 or float64)
  double *pa, *pn;                // dot partials, norm partials
  double *H1, *cs1, *sn1, *g1;
  double *H2, *cs2, *sn2, *g2;
  double *H3, *cs3, *sn3, *g3;
  int32_t *j1;
  Poll *poll;
  size_t bytes;
};

F3RWork carve_f3r(void *ws, int64_t n, const pksell_f3r_params &p, size_t vsz) {
  Carver c(ws);
  F3RWork w;
  const size_t N = (size_t)n;
  w.V1 = c.take<double>((p.m1 + 1) * N);
  w.Z1 = c.take<double>(p.m1 * N);
  w.zbuf = c.take<double>(N);
  w.wbuf = c.take<double>(N);
  auto vec = [&](size_t count) { return (void *)c.take<char>(count * N * vsz); };
  w.V2 = vec(p.m2 + 1);
  w.Z2 = vec(p.m2);
  w.V3 = vec(p.m3 + 1);
  w.Z3 = vec(p.m3);
  w.t4 = vec(1);
  const int mmax = std::max(p.m1, std::max(p.m2, p.m3)) + 1;
  w.pa = c.take<double>((size_t)mmax * kFBlocks);
  w.pn = c.take<double>(kFBlocks);
  auto hess = [&](int m, double **H, double **cs, double **sn, double **g) {
    *H = c.take<double>((size_t)(m + 1) * m);
    *cs = c.take<double>(m);
    *sn = c.take<double>(m);
    *g = c.take<double>(m + 1);
  };
  hess(p.m1, &w.H1, &w.cs1, &w.sn1, &w.g1);
  hess(p.m2, &w.H2, &w.cs2, &w.sn2, &w.g2);
  hess(p.m3, &w.H3, &w.cs3, &w.sn3, &w.g3);
  w.j1 = c.take<int32_t>(1);
  w.poll = c.take<Poll>(1);
  w.bytes = c.used;
  return w;
}

template <typename T>
struct F3RSolve {
  Op a1, a2, a3;  // outer, second-layer and inner-layer products
  pksell_f3r_params p;
  F3RWork w;
  uint32_t n, nb;  // rows; vector blocks
  hipStream_t s;
  const double *b;
  double *x;

  Hess h1() const { return Hess{w.H1, w.cs1, w.sn1, w.g1, p.m1 + 1}; }
  Hess h2() const { return Hess{w.H2, w.cs2, w.sn2, w.g2, p.m2 + 1}; }
  Hess h3() const { return Hess{w.H3, w.cs3, w.sn3, w.g3, p.m3 + 1}; }
  T *v2(int q) const { return static_cast<T *>(w.V2) + (size_t)q * n; }
  T *z2(int q) const { return static_cast<T *>(w.Z2) + (size_t)q * n; }
  T *v3(int q) const { return static_cast<T *>(w.V3) + (size_t)q * n; }
  T *z3(int q) const { return static_cast<T *>(w.Z3) + (size_t)q * n; }

  // Two Gram-Schmidt passes of wv against the basis V[0..j] (j fixed, or
  // *jdev), then the partials of ||wv||^2 in w.pn.
  template <typename TV>
  int orthogonalise(const TV *V, int j, const int32_t *jdev, TV *wv, Hess hs) {
    for (int pass = 0; pass < 2; ++pass) {
      double *np = pass == 1 ? w.pn : nullptr;
      if (jdev == nullptr && j + 1 <= kDotChunk) {  // basis size known now
#define PKS_GS(NC)                                                                         \
  case NC:                                                                                 \
    k_mdot_n<TV, NC><<<nb, kFB, 0, s>>>(V, n, wv, n, w.pa);                                \
    k_maxpy_n<TV, NC><<<nb, kFB, 0, s>>>(V, n, w.pa, wv, n, hs, j, pass, np);              \
    break;
        switch (j + 1) {
          PKS_GS(1) PKS_GS(2) PKS_GS(3) PKS_GS(4) PKS_GS(5) PKS_GS(6) PKS_GS(7)
          default: k_mdot_n<TV, 8><<<nb, kFB, 0, s>>>(V, n, wv, n, w.pa);
                   k_maxpy_n<TV, 8><<<nb, kFB, 0, s>>>(V, n, w.pa, wv, n, hs, j, pass, np);
        }
#undef PKS_GS
        PKS_LAUNCHED();
        continue;
      }
      k_mdot<TV><<<nb, kFB, 0, s>>>(V, n, j + 1, jdev, wv, n, w.pa);
      PKS_LAUNCHED();
      k_maxpy<TV><<<nb, kFB, 0, s>>>(V, n, j + 1, jdev, w.pa, wv, n, hs, j, pass, np);
      PKS_LAUNCHED();
    }
    return PKSELL_OK;
  }

  // Richardson: z = M4(v).
  int layer4(const T *v, T *z) {
    if (p.m4 == 1) {
      k_rich<T><<<nb, kFB, 0, s>>>(v, nullptr, z, n, p.omega, 0);
      PKS_LAUNCHED();
      return PKSELL_OK;
    }
    int rc = a3.run(v, w.t4, s);
    if (rc) return rc;
    k_rich<T><<<nb, kFB, 0, s>>>(v, static_cast<T *>(w.t4), z, n, p.omega, 1);
    PKS_LAUNCHED();
    for (int it = 2; it < p.m4; ++it) {
      if ((rc = a3.run(z, w.t4, s))) return rc;
      k_rich<T><<<nb, kFB, 0, s>>>(v, static_cast<T *>(w.t4), z, n, p.omega, 2);
      PKS_LAUNCHED();
    }
    return PKSELL_OK;
  }

  // One FGMRES(m3) cycle from zero: z = M3(u).
  int layer3(const T *u, T *z) {
    k_load_rhs<T, T><<<nb, kFB, 0, s>>>(u, 0, nullptr, v3(0), n, w.pn);
    PKS_LAUNCHED();
    k_scale_rotate<T><<<nb, kFB, 0, s>>>(v3(0), v3(0), 0, nullptr, n, w.pn, nb, h3(), -1, nullptr);
    PKS_LAUNCHED();
    int rc;
    for (int j = 0; j < p.m3; ++j) {
      if ((rc = layer4(v3(j), z3(j)))) return rc;
      if ((rc = a3.run(z3(j), v3(j + 1), s))) return rc;
      if ((rc = orthogonalise<T>(v3(0), j, nullptr, v3(j + 1), h3()))) return rc;
      k_scale_rotate<T><<<nb, kFB, 0, s>>>(v3(j + 1), v3(j + 1), 0, nullptr, n, w.pn, nb, h3(), j,
                                           nullptr);
      PKS_LAUNCHED();
    }
    launch_combine<T, T>(nb, s, z3(0), n, p.m3, h3(), z, 0, nullptr, nullptr, n, 0);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }

  // One outer step j1 (device): z = M2(v1_j) by one FGMRES(m2) cycle, stored
  // in Z1[j1]; w = A1 z; orthogonalised against V1[0..j1]; V1[j1+1] = w/h.
  int outer_step() {
    k_load_rhs<double, T><<<nb, kFB, 0, s>>>(w.V1, n, w.j1, v2(0), n, w.pn);
    PKS_LAUNCHED();
    k_scale_rotate<T><<<nb, kFB, 0, s>>>(v2(0), v2(0), 0, nullptr, n, w.pn, nb, h2(), -1, nullptr);
    PKS_LAUNCHED();
    int rc;
    for (int j = 0; j < p.m2; ++j) {
      if ((rc = layer3(v2(j), z2(j)))) return rc;
      if ((rc = a2.run(z2(j), v2(j + 1), s))) return rc;
      if ((rc = orthogonalise<T>(v2(0), j, nullptr, v2(j + 1), h2()))) return rc;
      k_scale_rotate<T><<<nb, kFB, 0, s>>>(v2(j + 1), v2(j + 1), 0, nullptr, n, w.pn, nb, h2(), j,
                                           nullptr);
      PKS_LAUNCHED();
    }
    launch_combine<T, double>(nb, s, z2(0), n, p.m2, h2(), w.Z1, n, w.j1, w.zbuf, n, 0);
    PKS_LAUNCHED();
    if ((rc = a1.run(w.zbuf, w.wbuf, s))) return rc;
    if ((rc = orthogonalise<double>(w.V1, 0, w.j1, w.wbuf, h1()))) return rc;
    k_scale_rotate<double><<<nb, kFB, 0, s>>>(w.wbuf, w.V1, n, w.j1, n, w.pn, nb, h1(), 0, w.poll);
    PKS_LAUNCHED();
    k_next_step<<<1, 1, 0, s>>>(w.j1);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }

  // r = b - A1 x into V1[0], then V1[0] = r / ||r||, g1 = ||r|| e1, j1 = 0.
  int restart() {
    int rc = a1.run(x, w.V1, s);
    if (rc) return rc;
    k_residual<<<nb, kFB, 0, s>>>(b, w.V1, n, w.pn);
    PKS_LAUNCHED();
    k_set_step<<<1, 1, 0, s>>>(w.j1, 0);
    PKS_LAUNCHED();
    k_scale_rotate<double><<<nb, kFB, 0, s>>>(w.V1, w.V1, 0, nullptr, n, w.pn, nb, h1(), -1,
                                              w.poll);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }

  // x += Z1 y over the steps of the current cycle.
  int finish_cycle() {
    k_combine<double, double><<<nb, kFB, 0, s>>>(w.Z1, n, 0, w.j1, h1(), x, 0, nullptr, nullptr,
                                                 n, 1);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
};

int read_poll(const F3RWork &w, Poll &h, hipStream_t s) {
  PKS_HIP(hipMemcpyAsync(&h, w.poll, sizeof(Poll), hipMemcpyDeviceToHost, s));
  PKS_HIP(hipStreamSynchronize(s));
  return PKSELL_OK;
}

template <typename F>
int capture_graph(hipStream_t s, F enqueue, hipGraphExec_t *exec) {
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

template <typename T>
int solve_f3r(F3RSolve<T> &sv, double tol, pksell_pcg_info *info) {
  hipStream_t s = sv.s;
  const uint32_t n = sv.n, nb = sv.nb;
  // ||b||: copy b with its norm partials, then the start form of the
  // scale kernel reduces them into poll->beta
  k_load_rhs<double, double><<<nb, kFB, 0, s>>>(sv.b, 0, nullptr, sv.w.wbuf, n, sv.w.pn);
  PKS_LAUNCHED();
  k_scale_rotate<double><<<nb, kFB, 0, s>>>(sv.w.wbuf, sv.w.wbuf, 0, nullptr, n, sv.w.pn, nb,
                                            sv.h1(), -1, sv.w.poll);
  PKS_LAUNCHED();
  Poll h{};
  int rc = read_poll(sv.w, h, s);
  if (rc) return rc;
  const double bnorm = h.beta;
  if (bnorm == 0.0) {  // b = 0: x = 0
    k_rich<double><<<nb, kFB, 0, s>>>(sv.b, nullptr, sv.x, n, 1.0, 0);  // x = 1 * b = 0
    PKS_LAUNCHED();
    PKS_HIP(hipStreamSynchronize(s));
    info->rel_residual = 0.0;
    return PKSELL_OK;
  }
  if ((rc = sv.restart()) || (rc = read_poll(sv.w, h, s))) return rc;
  double rel = h.beta / bnorm;
  if (!(rel >= tol)) {
    info->rel_residual = rel;
    return PKSELL_OK;
  }
  hipGraphExec_t exec = nullptr;
  if ((rc = capture_graph(s, [&] { return sv.outer_step(); }, &exec))) return rc;
  int status = PKSELL_OK, steps = 0, cycles = 0;
  for (;;) {
    ++cycles;
    for (int j = 0; j < sv.p.m1; ++j) {
      hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        set_error("graph launch: %s", hipGetErrorString(e));
        status = PKSELL_EHIP;
        break;
      }
      if ((status = read_poll(sv.w, h, s))) break;
      ++steps;
      if (!std::isfinite(h.est)) {
        set_error("breakdown: the residual estimate is not finite after %d steps", steps);
        status = PKSELL_EBREAKDOWN;
        break;
      }
      if (h.est < tol * bnorm) break;
    }
    if (status) break;
    if ((status = sv.finish_cycle()) || (status = sv.restart()) ||
        (status = read_poll(sv.w, h, s)))
      break;
    rel = h.beta / bnorm;
    if (!std::isfinite(rel)) {
      set_error("breakdown: the true residual is not finite after %d steps", steps);
      status = PKSELL_EBREAKDOWN;
      break;
    }
    if (rel < tol) break;
    if (cycles >= sv.p.max_cycles) {
      set_error("no convergence in %d cycles (%d steps; relative residual %.3e)", cycles, steps,
                rel);
      status = PKSELL_ENOTCONV;
      break;
    }
  }
  (void)hipGraphExecDestroy(exec);
  info->outer_iterations = steps;
  info->inner_iterations = steps * sv.p.m2;
  info->rel_residual = rel;
  return status;
}

int check_params(const pksell_f3r_params *p) {
  PKS_CHECK(p, PKSELL_EINVAL, "null parameters");
  PKS_CHECK(p->m1 >= 1 && p->m1 <= kMaxM, PKSELL_EINVAL, "m1 must be in [1, %d]", kMaxM);
  PKS_CHECK(p->m2 >= 1 && p->m2 <= 32 && p->m3 >= 1 && p->m3 <= 32 && p->m4 >= 1 && p->m4 <= 32,
            PKSELL_EINVAL, "m2, m3 and m4 must be in [1, 32]");
  PKS_CHECK(std::isfinite(p->omega) && p->omega > 0.0, PKSELL_EINVAL, "omega must be > 0");
  PKS_CHECK(p->max_cycles >= 1, PKSELL_EINVAL, "max_cycles must be >= 1");
  return PKSELL_OK;
}

// dtype2: a second accepted value type (0: none).
int check_sell(const pksell_sell *S, int64_t n, int32_t dtype, const char *what,
               int32_t dtype2 = 0) {
  PKS_CHECK(S->n == n && S->m == n, PKSELL_EINVAL, "%s: shape mismatch", what);
  PKS_CHECK(S->dtype == dtype || (dtype2 && S->dtype == dtype2), PKSELL_EINVAL,
            "%s: wrong value type", what);
  PKS_CHECK(S->perm_mode == PKSELL_IMPLICIT && S->perm && S->offset && S->val &&
                (S->col || S->dtype == PKSELL_F32_PAIRED),
            PKSELL_EINVAL, "%s: needs implicit row order with arrays set", what);
  return PKSELL_OK;
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_f3r_workspace(int64_t n, int32_t mixed, const pksell_f3r_params *prm,
                         size_t *ws_bytes) {
  int rc = check_params(prm);
  if (rc) return rc;
  PKS_CHECK(ws_bytes && n >= 1 && n < (int64_t(1) << 30), PKSELL_EINVAL, "bad n or null pointer");
  *ws_bytes = carve_f3r(nullptr, n, *prm, mixed ? sizeof(float) : sizeof(double)).bytes;
  return PKSELL_OK;
}

int pksell_f3r(const pksell_sell *A1, const pksell_sell *A2, const pksell_sell *A3_sell,
               const pksell_matrix *A3_pack, const double *b, double *x, double tol,
               const pksell_f3r_params *prm, pksell_pcg_info *info, void *ws, size_t ws_bytes,
               void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  PKS_CHECK(A1 && b && x && info, PKSELL_EINVAL, "null argument");
  std::memset(info, 0, sizeof(*info));
  int rc = check_params(prm);
  if (rc) return rc;
  PKS_CHECK(tol > 0.0, PKSELL_EINVAL, "tol must be > 0");
  const int64_t n = A1->n;
  PKS_CHECK(n >= 1 && n < (int64_t(1) << 30), PKSELL_EINVAL, "n must be in [1, 2^30)");
  if ((rc = check_sell(A1, n, PKSELL_F64, "A1"))) return rc;
  const bool mixed = A2 != nullptr;
  if (mixed) {
    if ((rc = check_sell(A2, n, PKSELL_F32, "A2", PKSELL_F32_PAIRED))) return rc;
    PKS_CHECK((A3_sell != nullptr) != (A3_pack != nullptr), PKSELL_EINVAL,
              "give exactly one inner operator (A3_sell or A3_pack)");
    if (A3_sell) {
      PKS_CHECK(A3_sell->dtype == PKSELL_F16 || A3_sell->dtype == PKSELL_F32 ||
                    A3_sell->dtype == PKSELL_F32_PAIRED,
                PKSELL_EINVAL, "A3_sell must hold half or float32 values");
      if ((rc = check_sell(A3_sell, n, A3_sell->dtype, "A3_sell"))) return rc;
    } else {
      const pksell_matrix *P = A3_pack;
      PKS_CHECK(P->n == n && P->m == n, PKSELL_EINVAL, "A3_pack: shape mismatch");
      PKS_CHECK(P->fmt == PKSELL_FP16 || P->fmt == PKSELL_E8MY || P->fmt == PKSELL_FIX,
                PKSELL_EINVAL, "A3_pack must have 32-bit words (FP16, E8MY or FIX)");
      PKS_CHECK(P->perm_mode == PKSELL_IMPLICIT && P->perm && P->pack && P->offset,
                PKSELL_EINVAL, "A3_pack: needs implicit row order with arrays set");
      PKS_CHECK(P->split_words == 0, PKSELL_EINVAL, "A3_pack: no split or chunk plan");
    }
  } else {
    PKS_CHECK(!A3_sell && !A3_pack, PKSELL_EINVAL,
              "the all-float64 form takes no inner operators (A2 = NULL)");
  }
  size_t need = 0;
  if ((rc = pksell_f3r_workspace(n, mixed, prm, &need))) return rc;
  PKS_CHECK(ws && ws_bytes >= need, PKSELL_EWORKSPACE, "workspace: need %zu bytes", need);
  const uint32_t nb = (uint32_t)std::min<int64_t>(kFBlocks, cdiv(n, kFB));
  PKS_HIP(hipStreamSynchronize(as_stream(stream)));
  hipStream_t s = nullptr;
  PKS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (mixed) {
    F3RSolve<float> sv;
    sv.a1.sell = A1;
    sv.a2.sell = A2;
    sv.a3.sell = A3_sell;
    sv.a3.pack = A3_pack;
    sv.p = *prm;
    sv.w = carve_f3r(ws, n, *prm, sizeof(float));
    sv.n = (uint32_t)n;
    sv.nb = nb;
    sv.s = s;
    sv.b = b;
    sv.x = x;
    rc = solve_f3r(sv, tol, info);
  } else {
    F3RSolve<double> sv;
    sv.a1.sell = sv.a2.sell = sv.a3.sell = A1;
    sv.p = *prm;
    sv.w = carve_f3r(ws, n, *prm, sizeof(double));
    sv.n = (uint32_t)n;
    sv.nb = nb;
    sv.s = s;
    sv.b = b;
    sv.x = x;
    rc = solve_f3r(sv, tol, info);
  }
  hipError_t e = hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  if (rc == PKSELL_OK && e != hipSuccess) {
    set_error("f3r: %s", hipGetErrorString(e));
    rc = PKSELL_EHIP;
  }
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

}  // extern "C"
