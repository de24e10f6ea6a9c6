// Adjoint products over the same packed words.
//
// For y = A_q x and a cotangent g: grad_x = A_q^T g (every flag-1 word at
// row i, column c adds v * g_i to grad_x[c]) and grad of each stored value
// a_ic is g_i * x_c (the product is linear in the values; quantisation is
// treated as the identity).  The transposed product scatters with float32
// atomics from the same lane-per-row walk as the forward product, so its
// summation order is not fixed.
#include "codec.hpp"

namespace pksell {

int zero_f32(float *p, int64_t len, hipStream_t st);
int check_matrix_public(const pksell_matrix *A);

namespace {

constexpr int kBlock = 256;

struct AdjArgs {
  const uint32_t *pack;
  const int64_t *offset;
  const void *perm;
  const int16_t *row_exp;
  int64_t n, m, n_slices, k_left;
  int32_t C, sigma, perm_bytes, k;
  Codec cd;
};

__device__ inline int64_t orig_row(const AdjArgs &a, int64_t t) {
  int64_t blk = (t / a.sigma) * a.sigma;
  return blk + (a.perm_bytes == 1 ? (int64_t) static_cast<const uint8_t *>(a.perm)[t]
                                  : (int64_t) static_cast<const uint16_t *>(a.perm)[t]);
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_spmv_t(AdjArgs a, bool implicit, const float *g,
                                                   float *y) {
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t t = b * kBlock + threadIdx.x;
  if (t >= a.n) return;
  const int64_t k = t / a.C, l = t - k * a.C;
  const int64_t s = a.offset[k];
  const int64_t w = (a.offset[k + 1] - s) / a.C;
  const int64_t gi = implicit ? orig_row(a, t) : t;
  float scale = 1.0f;
  if constexpr (FMT == PKSELL_FIX) scale = ldexpf(1.0f, (int)a.row_exp[t] - (a.cd.D + 1));
  uint32_t c = left_offset(t, a.sigma, a.k_left);
  const uint32_t *P = a.pack + s + l;
  for (int64_t j = 0; j < w; ++j) {
    const uint32_t p = __builtin_nontemporal_load(P + j * a.C);
    Unpacked u = unpack(p, a.cd);
    c += u.delta;
    if (p & 1u) {
      const float v = decode_value<FMT>(u.vbits) * scale;
      for (int r = 0; r < a.k; ++r)
        unsafeAtomicAdd(y + (int64_t)c * a.k + r, v * g[gi * a.k + r]);
    }
  }
}

// grad[rowptr[r] + q] = sum over right-hand sides s of g[r, s] * x[c, s]
// for the q-th flag-1 word of original row r (column c).
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_grad_values(AdjArgs a, bool implicit,
                                                        const int64_t *__restrict__ rowptr,
                                                        const float *__restrict__ g,
                                                        const float *__restrict__ x,
                                                        float *__restrict__ grad) {
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t t = b * kBlock + threadIdx.x;
  if (t >= a.n) return;
  const int64_t k = t / a.C, l = t - k * a.C;
  const int64_t s = a.offset[k];
  const int64_t w = (a.offset[k + 1] - s) / a.C;
  const int64_t r = orig_row(a, t);
  const float *gr = g + (implicit ? r : t) * a.k;
  int64_t e = rowptr[r];
  uint32_t c = left_offset(t, a.sigma, a.k_left);
  const uint32_t *P = a.pack + s + l;
  for (int64_t j = 0; j < w; ++j) {
    const uint32_t p = P[j * a.C];
    Unpacked u = unpack(p, a.cd);
    c += u.delta;
    if (p & 1u) {
      const float *xc = x + (int64_t)c * a.k;
      float acc = gr[0] * xc[0];
      for (int q = 1; q < a.k; ++q) acc = fmaf(gr[q], xc[q], acc);
      grad[e++] = acc;
    }
  }
}

AdjArgs make_adj(const pksell_matrix *A, int64_t k) {
  AdjArgs a;
  a.pack = A->pack;
  a.offset = A->offset;
  a.perm = A->perm;
  a.row_exp = A->row_exp;
  a.n = A->n;
  a.m = A->m;
  a.n_slices = A->n_slices;
  a.k_left = A->k_left;
  a.C = A->C;
  a.sigma = A->sigma;
  a.perm_bytes = A->perm_bytes;
  a.k = (int32_t)k;
  a.cd = make_codec(A->D);
  return a;
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_spmv_t(const pksell_matrix *A, const float *g, float *y, int64_t k, void *stream) {
  int rc = check_matrix_public(A);
  if (rc) return rc;
  PKS_CHECK(k >= 1 && k <= 64, PKSELL_EINVAL, "k must be in [1, 64]");
  PKS_CHECK(A->m == 0 || y, PKSELL_EINVAL, "null y");
  PKS_CHECK(A->n == 0 || g, PKSELL_EINVAL, "null g");
  hipStream_t st = as_stream(stream);
  rc = zero_f32(y, A->m * k, st);
  if (rc || A->n == 0 || A->m == 0) return rc;
  AdjArgs a = make_adj(A, k);
  const bool implicit = A->perm_mode == PKSELL_IMPLICIT;
  const int64_t grid = cdiv(A->n, kBlock);
  switch (A->fmt) {
    case PKSELL_FP16: k_spmv_t<PKSELL_FP16><<<grid, kBlock, 0, st>>>(a, implicit, g, y); break;
    case PKSELL_E8MY: k_spmv_t<PKSELL_E8MY><<<grid, kBlock, 0, st>>>(a, implicit, g, y); break;
    default: k_spmv_t<PKSELL_FIX><<<grid, kBlock, 0, st>>>(a, implicit, g, y); break;
  }
  PKS_LAUNCHED();
  return PKSELL_OK;
}

int pksell_grad_values(const pksell_matrix *A, const int64_t *rowptr, const float *g,
                       const float *x, float *grad, int64_t k, void *stream) {
  int rc = check_matrix_public(A);
  if (rc) return rc;
  PKS_CHECK(k >= 1 && k <= 64, PKSELL_EINVAL, "k must be in [1, 64]");
  PKS_CHECK(A->n == 0 || A->perm, PKSELL_EINVAL,
            "grad_values needs perm (the stored-to-original row map) in both modes");
  PKS_CHECK(A->nnz == 0 || (rowptr && g && x && grad), PKSELL_EINVAL, "null argument");
  if (A->nnz == 0) return PKSELL_OK;
  hipStream_t st = as_stream(stream);
  AdjArgs a = make_adj(A, k);
  const bool implicit = A->perm_mode == PKSELL_IMPLICIT;
  const int64_t grid = cdiv(A->n, kBlock);
  switch (A->fmt) {
    case PKSELL_FP16:
      k_grad_values<PKSELL_FP16><<<grid, kBlock, 0, st>>>(a, implicit, rowptr, g, x, grad);
      break;
    case PKSELL_E8MY:
      k_grad_values<PKSELL_E8MY><<<grid, kBlock, 0, st>>>(a, implicit, rowptr, g, x, grad);
      break;
    default:
      k_grad_values<PKSELL_FIX><<<grid, kBlock, 0, st>>>(a, implicit, rowptr, g, x, grad);
      break;
  }
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // extern "C"
