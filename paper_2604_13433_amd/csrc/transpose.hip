// CSR of A -> CSR of A^T on the device, so that A^T can be encoded as a
// PackSELL matrix of its own and the adjoint product becomes a plain
// forward product (no atomics).
//
// The entries arrive in row-major order.  A stable radix sort by column
// (hipCUB) therefore leaves every column's entries in ascending row order;
// the boundaries between columns become the new row pointers, and each
// sorted entry takes its original row as its new column index.  The result
// is deterministic.
#include <hipcub/hipcub.hpp>

#include "common.hpp"

namespace pksell {

namespace {

constexpr int kB = 256;

// One thread per row: the row index of each of its entries; flags a
// malformed rowptr instead of writing out of bounds.
__global__ void k_rows_of(const int64_t *__restrict__ rowptr, int64_t n, int64_t nnz,
                          int32_t *__restrict__ row_of, int32_t *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int64_t rb = rowptr[i], re = rowptr[i + 1];
  if (rb < 0 || re > nnz || rb > re || (i == 0 && rb != 0) || (i == n - 1 && re != nnz)) {
    atomicOr(err, 1);
    return;
  }
  for (int64_t e = rb; e < re; ++e) row_of[e] = (int32_t)i;
}

__global__ void k_iota(int32_t *__restrict__ v, int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < len) v[e] = (int32_t)e;
}

// Columns must lie in [0, m): checked before the sort (a key past the sorted
// bit range would be misplaced).
__global__ void k_check_cols(const int32_t *__restrict__ col, int64_t nnz, int64_t m,
                             int32_t *__restrict__ err) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < nnz && (col[e] < 0 || (int64_t)col[e] >= m)) atomicOr(err, 2);
}

// New row pointers from the sorted columns: t_rowptr[c] = first position
// whose column is >= c.
__global__ void k_bounds(const int32_t *__restrict__ keys, int64_t nnz, int64_t m,
                         int64_t *__restrict__ t_rowptr) {
  const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (p >= nnz) return;
  const int64_t c = keys[p];
  const int64_t prev = p > 0 ? (int64_t)keys[p - 1] : -1;
  for (int64_t cc = prev + 1; cc <= c; ++cc) t_rowptr[cc] = p;
  if (p == nnz - 1)
    for (int64_t cc = c + 1; cc <= m; ++cc) t_rowptr[cc] = nnz;
}

__global__ void k_zero_i64(int64_t *__restrict__ v, int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < len) v[e] = 0;
}

template <typename VT>
__global__ void k_take(const int32_t *__restrict__ src, const int32_t *__restrict__ row_of,
                       const VT *__restrict__ val, int64_t nnz, int32_t *__restrict__ t_col,
                       VT *__restrict__ t_val) {
  const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (p >= nnz) return;
  const int32_t e = src[p];
  t_col[p] = row_of[e];
  t_val[p] = val[e];
}

int key_bits(int64_t m) {
  int b = 1;
  while (b < 31 && (int64_t(1) << b) < m) ++b;
  return b;
}

struct TPlan {
  int32_t *err, *keys, *idx_in, *idx_out, *row_of;
  void *temp;
  size_t temp_bytes, bytes;
};

int plan(void *ws, int64_t m, int64_t nnz, TPlan &p) {
  size_t temp = 0;
  const int items = (int)(nnz > 0 ? nnz : 1);
  PKS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const int32_t *)nullptr,
                                             (int32_t *)nullptr, (const int32_t *)nullptr,
                                             (int32_t *)nullptr, items, 0, key_bits(m)));
  Carver cv(ws);
  const size_t len = (size_t)(nnz > 0 ? nnz : 1);
  p.err = cv.take<int32_t>(1);
  p.keys = cv.take<int32_t>(len);
  p.idx_in = cv.take<int32_t>(len);
  p.idx_out = cv.take<int32_t>(len);
  p.row_of = cv.take<int32_t>(len);
  p.temp = cv.take<char>(temp > 0 ? temp : 1);
  p.temp_bytes = temp;
  p.bytes = cv.used;
  return PKSELL_OK;
}

int check_sizes(int64_t n, int64_t m, int64_t nnz) {
  PKS_CHECK(n >= 0 && m >= 0 && nnz >= 0, PKSELL_EINVAL, "negative size");
  PKS_CHECK(n < (int64_t(1) << 30) && m < (int64_t(1) << 30), PKSELL_ERANGE,
            "n and m must be below 2^30");
  PKS_CHECK(nnz < (int64_t(1) << 31) - 1, PKSELL_ERANGE, "the transpose needs nnz < 2^31 - 1");
  return PKSELL_OK;
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_csr_transpose_query(int64_t n, int64_t m, int64_t nnz, size_t *ws_bytes) {
  PKS_CHECK(ws_bytes, PKSELL_EINVAL, "null argument");
  int rc = check_sizes(n, m, nnz);
  if (rc) return rc;
  TPlan p;
  rc = plan(nullptr, m, nnz, p);
  if (rc) return rc;
  *ws_bytes = p.bytes;
  return PKSELL_OK;
}

int pksell_csr_transpose(const int64_t *rowptr, const int32_t *col, const void *val,
                         int32_t val_dtype, int64_t n, int64_t m, int64_t nnz, int64_t *t_rowptr,
                         int32_t *t_col, void *t_val, void *ws, size_t ws_bytes, void *stream) {
  int rc = check_sizes(n, m, nnz);
  if (rc) return rc;
  PKS_CHECK(val_dtype == PKSELL_F32 || val_dtype == PKSELL_F64, PKSELL_EINVAL, "bad val_dtype");
  PKS_CHECK(t_rowptr && (n == 0 || rowptr), PKSELL_EINVAL, "null rowptr");
  PKS_CHECK(nnz == 0 || (col && val && t_col && t_val), PKSELL_EINVAL, "null entry arrays");
  TPlan p;
  rc = plan(ws, m, nnz, p);
  if (rc) return rc;
  PKS_CHECK(ws && ws_bytes >= p.bytes, PKSELL_EWORKSPACE, "workspace: need %zu bytes", p.bytes);
  hipStream_t st = as_stream(stream);
  int32_t zero = 0, err = 0;
  PKS_HIP(hipMemcpyAsync(p.err, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
  if (n > 0) {
    k_rows_of<<<cdiv(n, kB), kB, 0, st>>>(rowptr, n, nnz, p.row_of, p.err);
    PKS_LAUNCHED();
  }
  if (nnz > 0) {
    k_check_cols<<<cdiv(nnz, kB), kB, 0, st>>>(col, nnz, m, p.err);
    PKS_LAUNCHED();
  }
  PKS_HIP(hipMemcpyAsync(&err, p.err, sizeof(err), hipMemcpyDeviceToHost, st));
  PKS_HIP(hipStreamSynchronize(st));
  PKS_CHECK(err == 0, PKSELL_EINVAL, "malformed CSR (flags 0x%x: 1 rowptr, 2 column range)", err);
  if (nnz == 0) {
    k_zero_i64<<<cdiv(m + 1, kB), kB, 0, st>>>(t_rowptr, m + 1);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  k_iota<<<cdiv(nnz, kB), kB, 0, st>>>(p.idx_in, nnz);
  PKS_LAUNCHED();
  size_t temp = p.temp_bytes;
  PKS_HIP(hipcub::DeviceRadixSort::SortPairs(p.temp, temp, col, p.keys, p.idx_in, p.idx_out,
                                             (int)nnz, 0, key_bits(m), st));
  k_bounds<<<cdiv(nnz, kB), kB, 0, st>>>(p.keys, nnz, m, t_rowptr);
  PKS_LAUNCHED();
  if (val_dtype == PKSELL_F32)
    k_take<float><<<cdiv(nnz, kB), kB, 0, st>>>(p.idx_out, p.row_of,
                                                static_cast<const float *>(val), nnz, t_col,
                                                static_cast<float *>(t_val));
  else
    k_take<double><<<cdiv(nnz, kB), kB, 0, st>>>(p.idx_out, p.row_of,
                                                 static_cast<const double *>(val), nnz, t_col,
                                                 static_cast<double *>(t_val));
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // extern "C"
