// Sparse triangular solves on CSR-packed words, level by level.
//
// The paper names sparse triangular solves as a kernel its packing should
// suit (sec. 6).  L is lower triangular with every row ending in its
// diagonal, or upper triangular with every row starting with it; packed as
// CSR-based words (one-row slices, no sort), a row's words are contiguous
// and its last (lower) or first value word (upper) is the diagonal.  The
// solve
//   y_i = (b_i - sum_{j<i, or j>i} (L_q)_ij y_j) / (L_q)_ii
// runs one launch per level of a level schedule (rows whose off-diagonal
// columns all lie in lower levels), one thread per row: the thread walks
// its row's words, rebuilding columns as running sums of deltas from the
// row's eq. 4 left offset, and gathers y from rows solved by earlier
// launches.  The schedule is built on the host from the CSR structure (one
// pass in row order), once per matrix.
#include <algorithm>
#include <vector>

#include "codec.hpp"
#include "common.hpp"

namespace pksell {

namespace {

constexpr int kTrsvBlock = 256;

struct TrsvArgs {
  const uint32_t *pack;
  const int64_t *offset;
  const int16_t *row_exp;
  const float *b;
  float *y;
  uint32_t n, k_left;
  int32_t D;
  Codec cd;
};

constexpr int kTrsvGroup = 8;  // words (entries) of a row in flight together

// One launch per level, one thread per row.  A row's words are loaded a
// group at a time, all loads of a group first, then all its gathers of y,
// so a short row costs one round of each rather than one per word.
template <int FMT, bool UPPER>
__global__ __launch_bounds__(kTrsvBlock) void k_trsv_level(TrsvArgs a, const int32_t *rows,
                                                           uint32_t count) {
  const uint32_t t = blockIdx.x * kTrsvBlock + threadIdx.x;
  if (t >= count) return;
  const uint32_t i = (uint32_t)rows[t];
  if (i >= a.n) return;
  const int64_t s = a.offset[i], e = a.offset[i + 1];
  if (e <= s) return;  // rejected by the level analysis
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(a.y, a.n * 4u);
  const uint32_t oob = a.n * 4u;
  uint32_t col = i > a.k_left ? i - a.k_left : 0u;
  float acc = 0.0f;
  float d = 0.0f;
  bool have_d = false;  // upper: the first value word is the diagonal
  for (int64_t p = s; p < e; p += kTrsvGroup) {
    uint32_t w[kTrsvGroup];
#pragma unroll
    for (int j = 0; j < kTrsvGroup; ++j) w[j] = p + j < e ? a.pack[p + j] : 0u;
    float yv[kTrsvGroup], v[kTrsvGroup];
#pragma unroll
    for (int j = 0; j < kTrsvGroup; ++j) {
      const Unpacked u = unpack(w[j], a.cd);
      col += u.delta;
      v[j] = decode_value<FMT>(u.vbits);
      // the diagonal and flag-0 words gather nothing
      const bool live = w[j] & 1u;
      const bool diag = UPPER ? live && !have_d : p + j == e - 1;
      if (diag) {
        d = v[j];
        v[j] = 0.0f;
        have_d = true;
      }
      yv[j] = buffer_load_f32(ry, live && !diag ? col * 4u : oob);
    }
#pragma unroll
    for (int j = 0; j < kTrsvGroup; ++j) acc = fmaf(v[j], yv[j], acc);
  }
  if constexpr (FMT == PKSELL_FIX) {
    const int sh = (int)a.row_exp[i] - a.D - 1;
    acc = ldexpf(acc, sh);
    d = ldexpf(d, sh);
  }
  a.y[i] = (a.b[i] - acc) / d;
}

// The same solve on plain CSR (int32 columns, float32 values): the
// comparator at 8 bytes per stored entry, grouped the same way.
template <bool UPPER>
__global__ __launch_bounds__(kTrsvBlock) void k_trsv_csr_level(
    const int64_t *rowptr, const int32_t *col, const float *val, const float *b, float *y,
    uint32_t n, const int32_t *rows, uint32_t count) {
  const uint32_t t = blockIdx.x * kTrsvBlock + threadIdx.x;
  if (t >= count) return;
  const uint32_t i = (uint32_t)rows[t];
  if (i >= n) return;
  const int64_t s = rowptr[i], e = rowptr[i + 1];
  if (e <= s) return;
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y, n * 4u);
  const uint32_t oob = n * 4u;
  float acc = 0.0f;
  // off-diagonal entries: [s, e - 1) below the diagonal, [s + 1, e) above it
  const int64_t os = UPPER ? s + 1 : s, oe = UPPER ? e : e - 1;
  for (int64_t p = os; p < oe; p += kTrsvGroup) {
    uint32_t c[kTrsvGroup];
    float v[kTrsvGroup], yv[kTrsvGroup];
#pragma unroll
    for (int j = 0; j < kTrsvGroup; ++j) {
      const bool in = p + j < oe;
      c[j] = in ? (uint32_t)col[p + j] * 4u : oob;
      v[j] = in ? val[p + j] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kTrsvGroup; ++j) yv[j] = buffer_load_f32(ry, c[j]);
#pragma unroll
    for (int j = 0; j < kTrsvGroup; ++j) acc = fmaf(v[j], yv[j], acc);
  }
  y[i] = (b[i] - acc) / val[UPPER ? s : e - 1];
}

}  // namespace

}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_trsv_levels(const int64_t *rowptr, const int32_t *col, int64_t n, int32_t upper,
                       int32_t *order, int64_t *level_ptr, int64_t *n_levels, void *stream) {
  PKS_CHECK(n_levels && level_ptr, PKSELL_EINVAL, "null argument");
  PKS_CHECK(n >= 0 && n < (int64_t(1) << 30), PKSELL_ERANGE, "n must be in [0, 2^30)");
  *n_levels = 0;
  level_ptr[0] = 0;
  if (n == 0) return PKSELL_OK;
  PKS_CHECK(rowptr && col && order, PKSELL_EINVAL, "null argument");
  hipStream_t st = as_stream(stream);
  std::vector<int64_t> rp(n + 1);
  PKS_HIP(hipMemcpyAsync(rp.data(), rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
  PKS_HIP(hipStreamSynchronize(st));
  const int64_t nnz = rp[n];
  PKS_CHECK(rp[0] == 0 && nnz >= n && nnz < (int64_t(1) << 40), PKSELL_EINVAL, "bad rowptr");
  std::vector<int32_t> cl(nnz);
  PKS_HIP(hipMemcpyAsync(cl.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
  PKS_HIP(hipStreamSynchronize(st));
  // level(i) = 1 + max level over the row's off-diagonal columns (0 if
  // none), rows in dependency order: ascending (lower) or descending (upper)
  std::vector<int32_t> lev(n);
  int32_t top = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = upper ? n - 1 - k : k;
    const int64_t s = rp[i], e = rp[i + 1];
    PKS_CHECK(e > s && e <= nnz, PKSELL_EINVAL, "row %lld: no entries (needs its diagonal)",
              (long long)i);
    PKS_CHECK(cl[upper ? s : e - 1] == i, PKSELL_EINVAL,
              "row %lld: the %s entry is not the diagonal", (long long)i,
              upper ? "first" : "last");
    int32_t l = -1;
    int64_t prev = upper ? i : -1;
    for (int64_t p = upper ? s + 1 : s; p < (upper ? e : e - 1); ++p) {
      PKS_CHECK(cl[p] > prev && (upper ? cl[p] < n : cl[p] < i), PKSELL_EINVAL,
                "row %lld: columns must increase and lie on one side of the diagonal",
                (long long)i);
      prev = cl[p];
      l = std::max(l, lev[cl[p]]);
    }
    lev[i] = l + 1;
    top = std::max(top, lev[i]);
  }
  // counting sort by level, stable in row order
  const int64_t nl = (int64_t)top + 1;
  std::vector<int64_t> ptr(nl + 1, 0);
  for (int64_t i = 0; i < n; ++i) ++ptr[lev[i] + 1];
  for (int64_t l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
  std::vector<int32_t> ord(n);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t i = 0; i < n; ++i) ord[fill[lev[i]]++] = (int32_t)i;
  PKS_HIP(hipMemcpyAsync(order, ord.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  PKS_HIP(hipStreamSynchronize(st));
  for (int64_t l = 0; l <= nl; ++l) level_ptr[l] = ptr[l];
  *n_levels = nl;
  return PKSELL_OK;
}

int pksell_trsv(const pksell_matrix *L, int32_t upper, const int32_t *order,
                const int64_t *level_ptr, int64_t n_levels, const float *b, float *y,
                void *stream) {
  PKS_CHECK(L, PKSELL_EINVAL, "null matrix");
  PKS_CHECK(L->C == 1 && L->sigma == 1, PKSELL_EINVAL,
            "triangular solves need a CSR-packed matrix (C = 1, sigma = 1)");
  PKS_CHECK(L->fmt == PKSELL_FP16 || L->fmt == PKSELL_E8MY || L->fmt == PKSELL_FIX,
            PKSELL_EINVAL, "triangular solves need 32-bit words (FP16, E8MY, FIX)");
  PKS_CHECK(L->n == L->m, PKSELL_EINVAL, "L must be square");
  if (L->n == 0) return PKSELL_OK;
  PKS_CHECK(L->offset && L->pack && order && level_ptr && b && y, PKSELL_EINVAL,
            "null argument");
  PKS_CHECK(L->fmt != PKSELL_FIX || L->row_exp, PKSELL_EINVAL, "FIX needs row_exp");
  PKS_CHECK(n_levels >= 1 && level_ptr[0] == 0 && level_ptr[n_levels] == L->n, PKSELL_EINVAL,
            "level_ptr does not cover the n rows");
  hipStream_t st = as_stream(stream);
  TrsvArgs a;
  a.pack = L->pack;
  a.offset = L->offset;
  a.row_exp = L->row_exp;
  a.b = b;
  a.y = y;
  a.n = (uint32_t)L->n;
  a.k_left = (uint32_t)L->k_left;
  a.D = L->D;
  a.cd = make_codec(L->D);
  for (int64_t l = 0; l < n_levels; ++l) {
    const int64_t s = level_ptr[l], cnt = level_ptr[l + 1] - s;
    PKS_CHECK(cnt >= 0 && s + cnt <= L->n, PKSELL_EINVAL, "level_ptr must ascend");
    if (cnt == 0) continue;
    const uint32_t g = (uint32_t)cdiv(cnt, kTrsvBlock);
#define PKS_TRSV(F)                                                                   \
  {                                                                                   \
    if (upper) k_trsv_level<F, true><<<g, kTrsvBlock, 0, st>>>(a, order + s, (uint32_t)cnt); \
    else k_trsv_level<F, false><<<g, kTrsvBlock, 0, st>>>(a, order + s, (uint32_t)cnt);      \
  }
    switch (L->fmt) {
      case PKSELL_FP16: PKS_TRSV(PKSELL_FP16); break;
      case PKSELL_E8MY: PKS_TRSV(PKSELL_E8MY); break;
      default: PKS_TRSV(PKSELL_FIX); break;
    }
#undef PKS_TRSV
    PKS_LAUNCHED();
  }
  return PKSELL_OK;
}

int pksell_trsv_csr(const int64_t *rowptr, const int32_t *col, const float *val, int64_t n,
                    int32_t upper, const int32_t *order, const int64_t *level_ptr,
                    int64_t n_levels, const float *b, float *y, void *stream) {
  PKS_CHECK(n >= 0 && n < (int64_t(1) << 30), PKSELL_ERANGE, "n must be in [0, 2^30)");
  if (n == 0) return PKSELL_OK;
  PKS_CHECK(rowptr && col && val && order && level_ptr && b && y, PKSELL_EINVAL,
            "null argument");
  PKS_CHECK(n_levels >= 1 && level_ptr[0] == 0 && level_ptr[n_levels] == n, PKSELL_EINVAL,
            "level_ptr does not cover the n rows");
  hipStream_t st = as_stream(stream);
  for (int64_t l = 0; l < n_levels; ++l) {
    const int64_t s = level_ptr[l], cnt = level_ptr[l + 1] - s;
    PKS_CHECK(cnt >= 0 && s + cnt <= n, PKSELL_EINVAL, "level_ptr must ascend");
    if (cnt == 0) continue;
    const uint32_t g = (uint32_t)cdiv(cnt, kTrsvBlock);
    if (upper)
      k_trsv_csr_level<true><<<g, kTrsvBlock, 0, st>>>(rowptr, col, val, b, y, (uint32_t)n,
                                                      order + s, (uint32_t)cnt);
    else
      k_trsv_csr_level<false><<<g, kTrsvBlock, 0, st>>>(rowptr, col, val, b, y, (uint32_t)n,
                                                       order + s, (uint32_t)cnt);
    PKS_LAUNCHED();
  }
  return PKSELL_OK;
}

}  // extern "C"
