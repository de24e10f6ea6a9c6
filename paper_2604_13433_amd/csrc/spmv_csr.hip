// Products of CSR-packed matrices balanced over words.
//
// A CSR-packed matrix is PackSELL with one-row slices (C = 1) and no row
// sort (sigma = 1): every row's words sit together, in order, with no
// padding, and the slice offsets are a word row pointer.  The paper names
// delta-value packing in a CSR-based format as future work (sec. 6), noting
// that it needs care with load balancing and communication between
// threads; this is the design used here.
//
// The word stream is cut into chunks of T = 64 K words, one per wave,
// whatever rows they fall in, so every wave moves the same bytes however
// uneven the rows are.  Lane l takes the K consecutive words at c T + l K
// (loaded as 16-byte vectors) and walks them in order:
//
//  * Row starts ("heads") come from the rows the chunk owns (those whose
//    words start inside it, lo[c] .. lo[c+1] - 1, from the plan): each lane
//    marks one row's head in a per-wave bitmap in LDS, and writes y = 0 for
//    an empty row.
//  * Columns are running sums of deltas (sec. 4.4) from each row's eq. 4
//    left offset.  A lane knows its columns from its first head on; before
//    it, it needs the column reached at the end of the lane before.  A
//    segmented scan over the 64 lanes (a head restarts the sum) gives it,
//    seeded by the chunk's anchor (the running column before its first
//    word, from the plan).
//  * Products are summed per row in word order inside a lane; a row that
//    continues across lanes is finished by a second segmented scan of the
//    lanes' open sums, and the lane where it ends writes y.
//  * A row that continues past the chunk leaves its piece in the chunk's
//    scratch (the piece before the first head, and the open piece after
//    the last), and a second kernel adds the pieces of each such row in
//    chunk order.  Every sum has a fixed order: results are deterministic.
#include "codec.hpp"
#include "common.hpp"
#include "rowdot.hpp"

namespace pksell {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCsrWaves = 4;  // waves (chunks) per workgroup

// FMT value of the float32 CSR comparator: 8-byte entries (column in the
// low half, float32 value bits in the high half), absolute columns, no
// words to decode.  Its product reuses the chunk kernel below.
constexpr int kCsr32 = -1;
constexpr int kCsrBlock = kCsrWaves * kWave;

struct CsrArgs {
  const uint32_t *pack;
  const int64_t *rowptr;  // word row pointer (the slice offsets), n + 1
  const uint32_t *lo;     // n_chunks + 1
  const uint32_t *anchor; // n_chunks
  const int16_t *row_exp;
  const float *x;
  float *y;
  float *head_part;   // n_chunks: the piece of the row continued from earlier chunks
  float *tail_part;   // n_chunks: the open piece of the chunk's last row
  int32_t *tail_row;  // n_chunks: that row, or -1
  int64_t n_words;
  uint32_t n, m, n_chunks, k_left;
  uint32_t nr;  // right-hand sides (1, 2 or 4): x is m x nr, y n x nr, row-major
  int32_t D;
  Codec cd;
};

// Eq. 4 with one-row windows.
__device__ inline uint32_t row_base(uint32_t r, uint32_t k_left) {
  return r > k_left ? r - k_left : 0u;
}

template <int FMT>
__device__ inline float row_scaled(float v, const CsrArgs &a, uint32_t r) {
  if constexpr (FMT == PKSELL_FIX) return ldexpf(v, (int)a.row_exp[r] - a.D - 1);
  else return v;
}

// Inclusive segmented scan over the wave in lane order: a lane with ``f``
// set starts a new segment.  On return f tells whether a head lies at or
// before this lane, and v (and r, the row of the last head) hold the
// running values.
__device__ inline void seg_scan_col(bool &f, uint32_t &v, uint32_t &r, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t pv = __shfl_up(v, o, kWave);
    const uint32_t pr = __shfl_up(r, o, kWave);
    const bool pf = __shfl_up((int)f, o, kWave) != 0;
    if (lane >= (uint32_t)o && !f) {
      v += pv;
      r = pr;
      f = pf;
    }
  }
}

__device__ inline void seg_scan_sum(bool f, float &s, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const float ps = __shfl_up(s, o, kWave);
    const bool pf = __shfl_up((int)f, o, kWave) != 0;
    if (lane >= (uint32_t)o && !f) {
      s += ps;
      f = pf;
    }
  }
}

// Per-lane entry registers: K for the float32 CSR comparator, 1 (unused)
// for words.
template <int FMT, int K>
constexpr int kCsrEntries = FMT == kCsr32 ? K : 1;

template <int FMT, int K, int NR>
__global__ __launch_bounds__(kCsrBlock) void k_csr_chunks(CsrArgs a) {
  constexpr uint32_t T = K * kWave;
  __shared__ uint32_t s_heads[kCsrWaves][kWave];  // bit j of word l: position l K + j is a head
  __shared__ uint32_t s_row[kCsrWaves][T];        // the row at each head position
  const uint32_t wv = threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t c =
      __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * kCsrWaves + wv);
  if (c >= a.n_chunks) return;
  uint32_t *heads = s_heads[wv];
  uint32_t *hrow = s_row[wv];
  const int64_t p0 = (int64_t)c * T;
  const uint32_t rlo = a.lo[c];
  const uint32_t rhi = min(a.lo[c + 1], a.n);
  const bool last = c + 1 == a.n_chunks;
  // closed: the chunk's last word ends its row
  const bool closed = last || a.rowptr[rhi] == p0 + T;

  heads[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (uint32_t r = rlo + lane; r < rhi; r += kWave) {
    const int64_t s = a.rowptr[r], e = a.rowptr[r + 1];
    const uint64_t p = (uint64_t)(s - p0);
    if (s == e) {
#pragma unroll
      for (int q = 0; q < NR; ++q) a.y[(int64_t)r * NR + q] = 0.0f;
    } else if (p < T) {  // always, for a plan built by the encoder
      hrow[p] = r;
      atomicOr(&heads[p / K], 1u << (p % K));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const uint32_t hb = heads[lane];

  // the lane's K words (zero words past the end: delta 0, no value), or
  // its K float32 CSR entries
  const int64_t q0 = p0 + (int64_t)lane * K;
  uint32_t w[K];
  uint32_t ecol[kCsrEntries<FMT, K>], eval[kCsrEntries<FMT, K>];
  if constexpr (FMT == kCsr32) {
    const uint64_t *ent = reinterpret_cast<const uint64_t *>(a.pack);
    if (q0 + K <= a.n_words) {
      const u32x4 *p4 = reinterpret_cast<const u32x4 *>(ent + q0);
#pragma unroll
      for (int i = 0; i < K / 2; ++i) {
        const u32x4 u = __builtin_nontemporal_load(p4 + i);
        ecol[2 * i] = u.x;
        eval[2 * i] = u.y;
        ecol[2 * i + 1] = u.z;
        eval[2 * i + 1] = u.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint64_t e = q0 + j < a.n_words ? ent[q0 + j] : 0ull;
        ecol[j] = (uint32_t)e;
        eval[j] = (uint32_t)(e >> 32);
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) w[j] = q0 + j < a.n_words ? 1u : 0u;  // live entries
  } else if (q0 + K <= a.n_words) {
    const u32x4 *p4 = reinterpret_cast<const u32x4 *>(a.pack + q0);
#pragma unroll
    for (int i = 0; i < K / 4; ++i) {
      const u32x4 u = __builtin_nontemporal_load(p4 + i);
      w[4 * i] = u.x;
      w[4 * i + 1] = u.y;
      w[4 * i + 2] = u.z;
      w[4 * i + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) w[j] = q0 + j < a.n_words ? a.pack[q0 + j] : 0u;
  }

  // pass 1: the lane's column aggregate (absolute after a head, else a
  // delta sum) and the row of its last head
  // (float32 CSR entries carry their columns: only the rows are scanned)
  uint32_t run = 0, lrow = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t d = FMT == kCsr32 ? 0u : unpack(w[j], a.cd).delta;
    if ((hb >> j) & 1u) {
      lrow = hrow[lane * K + j];
      run = FMT == kCsr32 ? 0u : row_base(lrow, a.k_left) + d;
    } else {
      run += d;
    }
  }
  const bool has_head = hb != 0u;
  bool f = has_head;
  uint32_t v = run, rr = lrow;
  seg_scan_col(f, v, rr, lane);
  // exclusive values: what the lanes before this one leave open
  bool ef = __shfl_up((int)f, 1, kWave) != 0;
  uint32_t ev = __shfl_up(v, 1, kWave);
  uint32_t er = __shfl_up(rr, 1, kWave);
  if (lane == 0) {
    ef = false;
    ev = 0u;
    er = rlo - 1u;
  }
  const uint32_t anchor = FMT == kCsr32 ? 0u : a.anchor[c];
  uint32_t col = ef ? ev : anchor + ev;

  // pass 2: columns, gathers, per-row sums in word order
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * 4u * NR);
  const uint32_t oob = a.m * 4u * NR;
  float xv[K][NR], val[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if constexpr (FMT == kCsr32) {
      col = ecol[j];
      val[j] = __builtin_bit_cast(float, eval[j]);
    } else {
      const Unpacked u = unpack(w[j], a.cd);
      if ((hb >> j) & 1u) col = row_base(hrow[lane * K + j], a.k_left) + u.delta;
      else col += u.delta;
      val[j] = decode_value<FMT>(u.vbits);
    }
    const uint32_t off = (w[j] & 1u) ? col * 4u * NR : oob;
    if constexpr (NR == 4) {
      const f32x4 v4 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rx, off, 0, 0));
      xv[j][0] = v4.x;
      xv[j][1] = v4.y;
      xv[j][2] = v4.z;
      xv[j][3] = v4.w;
    } else {
#pragma unroll
      for (int q = 0; q < NR; ++q) xv[j][q] = buffer_load_f32(rx, off + 4u * q);
    }
  }
  // stores row r's NR sums
  auto put = [&](uint32_t r, const float (&v)[NR]) {
#pragma unroll
    for (int q = 0; q < NR; ++q) a.y[(int64_t)r * NR + q] = row_scaled<FMT>(v[q], a, r);
  };
  float acc[NR], lead[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = lead[q] = 0.0f;
  bool open = false;
  uint32_t cur = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if ((hb >> j) & 1u) {
      if (open) put(cur, acc);  // a row inside the lane
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (!open) lead[q] = acc[q];
        acc[q] = 0.0f;
      }
      open = true;
      cur = hrow[lane * K + j];
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = fmaf(val[j], xv[j][q], acc[q]);
  }
  if (!open) {
#pragma unroll
    for (int q = 0; q < NR; ++q) lead[q] = acc[q];
  }

  // the lanes' open sums: segmented by the same heads as the columns
  float s[NR], es[NR], total[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    s[q] = has_head ? acc[q] : lead[q];
    seg_scan_sum(has_head, s[q], lane);
    es[q] = __shfl_up(s[q], 1, kWave);
    if (lane == 0) es[q] = 0.0f;
    total[q] = es[q] + lead[q];
  }
  if (has_head) {
    // the row that ends just before this lane's first head
    if (ef) {
      put(er, total);
    } else {
#pragma unroll
      for (int q = 0; q < NR; ++q) a.head_part[(int64_t)c * NR + q] = total[q];  // continued
    }
  }
  if (lane == kWave - 1) {
    // f, s, rr: the chunk's last segment
    if (closed && f) {
      put(rr, s);
      a.tail_row[c] = -1;
    } else if (f) {
#pragma unroll
      for (int q = 0; q < NR; ++q) a.tail_part[(int64_t)c * NR + q] = s[q];
      a.tail_row[c] = (int32_t)rr;
    } else {
#pragma unroll
      for (int q = 0; q < NR; ++q) a.head_part[(int64_t)c * NR + q] = s[q];
      a.tail_row[c] = -1;
    }
  }
}

// Rows that continue past the chunk where they start: the open piece of
// that chunk plus the leading pieces of the following chunks, in chunk
// order.
template <int FMT, int NR>
__global__ void k_csr_rows_across(CsrArgs a, uint32_t T) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_chunks) return;
  const int32_t r = a.tail_row[c];
  if (r < 0) return;
  const int64_t end = a.rowptr[r + 1];
  const uint32_t c_end = (uint32_t)min<int64_t>((end - 1) / T, a.n_chunks - 1);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    float s = a.tail_part[(int64_t)c * NR + q];
    for (uint32_t k = c + 1; k <= c_end; ++k) s += a.head_part[(int64_t)k * NR + q];
    a.y[(int64_t)r * NR + q] = row_scaled<FMT>(s, a, (uint32_t)r);
  }
}

__global__ void k_csr_zero(float *y, int64_t n) {  // n = rows * right-hand sides
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0f;
}

template <int FMT, int NR>
int launch_chunks_nr(const CsrArgs &a, int K, hipStream_t st) {
  const uint32_t blocks = (uint32_t)cdiv(a.n_chunks, kCsrWaves);
  switch (K) {
    case 4: k_csr_chunks<FMT, 4, NR><<<blocks, kCsrBlock, 0, st>>>(a); break;
    case 8: k_csr_chunks<FMT, 8, NR><<<blocks, kCsrBlock, 0, st>>>(a); break;
    default: k_csr_chunks<FMT, 16, NR><<<blocks, kCsrBlock, 0, st>>>(a); break;
  }
  PKS_LAUNCHED();
  k_csr_rows_across<FMT, NR><<<cdiv(a.n_chunks, 256), 256, 0, st>>>(a, (uint32_t)(K * kWave));
  PKS_LAUNCHED();
  return PKSELL_OK;
}

template <int FMT>
int launch_chunks(const CsrArgs &a, int K, hipStream_t st) {
  switch (a.nr) {
    case 1: return launch_chunks_nr<FMT, 1>(a, K, st);
    case 2: return launch_chunks_nr<FMT, 2>(a, K, st);
    default: return launch_chunks_nr<FMT, 4>(a, K, st);
  }
}

}  // namespace

// y = A_q x for a CSR-packed matrix with a chunk plan (C = 1, sigma = 1,
// split_words = T); called by pksell_spmv for k = 1, 2 or 4.
int spmv_chunks(const pksell_matrix *A, const float *x, float *y, int64_t k, hipStream_t st) {
  const int64_t T = A->split_words;
  PKS_CHECK(A->C == 1 && A->sigma == 1 && (T == 256 || T == 512 || T == 1024), PKSELL_EINVAL,
            "chunked products need C = 1, sigma = 1 and split_words 256, 512 or 1024");
  PKS_CHECK(A->n_units == cdiv(A->n_words, T), PKSELL_EINVAL, "n_units does not match n_words");
  PKS_CHECK(A->n_units < (int64_t(1) << 31), PKSELL_ERANGE, "too many chunks");
  PKS_CHECK(A->n_units == 0 || (A->units && A->ckpt && A->partial), PKSELL_EINVAL,
            "chunked products need units, ckpt and partial");
  PKS_CHECK(((uintptr_t)A->pack & 15) == 0, PKSELL_EINVAL,
            "chunked products need 16-byte aligned words");
  PKS_CHECK(k == 1 || k == 2 || k == 4, PKSELL_EINVAL, "chunked products take k = 1, 2 or 4");
  PKS_CHECK(k != 4 || ((uintptr_t)x & 15) == 0, PKSELL_EINVAL,
            "chunked products with k = 4 need 16-byte aligned x");
  if (A->n_units == 0) {  // no words: every row is empty
    k_csr_zero<<<cdiv(A->n * k, 256), 256, 0, st>>>(y, A->n * k);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  CsrArgs a;
  a.pack = A->pack;
  a.rowptr = A->offset;
  a.lo = A->units;
  a.anchor = A->ckpt;
  a.row_exp = A->row_exp;
  a.x = x;
  a.y = y;
  a.head_part = A->partial;
  a.tail_part = A->partial + k * A->n_units;
  a.tail_row = reinterpret_cast<int32_t *>(A->partial + 2 * k * A->n_units);
  a.nr = (uint32_t)k;
  a.n_words = A->n_words;
  a.n = (uint32_t)A->n;
  a.m = (uint32_t)A->m;
  a.n_chunks = (uint32_t)A->n_units;
  a.k_left = (uint32_t)A->k_left;
  a.D = A->D;
  a.cd = make_codec(A->D);
  const int K = (int)(T / kWave);
  switch (A->fmt) {
    case PKSELL_FP16: return launch_chunks<PKSELL_FP16>(a, K, st);
    case PKSELL_E8MY: return launch_chunks<PKSELL_E8MY>(a, K, st);
    default: return launch_chunks<PKSELL_FIX>(a, K, st);
  }
}


namespace {

// lo[c] = the first row whose entries start at or after entry c T; lo[n_chunks] = n.
__global__ void k_csr32_lo(const int64_t *__restrict__ rowptr, int64_t n, int64_t n_chunks,
                           int64_t T, uint32_t *__restrict__ lo) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_chunks) return;
  if (c == n_chunks) {
    lo[c] = (uint32_t)n;
    return;
  }
  const int64_t p = c * T;
  int64_t lo_i = 0, hi_i = n;
  while (lo_i < hi_i) {
    const int64_t mid = (lo_i + hi_i) / 2;
    if (rowptr[mid] < p) lo_i = mid + 1;
    else hi_i = mid;
  }
  lo[c] = (uint32_t)lo_i;
}

template <typename V>
__global__ void k_csr32_fill(const int32_t *__restrict__ col, const V *__restrict__ val,
                             int64_t nnz, uint64_t *__restrict__ ent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const float v = (float)val[i];
  ent[i] = (uint64_t)(uint32_t)col[i] | ((uint64_t)__builtin_bit_cast(uint32_t, v) << 32);
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_csr32_query(int64_t n, int64_t m, int64_t nnz, int32_t T, pksell_csr32 *A) {
  PKS_CHECK(A, PKSELL_EINVAL, "null descriptor");
  PKS_CHECK(T == 256 || T == 512 || T == 1024, PKSELL_EINVAL, "T must be 256, 512 or 1024");
  PKS_CHECK(n >= 0 && m >= 0 && n < (int64_t(1) << 30) && m < (int64_t(1) << 30), PKSELL_EINVAL,
            "n and m must be in [0, 2^30)");
  PKS_CHECK(nnz >= 0 && nnz < (int64_t(1) << 31), PKSELL_EINVAL, "nnz must be in [0, 2^31)");
  std::memset(A, 0, sizeof(*A));
  A->n = n;
  A->m = m;
  A->nnz = nnz;
  A->T = T;
  A->n_chunks = cdiv(nnz, T);
  return PKSELL_OK;
}

int pksell_csr32_encode(const int32_t *col, const void *val, int32_t val_dtype, pksell_csr32 *A,
                        void *stream) {
  PKS_CHECK(A, PKSELL_EINVAL, "null descriptor");
  PKS_CHECK(val_dtype == PKSELL_F32 || val_dtype == PKSELL_F64, PKSELL_EINVAL,
            "val_dtype must be PKSELL_F32 or PKSELL_F64");
  PKS_CHECK(A->n_chunks == cdiv(A->nnz, A->T), PKSELL_EINVAL, "descriptor not from the query");
  PKS_CHECK(A->rowptr && A->lo && (A->nnz == 0 || (A->ent && col && val)), PKSELL_EINVAL,
            "arrays not set");
  hipStream_t st = as_stream(stream);
  if (A->nnz > 0) {
    if (val_dtype == PKSELL_F32)
      k_csr32_fill<float><<<cdiv(A->nnz, 256), 256, 0, st>>>(col, static_cast<const float *>(val),
                                                            A->nnz, A->ent);
    else
      k_csr32_fill<double><<<cdiv(A->nnz, 256), 256, 0, st>>>(
          col, static_cast<const double *>(val), A->nnz, A->ent);
    PKS_LAUNCHED();
  }
  k_csr32_lo<<<cdiv(A->n_chunks + 1, 256), 256, 0, st>>>(A->rowptr, A->n, A->n_chunks, A->T,
                                                         A->lo);
  PKS_LAUNCHED();
  return PKSELL_OK;
}

int pksell_csr32_spmv(const pksell_csr32 *A, const float *x, float *y, void *stream) {
  PKS_CHECK(A, PKSELL_EINVAL, "null descriptor");
  PKS_CHECK(A->T == 256 || A->T == 512 || A->T == 1024, PKSELL_EINVAL, "bad T");
  PKS_CHECK(A->n_chunks == cdiv(A->nnz, A->T), PKSELL_EINVAL, "descriptor not from the query");
  PKS_CHECK(A->n == 0 || y, PKSELL_EINVAL, "null y");
  hipStream_t st = as_stream(stream);
  if (A->n == 0) return PKSELL_OK;
  if (A->n_chunks == 0) {  // no entries: every row is empty
    k_csr_zero<<<cdiv(A->n, 256), 256, 0, st>>>(y, A->n);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  PKS_CHECK(x && A->rowptr && A->ent && A->lo && A->partial, PKSELL_EINVAL, "arrays not set");
  PKS_CHECK(((uintptr_t)A->ent & 15) == 0, PKSELL_EINVAL, "ent must be 16-byte aligned");
  CsrArgs a{};
  a.pack = reinterpret_cast<const uint32_t *>(A->ent);
  a.rowptr = A->rowptr;
  a.lo = A->lo;
  a.anchor = nullptr;
  a.row_exp = nullptr;
  a.x = x;
  a.y = y;
  a.head_part = A->partial;
  a.tail_part = A->partial + A->n_chunks;
  a.tail_row = reinterpret_cast<int32_t *>(A->partial + 2 * A->n_chunks);
  a.nr = 1;
  a.n_words = A->nnz;
  a.n = (uint32_t)A->n;
  a.m = (uint32_t)A->m;
  a.n_chunks = (uint32_t)A->n_chunks;
  a.k_left = 0;
  a.D = 0;
  return launch_chunks_nr<kCsr32, 1>(a, A->T / kWave, st);
}

}  // extern "C"
