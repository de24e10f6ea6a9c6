/* pksell.h -- PackSELL sparse matrix-vector products on AMD MI355X (gfx950).
 *
 * PackSELL (Suzuki & Iwashita, "PackSELL: A Sparse Matrix Format for
 * Precision-Agnostic High-Performance SpMV") is sliced ELLPACK in which every
 * stored element is one 32-bit word holding a column delta and a quantised
 * value.  Word layout (sec. 4.2.1, W = V + D + 1 = 32): bit 0 is a flag;
 * flag = 1 puts the value in the upper V bits and a delta < 2^D in bits
 * 1..D; flag = 0 puts a delta up to 2^31 - 1 in bits 1..31 and no value (a
 * "dummy", inserted before an element whose delta does not fit, sec. 4.3).
 * The all-zero word is padding.  Column indices are rebuilt as running sums
 * of deltas from a left offset that is uniform within each sigma-block of
 * rows (eq. 4).  Rows are grouped in slices of C rows stored column-major,
 * after a descending sort by stored-word count inside windows of sigma rows
 * (SELL-C-sigma, sec. 3).
 *
 * Conventions for every call:
 *  - Pointers named in a call are DEVICE pointers unless said otherwise; the
 *    caller allocates and owns all of them.  The library allocates no device
 *    memory; scratch space is passed in as a workspace (``ws``).
 *  - ``stream`` is a hipStream_t (NULL = the default stream).  All device
 *    work is enqueued on it asynchronously unless a call says it
 *    synchronises.
 *  - Every call returns a status code (PKSELL_OK = 0, negative on error);
 *    pksell_status_string() names it, and pksell_last_error() gives detail
 *    for the calling thread.  Inputs are never modified.
 *  - Sizes: n, m < 2^30 (so byte offsets into x fit 32 bits), columns < m.
 */
#ifndef PKSELL_H
#define PKSELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PKSELL_OK 0
#define PKSELL_EINVAL (-1)      /* bad argument, shape or CSR structure */
#define PKSELL_ERANGE (-2)      /* a size exceeds what the format or kernels address */
#define PKSELL_EWORKSPACE (-3)  /* workspace missing or too small */
#define PKSELL_EHIP (-4)        /* a HIP runtime call failed */
#define PKSELL_ENOTCONV (-5)    /* solver hit its iteration limit */
#define PKSELL_EBREAKDOWN (-6)  /* solver breakdown (p^T A p <= 0 or NaN) */

/* ---- value formats (sec. 4.2.2) ---------------------------------------- */
#define PKSELL_FP16 0 /* IEEE binary16 in the upper 16 bits; D must be 15 */
#define PKSELL_E8MY 1 /* FP32-compatible float, Y = 22 - D mantissa bits; 1 <= D <= 22 */
#define PKSELL_FIX 2  /* (31-D)-bit two's-complement integer times a per-row
                         power of two; 1 <= D <= 29 */
#define PKSELL_E11MY 3 /* 64-bit words (sec. 4.2.1 with W = 64): an
                          FP64-compatible float with Y = 51 - D mantissa bits,
                          the E8MY construction applied to FP64; 1 <= D <= 51.
                          Products in float64 through pksell_spmv_f64 only. */
/* 16-bit words (sec. 4.2.1 with W = 16): a value word has its delta in bits
 * 1..D and 15 - D value bits; a dummy carries at most 2^15 - 1, so a larger
 * delta takes a chain of dummies (all but the last carrying 2^15 - 1)
 * before its value word.  C must be 64.  Products through pksell_spmv
 * (any k), and the solvers' inner operator (pksell_pcg, pksell_pcg64);
 * every other entry point rejects these formats. */
#define PKSELL_E5MY 4  /* binary16-compatible float, Y = 9 - D mantissa bits
                          (the E8MY construction applied to binary16; D = 7 is
                          8-bit E5M2); 1 <= D <= 8 */
#define PKSELL_FIX16 5 /* (15-D)-bit two's-complement integer times a per-row
                          power of two (D = 7: int8); 1 <= D <= 13 */

/* ---- row permutation modes (sec. 3) ------------------------------------ */
#define PKSELL_EXPLICIT 0 /* results are produced in stored (sorted) row order */
#define PKSELL_IMPLICIT 1 /* results are produced in the original row order via perm */

/* ---- value input types ------------------------------------------------- */
#define PKSELL_F32 4
#define PKSELL_F64 8
/* SELL values only: IEEE binary16 values (rounded from float32 with ties to
 * even, float64 input rounded to float32 first, as for PackSELL FP16 words),
 * float32 x and y, float32 accumulation: the plain-SELL counterpart of the
 * FP16 PackSELL words (int32 column + 2-byte value per slot). */
#define PKSELL_F16 2
/* SELL values only: float32 values with their int32 columns side by side,
 * one 8-byte slot per entry (column in the low 4 bytes, value bits in the
 * high 4), float32 vectors: one load per slot instead of two.  S->val
 * points to the uint64 slots; S->col is not used (may be NULL). */
#define PKSELL_F32_PAIRED 12

/* A PackSELL matrix.  pksell_encode_query() fills the shape and parameter
 * fields; the analyse phase of pksell_encode() fills n_words, n_dummies and
 * k_left; the caller allocates the device arrays.
 *
 *   pack     uint32[n_words]     slice k occupies [offset[k], offset[k+1]),
 *                                word j of lane l at offset[k] + j*C + l
 *                                (E11MY: uint64[n_words], 64-bit words, the
 *                                same layout; the pointer is cast.  E5MY and
 *                                FIX16: uint32[n_words / 2], 16-bit words two
 *                                per slot -- words 2i (low half) and 2i + 1
 *                                (high half) of lane l in slot offset[k]/2 +
 *                                i*C + l; every lane's word count is rounded
 *                                up to even with a zero padding word)
 *   offset   int64[n_slices + 1] slice starts in words (sec. 3)
 *   perm     uint8 (sigma <= 256) or uint16 [n]  original row minus its
 *                                window start, per stored row (implicit mode
 *                                only; may be NULL in explicit mode)
 *   row_exp  int16[n]            FIX and FIX16: row scale exponent e, stored order
 *                                (decoded value = q * 2^e)
 *
 * Wide-slice splitting (C = 64 only; optional).  Set split_words = J (a
 * multiple of 8, 0 = off) after pksell_encode_query.  The analyse phase then
 * counts the work units: a slice wider than J words per lane becomes
 * ceil(w / J) units of J words, a narrower slice one unit.  When some slice
 * is split (n_split_units > 0) the caller also allocates
 *   units    uint32[4 * n_units]        {slice, chunk, chunks, base} per unit
 *   splits   uint32[4 * n_split_slices] {slice, base, chunks, 0} per split slice
 *   ckpt     uint32[64 * n_split_units] column reached by each lane at the
 *                                       start of each chunk (index base + chunk)
 *   partial  float[64 * n_split_units]  per-chunk sums (scratch of pksell_spmv:
 *                                       one product at a time per matrix)
 * and the fill phase writes units, splits and ckpt.  Products with k = 1 then
 * run one work unit per wave and add each split slice's chunk sums in chunk
 * order (deterministic); other calls ignore the split arrays.
 *
 * CSR-packed matrices (C = 1 and sigma = 1; 32-bit words).  With one-row
 * slices and no sort, every row's words lie together in row order with no
 * padding, and offset is a word row pointer: delta-value packing in a
 * CSR-based layout, which the paper leaves to future work (sec. 6).  Set
 * split_words = T (256, 512 or 1024) after pksell_encode_query to give
 * pksell_spmv (k = 1, 2, or 4 with 16-byte aligned x; a k = 4 product with
 * misaligned x runs the one-row-slice product instead) a product
 * balanced over words: the word stream is
 * cut into n_units = ceil(n_words / T) chunks of T words, one per wave,
 * whatever rows they fall in.  The analyse phase sets n_units
 * (n_split_units = n_split_slices = 0); the caller then allocates
 *   units    uint32[n_units + 1]  first row whose words start at or after
 *                                 word c*T (units[n_units] = n)
 *   ckpt     uint32[n_units]      column reached before word c*T (the row's
 *                                 eq. 4 left offset when a row starts there)
 *   partial  float[9 * n_units]   scratch of pksell_spmv (one product at a
 *                                 time per matrix): pieces of the rows that
 *                                 cross chunk edges (k per chunk and side)
 *                                 and those rows' indices
 * and the fill phase writes units and ckpt.  pack must be 16-byte aligned
 * for these products.  Rows crossing chunk edges are summed piece by piece
 * in chunk order by a second kernel: results are deterministic.  Products
 * with other k and the other entry points ignore the plan.
 */
typedef struct pksell_matrix {
  int64_t n, m, nnz;
  int32_t C, sigma, D, fmt, perm_mode, perm_bytes;
  int64_t n_slices;
  int64_t n_words, n_dummies, k_left;
  uint32_t *pack;
  int64_t *offset;
  void *perm;
  int16_t *row_exp;
  int32_t split_words, cache_hint; /* cache_hint: PKSELL_CACHE_* below */
  int64_t n_units, n_split_units, n_split_slices;
  uint32_t *units;
  uint32_t *splits;
  uint32_t *ckpt;
  float *partial;
} pksell_matrix;

/* How the single-vector products with C = 64 (pksell_spmv with k = 1 on
 * 32-bit words; pksell_sell_spmv with float32 vectors) load the matrix;
 * other products ignore it.  pksell_encode_query and pksell_sell_query set
 * 0; the caller may change it at any time between products.  Any other
 * value acts as PKSELL_CACHE_STREAM.
 *   PKSELL_CACHE_STREAM    streaming cache policy: the product reads each
 *                          word once and keeps none (the fastest policy
 *                          when the matrix is not read again soon);
 *   PKSELL_CACHE_RESIDENT  default policy: for a matrix applied many times
 *                          in a row (an iterative method), so that one that
 *                          fits in the 256 MB last-level cache stays there
 *                          between products.
 * The results are the same either way, bit for bit. */
#define PKSELL_CACHE_STREAM 0
#define PKSELL_CACHE_RESIDENT 1

/* Plain SELL-C-sigma (sec. 3) with float32 or float64 values and int32
 * columns -- the same-GPU comparator and the float64 operator of the outer
 * solver.  Padding slots hold value 0 and the row's last column.
 *   val  float or double [n_slots], col int32[n_slots], offset int64[n_slices+1]
 */
typedef struct pksell_sell {
  int64_t n, m, nnz;
  int32_t C, sigma, perm_mode, perm_bytes, dtype; /* PKSELL_F32/F64/F16 */
  int32_t cache_hint; /* PKSELL_CACHE_* (above) */
  int64_t n_slices, n_slots;
  int64_t *offset;
  void *perm;
  int32_t *col;
  void *val;
} pksell_sell;

/* Plain CSR with float32 values, the comparator of the CSR-packed product:
 * entries in row order, each 8 bytes (column in the low 32 bits, float32
 * value bits in the high 32), and a chunk plan over entries.
 *   rowptr int64[n + 1] (the caller's; rowptr[0] = 0, non-decreasing,
 *          rowptr[n] = nnz), ent uint64[nnz], lo uint32[n_chunks + 1]
 *          (the first row starting at or after entry c T, then n),
 *   partial float32[3 n_chunks] (scratch of the product) */
typedef struct pksell_csr32 {
  int64_t n, m, nnz;
  int32_t T;        /* entries per chunk: 256, 512 or 1024 */
  int32_t reserved;
  int64_t n_chunks; /* ceil(nnz / T) */
  const int64_t *rowptr;
  uint64_t *ent;
  uint32_t *lo;
  float *partial;
} pksell_csr32;

/* Result of pksell_pcg (host struct). */
typedef struct pksell_pcg_info {
  int32_t outer_iterations; /* outer (FCG) iterations, or CG iterations */
  int32_t inner_iterations; /* total inner iterations */
  double rel_residual;      /* final true ||b - A x||_2 / ||b||_2 */
  double seconds;           /* wall time of the solve on the host clock */
} pksell_pcg_info;

/* Library version (major*10000 + minor*100 + patch). */
int pksell_version(void);

/* Static name of a status code. */
const char *pksell_status_string(int status);

/* Detail of the last failing call on the calling host thread (static buffer). */
const char *pksell_last_error(void);

/* ------------------------------------------------------------------------
 * Encoding CSR -> PackSELL (sec. 4.1 delta encoding with eq. 4 left offsets,
 * sec. 4.2 packing, sec. 4.3 dummies, padding and the sigma-window sort).
 * ---------------------------------------------------------------------- */

/* Validates (n, m, nnz, C, sigma, D, fmt, perm_mode), fills A's shape and
 * parameter fields (n_slices = ceil(n/C), perm_bytes), sets its array
 * pointers to NULL, and writes the workspace size pksell_encode needs to
 * *ws_bytes (host pointers).  C is a power of two in [1, 64]; sigma in
 * [1, 65536].  Returns PKSELL_EINVAL on bad parameters, PKSELL_ERANGE when n
 * or m reaches 2^30.  No device work. */
int pksell_encode_query(int64_t n, int64_t m, int64_t nnz, int32_t C,
                        int32_t sigma, int32_t D, int32_t fmt,
                        int32_t perm_mode, pksell_matrix *A, size_t *ws_bytes);

/* Encodes a device CSR matrix (rowptr int64[n+1], col int32[nnz] strictly
 * increasing within each row, val float32 or float64 [nnz] per val_dtype;
 * float64 values are rounded to float32 first, as sec. 4.2.2 converts from
 * float).  Two phases, chosen by A->pack:
 *
 *  - A->pack == NULL (analyse): needs A->offset (and A->perm in implicit
 *    mode).  Validates the CSR on the device, computes the lower bandwidth
 *    k_left, the per-row word counts (nonzeros + dummies), the sigma-window
 *    sort and the slice offsets; then SYNCHRONISES the stream and fills
 *    A->n_words, A->n_dummies, A->k_left.  The caller then allocates
 *    A->pack (n_words) and, for FIX, A->row_exp (n).
 *  - A->pack != NULL (fill): writes every word of A->pack (padding included)
 *    and A->row_exp; asynchronous.  ``ws`` must still hold what the analyse
 *    phase left in it.
 *
 * Errors: PKSELL_EINVAL for a malformed CSR (unsorted or duplicate columns,
 * column >= m, bad rowptr) or non-finite values in FIX; PKSELL_EWORKSPACE
 * when ws_bytes is below pksell_encode_query's size. */
int pksell_encode(const int64_t *rowptr, const int32_t *col, const void *val,
                  int32_t val_dtype, pksell_matrix *A, void *ws,
                  size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Products (sec. 4.4 PackSELL SpMV).  k right-hand sides are row-major
 * blocks: x is m x k, y is n x k (element (r, c) at r*k + c).
 * ---------------------------------------------------------------------- */

/* y = A_q x with float32 accumulation; y is overwritten (no beta term).  In
 * implicit mode y is in the original row order, in explicit mode in stored
 * order.  1 <= k <= 64.  With k a multiple of 4 and x, y 16-byte aligned, x
 * is gathered and y stored four columns at a time.  16-bit words (E5MY,
 * FIX16) take any such k too: k > 1 runs in passes of up to eight columns
 * over the words. */
int pksell_spmv(const pksell_matrix *A, const float *x, float *y, int64_t k,
                void *stream);

/* pksell_spmv for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product and the same result, bit for bit, but the scratch that
 * products of CSR-packed matrices with a chunk plan (k = 1, 2, or 4 with
 * 16-byte aligned x) and of split wide slices (k = 1) need comes from one
 * 16 MiB float32 array that the library holds on each GPU until the process
 * ends, instead of A->partial (which may then be NULL).  Such a product
 * needs (2k + 1) * n_units floats (chunk plan) or 64 * n_split_units
 * (split slices); beyond 2^22 floats the call returns PKSELL_ERANGE before
 * any device work.  Other products need no scratch and run as pksell_spmv.
 * The call allocates nothing.  Its first call on a device looks up that
 * device's array (the stream must belong to the current device, else
 * PKSELL_EINVAL).  Every call on one GPU shares that GPU's array, and each
 * product writes all the scratch it reads: calls that overlap on one GPU
 * (on different streams, or on one stream with a concurrent graph replay)
 * race, so serialise them. */
int pksell_spmv_static(const pksell_matrix *A, const float *x, float *y, int64_t k,
                       void *stream);

/* y = A_q^T g (the adjoint: grad_x of <g, A x>).  g is n x k in the row
 * order pksell_spmv produces; y (m x k) is zeroed on the stream and then
 * accumulated with float32 atomics, so the summation order is not fixed. */
int pksell_spmv_t(const pksell_matrix *A, const float *g, float *y,
                  int64_t k, void *stream);

/* Gradient of <g, A x> with respect to every stored value:
 * grad[e] = sum_s g[i, s] * x[j, s] for each stored nonzero e = (i, j) of the
 * CSR matrix the words were encoded from, in that CSR's order (rowptr
 * int64[n+1] of the ORIGINAL matrix; quantisation is treated as the
 * identity).  g (n x k) in pksell_spmv's row order, x (m x k), row-major.
 * Needs A->perm (the stored-to-original row map) in both modes. */
int pksell_grad_values(const pksell_matrix *A, const int64_t *rowptr,
                       const float *g, const float *x, float *grad, int64_t k,
                       void *stream);

/* The transpose of a CSR matrix on the device, for a PackSELL copy of A^T
 * (not in the paper).  With the element-wise quantisers (FP16, E8MY) the
 * encoded copy holds exactly (A_q)^T, so grad_x = A_q^T g becomes a forward
 * pksell_spmv on it, with no atomics; FIX quantises per row, so its A^T
 * copy would hold different values and its adjoint stays pksell_spmv_t.
 *
 * Input: rowptr int64[n+1], col int32[nnz] (in [0, m), strictly increasing
 * per row), val (float32 or float64 per val_dtype) [nnz].  Output (caller
 * allocated): t_rowptr int64[m+1], t_col int32[nnz] (rows of A, ascending
 * per column), t_val [nnz] in the input's value type.  A stable radix sort
 * by column: deterministic.  Needs nnz < 2^31 - 1.  Validates rowptr and the
 * column range first (EINVAL on malformed input, no writes), which
 * SYNCHRONISES once; the rest is asynchronous on ``stream``.
 * pksell_csr_transpose_query sizes the workspace; it asks the current
 * device for the sort's scratch size, so it needs a GPU. */
int pksell_csr_transpose_query(int64_t n, int64_t m, int64_t nnz, size_t *ws_bytes);
int pksell_csr_transpose(const int64_t *rowptr, const int32_t *col,
                         const void *val, int32_t val_dtype, int64_t n,
                         int64_t m, int64_t nnz, int64_t *t_rowptr,
                         int32_t *t_col, void *t_val, void *ws,
                         size_t ws_bytes, void *stream);

/* Measurement helper (not in the paper): one streaming read of ``bytes``
 * (a positive multiple of 16; src 16-byte aligned) in a single launch, to
 * measure the practical HBM read ceiling for a transfer of that size.  Each
 * wave reads ``chunks`` (1..4096) consecutive pieces of 64 lanes x ``width``
 * (4 or 16) bytes with nontemporal loads, eight in flight per lane.
 * ``out`` (device, >= 1 float) is only there so the loads are kept; its
 * contents carry no meaning. */
int pksell_stream_read(const void *src, size_t bytes, int32_t width,
                       int32_t chunks, float *out, void *stream);

/* y = A_q x in float64 for 64-bit-word matrices (fmt E11MY): x float64[m x k]
 * and y float64[n x k], row-major, k in [1, 64] right-hand sides (rows of y
 * in original order in implicit mode, stored order in explicit mode), each
 * column accumulated in float64 in word order.  m * k < 2^29, else ERANGE.
 * Not in the paper as such: its W = 64 word with the E8MY value
 * construction applied to FP64, for FP64 operators at 8 bytes per stored
 * word.  Other product, adjoint, batched and solver entry points reject
 * E11MY. */
int pksell_spmv_f64(const pksell_matrix *A, const double *x, double *y, int64_t k,
                    void *stream);

/* Decodes every word position: cols[p] = column reconstructed at word p
 * (running sum of deltas from the left offset), vals[p] = decoded value
 * (0 for flag-0 words; FIX: q * 2^e).  Positions of phantom rows past n are
 * left untouched.  For checking encoders against a reference. */
int pksell_decode(const pksell_matrix *A, int32_t *cols, float *vals,
                  void *stream);

/* ------------------------------------------------------------------------
 * Sparse triangular solves on CSR-packed words (not in the paper as such:
 * it names triangular solves as a kernel its packing should suit, sec. 6).
 * L is n x n and triangular: lower (upper = 0) with every row ending in its
 * diagonal entry, or upper (upper = 1) with every row starting with it.  It
 * is encoded as a CSR-packed matrix (C = 1, sigma = 1, no split_words
 * needed) with FP16, E8MY or FIX words, so the solve uses the quantised L_q.
 * ---------------------------------------------------------------------- */

/* Level schedule: level(i) = 0 for a row with only its diagonal, else
 * 1 + the largest level among its off-diagonal columns (rows taken in
 * ascending order for lower, descending for upper).  Input: the device
 * CSR of L (rowptr int64[n+1], col int32[nnz]) and ``upper``.  Output: order (device
 * int32[n]: rows by ascending level, ascending row order inside a level),
 * level_ptr (HOST int64[n + 1]: level l holds order[level_ptr[l] ..
 * level_ptr[l+1])) and *n_levels (host).  Copies the CSR structure to the
 * host and walks it once; SYNCHRONISES the stream.  EINVAL when a row is
 * empty, its diagonal is not where ``upper`` puts it, or its other columns
 * do not increase on that side of the diagonal. */
int pksell_trsv_levels(const int64_t *rowptr, const int32_t *col, int64_t n,
                       int32_t upper, int32_t *order, int64_t *level_ptr,
                       int64_t *n_levels, void *stream);

/* Solves L_q y = b (float32 b and y, device, n each; y must not alias b):
 * y_i = (b_i - sum_{j != i} (L_q)_ij y_j) / (L_q)_ii with float32 sums in
 * word order, one launch per level on ``stream`` (order on the device,
 * level_ptr on the host, from pksell_trsv_levels on the same CSR and the
 * same ``upper``).  A zero diagonal gives inf or NaN.  EINVAL unless L is
 * CSR-packed with 32-bit words, square, and level_ptr spans its n rows. */
int pksell_trsv(const pksell_matrix *L, int32_t upper, const int32_t *order,
                const int64_t *level_ptr, int64_t n_levels, const float *b,
                float *y, void *stream);

/* The same level-scheduled solve on plain CSR (int32 columns, float32
 * values, 8 bytes per entry): the comparator for pksell_trsv. */
int pksell_trsv_csr(const int64_t *rowptr, const int32_t *col,
                    const float *val, int64_t n, int32_t upper,
                    const int32_t *order, const int64_t *level_ptr,
                    int64_t n_levels, const float *b, float *y, void *stream);

/* ------------------------------------------------------------------------
 * Plain SELL-C-sigma (sec. 3), the comparator and the float64 operator.
 * ---------------------------------------------------------------------- */

/* As pksell_encode_query for SELL; dtype is PKSELL_F32, PKSELL_F64,
 * PKSELL_F16 or PKSELL_F32_PAIRED (the value type and slot layout; vectors
 * are float32 for F16 and F32_PAIRED). */
int pksell_sell_query(int64_t n, int64_t m, int64_t nnz, int32_t C,
                      int32_t sigma, int32_t dtype, int32_t perm_mode,
                      pksell_sell *S, size_t *ws_bytes);

/* As pksell_encode: analyse when S->val == NULL (needs S->offset, S->perm;
 * synchronises; fills S->n_slots), fill otherwise (needs S->val, and S->col
 * unless the slots are paired). */
int pksell_sell_encode(const int64_t *rowptr, const int32_t *col,
                       const void *val, int32_t val_dtype, pksell_sell *S,
                       void *ws, size_t ws_bytes, void *stream);

/* y = S x in S->dtype (x: m, y: n, of S->dtype), accumulated in S->dtype
 * with one fused multiply-add per slot in slot order; for PKSELL_F16 and
 * PKSELL_F32_PAIRED, x and y are float32 and the sums float32. */
int pksell_sell_spmv(const pksell_sell *S, const void *x, void *y,
                     void *stream);

/* ------------------------------------------------------------------------
 * Float32 CSR balanced over entries: the comparator for the CSR-packed
 * product (not in the paper).  The entry stream is cut into chunks of T
 * entries, one 64-lane wave each, with the chunk kernel of the CSR-packed
 * words: lane-sequential entries, segmented wave scans for the row sums,
 * rows across chunks added in chunk order.
 * ---------------------------------------------------------------------- */

/* Fills A's sizes (n, m, nnz, T, n_chunks) from the arguments; no device
 * work.  EINVAL unless T is 256, 512 or 1024, n, m < 2^30 and
 * nnz < 2^31. */
int pksell_csr32_query(int64_t n, int64_t m, int64_t nnz, int32_t T, pksell_csr32 *A);

/* Builds ent (float32 values; float64 input rounded to nearest) and lo
 * from a device CSR (rowptr as above; col int32[nnz] in [0, m); val
 * float32 or float64 [nnz] per val_dtype).  Asynchronous on ``stream``.
 * Needs A->rowptr, A->ent and A->lo set; A->rowptr must stay valid for
 * the products. */
int pksell_csr32_encode(const int32_t *col, const void *val, int32_t val_dtype,
                        pksell_csr32 *A, void *stream);

/* y = A x, float32, each row's products summed in entry order within a
 * lane and then across lanes and chunks in a fixed order (deterministic).
 * x float32[m], y float32[n]; A->partial must hold 3 n_chunks floats.
 * Columns out of range read 0. */
int pksell_csr32_spmv(const pksell_csr32 *A, const float *x, float *y, void *stream);

/* ------------------------------------------------------------------------
 * Batched products: many PackSELL matrices (uneven sizes, one value format,
 * C = 64, each with its own D) and k right-hand sides in one persistent
 * launch.  Not in the paper; the per-matrix arithmetic is pksell_spmv's.
 * ---------------------------------------------------------------------- */

/* One matrix of a batch: A (host pointer to its descriptor) and its input
 * and output blocks (device, row-major).  Forward: in = x (m x k),
 * out = y (n x k).  Transposed: in = g (n x k), out = A^T g (m x k). */
typedef struct pksell_batch_item {
  const pksell_matrix *A;
  const float *in;
  float *out;
} pksell_batch_item;

/* A batch plan (host struct; ``items`` and ``unit_start`` point into the
 * plan workspace on the device). */
typedef struct pksell_batch {
  int32_t count, fmt, k, transpose;
  int64_t total_units;      /* work units over all matrices: slices x group */
  int32_t units_per_wave, waves;  /* wave w takes units w, w + waves, ... */
  int32_t vec4;             /* k % 4 == 0 and 16-byte aligned blocks: 16-byte gathers */
  int32_t group;            /* lanes per row: L = 2..16 (forward, vec4, k >= 8), else 1 */
  int32_t words_per_group;  /* k = 1 loop: words per group, from the batch's average
                               slice width (4..8) */
  int32_t pair_units;       /* k = 1 forward: slice pairs over all matrices, each one
                               wave of the two-slice product (0: the pipelined loop) */
  void *items;
  void *unit_start;
} pksell_batch;

/* Device workspace bytes of a plan for ``count`` matrices (host call). */
int pksell_batch_plan_bytes(int32_t count, size_t *bytes);

/* Validates the items and writes the plan's device table into ``ws`` (which
 * must stay alive and unchanged while the plan is used); SYNCHRONISES once.
 * transpose != 0 plans out = A^T in. */
int pksell_batch_plan(const pksell_batch_item *items, int32_t count, int64_t k,
                      int32_t transpose, pksell_batch *plan, void *ws,
                      size_t ws_bytes, void *stream);

/* Runs a plan: k = 1 forward plans with pair_units > 0, one launch of the
 * two-slice product over every slice pair of the batch; otherwise one
 * persistent launch (lane groups, group > 1: every k in one pass; else one
 * launch per pass of up to 32 right-hand sides) (a transposed plan first
 * zeroes its outputs with a kernel, then scatters with float32 atomics).
 * Asynchronous, and safe to capture in a graph. */
int pksell_spmv_batched(const pksell_batch *plan, void *stream);

/* ------------------------------------------------------------------------
 * Solvers (sec. 5.2): A x = b with ||b - A x||_2 / ||b||_2 < tol (eq. 6).
 * ---------------------------------------------------------------------- */

/* Workspace bytes pksell_pcg needs for these matrices (A_lo may be NULL). */
int pksell_pcg_workspace(const pksell_matrix *A_lo, const pksell_sell *A_hi,
                         size_t *ws_bytes);

/* Solves A x = b for a symmetric positive definite A given as A_hi, a
 * float64 SELL matrix in implicit row order.  x (float64, n) holds the
 * initial guess on entry and the solution on return; b (float64, n).
 *
 *  - A_lo != NULL: the inner-outer CG of sec. 5.2.2.  Outer iterations are
 *    flexible CG (one previous direction kept) in float64 on A_hi; each is
 *    preconditioned by m_in float32 CG iterations on A_lo, the PackSELL
 *    encoding of the same matrix (implicit row order; FP16, E8MY or FIX
 *    words, or 16-bit E5MY or FIX16 words with C = 64), started from zero on
 *    the right-hand side r / ||r||.  Inner dot products, alpha and beta are
 *    accumulated in float64.  max_outer bounds outer iterations.
 *  - A_lo == NULL: plain float64 CG on A_hi (the baseline); max_outer bounds
 *    iterations, m_in is ignored.
 *
 * No preconditioner is applied beyond the inner solve: scale the system
 * symmetrically (Gbar^-1 A Gbar^-1, unit diagonal, sec. 5.2) beforehand so
 * that Jacobi is the identity.  Convergence is judged on the recursively
 * updated residual and confirmed on the true residual b - A x in float64
 * (otherwise the iteration restarts from it).  ``info`` (host) receives
 * iteration counts, the final true relative residual and the wall time.
 * The call SYNCHRONISES: it waits for ``stream``, runs on a private stream
 * (iterations replayed from captured HIP graphs, the host polling a few
 * device scalars per replay) and returns when done.
 * Returns PKSELL_ENOTCONV at the iteration limit (x holds the last
 * iterate), PKSELL_EBREAKDOWN when p^T A p <= 0 or is not finite. */
int pksell_pcg(const pksell_matrix *A_lo, const pksell_sell *A_hi,
               const double *b, double *x, double tol, int32_t m_in,
               int32_t max_outer, pksell_pcg_info *info, void *ws,
               size_t ws_bytes, void *stream);

/* The same solvers with the float64 operator A_hi given as a 64-bit-word
 * PackSELL matrix (fmt E11MY, implicit row order, no split units) instead
 * of float64 SELL: 8 bytes per stored word for the outer products and the
 * true residual, instead of 12 per SELL slot.  Everything else (A_lo,
 * arguments, synchronisation, status codes) is as in pksell_pcg; the system
 * solved is the one whose matrix A_hi holds, i.e. A with its values rounded
 * to 52 - D significant bits.  Both calls return PKSELL_EINVAL, before any
 * device work, when A_hi is not an E11MY matrix; pksell_pcg64 also when it
 * is not square or not in implicit row order. */
int pksell_pcg64_workspace(const pksell_matrix *A_lo, const pksell_matrix *A_hi,
                           size_t *ws_bytes);
int pksell_pcg64(const pksell_matrix *A_lo, const pksell_matrix *A_hi,
                 const double *b, double *x, double tol, int32_t m_in,
                 int32_t max_outer, pksell_pcg_info *info, void *ws,
                 size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * F3R nested Krylov solver (sec. 5.2.1): A x = b with
 * ||b - A x||_2 / ||b||_2 < tol (eq. 6), for square (not necessarily
 * symmetric) A.
 * ---------------------------------------------------------------------- */

/* Layer parameters.  The paper takes them from the solver's own defaults
 * and names no values; ours are the caller's choice (the Python binding
 * uses m1 = 100, m2 = 8, m3 = 4, m4 = 2, omega = 1). */
typedef struct pksell_f3r_params {
  int32_t m1;         /* outer FGMRES steps per restart cycle, 1..200 */
  int32_t m2;         /* second-layer FGMRES steps (one cycle from zero), 1..32 */
  int32_t m3;         /* third-layer FGMRES steps (one cycle from zero), 1..32 */
  int32_t m4;         /* Richardson iterations from zero, 1..32 */
  double omega;       /* Richardson weight (> 0); its preconditioner is the identity */
  int32_t max_cycles; /* outer restart cycles before PKSELL_ENOTCONV, >= 1 */
  int32_t reserved;
} pksell_f3r_params;

/* Workspace bytes of pksell_f3r for n rows; mixed != 0 for the
 * mixed-precision form (float32 inner vectors), 0 for the all-float64 form.
 * About (2 m1 + 3) n float64 values plus (2 m2 + 2 m3 + 3) n inner values. */
int pksell_f3r_workspace(int64_t n, int32_t mixed, const pksell_f3r_params *prm,
                         size_t *ws_bytes);

/* F3R: an outer flexible GMRES(m1) in float64 on A1 (float64 SELL),
 * restarted until the true relative residual passes tol, preconditioned by
 * one FGMRES(m2) cycle, preconditioned by one FGMRES(m3) cycle,
 * preconditioned by m4 Richardson iterations.  The inner layers run a fixed
 * number of steps from zero, with no convergence test.
 *
 *  - A2 == NULL: every layer uses A1 with float64 vectors (FP64-F3R); A3_sell
 *    and A3_pack must be NULL.
 *  - A2 != NULL (float32 SELL, plain or paired slots): layers 2-4 keep
 *    float32 vectors; layer 2
 *    multiplies with A2, layers 3 and 4 with exactly one of A3_sell (SELL
 *    with half or float32 values) and A3_pack (32-bit PackSELL words: FP16,
 *    E8MY or FIX, no split).  Half-value SELL and FP16 PackSELL words of the
 *    same matrix give bit-identical products, so the two forms give
 *    bit-identical iterates (the paper's FP16-F3R and PackSELL-F3R).
 *
 * All matrices are n x n in implicit (original) row order.  Gram-Schmidt is
 * classical with one reorthogonalisation; dot products, the Hessenberg
 * matrices, rotations and the small triangular solves are float64, each
 * reduction in one fixed order (results repeat bit for bit).  No
 * preconditioner is applied inside the Richardson layer: scale the system
 * (Gbar^-1 A Gbar^-1, sec. 5.2) beforehand.  x (float64, n) holds the
 * initial guess on entry and the solution on return.  The outer layer
 * checks its residual estimate after every step and the true residual
 * b - A1 x (float64) at the end of each cycle, restarting from it.
 * ``info``: outer_iterations = outer steps over all cycles,
 * inner_iterations = second-layer steps (outer steps x m2), the final true
 * relative residual and the wall time.  The call SYNCHRONISES: it waits for
 * ``stream``, runs on a private stream (each outer step replayed from one
 * captured HIP graph, the host polling the residual estimate) and returns
 * when done.  PKSELL_ENOTCONV after max_cycles cycles (x holds the last
 * iterate), PKSELL_EBREAKDOWN when a residual is not finite,
 * PKSELL_EWORKSPACE when ws_bytes is below pksell_f3r_workspace's size. */
int pksell_f3r(const pksell_sell *A1, const pksell_sell *A2, const pksell_sell *A3_sell,
               const pksell_matrix *A3_pack, const double *b, double *x, double tol,
               const pksell_f3r_params *prm, pksell_pcg_info *info, void *ws, size_t ws_bytes,
               void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PKSELL_H */
