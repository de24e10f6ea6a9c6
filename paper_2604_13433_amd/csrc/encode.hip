// CSR -> PackSELL and CSR -> SELL-C-sigma encoders on the device.
//
// Analyse phase: validate the CSR and take the lower bandwidth k_left
// (sec. 4.1); count each row's stored words, nonzeros plus dummies for
// deltas >= 2^D (eq. 2 with the left offset of eq. 4, sec. 4.3); rank the
// rows of every sigma-window by descending count, ties by row index (the
// SELL-C-sigma sort, sec. 3, counting dummies as sec. 4.3 asks); take slice
// widths and scan them into offsets; with wide-slice splitting on, count
// each slice's work units and scan those too.  Fill phase: one thread per
// stored row writes its words down its slice lane, pads the lane with zero
// words and records, for split slices, the column reached at every chunk
// start.
#include "codec.hpp"

#include <cstdarg>

namespace pksell {

namespace {

constexpr int kBlock = 256;

enum : int32_t {
  kErrRowptr = 1,
  kErrColRange = 2,
  kErrColOrder = 4,
  kErrNonFinite = 8,
};

struct EncInfo {
  int32_t err;
  int32_t k_left;
  unsigned long long n_dummies;
  long long n_words;
  long long units;         // low 32 bits: work units, high 32: units of split slices
  long long split_slices;
};

// ---- analyse -----------------------------------------------------------------

// One thread per row: rowptr sane, columns in range and strictly
// increasing, values finite when ``val`` is given (FIX needs a finite row
// maximum); k_left = max over rows of i - (leftmost column), at least 0.
template <typename VT>
__global__ void k_check_rows(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                             const VT *__restrict__ val, int64_t n, int64_t m, int64_t nnz,
                             EncInfo *info) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int err = 0;
  int kl = 0;
  if (i < n) {
    int64_t rb = rowptr[i], re = rowptr[i + 1];
    if (rb < 0 || re > nnz || rb > re || (i == 0 && rb != 0) || (i == n - 1 && re != nnz)) {
      err |= kErrRowptr;
    } else {
      int64_t prev = -1;
      for (int64_t e = rb; e < re; ++e) {
        int64_t c = col[e];
        if (c < 0 || c >= m) err |= kErrColRange;
        if (c <= prev) err |= kErrColOrder;
        prev = c;
        if (val != nullptr && !isfinite((float)val[e])) err |= kErrNonFinite;
      }
      if (re > rb) {
        int64_t d = i - (int64_t)col[rb];  // the leftmost column gives max(i - j)
        kl = d > 0 ? (int)d : 0;
      }
    }
  }
  kl = wave_max(kl);
  err = wave_or(err);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (kl) atomicMax(&info->k_left, kl);
    if (err) atomicOr(&info->err, err);
  }
}

// Stored words per row: nonzeros plus the dummies of every delta >= 2^D
// (D = 31: plain SELL, no dummies): one with 32- and 64-bit words, a chain
// of ceil(d / (2^15 - 1)) with 16-bit words (``chain``).
constexpr uint32_t kDummyMax16 = (1u << 15) - 1u;

__global__ void k_count(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                        int64_t n, int32_t sigma, int64_t k_left, int32_t D, int32_t chain,
                        int32_t *__restrict__ cnt, EncInfo *info) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long dum = 0;
  if (i < n) {
    int64_t rb = rowptr[i], re = rowptr[i + 1];
    uint32_t prev = left_offset(i, sigma, k_left);
    const uint32_t lim = D >= 31 ? 0xFFFFFFFFu : (1u << D);
    for (int64_t e = rb; e < re; ++e) {
      uint32_t c = (uint32_t)col[e];
      const uint32_t d = c - prev;
      if (d >= lim) dum += chain ? (d + kDummyMax16 - 1) / kDummyMax16 : 1u;
      prev = c;
    }
    cnt[i] = (int32_t)(re - rb + dum);
  }
  dum = wave_sum(dum);
  if ((threadIdx.x & (kWave - 1)) == 0 && dum) atomicAdd(&info->n_dummies, dum);
}

// Rank of each row inside its sigma-window: rows with a larger count come
// first, equal counts keep ascending row order (a stable descending sort).
// Each block ranks up to 256 rows of one window against every row of the
// window, staged through LDS 256 counts at a time.
__global__ void k_sigma_rank(const int32_t *__restrict__ cnt, int64_t n, int32_t sigma,
                             int64_t chunks, int32_t *__restrict__ stored_rows,
                             void *perm, int32_t perm_bytes) {
  __shared__ int32_t tile[kBlock];
  int64_t win = blockIdx.x / chunks;
  int64_t chunk = blockIdx.x - win * chunks;
  int64_t base = win * sigma;
  int64_t wlen = n - base < sigma ? n - base : sigma;
  int64_t t = chunk * kBlock + threadIdx.x;
  bool live = t < wlen;
  int32_t mine = live ? cnt[base + t] : 0;
  int64_t rank = 0;
  for (int64_t t0 = 0; t0 < wlen; t0 += kBlock) {
    int64_t j = t0 + threadIdx.x;
    tile[threadIdx.x] = j < wlen ? cnt[base + j] : -1;
    __syncthreads();
    int lim = (int)(wlen - t0 < kBlock ? wlen - t0 : kBlock);
    for (int q = 0; q < lim; ++q) {
      int32_t c = tile[q];
      rank += (c > mine) | ((c == mine) & (t0 + q < t));
    }
    __syncthreads();
  }
  if (live) {
    int64_t s = base + rank;
    stored_rows[s] = (int32_t)(base + t);
    if (perm) {
      if (perm_bytes == 1)
        static_cast<uint8_t *>(perm)[s] = (uint8_t)t;
      else
        static_cast<uint16_t *>(perm)[s] = (uint16_t)t;
    }
  }
}

// offset[k + 1] = C * (max count over the slice's stored rows), rounded up
// to even for 16-bit words (two per 32-bit slot); offset[0] = 0.
__global__ void k_slice_width(const int32_t *__restrict__ cnt, const int32_t *__restrict__ stored_rows,
                              int64_t n, int32_t C, int64_t n_slices, int32_t even,
                              int64_t *__restrict__ offset) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) offset[0] = 0;
  if (k >= n_slices) return;
  int32_t w = 0;
  for (int l = 0; l < C; ++l) {
    int64_t i = k * C + l;
    if (i < n) {
      int32_t c = cnt[stored_rows[i]];
      w = c > w ? c : w;
    }
  }
  if (even) w += w & 1;
  offset[k + 1] = (int64_t)C * w;
}

// ---- inclusive scan of int64 values in place (3 phases) ---------------------

constexpr int kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kBlock * kScanItems;

__device__ inline int64_t block_inclusive_scan(int64_t v, int64_t *warp_tot) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  if (lane == kWave - 1) warp_tot[w] = v;
  __syncthreads();
  int64_t add = 0;
  for (int q = 0; q < w; ++q) add += warp_tot[q];
  __syncthreads();
  return v + add;
}

__global__ void k_scan_tiles(const int64_t *__restrict__ a, int64_t len, int64_t *__restrict__ tile_sums) {
  __shared__ int64_t wt[kBlock / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < len) s += a[base + q];
  int64_t incl = block_inclusive_scan(s, wt);
  if (threadIdx.x == kBlock - 1) tile_sums[blockIdx.x] = incl;
}

// Exclusive scan of the tile sums, by one block walking them with a carry.
__global__ void k_scan_sums(int64_t *__restrict__ tile_sums, int64_t ntiles) {
  __shared__ int64_t wt[kBlock / kWave];
  __shared__ int64_t last;
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < ntiles; t0 += kBlock) {
    int64_t j = t0 + threadIdx.x;
    int64_t v = j < ntiles ? tile_sums[j] : 0;
    int64_t incl = block_inclusive_scan(v, wt);
    if (j < ntiles) tile_sums[j] = carry + incl - v;
    if (threadIdx.x == kBlock - 1) last = incl;
    __syncthreads();
    carry += last;
    __syncthreads();
  }
}

__global__ void k_scan_apply(int64_t *__restrict__ a, int64_t len, const int64_t *__restrict__ tile_pre) {
  __shared__ int64_t wt[kBlock / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = base + q < len ? a[base + q] : 0;
    s += v[q];
  }
  int64_t run = block_inclusive_scan(s, wt) - s + tile_pre[blockIdx.x];
  for (int q = 0; q < kScanItems; ++q) {
    run += v[q];
    if (base + q < len) a[base + q] = run;
  }
}

// ---- work units of wide-slice splitting (C = 64) --------------------------------

// A slice of w > J words per lane is split into ceil(w / J) units of J
// words (the last one shorter); a narrower slice is one unit.  ucnt[k + 1]
// packs the slice's unit count (low 32 bits) and its split-unit count (high
// 32 bits), scnt[k + 1] is 1 for a split slice; both are scanned afterwards
// so that index k holds the exclusive prefix.
__global__ void k_unit_counts(const int64_t *__restrict__ offset, int64_t n_slices, int32_t J,
                              int64_t *__restrict__ ucnt, int64_t *__restrict__ scnt) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    ucnt[0] = 0;
    scnt[0] = 0;
  }
  if (k >= n_slices) return;
  const int64_t w = (offset[k + 1] - offset[k]) / kWave;
  const int64_t u = w > J ? (w + J - 1) / J : 1;
  ucnt[k + 1] = u | (w > J ? u << 32 : 0);
  scnt[k + 1] = w > J ? 1 : 0;
}

// Unit table {slice, chunk, chunks, base} and split table {slice, base,
// chunks, 0}; base is the index of the slice's first chunk among all split
// units (it addresses the checkpoints and the chunk sums).
__global__ void k_unit_tables(const int64_t *__restrict__ ucnt, const int64_t *__restrict__ scnt,
                              int64_t n_slices, uint32_t *__restrict__ units,
                              uint32_t *__restrict__ splits) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_slices) return;
  const uint64_t u0 = (uint64_t)ucnt[k], u1 = (uint64_t)ucnt[k + 1];
  const uint32_t first = (uint32_t)u0, base = (uint32_t)(u0 >> 32);
  const uint32_t chunks = (uint32_t)u1 - first;
  const bool split = (uint32_t)(u1 >> 32) != base;
  for (uint32_t c = 0; c < chunks; ++c) {
    uint32_t *d = units + 4 * (uint64_t)(first + c);
    d[0] = (uint32_t)k;
    d[1] = c;
    d[2] = chunks;
    d[3] = split ? base : 0u;
  }
  if (split) {
    uint32_t *d = splits + 4 * (uint64_t)scnt[k];
    d[0] = (uint32_t)k;
    d[1] = base;
    d[2] = chunks;
    d[3] = 0u;
  }
}

__global__ void k_finish(const int64_t *__restrict__ offset, int64_t n_slices,
                         const int64_t *__restrict__ ucnt, const int64_t *__restrict__ scnt,
                         EncInfo *info) {
  info->n_words = offset[n_slices];
  info->units = ucnt ? ucnt[n_slices] : 0;
  info->split_slices = scnt ? scnt[n_slices] : 0;
}

// ---- fill --------------------------------------------------------------------

// Loads a value as float32.  A float64 input is rounded to float32 first
// (to nearest even), and the result is pinned in a register so the
// compiler cannot fuse it with a later float32 -> half conversion into one
// direct float64 -> half rounding (the two roundings differ on ties).
template <typename VT>
__device__ inline float load_value(const VT *v, int64_t e) {
  float f = (float)v[e];
  asm volatile("" : "+v"(f));
  return f;
}

// One thread per stored row position (phantom rows past n only pad).
template <int FMT, typename VT>
__global__ void k_fill_packsell(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                const VT *__restrict__ val, int64_t n, int32_t C, int32_t sigma,
                                int64_t k_left, int32_t D, int64_t n_slices,
                                const int32_t *__restrict__ stored_rows,
                                const int64_t *__restrict__ offset, uint32_t *__restrict__ pack,
                                int16_t *__restrict__ row_exp, int32_t J,
                                const int64_t *__restrict__ ucnt, uint32_t *__restrict__ ckpt,
                                int64_t T, uint32_t *__restrict__ anchor) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slices * C) return;
  int64_t k = i / C, l = i - k * C;
  int64_t s = offset[k];
  int64_t w = (offset[k + 1] - s) / C;
  uint32_t *out = pack + s + l;
  int64_t j = 0;
  // Split slice (J > 0 and w > J): the column reached before word j is
  // recorded whenever j starts a chunk (j a multiple of J).
  uint32_t *ck = nullptr;
  if (J > 0 && w > J) ck = ckpt + (uint64_t)(((uint64_t)ucnt[k]) >> 32) * kWave + l;
  uint32_t run = left_offset(i < n ? stored_rows[i] : i, sigma, k_left);
  // CSR-packed chunks (C = 1, T > 0): the column reached before every word
  // position that starts a chunk of T words.
  auto put = [&](uint32_t word, uint32_t col_after) {
    if (ck && j % J == 0) ck[(j / J) * kWave] = run;
    if (anchor && (s + j) % T == 0) anchor[(s + j) / T] = run;
    out[j * C] = word;
    run = col_after;
    ++j;
  };
  if (i < n) {
    int64_t r = stored_rows[i];
    int64_t rb = rowptr[r], re = rowptr[r + 1];
    int32_t ex = 0;
    if constexpr (FMT == PKSELL_FIX) {
      float mx = 0.0f;  // values were checked finite by the analyse phase
      for (int64_t e = rb; e < re; ++e) mx = fmaxf(mx, fabsf(load_value(val, e)));
      ex = fix_row_exponent(mx, D);
      row_exp[i] = (int16_t)ex;
    }
    uint32_t prev = left_offset(r, sigma, k_left);
    const uint32_t lim = 1u << D;
    for (int64_t e = rb; e < re; ++e) {
      uint32_t c = (uint32_t)col[e];
      uint32_t d = c - prev;
      prev = c;
      float v = load_value(val, e);
      uint32_t vb;
      if constexpr (FMT == PKSELL_FP16)
        vb = quant_fp16(v);
      else if constexpr (FMT == PKSELL_E8MY)
        vb = quant_e8my(v, D);
      else
        vb = quant_fix(v, ex, D);
      if (d >= lim) {
        put(d << 1, c);  // dummy at the same column
        d = 0;
      }
      put(vb | (d << 1) | 1u, c);
    }
  }
  while (j < w) put(0u, run);
}

// 64-bit words (E11MY): one thread per stored row position, as
// k_fill_packsell; values are taken in float64.
template <typename VT>
__global__ void k_fill_packsell64(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                  const VT *__restrict__ val, int64_t n, int32_t C, int32_t sigma,
                                  int64_t k_left, int32_t D, int64_t n_slices,
                                  const int32_t *__restrict__ stored_rows,
                                  const int64_t *__restrict__ offset, uint64_t *__restrict__ pack) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slices * C) return;
  int64_t k = i / C, l = i - k * C;
  int64_t s = offset[k];
  int64_t w = (offset[k + 1] - s) / C;
  uint64_t *out = pack + s + l;
  int64_t j = 0;
  if (i < n) {
    int64_t r = stored_rows[i];
    uint32_t prev = left_offset(r, sigma, k_left);
    const uint32_t lim = D >= 31 ? 0xFFFFFFFFu : (1u << D);  // columns < 2^30
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const uint32_t c = (uint32_t)col[e];
      uint32_t d = c - prev;
      prev = c;
      const uint64_t vb = quant_e11my((double)val[e], D);
      if (d >= lim) {
        out[j * C] = (uint64_t)d << 1;  // dummy at the same column
        ++j;
        d = 0;
      }
      out[j * C] = vb | ((uint64_t)d << 1) | 1ull;
      ++j;
    }
  }
  for (; j < w; ++j) out[j * C] = 0ull;
}

// 16-bit words (E5MY, FIX16): one thread per stored row position, as
// k_fill_packsell; words 2i and 2i + 1 of a lane share one 32-bit slot
// (low and high half), and a delta >= 2^D is carried by a dummy chain.
template <int FMT, typename VT>
__global__ void k_fill_packsell16(const int64_t *__restrict__ rowptr,
                                  const int32_t *__restrict__ col, const VT *__restrict__ val,
                                  int64_t n, int32_t C, int32_t sigma, int64_t k_left, int32_t D,
                                  int64_t n_slices, const int32_t *__restrict__ stored_rows,
                                  const int64_t *__restrict__ offset, uint32_t *__restrict__ pack,
                                  int16_t *__restrict__ row_exp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slices * C) return;
  int64_t k = i / C, l = i - k * C;
  int64_t s = offset[k] / 2;             // in slots
  int64_t w2 = (offset[k + 1] - offset[k]) / (2 * C);
  uint32_t *out = pack + s + l;
  int64_t j = 0;      // words written
  uint32_t half = 0;  // the pending low word of a slot
  auto put = [&](uint32_t word) {
    if (j & 1) out[(j >> 1) * C] = half | (word << 16);
    else half = word;
    ++j;
  };
  if (i < n) {
    int64_t r = stored_rows[i];
    int64_t rb = rowptr[r], re = rowptr[r + 1];
    int32_t ex = 0;
    if constexpr (FMT == PKSELL_FIX16) {
      float mx = 0.0f;  // values were checked finite by the analyse phase
      for (int64_t e = rb; e < re; ++e) mx = fmaxf(mx, fabsf(load_value(val, e)));
      ex = fix16_row_exponent(mx, D);
      row_exp[i] = (int16_t)ex;
    }
    uint32_t prev = left_offset(r, sigma, k_left);
    const uint32_t lim = 1u << D;
    for (int64_t e = rb; e < re; ++e) {
      const uint32_t c = (uint32_t)col[e];
      uint32_t d = c - prev;
      prev = c;
      const float v = load_value(val, e);
      const uint32_t vb = FMT == PKSELL_E5MY ? quant_e5my(v, D) : quant_fix16(v, ex, D);
      if (d >= lim) {
        while (d > 0) {
          const uint32_t step = d < kDummyMax16 ? d : kDummyMax16;
          put(step << 1);
          d -= step;
        }
      }
      put(vb | (d << 1) | 1u);
    }
  }
  while (j < 2 * w2) put(0u);
}

// A SELL slot value: half values are rounded from float32 (float64 input
// first rounded to float32, the intermediate pinned by load_value), as the
// FP16 PackSELL words are.
template <typename OT, typename VT>
__device__ inline OT sell_value(const VT *v, int64_t e) {
  if constexpr (sizeof(OT) == 2) return (OT)load_value(v, e);
  else return (OT)v[e];
}

// One paired slot: the column in the low 4 bytes, the float32 value bits in
// the high 4 (float64 input rounded to float32 first).
template <typename VT>
__device__ inline uint64_t sell_slot(const VT *v, int64_t e, int32_t c) {
  const float f = (float)load_value(v, e);
  return (uint64_t)(uint32_t)c | ((uint64_t)__float_as_uint(f) << 32);
}

template <typename VT>
__global__ void k_fill_sell_paired(const int64_t *__restrict__ rowptr,
                                   const int32_t *__restrict__ col, const VT *__restrict__ val,
                                   int64_t n, int32_t C, int64_t n_slices,
                                   const int32_t *__restrict__ stored_rows,
                                   const int64_t *__restrict__ offset, uint64_t *__restrict__ slot) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slices * C) return;
  int64_t k = i / C, l = i - k * C;
  int64_t s = offset[k];
  int64_t w = (offset[k + 1] - s) / C;
  int64_t j = 0;
  int32_t last = 0;
  if (i < n) {
    int64_t r = stored_rows[i];
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e, ++j) {
      last = col[e];
      slot[s + j * C + l] = sell_slot(val, e, last);
    }
  }
  for (; j < w; ++j) slot[s + j * C + l] = (uint64_t)(uint32_t)last;  // value 0
}

template <typename VT, typename OT>
__global__ void k_fill_sell(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const VT *__restrict__ val, int64_t n, int32_t C, int64_t n_slices,
                            const int32_t *__restrict__ stored_rows,
                            const int64_t *__restrict__ offset, int32_t *__restrict__ scol,
                            OT *__restrict__ sval) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slices * C) return;
  int64_t k = i / C, l = i - k * C;
  int64_t s = offset[k];
  int64_t w = (offset[k + 1] - s) / C;
  int64_t j = 0;
  int32_t last = 0;
  if (i < n) {
    int64_t r = stored_rows[i];
    int64_t rb = rowptr[r], re = rowptr[r + 1];
    for (int64_t e = rb; e < re; ++e, ++j) {
      last = col[e];
      scol[s + j * C + l] = last;
      sval[s + j * C + l] = sell_value<OT>(val, e);
    }
  }
  for (; j < w; ++j) {
    scol[s + j * C + l] = last;
    sval[s + j * C + l] = (OT)0;
  }
}

// Chunk plan of a CSR-packed matrix: lo[c] = the first row whose words start
// at or after word c*T (offsets ascend; offset[n] = n_words > c*T for every
// chunk), lo[n_chunks] = n.
__global__ void k_csr_lo(const int64_t *__restrict__ offset, int64_t n, int64_t n_chunks,
                         int64_t T, uint32_t *__restrict__ lo) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_chunks) return;
  if (c == n_chunks) {
    lo[c] = (uint32_t)n;
    return;
  }
  const int64_t p = c * T;
  int64_t a = 0, b = n;
  while (a < b) {
    const int64_t mid = (a + b) / 2;
    if (offset[mid] < p) a = mid + 1;
    else b = mid;
  }
  lo[c] = (uint32_t)a;
}

// ---- shared host driver ------------------------------------------------------

struct Plan {
  EncInfo *info;
  int32_t *cnt;
  int32_t *stored_rows;
  int64_t *tile_sums;
  int64_t *ucnt;  // per-slice unit counts, scanned (n_slices + 1)
  int64_t *scnt;  // per-slice split flags, scanned (n_slices + 1)
  size_t bytes;
};

Plan carve(void *ws, int64_t n, int64_t n_slices) {
  Carver cv(ws);
  Plan p;
  p.info = cv.take<EncInfo>(1);
  p.cnt = cv.take<int32_t>(n > 0 ? n : 1);
  p.stored_rows = cv.take<int32_t>(n > 0 ? n : 1);
  p.tile_sums = cv.take<int64_t>(cdiv(n_slices > 0 ? n_slices : 1, kScanTile));
  p.ucnt = cv.take<int64_t>(n_slices + 1);
  p.scnt = cv.take<int64_t>(n_slices + 1);
  p.bytes = cv.used;
  return p;
}

int check_common(int64_t n, int64_t m, int64_t nnz, int32_t C, int32_t sigma,
                 int32_t perm_mode) {
  PKS_CHECK(n >= 0 && m >= 0 && nnz >= 0, PKSELL_EINVAL, "negative size");
  PKS_CHECK(n < (int64_t(1) << 30) && m < (int64_t(1) << 30), PKSELL_ERANGE,
            "n and m must be below 2^30");
  PKS_CHECK(nnz < (int64_t(1) << 40), PKSELL_ERANGE, "nnz too large");
  PKS_CHECK(C >= 1 && C <= 64 && (C & (C - 1)) == 0, PKSELL_EINVAL,
            "C must be a power of two in [1, 64]");
  PKS_CHECK(sigma >= 1 && sigma <= 65536, PKSELL_EINVAL, "sigma must be in [1, 65536]");
  PKS_CHECK(perm_mode == PKSELL_EXPLICIT || perm_mode == PKSELL_IMPLICIT, PKSELL_EINVAL,
            "bad perm_mode");
  return PKSELL_OK;
}

// Validation, counts, sort, widths, offsets.  Synchronises twice: after the
// CSR check (later kernels index col through rowptr) and at the end.
int analyse(const int64_t *rowptr, const int32_t *col, const void *finite_val,
            int32_t val_dtype, int64_t n, int64_t m, int64_t nnz, int32_t C, int32_t sigma,
            int32_t D, int64_t n_slices, int64_t *offset, void *perm, int32_t perm_bytes,
            int32_t split_words, bool w16, const Plan &p, hipStream_t st, EncInfo *host) {
  PKS_HIP(hipMemsetAsync(p.info, 0, sizeof(EncInfo), st));
  const int64_t rb = cdiv(n, kBlock);
  if (n > 0) {
    if (val_dtype == PKSELL_F64)
      k_check_rows<double><<<rb, kBlock, 0, st>>>(
          rowptr, col, static_cast<const double *>(finite_val), n, m, nnz, p.info);
    else
      k_check_rows<float><<<rb, kBlock, 0, st>>>(
          rowptr, col, static_cast<const float *>(finite_val), n, m, nnz, p.info);
    PKS_LAUNCHED();
  }
  PKS_HIP(hipMemcpyAsync(host, p.info, sizeof(EncInfo), hipMemcpyDeviceToHost, st));
  PKS_HIP(hipStreamSynchronize(st));
  PKS_CHECK(host->err == 0, PKSELL_EINVAL,
            "malformed input (flags 0x%x: 1 rowptr, 2 column range, 4 column order, "
            "8 non-finite value for FIX)", host->err);
  if (n > 0) {
    k_count<<<rb, kBlock, 0, st>>>(rowptr, col, n, sigma, host->k_left, D, w16 ? 1 : 0, p.cnt,
                                   p.info);
    PKS_LAUNCHED();
    const int64_t nwin = cdiv(n, sigma);
    const int64_t chunks = cdiv(n < sigma ? n : sigma, kBlock);
    k_sigma_rank<<<nwin * chunks, kBlock, 0, st>>>(p.cnt, n, sigma, chunks, p.stored_rows, perm,
                                                  perm_bytes);
    PKS_LAUNCHED();
    k_slice_width<<<cdiv(n_slices, kBlock), kBlock, 0, st>>>(p.cnt, p.stored_rows, n, C,
                                                            n_slices, w16 ? 1 : 0, offset);
    PKS_LAUNCHED();
    const int64_t ntiles = cdiv(n_slices, kScanTile);
    k_scan_tiles<<<ntiles, kBlock, 0, st>>>(offset + 1, n_slices, p.tile_sums);
    PKS_LAUNCHED();
    k_scan_sums<<<1, kBlock, 0, st>>>(p.tile_sums, ntiles);
    PKS_LAUNCHED();
    k_scan_apply<<<ntiles, kBlock, 0, st>>>(offset + 1, n_slices, p.tile_sums);
    PKS_LAUNCHED();
    if (split_words > 0) {
      k_unit_counts<<<cdiv(n_slices, kBlock), kBlock, 0, st>>>(offset, n_slices, split_words,
                                                              p.ucnt, p.scnt);
      PKS_LAUNCHED();
      for (int64_t *a : {p.ucnt, p.scnt}) {
        k_scan_tiles<<<ntiles, kBlock, 0, st>>>(a + 1, n_slices, p.tile_sums);
        PKS_LAUNCHED();
        k_scan_sums<<<1, kBlock, 0, st>>>(p.tile_sums, ntiles);
        PKS_LAUNCHED();
        k_scan_apply<<<ntiles, kBlock, 0, st>>>(a + 1, n_slices, p.tile_sums);
        PKS_LAUNCHED();
      }
    }
  } else {
    int64_t zero = 0;
    PKS_HIP(hipMemcpyAsync(offset, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
  }
  const bool units = split_words > 0 && n > 0;
  k_finish<<<1, 1, 0, st>>>(offset, n_slices, units ? p.ucnt : nullptr,
                            units ? p.scnt : nullptr, p.info);
  PKS_LAUNCHED();
  PKS_HIP(hipMemcpyAsync(host, p.info, sizeof(EncInfo), hipMemcpyDeviceToHost, st));
  PKS_HIP(hipStreamSynchronize(st));
  return PKSELL_OK;
}

}  // namespace

// ---- error state ---------------------------------------------------------------

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_version(void) { return 100; }

const char *pksell_status_string(int s) {
  switch (s) {
    case PKSELL_OK: return "ok";
    case PKSELL_EINVAL: return "invalid argument";
    case PKSELL_ERANGE: return "size out of range";
    case PKSELL_EWORKSPACE: return "workspace too small";
    case PKSELL_EHIP: return "HIP runtime error";
    case PKSELL_ENOTCONV: return "solver did not converge";
    case PKSELL_EBREAKDOWN: return "solver breakdown";
    default: return "unknown status";
  }
}

const char *pksell_last_error(void) { return g_err; }

int pksell_encode_query(int64_t n, int64_t m, int64_t nnz, int32_t C, int32_t sigma, int32_t D,
                        int32_t fmt, int32_t perm_mode, pksell_matrix *A, size_t *ws_bytes) {
  PKS_CHECK(A && ws_bytes, PKSELL_EINVAL, "null argument");
  int rc = check_common(n, m, nnz, C, sigma, perm_mode);
  if (rc) return rc;
  switch (fmt) {
    case PKSELL_FP16: PKS_CHECK(D == 15, PKSELL_EINVAL, "FP16 needs D = 15"); break;
    case PKSELL_E8MY: PKS_CHECK(D >= 1 && D <= 22, PKSELL_EINVAL, "E8MY needs 1 <= D <= 22"); break;
    case PKSELL_FIX: PKS_CHECK(D >= 1 && D <= 29, PKSELL_EINVAL, "FIX needs 1 <= D <= 29"); break;
    case PKSELL_E11MY: PKS_CHECK(D >= 1 && D <= 51, PKSELL_EINVAL, "E11MY needs 1 <= D <= 51"); break;
    case PKSELL_E5MY: PKS_CHECK(D >= 1 && D <= 8, PKSELL_EINVAL, "E5MY needs 1 <= D <= 8"); break;
    case PKSELL_FIX16: PKS_CHECK(D >= 1 && D <= 13, PKSELL_EINVAL, "FIX16 needs 1 <= D <= 13"); break;
    default: PKS_CHECK(false, PKSELL_EINVAL, "unknown format %d", fmt);
  }
  PKS_CHECK(!is_w16(fmt) || C == kWave, PKSELL_EINVAL, "16-bit words need C = 64");
  std::memset(A, 0, sizeof(*A));
  A->n = n;
  A->m = m;
  A->nnz = nnz;
  A->C = C;
  A->sigma = sigma;
  A->D = D;
  A->fmt = fmt;
  A->perm_mode = perm_mode;
  A->perm_bytes = sigma <= 256 ? 1 : 2;
  A->n_slices = cdiv(n, C);
  *ws_bytes = carve(nullptr, n, A->n_slices).bytes;
  return PKSELL_OK;
}

int pksell_encode(const int64_t *rowptr, const int32_t *col, const void *val, int32_t val_dtype,
                  pksell_matrix *A, void *ws, size_t ws_bytes, void *stream) {
  PKS_CHECK(A && rowptr && A->offset, PKSELL_EINVAL, "null argument");
  PKS_CHECK(A->nnz == 0 || (col && val), PKSELL_EINVAL, "null col/val");
  PKS_CHECK(val_dtype == PKSELL_F32 || val_dtype == PKSELL_F64, PKSELL_EINVAL, "bad val_dtype");
  PKS_CHECK(A->perm_mode == PKSELL_EXPLICIT || A->perm, PKSELL_EINVAL,
            "implicit mode needs perm");
  Plan p = carve(ws, A->n, A->n_slices);
  PKS_CHECK(ws && ws_bytes >= p.bytes, PKSELL_EWORKSPACE, "workspace: need %zu bytes", p.bytes);
  PKS_CHECK(A->split_words == 0 || (A->fmt != PKSELL_E11MY && !is_w16(A->fmt)), PKSELL_EINVAL,
            "split_words: 32-bit words only");
  const bool chunked = A->C == 1 && A->split_words > 0;
  PKS_CHECK(A->split_words == 0 ||
                (A->C == kWave && A->split_words % 8 == 0 && A->split_words >= 8 &&
                 A->split_words <= (1 << 24)) ||
                (chunked && A->sigma == 1 &&
                 (A->split_words == 256 || A->split_words == 512 || A->split_words == 1024)),
            PKSELL_EINVAL,
            "split_words must be 0, a multiple of 8 in [8, 2^24] with C = 64, or 256, 512 "
            "or 1024 with C = 1 and sigma = 1");
  hipStream_t st = as_stream(stream);
  if (A->pack == nullptr) {
    EncInfo h{};
    const bool fix = A->fmt == PKSELL_FIX || A->fmt == PKSELL_FIX16;
    int rc = analyse(rowptr, col, fix ? val : nullptr, val_dtype, A->n, A->m, A->nnz, A->C,
                     A->sigma, A->D, A->n_slices, A->offset, A->perm, A->perm_bytes,
                     chunked ? 0 : A->split_words, is_w16(A->fmt), p, st, &h);
    if (rc) return rc;
    A->k_left = h.k_left;
    A->n_dummies = (int64_t)h.n_dummies;
    A->n_words = h.n_words;
    PKS_CHECK(A->n_words < (int64_t(1) << 40), PKSELL_ERANGE, "too many words");
    if (chunked) {
      A->n_units = cdiv(A->n_words, A->split_words);
      A->n_split_units = 0;
      A->n_split_slices = 0;
      PKS_CHECK(A->n_units < (int64_t(1) << 31), PKSELL_ERANGE, "too many chunks");
      return PKSELL_OK;
    }
    A->n_units = (int64_t)(uint32_t)h.units;
    A->n_split_units = (int64_t)((uint64_t)h.units >> 32);
    A->n_split_slices = h.split_slices;
    return PKSELL_OK;
  }
  PKS_CHECK((A->fmt != PKSELL_FIX && A->fmt != PKSELL_FIX16) || A->row_exp, PKSELL_EINVAL,
            "FIX needs row_exp");
  const int64_t rows = A->n_slices * A->C;
  if (rows == 0) return PKSELL_OK;
  const bool split = !chunked && A->split_words > 0 && A->n_split_units > 0;
  PKS_CHECK(!split || (A->units && A->splits && A->ckpt), PKSELL_EINVAL,
            "split slices need units, splits and ckpt");
  const bool plan = chunked && A->n_units > 0;
  PKS_CHECK(!plan || (A->units && A->ckpt), PKSELL_EINVAL, "chunked matrices need units and ckpt");
  if (plan) {
    k_csr_lo<<<cdiv(A->n_units + 1, kBlock), kBlock, 0, st>>>(A->offset, A->n, A->n_units,
                                                              A->split_words, A->units);
    PKS_LAUNCHED();
  }
  if (split) {
    k_unit_tables<<<cdiv(A->n_slices, kBlock), kBlock, 0, st>>>(p.ucnt, p.scnt, A->n_slices,
                                                               A->units, A->splits);
    PKS_LAUNCHED();
  }
  const int64_t g = cdiv(rows, kBlock);
  if (A->fmt == PKSELL_E11MY) {
    uint64_t *pk = reinterpret_cast<uint64_t *>(A->pack);
    if (val_dtype == PKSELL_F32)
      k_fill_packsell64<float><<<g, kBlock, 0, st>>>(rowptr, col, static_cast<const float *>(val),
                                                     A->n, A->C, A->sigma, A->k_left, A->D,
                                                     A->n_slices, p.stored_rows, A->offset, pk);
    else
      k_fill_packsell64<double><<<g, kBlock, 0, st>>>(rowptr, col, static_cast<const double *>(val),
                                                      A->n, A->C, A->sigma, A->k_left, A->D,
                                                      A->n_slices, p.stored_rows, A->offset, pk);
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
  if (is_w16(A->fmt)) {
#define PKS_FILL16(F, VT)                                                                     \
  k_fill_packsell16<F, VT><<<g, kBlock, 0, st>>>(rowptr, col, static_cast<const VT *>(val), \
                                                 A->n, A->C, A->sigma, A->k_left, A->D,     \
                                                 A->n_slices, p.stored_rows, A->offset,     \
                                                 A->pack, A->row_exp)
    if (val_dtype == PKSELL_F32) {
      if (A->fmt == PKSELL_E5MY) PKS_FILL16(PKSELL_E5MY, float);
      else PKS_FILL16(PKSELL_FIX16, float);
    } else {
      if (A->fmt == PKSELL_E5MY) PKS_FILL16(PKSELL_E5MY, double);
      else PKS_FILL16(PKSELL_FIX16, double);
    }
#undef PKS_FILL16
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
#define PKS_FILL(F, VT)                                                                      \
  k_fill_packsell<F, VT><<<g, kBlock, 0, st>>>(rowptr, col, static_cast<const VT *>(val),   \
                                               A->n, A->C, A->sigma, A->k_left, A->D,       \
                                               A->n_slices, p.stored_rows, A->offset,       \
                                               A->pack, A->row_exp,                         \
                                               split ? A->split_words : 0, p.ucnt, A->ckpt, \
                                               plan ? A->split_words : 0,                   \
                                               plan ? A->ckpt : nullptr)
  if (val_dtype == PKSELL_F32) {
    if (A->fmt == PKSELL_FP16) PKS_FILL(PKSELL_FP16, float);
    else if (A->fmt == PKSELL_E8MY) PKS_FILL(PKSELL_E8MY, float);
    else PKS_FILL(PKSELL_FIX, float);
  } else {
    if (A->fmt == PKSELL_FP16) PKS_FILL(PKSELL_FP16, double);
    else if (A->fmt == PKSELL_E8MY) PKS_FILL(PKSELL_E8MY, double);
    else PKS_FILL(PKSELL_FIX, double);
  }
#undef PKS_FILL
  PKS_LAUNCHED();
  return PKSELL_OK;
}

int pksell_sell_query(int64_t n, int64_t m, int64_t nnz, int32_t C, int32_t sigma, int32_t dtype,
                      int32_t perm_mode, pksell_sell *S, size_t *ws_bytes) {
  PKS_CHECK(S && ws_bytes, PKSELL_EINVAL, "null argument");
  int rc = check_common(n, m, nnz, C, sigma, perm_mode);
  if (rc) return rc;
  PKS_CHECK(dtype == PKSELL_F32 || dtype == PKSELL_F64 || dtype == PKSELL_F16 ||
                dtype == PKSELL_F32_PAIRED,
            PKSELL_EINVAL, "bad dtype");
  std::memset(S, 0, sizeof(*S));
  S->n = n;
  S->m = m;
  S->nnz = nnz;
  S->C = C;
  S->sigma = sigma;
  S->perm_mode = perm_mode;
  S->perm_bytes = sigma <= 256 ? 1 : 2;
  S->dtype = dtype;
  S->n_slices = cdiv(n, C);
  *ws_bytes = carve(nullptr, n, S->n_slices).bytes;
  return PKSELL_OK;
}

int pksell_sell_encode(const int64_t *rowptr, const int32_t *col, const void *val,
                       int32_t val_dtype, pksell_sell *S, void *ws, size_t ws_bytes,
                       void *stream) {
  PKS_CHECK(S && rowptr && S->offset, PKSELL_EINVAL, "null argument");
  PKS_CHECK(S->nnz == 0 || (col && val), PKSELL_EINVAL, "null col/val");
  PKS_CHECK(val_dtype == PKSELL_F32 || val_dtype == PKSELL_F64, PKSELL_EINVAL, "bad val_dtype");
  PKS_CHECK(S->perm_mode == PKSELL_EXPLICIT || S->perm, PKSELL_EINVAL,
            "implicit mode needs perm");
  Plan p = carve(ws, S->n, S->n_slices);
  PKS_CHECK(ws && ws_bytes >= p.bytes, PKSELL_EWORKSPACE, "workspace: need %zu bytes", p.bytes);
  hipStream_t st = as_stream(stream);
  if (S->val == nullptr) {
    EncInfo h{};
    int rc = analyse(rowptr, col, nullptr, val_dtype, S->n, S->m, S->nnz, S->C, S->sigma, 31,
                     S->n_slices, S->offset, S->perm, S->perm_bytes, 0, false, p, st, &h);
    if (rc) return rc;
    S->n_slots = h.n_words;
    return PKSELL_OK;
  }
  const bool paired = S->dtype == PKSELL_F32_PAIRED;
  PKS_CHECK(paired || S->col, PKSELL_EINVAL, "null S->col");
  const int64_t rows = S->n_slices * S->C;
  if (rows == 0) return PKSELL_OK;
  const int64_t g = cdiv(rows, kBlock);
  if (paired) {
    if (val_dtype == PKSELL_F32)
      k_fill_sell_paired<float><<<g, kBlock, 0, st>>>(rowptr, col, static_cast<const float *>(val),
                                                      S->n, S->C, S->n_slices, p.stored_rows,
                                                      S->offset, static_cast<uint64_t *>(S->val));
    else
      k_fill_sell_paired<double><<<g, kBlock, 0, st>>>(rowptr, col,
                                                       static_cast<const double *>(val), S->n,
                                                       S->C, S->n_slices, p.stored_rows,
                                                       S->offset, static_cast<uint64_t *>(S->val));
    PKS_LAUNCHED();
    return PKSELL_OK;
  }
#define PKS_SFILL(VT, OT)                                                                   \
  k_fill_sell<VT, OT><<<g, kBlock, 0, st>>>(rowptr, col, static_cast<const VT *>(val), S->n, \
                                            S->C, S->n_slices, p.stored_rows, S->offset,     \
                                            S->col, static_cast<OT *>(S->val))
  if (val_dtype == PKSELL_F32) {
    if (S->dtype == PKSELL_F32) PKS_SFILL(float, float);
    else if (S->dtype == PKSELL_F16) PKS_SFILL(float, _Float16);
    else PKS_SFILL(float, double);
  } else {
    if (S->dtype == PKSELL_F32) PKS_SFILL(double, float);
    else if (S->dtype == PKSELL_F16) PKS_SFILL(double, _Float16);
    else PKS_SFILL(double, double);
  }
#undef PKS_SFILL
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // extern "C"
