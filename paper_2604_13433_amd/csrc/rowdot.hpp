// PackSELL slice geometry and the word loop shared by every product kernel.
#pragma once

#include "codec.hpp"

namespace pksell {

constexpr int kRowBlock = 256;  // threads per workgroup of the product kernels
constexpr int kUnroll = 8;      // words per group (loads in flight per lane)

// Original row of stored row t: its sigma-block start plus perm (implicit
// mode); t itself when perm is null (explicit mode).
__device__ inline uint32_t out_row(const void *perm, int32_t perm_bytes, uint32_t t,
                                   const RowGeo &g) {
  if (perm == nullptr) return t;
  return block_start(t, g) + (perm_bytes == 1 ? (uint32_t) static_cast<const uint8_t *>(perm)[t]
                                              : (uint32_t) static_cast<const uint16_t *>(perm)[t]);
}

// The destination of stored row t: block_start(t) + perm[t] in implicit
// order, t itself in explicit order; and, for FIX, the row's scale exponent.
// row_out issues the perm and row_exp loads at the start of the row's work,
// through buffer resources (lanes with t >= n read 0 and store nothing, so
// no divergent branch), and keeps the raw loaded values: they are combined
// only where the result is stored.  Using a loaded value right away would
// make the wave wait for that load before it issues its word loads.
struct RowOut {
  uint32_t base, p;
  uint32_t e;  // FIX: the raw int16 row exponent
  // The empty asm pins the use of the loaded value here: without it the
  // compiler may fold the addition back next to the load (into the blocks
  // that feed a loop-carried RowOut), which reintroduces the early wait.
  __device__ uint32_t row() const {
    uint32_t q = p;
    asm volatile("" : "+v"(q));
    return base + q;
  }
  __device__ int shift(const Codec &cd) const {
    uint32_t q = e;
    asm volatile("" : "+v"(q));
    return (int)(int16_t)q - (cd.D + 1);
  }
};

__device__ inline RowOut row_out(const void *perm, int32_t perm_bytes, uint32_t t, uint32_t n,
                                 const RowGeo &g) {
  RowOut r{t, 0u, 0u};
  if (perm != nullptr) {
    r.base = block_start(t, g);
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(perm, n * (uint32_t)perm_bytes);
    r.p = perm_bytes == 1 ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rp, t, 0, 0)
                          : (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rp, 2u * t, 0, 0);
  }
  return r;
}

template <int FMT>
__device__ inline RowOut row_out(const void *perm, int32_t perm_bytes, const int16_t *row_exp,
                                 uint32_t t, uint32_t n, const RowGeo &g) {
  RowOut r = row_out(perm, perm_bytes, t, n, g);
  if constexpr (FMT == PKSELL_FIX || FMT == PKSELL_FIX16)
    r.e = __builtin_amdgcn_raw_buffer_load_b16(make_rsrc(row_exp, 2u * n), 2u * t, 0, 0);
  return r;
}

// Slice coordinates of the calling lane: stored row t, slice k = t / C,
// lane l, slice start s (words) and width w.  With C = 64 a wave is exactly
// one slice, so k, s and w are made wave-uniform (scalar loads, scalar loop).
struct Lane {
  uint32_t k, l, t, w;
  int64_t s;
};

template <bool CWAVE>
__device__ inline bool lane_slice(const int64_t *offset, uint32_t n_slices, const RowGeo &g,
                                  Lane &ln) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  if constexpr (CWAVE) {
    ln.k = __builtin_amdgcn_readfirstlane(b * (kRowBlock / kWave) + (threadIdx.x / kWave));
    ln.l = threadIdx.x & (kWave - 1);
    ln.t = ln.k * kWave + ln.l;
  } else {
    ln.t = b * kRowBlock + threadIdx.x;
    ln.k = ln.t >> g.c_log2;
    ln.l = ln.t - (ln.k << g.c_log2);
  }
  if (ln.k >= n_slices) return false;
  ln.s = offset[ln.k];
  ln.w = (uint32_t)((offset[ln.k + 1] - ln.s) >> g.c_log2);
  return true;
}

// Word load: nontemporal when each word is read once (the stream should
// not evict x from the caches), plain when several waves share the words.
template <bool NT>
__device__ inline uint32_t load_word(const uint32_t *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// The word stream of one C = 64 slice through a buffer resource on its first
// word, loaded with cache-policy bits 2 (streaming).  On gfx950 this ran the
// single-vector product 3-4 % faster than nontemporal global loads, and
// policies 0 and 1 ran 8 % slower.  Byte offsets are 32-bit, so callers use
// it only while the packed words stay below 4 GiB.
constexpr int kStreamPolicy = 2;

__device__ inline __amdgpu_buffer_rsrc_t slice_words(const uint32_t *first, uint32_t w) {
  return make_rsrc(first, w * 256u);
}

// POL = 0 (default policy) instead serves a matrix applied many times in a
// row (cache_hint PKSELL_CACHE_RESIDENT): one that fits in the 256 MB
// last-level cache then stays there between products.
template <int POL = kStreamPolicy>
__device__ inline uint32_t stream_word(__amdgpu_buffer_rsrc_t rs, uint32_t lane, uint32_t j) {
  return __builtin_amdgcn_raw_buffer_load_b32(rs, (lane + j * kWave) * 4u, 0, POL);
}

// The word-load policy of a product: streaming, or the default policy for
// a matrix whose cache_hint is PKSELL_CACHE_RESIDENT.
template <bool RES>
constexpr int word_policy() {
  return RES ? 0 : kStreamPolicy;
}

// One float32 result of a single-vector product, stored through a buffer
// resource on y with the streaming policy: on the 128^3 FP16 product this
// took 14.26 us against 14.73 us for plain stores (other policies, 14.4 to
// 15.0 us).  Rows at or past n fall outside the resource and are dropped.
__device__ inline void store_result(float *y, uint32_t n, uint32_t row, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), make_rsrc(y, n * 4u),
                                        row * 4u, 0, kStreamPolicy);
}

// Element j of lane ``lane`` of a C = 64 slice of 2-, 4- or 8-byte
// elements (the SELL comparators' columns and values), loaded the same way.
template <typename T, int POL = kStreamPolicy>
__device__ inline T stream_elem(__amdgpu_buffer_rsrc_t rs, uint32_t lane, uint32_t j) {
  const uint32_t off = (lane + j * kWave) * (uint32_t)sizeof(T);
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, POL));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, POL));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, POL));
}

// The PackSELL row loop (sec. 4.4) for one lane: walks the w words of its
// slice lane in groups of kUnroll -- all loads of a group in flight
// together, columns as running sums of deltas from c, then all gathers
// together, then the products accumulated in word order.  The last partial
// group re-reads the lane's last word (clamped, in bounds) and turns the
// extra words into padding (delta 0, value 0).  ``gather(c, r, live)``
// returns the operand for column c and right-hand side r; live is false for
// flag-0 words (dummies and padding, value 0), whose gather the callers
// point past the end of their buffer resource so that it returns 0 without
// a memory request.
// ``word(j)`` returns word j of the lane (j < w).
template <int FMT, int KB, typename Word, typename Gather>
__device__ inline void packsell_row_f(Word word, uint32_t w, uint32_t c, const Codec &cd,
                                      Gather gather, float (&acc)[KB]) {
  auto group = [&](uint32_t j, bool full) {
    uint32_t p[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const uint32_t jj = full ? j + q : min(j + q, w - 1);
      p[q] = word(jj);
      if (!full && j + q >= w) p[q] = 0u;
    }
    uint32_t cq[kUnroll];
    float v[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const Unpacked u = unpack(p[q], cd);
      c += u.delta;
      cq[q] = c;
      v[q] = decode_value<FMT>(u.vbits);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r) {
      float xv[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) xv[q] = gather(cq[q], r, (p[q] & 1u) != 0u);
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) acc[r] = fmaf(v[q], xv[q], acc[r]);
    }
  };
  uint32_t j = 0;
  for (; j + kUnroll <= w; j += kUnroll) group(j, true);
  if (j < w) group(j, false);
}

// The same loop over the words at P, P + stride, ... (one lane's words).
template <int FMT, int KB, bool NT = true, typename Gather>
__device__ inline void packsell_row(const uint32_t *P, uint32_t stride, uint32_t w, uint32_t c,
                                    const Codec &cd, Gather gather, float (&acc)[KB]) {
  packsell_row_f<FMT, KB>([&](uint32_t j) { return load_word<NT>(P + j * stride); }, w, c, cd,
                          gather, acc);
}

// Four consecutive right-hand sides as one 16-byte gather (x rows hold k
// floats with k a multiple of 4, so every such group is 16-byte aligned).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 buffer_load_f32x4(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0));
}

// packsell_row for KB right-hand sides (KB a multiple of 4) gathered four at
// a time: ``gather4(c, g, live)`` returns columns 4g .. 4g+3 of x row c.
// Each accumulator still adds its products in word order.
template <int FMT, int KB, bool NT = true, typename Gather4>
__device__ inline void packsell_row_v4(const uint32_t *P, uint32_t stride, uint32_t w, uint32_t c,
                                       const Codec &cd, Gather4 gather4, float (&acc)[KB]) {
  static_assert(KB % 4 == 0, "KB must be a multiple of 4");
  auto group = [&](uint32_t j, bool full) {
    uint32_t p[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const uint32_t jj = full ? j + q : min(j + q, w - 1);
      p[q] = load_word<NT>(P + jj * stride);
      if (!full && j + q >= w) p[q] = 0u;
    }
    uint32_t cq[kUnroll];
    float v[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const Unpacked u = unpack(p[q], cd);
      c += u.delta;
      cq[q] = c;
      v[q] = decode_value<FMT>(u.vbits);
    }
#pragma unroll
    for (int g = 0; g < KB / 4; ++g) {
      f32x4 xv[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) xv[q] = gather4(cq[q], g, (p[q] & 1u) != 0u);
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        acc[4 * g + 0] = fmaf(v[q], xv[q].x, acc[4 * g + 0]);
        acc[4 * g + 1] = fmaf(v[q], xv[q].y, acc[4 * g + 1]);
        acc[4 * g + 2] = fmaf(v[q], xv[q].z, acc[4 * g + 2]);
        acc[4 * g + 3] = fmaf(v[q], xv[q].w, acc[4 * g + 3]);
      }
    }
  };
  uint32_t j = 0;
  for (; j + kUnroll <= w; j += kUnroll) group(j, true);
  if (j < w) group(j, false);
}

// Lane groups for k right-hand sides (k a multiple of 4): L lanes (a power
// of two, 4L >= k) share one row and lane q of the group owns columns
// 4q .. 4q+3, so a group gathers one contiguous 16L-byte piece of x row c
// per word (one cache line at k = 32) instead of L separate pieces, and
// any k <= 64 is one pass over the words.  A wave holds 64 / L rows; lanes
// with 4q >= k repeat the last live lane's loads (same addresses) and store
// nothing.  h selects which 64 / L rows of the slice the wave takes.
struct GroupLane {
  uint32_t l;  // row within the slice
  uint32_t q;  // column group (clamped to k / 4 - 1)
  bool live;   // owns columns 4q .. 4q+3
};

template <int L>
__device__ inline GroupLane group_lane(uint32_t h, uint32_t lane, uint32_t k4) {
  static_assert(L >= 2 && L <= 16 && (L & (L - 1)) == 0, "L must be 2, 4, 8 or 16");
  GroupLane g;
  g.l = h * (kWave / L) + lane / L;
  const uint32_t q = lane % L;
  g.live = q < k4;
  g.q = g.live ? q : k4 - 1;
  return g;
}

// Smallest lane-group size L (2..16) with 4L >= k, for 8 <= k <= 64.
inline int group_size(int64_t k) {
  const int64_t k4 = (k + 3) / 4;
  return k4 <= 2 ? 2 : k4 <= 4 ? 4 : k4 <= 8 ? 8 : 16;
}

}  // namespace pksell
