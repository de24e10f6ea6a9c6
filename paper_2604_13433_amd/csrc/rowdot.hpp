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

// The PackSELL row loop (sec. 4.4) for one lane: walks the w words of its
// slice lane in groups of kUnroll -- all loads of a group in flight
// together, columns as running sums of deltas from c, then all gathers
// together, then the products accumulated in word order.  The last partial
// group re-reads the lane's last word (clamped, in bounds) and turns the
// extra words into padding (delta 0, value 0).  ``gather(c, r)`` returns the
// operand for column c and right-hand side r.
template <int FMT, int KB, typename Gather>
__device__ inline void packsell_row(const uint32_t *P, uint32_t stride, uint32_t w, uint32_t c,
                                    const Codec &cd, Gather gather, float (&acc)[KB]) {
  auto group = [&](uint32_t j, bool full) {
    uint32_t p[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const uint32_t jj = full ? j + q : min(j + q, w - 1);
      p[q] = __builtin_nontemporal_load(P + jj * stride);
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
      for (int q = 0; q < kUnroll; ++q) xv[q] = gather(cq[q], r);
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) acc[r] = fmaf(v[q], xv[q], acc[r]);
    }
  };
  uint32_t j = 0;
  for (; j + kUnroll <= w; j += kUnroll) group(j, true);
  if (j < w) group(j, false);
}

}  // namespace pksell
