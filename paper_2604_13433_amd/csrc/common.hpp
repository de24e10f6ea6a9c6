// Shared host/device helpers of the PackSELL library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/pksell.h"

namespace pksell {

constexpr int kWave = 64;

// ---- error reporting -------------------------------------------------------

void set_error(const char *fmt, ...);

#define PKS_HIP(call)                                                       \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::pksell::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,        \
                          hipGetErrorString(e_));                           \
      return PKSELL_EHIP;                                                   \
    }                                                                       \
  } while (0)

#define PKS_CHECK(cond, code, ...)                                          \
  do {                                                                      \
    if (!(cond)) {                                                          \
      ::pksell::set_error(__VA_ARGS__);                                     \
      return (code);                                                        \
    }                                                                       \
  } while (0)

#define PKS_LAUNCHED()                                                      \
  do {                                                                      \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess) {                                                 \
      ::pksell::set_error("%s:%d launch: %s", __FILE__, __LINE__,           \
                          hipGetErrorString(e_));                           \
      return PKSELL_EHIP;                                                   \
    }                                                                       \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Formats with 16-bit words (two per 32-bit slot).
__host__ __device__ inline bool is_w16(int fmt) {
  return fmt == PKSELL_E5MY || fmt == PKSELL_FIX16;
}

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Carves aligned sub-buffers out of a caller workspace.
struct Carver {
  char *base;
  size_t used = 0;
  explicit Carver(void *p) : base(static_cast<char *>(p)) {}
  template <typename T>
  T *take(size_t count) {
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used = align_up(used + count * sizeof(T));
    return p;
  }
};

// ---- device helpers ------------------------------------------------------------

// Raw buffer resource over [p, p + bytes): out-of-range loads return 0, so a
// gather through it never faults (dword3 value for gfx9-class CDNA parts).
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           0x00020000);
}

__device__ inline float buffer_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// Two consecutive floats (8-byte aligned) in one load; 0 past the resource.
// The halves are taken from the 64-bit value by shifts: with this compiler,
// a bit cast of one element of the builtin's vector result (or of a vector
// copied from it) read element 0 for both halves.
__device__ inline float2 buffer_load_f32x2(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  const uint64_t v =
      __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  return make_float2(__builtin_bit_cast(float, lo), __builtin_bit_cast(float, hi));
}

// Left offset of eq. 4: uniform over each sigma-block of rows.
__device__ __host__ inline uint32_t left_offset(int64_t row, int32_t sigma, int64_t k_left) {
  int64_t blk = (row / sigma) * sigma;
  return (uint32_t)(k_left < blk ? blk - k_left : 0);
}

// 32-bit row geometry for the product kernels (rows < 2^30).  sig_log2 is
// log2(sigma) when sigma is a power of two, else 255.
struct RowGeo {
  uint32_t sigma, sig_log2, k_left, c_log2;
};

inline uint32_t log2_or_255(uint32_t v) {
  if (v == 0 || (v & (v - 1))) return 255;
  uint32_t r = 0;
  while ((1u << r) != v) ++r;
  return r;
}

inline RowGeo make_geo(int32_t sigma, int64_t k_left, int32_t C) {
  RowGeo g;
  g.sigma = (uint32_t)sigma;
  g.sig_log2 = log2_or_255((uint32_t)sigma);
  g.k_left = (uint32_t)k_left;
  g.c_log2 = log2_or_255((uint32_t)C);
  return g;
}

__device__ inline uint32_t block_start(uint32_t row, const RowGeo &g) {
  return g.sig_log2 < 32 ? (row >> g.sig_log2) << g.sig_log2 : (row / g.sigma) * g.sigma;
}

__device__ inline uint32_t left_offset32(uint32_t row, const RowGeo &g) {
  const uint32_t blk = block_start(row, g);
  return blk > g.k_left ? blk - g.k_left : 0u;
}

// Wave-wide reductions (wave64).
template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
template <typename T>
__device__ inline T wave_or(T v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// Maps a linear workgroup id so that each of the 8 XCDs (which receive
// workgroups round-robin and each own an L2) processes one contiguous range
// of the grid; neighbouring slices then share x in the same L2.
__device__ inline uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
  constexpr uint32_t kXcd = 8;
  const uint32_t per = nblocks / kXcd;        // full rounds
  const uint32_t rem = nblocks - per * kXcd;  // XCDs that get one extra block
  const uint32_t xcd = bid % kXcd;
  const uint32_t idx = bid / kXcd;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

}  // namespace pksell
