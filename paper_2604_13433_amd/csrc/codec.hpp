// PackSELL word codec on the device (sec. 4.2).
//
// Word (W = 32): bit 0 = flag.  flag 1: value field in the upper V = 31 - D
// bits, delta in bits 1..D.  flag 0: delta in bits 1..31, no value (dummy
// when the delta is nonzero, padding when the word is 0).
#pragma once

#include <hip/hip_fp16.h>

#include "common.hpp"

namespace pksell {

// Per-matrix decode constants, computed once on the host.
struct Codec {
  uint32_t dmask;  // 2^D - 1: the flag-1 delta field after >> 1
  uint32_t vmask;  // ~(2^(D+1) - 1): the value field
  int32_t D;
};

inline Codec make_codec(int D) {
  Codec c;
  c.D = D;
  c.dmask = (1u << D) - 1u;
  c.vmask = ~((2u << D) - 1u);
  return c;
}

// Branch-free unpack (sec. 4.2.1): the flag selects the delta width (D bits
// or 31) and zeroes the value field of flag-0 words.  ``nf`` is the flag
// sign-extended to all ones or zero.
struct Unpacked {
  uint32_t delta;
  uint32_t vbits;
};

__device__ inline Unpacked unpack(uint32_t p, const Codec &c) {
  uint32_t nf = (uint32_t)__builtin_amdgcn_sbfe((int)p, 0u, 1u);
  Unpacked u;
  u.delta = (p >> 1) & (c.dmask | ~nf);
  u.vbits = p & nf & c.vmask;
  return u;
}

// Value field -> float32 working value.  FIX returns q * 2^(D+1) (the
// integer field as stored); the row scale 2^(e - D - 1) is applied once per
// row by the caller.
template <int FMT>
__device__ inline float decode_value(uint32_t vbits) {
  if constexpr (FMT == PKSELL_FP16) {
    return __half2float(__ushort_as_half((unsigned short)(vbits >> 16)));
  } else if constexpr (FMT == PKSELL_E8MY) {
    return __uint_as_float(vbits);
  } else {
    return (float)(int32_t)vbits;
  }
}

// ---- quantisers (encoder side) ---------------------------------------------

// FP16: IEEE binary16 with round to nearest even; NaN -> 0x7E00.
__device__ inline uint32_t quant_fp16(float v) {
  if (v != v) return 0x7E00u << 16;
  return (uint32_t)__half_as_ushort(__float2half_rn(v)) << 16;
}

// E8MY: magnitude bits rounded to a multiple of 2^(D+1) units in the last
// place with ties away from zero (the integer form of the conversion in
// sec. 4.2.2), saturating to infinity; NaN -> 0x7FC00000; +-0, +-inf kept.
__device__ inline uint32_t quant_e8my(float v, int D) {
  uint32_t b = __float_as_uint(v);
  uint32_t sign = b & 0x80000000u;
  uint32_t mag = b & 0x7FFFFFFFu;
  if (mag > 0x7F800000u) return 0x7FC00000u;
  if (mag == 0x7F800000u) return b;
  uint32_t r = (mag + (1u << D)) & ~((2u << D) - 1u);
  if (r > 0x7F800000u) r = 0x7F800000u;
  return sign | r;
}

// E11MY (64-bit words): the same integer rule on the FP64 pattern -- round
// the magnitude bits to a multiple of 2^(D+1), ties away from zero, past the
// largest finite value to infinity; NaN becomes 0x7FF8000000000000.
__device__ inline uint64_t quant_e11my(double v, int D) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t sign = b & 0x8000000000000000ull;
  const uint64_t mag = b & 0x7FFFFFFFFFFFFFFFull;
  if (mag > 0x7FF0000000000000ull) return 0x7FF8000000000000ull;
  if (mag == 0x7FF0000000000000ull) return b;
  uint64_t r = (mag + (1ull << D)) & ~((2ull << D) - 1ull);
  if (r > 0x7FF0000000000000ull) r = 0x7FF0000000000000ull;
  return sign | r;
}

// FIX: row exponent e = e(M) - (V - 1) with M = max |a| = f * 2^e(M),
// 1/2 <= f < 1 (0 for M == 0); q = clamp(round_half_away(v * 2^-e),
// +-(2^(V-1) - 1)) in the upper V bits.
__device__ inline int32_t fix_row_exponent(float absmax, int D) {
  if (absmax == 0.0f) return 0;
  int e;
  frexpf(absmax, &e);
  return e - (31 - D - 1);
}

__device__ inline uint32_t quant_fix(float v, int32_t e, int D) {
  const int V = 31 - D;
  const int64_t lim = (int64_t(1) << (V - 1)) - 1;
  // |v| <= M < 2^e(M), so v * 2^-e < 2^(V-1): the scaling is exact and the
  // rounded value (roundf: half away from zero) is an exact integer.  The
  // clamp is done on integers because 2^(V-1) - 1 is not a float for V > 24.
  int64_t q = (int64_t)roundf(ldexpf(v, -e));
  q = q < -lim ? -lim : (q > lim ? lim : q);
  return ((uint32_t)(int32_t)q) << (D + 1);
}

// ---- 16-bit words --------------------------------------------------------------

// E5MY (16-bit words, Y = 9 - D): the binary16 pattern with its low D + 1
// bits given to the delta and the flag.  The float32 input is rounded once,
// straight onto that grid, with ties away from zero: for |v| >= 2^-14 by
// the integer rule on the float32 magnitude (keep Y mantissa bits), below
// it on the grid 2^(D + 1 - 24); past the largest finite value
// (2 - 2^-Y) * 2^15 the result is infinity; NaN -> 0x7E00.  The result is
// a binary16 value, so the final conversion is exact.  Returns the 16-bit
// field in the low half.
__device__ inline uint32_t quant_e5my(float v, int D) {
  const uint32_t b = __float_as_uint(v);
  const uint32_t sign16 = (b >> 16) & 0x8000u;
  const uint32_t mag = b & 0x7FFFFFFFu;
  if (mag > 0x7F800000u) return 0x7E00u;
  if (mag == 0x7F800000u) return sign16 | 0x7C00u;
  const int Y = 9 - D;
  const float a = __uint_as_float(mag);
  float q;
  if (a >= 0x1p-14f) {
    const uint32_t sh = 23u - (uint32_t)Y;  // dropped float32 mantissa bits
    q = __uint_as_float((mag + (1u << (sh - 1))) & ~((1u << sh) - 1u));
  } else {
    q = ldexpf(roundf(ldexpf(a, 23 - D)), D - 23);
  }
  if (q > ldexpf(2.0f - ldexpf(1.0f, -Y), 15)) return sign16 | 0x7C00u;
  return sign16 | (uint32_t)__half_as_ushort(__float2half_rn(q));
}

// FIX16: FIX with a V = 15 - D bit field: e = e(M) - (V - 1), q as in
// quant_fix, returned in the upper V bits of the low half.
__device__ inline int32_t fix16_row_exponent(float absmax, int D) {
  if (absmax == 0.0f) return 0;
  int e;
  frexpf(absmax, &e);
  return e - (15 - D - 1);
}

__device__ inline uint32_t quant_fix16(float v, int32_t e, int D) {
  const int32_t lim = (1 << (15 - D - 1)) - 1;
  int32_t q = (int32_t)roundf(ldexpf(v, -e));
  q = q < -lim ? -lim : (q > lim ? lim : q);
  return ((uint32_t)q << (D + 1)) & 0xFFFFu;
}

}  // namespace pksell
