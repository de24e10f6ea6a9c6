"""Value formats and the 32-bit PackSELL word (oracle; test infrastructure).

Word layout (sec. 4.2.1, W = V + D + 1 = 32): bit 0 is a flag.  With
flag = 1 the upper V bits hold a value and bits 1..D a delta smaller than
2^D.  With flag = 0 bits 1..31 hold a delta (up to 2^31 - 1) and there is no
value; such words are dummies (sec. 4.3), and the all-zero word is padding.

Value formats (sec. 4.2.2):

* FP16 (V = 16, D = 15): IEEE binary16 in the upper 16 bits.
* E8MY (V = 31 - D, Y = 22 - D): an FP32-compatible float with Y mantissa
  bits; the low D + 1 bits of the FP32 pattern are given to delta and flag.
* FIX (V = 31 - D): a V-bit two's-complement integer q with one power-of-two
  scale per row, decoded value q * 2^e_row.  The paper names integer and
  fixed-point values but defines none; this reading is ours.
"""
from __future__ import annotations

import struct

import numpy as np

FMT_FP16 = 0
FMT_E8MY = 1
FMT_FIX = 2

FMT_NAMES = {FMT_FP16: "fp16", FMT_E8MY: "e8my", FMT_FIX: "fix"}


def d_range(fmt: int):
    """Admissible delta widths D for each value format.

    FP16 fixes V = 16, so D = 15.  E8MY needs Y = 22 - D >= 0.  FIX keeps at
    least two value bits (sign and one magnitude bit).  D = 0 is excluded: the unpacking shifts would reach
    32 (sec. 4.3 allows D "as small as 1 bit").
    """
    if fmt == FMT_FP16:
        return (15, 15)
    if fmt == FMT_E8MY:
        return (1, 22)
    if fmt == FMT_FIX:
        return (1, 29)
    raise ValueError(fmt)


def _round_half_away(x: np.ndarray) -> np.ndarray:
    """Round to nearest integer, ties away from zero (C's round / std::round)."""
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


# ---------------------------------------------------------------------------
# FP16 (sec. 4.2.2, first example)
# ---------------------------------------------------------------------------

def fp16_value_bits(v32: np.ndarray) -> np.ndarray:
    """Upper-16-bit value field for FP16: IEEE binary16 of the float32 value,
    round to nearest even (a half-precision cast), placed << 16.

    Readings: |v| >= 65520 becomes +-inf; half subnormals are kept; NaN is
    stored as the canonical quiet NaN 0x7E00.
    """
    v32 = np.asarray(v32, dtype=np.float32)
    h = v32.astype(np.float16)
    bits = h.view(np.uint16).astype(np.uint32)
    bits[np.isnan(v32)] = 0x7E00
    return bits << np.uint32(16)


def fp16_value_bits_scalar(v: float) -> int:
    """Same as ``fp16_value_bits`` for one Python float, through the struct
    module's binary16 packing (round half to even) -- kept for cross-checks."""
    if v != v:
        return 0x7E00 << 16
    try:
        (h,) = struct.unpack("<H", struct.pack("<e", float(np.float32(v))))
    except OverflowError:
        h = 0x7C00 | (0x8000 if v < 0 else 0)
    return h << 16


# ---------------------------------------------------------------------------
# E8MY (sec. 4.2.2, second example)
# ---------------------------------------------------------------------------

def e8my_grid_neighbours(v32: np.ndarray, D: int):
    """The two E8MY values that enclose each float32 v (sec. 4.2.2): E8MY
    holds the float32 values whose low D + 1 pattern bits are zero, so the
    neighbour toward zero has those bits cleared and the one away from zero
    is the next such pattern (possibly the infinity pattern)."""
    b = np.asarray(v32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    low = np.uint64((1 << (D + 1)) - 1)
    toward = b & ~low & np.uint64(0xFFFFFFFF)
    sign = toward & np.uint64(0x80000000)
    mag = (toward & np.uint64(0x7FFFFFFF)) + np.uint64(1 << (D + 1))
    away = sign | np.minimum(mag, np.uint64(0x7F800000))
    return toward.astype(np.uint32), away.astype(np.uint32)


def e8my_value_bits(v32: np.ndarray, D: int) -> np.ndarray:
    """float32 -> E8MY value field (Y = 22 - D, sec. 4.2.2): the nearest
    E8MY value, ties away from zero (the conversion rounds with C's round).

    Distances to the two neighbours are exact in float64; the infinity
    pattern stands for 2^128, the first value past the float32 range, so a
    value at or past the midpoint above the largest finite E8MY value
    becomes infinity.  Readings: the same rule on the subnormal grid; +-0
    and +-inf kept; NaN -> 0x7FC00000.
    """
    if not (1 <= D <= 22):
        raise ValueError("E8MY needs 1 <= D <= 22")
    v32 = np.asarray(v32, dtype=np.float32)
    toward, away = e8my_grid_neighbours(v32, D)

    def magnitude(bits):
        m = np.abs(bits.view(np.float32).astype(np.float64))
        return np.where((bits & np.uint32(0x7FFFFFFF)) == 0x7F800000, 2.0 ** 128, m)

    a = np.abs(v32.astype(np.float64))
    with np.errstate(invalid="ignore"):
        d_toward = a - magnitude(toward)
        d_away = magnitude(away) - a
        out = np.where(d_away <= d_toward, away, toward).astype(np.uint32)
    out[np.isinf(v32)] = v32.view(np.uint32)[np.isinf(v32)]
    out[np.isnan(v32)] = 0x7FC00000
    return out


# ---------------------------------------------------------------------------
# FIX (integer value with a per-row power-of-two scale; our reading)
# ---------------------------------------------------------------------------

def fix_row_exponent(row_absmax: np.ndarray, D: int) -> np.ndarray:
    """e_row = e(M) - (V - 1) where M = max |a| over the row and e(M) is the
    binary exponent with M = f * 2^e(M), 1/2 <= f < 1; this puts
    |a| / 2^e_row below 2^(V - 1).  Empty or all-zero rows get e_row = 0."""
    V = 31 - D
    M = np.asarray(row_absmax, dtype=np.float64)
    _, e = np.frexp(M)
    e = e.astype(np.int64) - (V - 1)
    e[M == 0] = 0
    return e


def fix_value_bits(v32: np.ndarray, e_row: np.ndarray, D: int) -> np.ndarray:
    """q = clamp(round_half_away(v / 2^e_row), +-(2^(V-1) - 1)) as a V-bit
    two's-complement field in the upper V bits of the word."""
    if not (1 <= D <= 29):
        raise ValueError("FIX needs 1 <= D <= 29")
    V = 31 - D
    v = np.asarray(v32, dtype=np.float32).astype(np.float64)
    if not np.all(np.isfinite(v)):
        raise ValueError("FIX values must be finite")
    q = _round_half_away(np.ldexp(v, -np.asarray(e_row, dtype=np.int64)))
    lim = 2.0 ** (V - 1) - 1
    q = np.clip(q, -lim, lim).astype(np.int64)
    return ((q << (D + 1)) & 0xFFFFFFFF).astype(np.uint32)


# ---------------------------------------------------------------------------
# Word codec (sec. 4.2.1, packing and unpacking)
# ---------------------------------------------------------------------------

def pack_value_word(value_bits: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """Flag-1 word: value field (already in the upper V bits) OR delta << 1
    OR 1.  The caller guarantees delta < 2^D."""
    value_bits = np.asarray(value_bits, dtype=np.uint32)
    delta = np.asarray(delta, dtype=np.uint64)
    return (value_bits | (delta << np.uint64(1)).astype(np.uint32) | np.uint32(1)).astype(np.uint32)


def pack_delta_word(delta: np.ndarray) -> np.ndarray:
    """Flag-0 word (dummy): the whole upper 31 bits hold the delta."""
    delta = np.asarray(delta, dtype=np.uint64)
    if np.any(delta > 0x7FFFFFFF):
        raise OverflowError("delta does not fit in 31 bits")
    return (delta << np.uint64(1)).astype(np.uint32)


def unpack_word(p: np.ndarray, D: int):
    """(flag, delta, value_bits) of 32-bit words (sec. 4.2.1): bit 0 is the
    flag; a flag-1 word has its delta in bits 1..D and its value field in
    bits D+1..31, a flag-0 word its delta in bits 1..31 and no value."""
    p = np.asarray(p, dtype=np.uint32)
    flag = p & np.uint32(1)
    one = flag == 1
    delta = np.where(one, (p >> np.uint32(1)) & np.uint32((1 << D) - 1), p >> np.uint32(1))
    value_bits = np.where(one, p & np.uint32((0xFFFFFFFF << (D + 1)) & 0xFFFFFFFF), np.uint32(0))
    return flag.astype(np.uint32), delta.astype(np.uint32), value_bits.astype(np.uint32)


def value_from_bits(value_bits: np.ndarray, fmt: int, D: int) -> np.ndarray:
    """Reinterpret a value field as a float64 number (FIX: the integer q;
    the row scale is applied by the caller)."""
    b = np.asarray(value_bits, dtype=np.uint32)
    if fmt == FMT_FP16:
        return (b >> np.uint32(16)).astype(np.uint16).view(np.float16).astype(np.float64)
    if fmt == FMT_E8MY:
        return b.view(np.float32).astype(np.float64)
    if fmt == FMT_FIX:
        return (b.view(np.int32).astype(np.int64) >> (D + 1)).astype(np.float64)
    raise ValueError(fmt)
