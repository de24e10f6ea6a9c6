"""PackSELL with 16-bit words and 8-bit-class values (oracle; test
infrastructure only: nothing on the product path imports it).

Sec. 4.2.1 fixes the word layout for any word width W: bit 0 is a flag;
with flag = 1 the upper V = W - 1 - D bits hold the value and bits 1..D a
delta below 2^D; with flag = 0 the upper W - 1 bits hold a delta and there
is no value (a dummy, sec. 4.3); the all-zero word is padding.  The paper
spells out the value formats for W = 32 only.  Our readings for W = 16:

* E5MY values (Y = 9 - D, 1 <= D <= 8): the E8MY construction of sec.
  4.2.2 applied to IEEE binary16 -- the binary16 bit pattern whose low D + 1
  bits are given to the delta and the flag.  The float32 input is rounded
  directly onto that grid (one rounding, not float32 -> binary16 -> E5MY),
  to nearest with ties away from zero as for E8MY: for |v| >= 2^-14 the
  step is 2^(e - Y) with 2^e <= |v| < 2^(e + 1); below 2^-14 the step is
  2^(D + 1 - 24) (the binary16 subnormal grid with D + 1 bits dropped); a
  result above the largest finite value (2 - 2^-Y) * 2^15 becomes +-inf;
  +-0 and +-inf are kept; NaN becomes 0x7E00.  With D = 7 the values are
  those of the 8-bit E5M2 format (1 sign, 5 exponent, 2 mantissa bits).
* FIX16 values (V = 15 - D, 1 <= D <= 13): the FIX format with a V-bit
  two's-complement field and a per-row exponent, as for W = 32; with
  D = 7 the field is an int8.
* Dummy chains: a flag-0 word carries at most 2^15 - 1, so a delta
  d >= 2^D is carried by ceil(d / (2^15 - 1)) dummies, each with 2^15 - 1
  except the last, which holds the remainder, followed by the value word
  with delta 0.  For d < 2^15 this is the single dummy of sec. 4.3.

The encoder takes the steps E0 - E8 of the 32-bit oracle (oracle/packsell.py)
with these words; ``pack`` is column-major per slice in 16-bit words, as
the paper lays out words of any width.  The SpMV is the algorithm of sec.
4.4 in float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .packsell import row_columns, row_words

W = 16
FMT_E5MY = 4
FMT_FIX16 = 5
DUMMY_MAX = (1 << 15) - 1
PERM_EXPLICIT = 0
PERM_IMPLICIT = 1


def d_range(fmt: int):
    if fmt == FMT_E5MY:
        return 1, 8
    if fmt == FMT_FIX16:
        return 1, 13
    raise ValueError(f"unknown 16-bit format {fmt}")


def _round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def e5my_value_bits(v32: np.ndarray, D: int) -> np.ndarray:
    """float32 -> E5MY value field (uint16, low D + 1 bits zero)."""
    lo, hi = d_range(FMT_E5MY)
    if not (lo <= D <= hi):
        raise ValueError("E5MY needs 1 <= D <= 8")
    Y = 9 - D
    v = np.asarray(v32, dtype=np.float32).astype(np.float64)
    a = np.abs(v)
    q = np.zeros(v.shape, dtype=np.float64)
    finite = np.isfinite(v)
    normal = finite & (a >= 2.0 ** -14)
    sub = finite & ~normal
    if normal.any():
        _, ex = np.frexp(a[normal])  # a = f 2^ex, 1/2 <= f < 1, so e = ex - 1
        step = np.ldexp(1.0, ex - 1 - Y)
        q[normal] = np.floor(a[normal] / step + 0.5) * step
    if sub.any():
        step = 2.0 ** (D + 1 - 24)
        q[sub] = np.floor(a[sub] / step + 0.5) * step
    q[~finite] = np.inf
    q[q > (2.0 - 2.0 ** -Y) * 2.0 ** 15] = np.inf
    bits = q.astype(np.float16).view(np.uint16).copy()  # q is a binary16 value: exact
    bits[np.signbit(v)] |= np.uint16(0x8000)
    bits[np.isnan(v)] = np.uint16(0x7E00)
    return bits


def fix16_row_exponent(row_absmax: np.ndarray, D: int) -> np.ndarray:
    """e_row = e(M) - (V - 1), V = 15 - D, with M = f 2^e(M), 1/2 <= f < 1
    the row's largest magnitude; empty or all-zero rows get 0."""
    V = 15 - D
    M = np.asarray(row_absmax, dtype=np.float64)
    _, e = np.frexp(M)
    e = e.astype(np.int64) - (V - 1)
    e[M == 0] = 0
    return e


def fix16_value_bits(v32: np.ndarray, e_row: np.ndarray, D: int) -> np.ndarray:
    """q = clamp(round_half_away(v / 2^e_row), +-(2^(V-1) - 1)) as a V-bit
    two's-complement field in the upper V bits of the 16-bit word."""
    lo, hi = d_range(FMT_FIX16)
    if not (lo <= D <= hi):
        raise ValueError("FIX16 needs 1 <= D <= 13")
    V = 15 - D
    v = np.asarray(v32, dtype=np.float32).astype(np.float64)
    if not np.all(np.isfinite(v)):
        raise ValueError("FIX16 values must be finite")
    q = _round_half_away(np.ldexp(v, -np.asarray(e_row, dtype=np.int64)))
    lim = 2.0 ** (V - 1) - 1
    q = np.clip(q, -lim, lim).astype(np.int64)
    return ((q << (D + 1)) & 0xFFFF).astype(np.uint16)


def value_from_bits(bits: np.ndarray, fmt: int, D: int) -> np.ndarray:
    """A value field as a float64 number (FIX16: the integer q; the row
    scale 2^e_row is applied by the caller)."""
    b = np.asarray(bits, dtype=np.uint16)
    if fmt == FMT_E5MY:
        return b.view(np.float16).astype(np.float64)
    return (b.view(np.int16).astype(np.int64) >> (D + 1)).astype(np.float64)


def pack_value_word(value_bits, delta):
    delta = np.asarray(delta, dtype=np.uint32)
    return (np.asarray(value_bits, np.uint16).astype(np.uint32) | (delta << 1) | 1).astype(np.uint16)


def pack_delta_word(delta):
    delta = np.asarray(delta, dtype=np.uint32)
    if np.any(delta > DUMMY_MAX):
        raise OverflowError("a dummy carries at most 2^15 - 1")
    return (delta << 1).astype(np.uint16)


def unpack_word(p, D: int):
    """(flag, delta, value_bits) of 16-bit words: a flag-1 word has its delta
    in bits 1..D and its value in bits D+1..15; a flag-0 word has its delta
    in bits 1..15 and no value."""
    p = np.asarray(p, dtype=np.uint16).astype(np.uint32)
    flag = p & 1
    delta = np.where(flag == 1, (p >> 1) & ((1 << D) - 1), p >> 1)
    vmask = 0xFFFF & ~((1 << (D + 1)) - 1)
    value_bits = np.where(flag == 1, p & vmask, 0).astype(np.uint16)
    return flag.astype(np.uint16), delta.astype(np.int64), value_bits


def dummies_for(d, D: int):
    """Dummies that carry a delta d: 0 when d < 2^D, else ceil(d / (2^15 - 1))."""
    d = np.asarray(d, dtype=np.int64)
    return np.where(d >= (1 << D), (d + DUMMY_MAX - 1) // DUMMY_MAX, 0)


@dataclass
class Encoded16:
    n: int
    m: int
    fmt: int
    C: int
    sigma: int
    D: int
    k_left: int
    perm_mode: int
    offset: np.ndarray       # int64[n_slices + 1], in 16-bit words
    pack: np.ndarray         # uint16[n_words], column-major per slice
    perm: np.ndarray         # int64[n]: original row - window start, per stored row
    stored_rows: np.ndarray  # int64[n]
    n_dummies: int
    row_exp: np.ndarray | None  # int64[n], FIX16 exponents in stored order

    @property
    def n_words(self) -> int:
        return int(self.pack.size)


def left_offsets(n: int, sigma: int, k_left: int) -> np.ndarray:
    """eq. 4: the block-uniform left offset of every row."""
    blk = (np.arange(n, dtype=np.int64) // sigma) * sigma
    return np.where(k_left < blk, blk - k_left, 0)


def value_field(val, rowptr, fmt: int, D: int, n: int):
    """E0 + quantisation: float32 values, then the value fields (and, for
    FIX16, the per-row exponents in original row order)."""
    v32 = np.asarray(val).astype(np.float32)
    if fmt == FMT_E5MY:
        return e5my_value_bits(v32, D), None
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    mx = np.zeros(n)
    if v32.size:
        np.maximum.at(mx, rows, np.abs(v32.astype(np.float64)))
    e_row = fix16_row_exponent(mx, D)
    return fix16_value_bits(v32, e_row[rows], D), e_row


def quantized(rowptr, val, n: int, fmt: int, D: int) -> np.ndarray:
    """The decoded values q(a_ij) as float64, in CSR order."""
    bits, e_row = value_field(val, rowptr, fmt, D, n)
    q = value_from_bits(bits, fmt, D)
    if fmt == FMT_FIX16:
        rows = np.repeat(np.arange(n), np.diff(rowptr))
        q = np.ldexp(q, e_row[rows])
    return q


def encode(rowptr, col, val, n: int, m: int, fmt: int, D: int, C: int, sigma: int,
           perm_mode: int = PERM_IMPLICIT) -> Encoded16:
    lo, hi = d_range(fmt)
    if not (lo <= D <= hi):
        raise ValueError("D out of range")
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    # E1: lower bandwidth on the original order
    k_left = int(max(0, (rows - col).max())) if col.size else 0
    # E2/E3: deltas from the eq. 4 offsets, dummy chains for deltas >= 2^D
    start = left_offsets(n, sigma, k_left)
    prev = np.empty(col.size, np.int64)
    if col.size:
        prev[:] = col
        prev[1:] = col[:-1]
        first = rowptr[:-1][np.diff(rowptr) > 0]
        prev[first] = start[rows[first]]
    delta = col - prev
    nd = dummies_for(delta, D)
    # E4: words per row
    cnt = np.diff(rowptr) + np.bincount(rows, weights=nd, minlength=n).astype(np.int64)
    # E5: stable descending sort by count within each sigma-window
    win = np.arange(n, dtype=np.int64) // sigma
    stored_rows = np.lexsort((np.arange(n), -cnt, win)).astype(np.int64)
    perm = stored_rows - (stored_rows // sigma) * sigma
    # E6: slice widths and offsets
    n_slices = -(-n // C)
    cnt_stored = np.zeros(n_slices * C, np.int64)
    cnt_stored[:n] = cnt[stored_rows]
    width = cnt_stored.reshape(n_slices, C).max(axis=1) if n else np.zeros(0, np.int64)
    offset = np.zeros(n_slices + 1, np.int64)
    offset[1:] = np.cumsum(C * width)
    # E7: the words of every row in order, column-major per slice; the
    # value word of entry e is word j_e of its row (entries before it and
    # all dummies up to and including its own chain come first); its chain
    # occupies words j_e - nd_e .. j_e - 1.
    bits, e_row = value_field(val, rowptr, fmt, D, n)
    pack = np.zeros(int(offset[-1]), np.uint16)
    if col.size:
        stored_index = np.empty(n, np.int64)
        stored_index[stored_rows] = np.arange(n)
        ncum = np.cumsum(nd)
        row_base = np.concatenate([[0], ncum])[rowptr[:-1]]  # dummies before each row
        j = (np.arange(col.size) - rowptr[rows]) + (ncum - row_base[rows])
        s_of = stored_index[rows]
        k, l = s_of // C, s_of % C
        pack[offset[k] + j * C + l] = pack_value_word(bits, np.where(nd > 0, 0, delta))
        # chains: entry e contributes nd_e dummies, words j_e - nd_e + t for t < nd_e
        ed = np.repeat(np.arange(col.size), nd)
        t = np.arange(ed.size) - np.repeat(np.cumsum(nd) - nd, nd)
        last = t == nd[ed] - 1
        dd = np.where(last, delta[ed] - DUMMY_MAX * (nd[ed] - 1), DUMMY_MAX)
        pack[offset[k[ed]] + (j[ed] - nd[ed] + t) * C + l[ed]] = pack_delta_word(dd)
    rexp = e_row[stored_rows] if e_row is not None else None
    return Encoded16(n, m, fmt, C, sigma, D, k_left, perm_mode, offset, pack, perm, stored_rows,
                     int(nd.sum()), rexp)


def spmv(E: Encoded16, x: np.ndarray) -> np.ndarray:
    """y = A_q x through the format (sec. 4.4), in float64: decode each
    stored row's words (columns from the eq. 4 left offset plus the running
    deltas), then take the dot product of its flag-1 values with x; y in the
    original order (implicit) or in stored order (explicit)."""
    x = np.asarray(x, np.float64)
    n = E.n
    row, pos, start = row_words(E.offset, n, E.C)
    flag, delta, vb = unpack_word(E.pack[pos], E.D)
    col = row_columns(delta, row, start, left_offsets(n, E.sigma, E.k_left))
    has = flag == 1
    prod = np.zeros(row.size)
    prod[has] = value_from_bits(vb[has], E.fmt, E.D) * x[col[has]]
    t = np.bincount(row, weights=prod, minlength=n)[:n] if n else np.zeros(0)
    if E.fmt == FMT_FIX16:
        t = np.ldexp(t, E.row_exp)
    y = np.zeros(n)
    if E.perm_mode == PERM_IMPLICIT:
        i = np.arange(n, dtype=np.int64)
        y[(i // E.sigma) * E.sigma + E.perm] = t
    else:
        y[:] = t
    return y
