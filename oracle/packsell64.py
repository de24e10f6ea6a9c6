"""PackSELL with 64-bit words and an FP64-compatible value (oracle; test
infrastructure only: nothing on the product path imports it).

Sec. 4.2.1 fixes the word layout for any word width W: bit 0 is a flag;
with flag = 1 the upper V = W - 1 - D bits hold the value and bits 1..D a
delta below 2^D; with flag = 0 the upper W - 1 bits hold a delta and there is
no value (a dummy, sec. 4.3); the all-zero word is padding.  Sec. 4.2.2
builds its E8MY format by giving the low D + 1 bits of the FP32 pattern to
the delta and the flag.  Here the same construction is applied to FP64
(our reading, since the paper spells it out for W = 32 only): with W = 64
the value is an E11MY float, the FP64 pattern with Y = 51 - D mantissa bits,
so 1 <= D <= 51, rounded to nearest with ties away from zero as E8MY is.
Readings as for E8MY: the same rule on the subnormal grid; +-0 and +-inf
are kept; NaN becomes the canonical quiet NaN 0x7FF8000000000000; a value
past the midpoint above the largest finite E11MY value becomes +-inf.

The encoder follows the same steps E0 - E8 as the 32-bit oracle
(oracle/packsell.py), written again here for 64-bit words: lower bandwidth
and eq. 4 offsets, deltas and dummies (eq. 2, sec. 4.3), the sigma-window
sort, slice widths and offsets, column-major packing.  The SpMV is the
algorithm of sec. 4.4 in float64 with float64 x.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .packsell import row_columns, row_words

W = 64
PERM_EXPLICIT = 0
PERM_IMPLICIT = 1


def e11my_value_bits(v: np.ndarray, D: int) -> np.ndarray:
    """float64 -> E11MY value field (uint64, low D + 1 bits zero): the
    nearest float64 value whose low D + 1 pattern bits are zero, ties away
    from zero, as E8MY rounds float32 (sec. 4.2.2).

    The two candidates are the pattern with those bits cleared (toward zero)
    and the next such pattern (away from zero; the infinity pattern past the
    largest finite value, standing for 2^1024).  Both distances are exact in
    float64 (Sterbenz); next to 2^1024 they are compared halved.  +-0 and
    +-inf are kept; NaN becomes 0x7FF8000000000000.
    """
    if not (1 <= D <= 51):
        raise ValueError("E11MY needs 1 <= D <= 51")
    v = np.asarray(v, dtype=np.float64)
    b = v.view(np.uint64)
    low = np.uint64((1 << (D + 1)) - 1)
    sign_bit = np.uint64(1 << 63)
    inf_pat = np.uint64(0x7FF0000000000000)
    toward = b & ~low
    sign = toward & sign_bit
    tmag = toward & ~sign_bit
    amag = np.minimum(tmag + np.uint64(1 << (D + 1)), inf_pat)
    away = sign | amag
    a = np.abs(v)
    t = tmag.view(np.float64)
    over = amag == inf_pat
    with np.errstate(invalid="ignore", over="ignore"):
        d_toward = np.where(over, 0.5 * a - 0.5 * t, a - t)
        d_away = np.where(over, 2.0 ** 1023 - 0.5 * a, amag.view(np.float64) - a)
        out = np.where(d_away <= d_toward, away, toward)
    out = np.where(np.isinf(v), b, out)
    out = np.where(np.isnan(v), np.uint64(0x7FF8000000000000), out)
    return out.astype(np.uint64)


def quantized(v: np.ndarray, D: int) -> np.ndarray:
    """The decoded values q(v) as float64."""
    return e11my_value_bits(v, D).view(np.float64)


def pack_value_word(value_bits, delta):
    return (np.asarray(value_bits, np.uint64) | (np.asarray(delta, np.uint64) << np.uint64(1))
            | np.uint64(1))


def pack_delta_word(delta):
    delta = np.asarray(delta, np.uint64)
    if np.any(delta >= np.uint64(1) << np.uint64(63)):
        raise OverflowError("delta does not fit in 63 bits")
    return delta << np.uint64(1)


def unpack_word(p, D: int):
    """(flag, delta, value_bits) of 64-bit words: a flag-1 word has its delta
    in bits 1..D and its value in bits D+1..63; a flag-0 word has its delta
    in bits 1..63 and no value."""
    p = np.asarray(p, dtype=np.uint64)
    flag = p & np.uint64(1)
    dmask = np.uint64((1 << D) - 1)
    delta = np.where(flag == 1, (p >> np.uint64(1)) & dmask, p >> np.uint64(1))
    vmask = np.uint64(((1 << 64) - 1) >> (D + 1) << (D + 1))
    value_bits = np.where(flag == 1, p & vmask, np.uint64(0))
    return flag, delta, value_bits


@dataclass
class Encoded64:
    n: int
    m: int
    C: int
    sigma: int
    D: int
    k_left: int
    perm_mode: int
    offset: np.ndarray       # int64[n_slices + 1], in words
    pack: np.ndarray         # uint64[n_words]
    perm: np.ndarray         # int64[n]: original row - window start, per stored row
    stored_rows: np.ndarray  # int64[n]
    n_dummies: int

    @property
    def n_words(self) -> int:
        return int(self.pack.size)


def left_offsets(n: int, sigma: int, k_left: int) -> np.ndarray:
    """eq. 4: the block-uniform left offset of every row."""
    blk = (np.arange(n, dtype=np.int64) // sigma) * sigma
    return np.where(k_left < blk, blk - k_left, 0)


def encode(rowptr, col, val, n: int, m: int, D: int, C: int, sigma: int,
           perm_mode: int = PERM_IMPLICIT) -> Encoded64:
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    val = np.asarray(val, np.float64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    # E1: lower bandwidth on the original order
    k_left = int(max(0, (rows - col).max())) if col.size else 0
    # E2/E3: deltas from the eq. 4 offsets, dummies for deltas >= 2^D
    start = left_offsets(n, sigma, k_left)
    prev = np.empty(col.size, np.int64)
    if col.size:
        prev[:] = col
        prev[1:] = col[:-1]
        first = rowptr[:-1][np.diff(rowptr) > 0]
        prev[first] = start[rows[first]]
    delta = col - prev
    dummy = delta >= (1 << D)
    cnt = np.diff(rowptr) + np.bincount(rows[dummy], minlength=n).astype(np.int64)
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
    # E7: words of every row in order, column-major per slice; padding = 0.
    # Entry e of row r is the word j = (e - rowptr[r]) + (dummies of row r
    # up to and including e); its dummy, if any, is word j - 1.
    qbits = e11my_value_bits(val, D)
    pack = np.zeros(int(offset[-1]), np.uint64)
    if col.size:
        stored_index = np.empty(n, np.int64)
        stored_index[stored_rows] = np.arange(n)
        dcum = np.cumsum(dummy.astype(np.int64))
        row_base = np.concatenate([[0], dcum])[rowptr[:-1]]  # dummies before each row
        j = (np.arange(col.size) - rowptr[rows]) + (dcum - row_base[rows])
        s_of = stored_index[rows]
        k, l = s_of // C, s_of % C
        pack[offset[k] + j * C + l] = pack_value_word(qbits, np.where(dummy, 0, delta))
        dm = np.nonzero(dummy)[0]
        pack[offset[k[dm]] + (j[dm] - 1) * C + l[dm]] = pack_delta_word(delta[dm])
    return Encoded64(n, m, C, sigma, D, k_left, perm_mode, offset, pack, perm, stored_rows,
                     int(dummy.sum()))


def spmv(E: Encoded64, x: np.ndarray) -> np.ndarray:
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
    prod[has] = vb[has].view(np.float64) * x[col[has]]
    t = np.bincount(row, weights=prod, minlength=n)[:n] if n else np.zeros(0)
    y = np.zeros(n)
    if E.perm_mode == PERM_IMPLICIT:
        i = np.arange(n, dtype=np.int64)
        y[(i // E.sigma) * E.sigma + E.perm] = t
    else:
        y[:] = t
    return y
