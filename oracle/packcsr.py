"""CSR-based delta-value packing (oracle; test infrastructure only, never
called by the product path).

The paper names extending its delta-value packing to CSR-based formats as
future work (sec. 6), for matrices whose row lengths vary so much that
SELL pads heavily.  Reading: the words of every row are the PackSELL words
of sec. 4 (32-bit words, sec. 4.2.1; FP16, E8MY and FIX values, sec. 4.2.2;
one dummy before a delta that does not fit, sec. 4.3), stored row after row
with no padding and no row sort, and a word row pointer in place of slice
offsets.  Every row's first delta is taken from its eq. 4 left offset with
a window of one row (row i - k_left when k_left < i, else 0).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import formats as F


@dataclasses.dataclass
class PackedCSR:
    n: int
    m: int
    nnz: int
    fmt: int
    D: int
    k_left: int
    n_words: int
    n_dummies: int
    pack: np.ndarray     # uint32[n_words], row after row
    wrowptr: np.ndarray  # int64[n + 1], row starts in words
    row_exp: np.ndarray | None  # int64[n] FIX exponents


def left_offset(i: np.ndarray, k_left: int) -> np.ndarray:
    """Eq. 4 with a window of one row: i - k_left when k_left < i, else 0."""
    i = np.asarray(i, dtype=np.int64)
    return np.where(k_left < i, i - k_left, 0)


def encode(rowptr, col, val, n: int, m: int, fmt: int, D: int) -> PackedCSR:
    """Words of each row in CSR order: for each stored (j, v), d = j - prev
    (prev = the row's left offset, then the previous column); a delta of
    2^D or more is preceded by a dummy carrying it (flag 0), after which the
    value word carries delta 0."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    lo, hi = F.d_range(fmt)
    if not (lo <= D <= hi) or fmt not in (F.FMT_FP16, F.FMT_E8MY, F.FMT_FIX):
        raise ValueError("bad format or D")
    if rowptr.shape != (n + 1,) or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise ValueError("bad rowptr")
    nnz = int(rowptr[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    if nnz and (col.min() < 0 or col.max() >= m):
        raise ValueError("column out of range")
    if np.any((rows[1:] == rows[:-1]) & (np.diff(col) <= 0)):
        raise ValueError("columns must strictly increase within a row")
    v32 = np.asarray(val, dtype=np.float64).astype(np.float32)
    k_left = int(max(0, int(np.max(rows - col)))) if nnz else 0
    # previous column of each entry: the row's left offset for its first one
    prev = np.empty(nnz, dtype=np.int64)
    if nnz:
        prev[1:] = col[:-1]
        starts = rowptr[:-1][np.diff(rowptr) > 0]
        prev[starts] = left_offset(rows[starts], k_left)
    delta = col - prev
    big = delta >= (1 << D)
    row_exp = None
    if fmt == F.FMT_FP16:
        vbits = F.fp16_value_bits(v32)
    elif fmt == F.FMT_E8MY:
        vbits = F.e8my_value_bits(v32, D)
    else:
        absmax = np.zeros(n)
        if nnz:
            np.maximum.at(absmax, rows, np.abs(v32.astype(np.float64)))
        row_exp = F.fix_row_exponent(absmax, D)
        vbits = F.fix_value_bits(v32, row_exp[rows], D)
    # one or two words per entry, in entry order
    end = np.cumsum(1 + big.astype(np.int64))
    pack = np.zeros(int(end[-1]) if nnz else 0, dtype=np.uint32)
    pack[end - 1] = F.pack_value_word(vbits, np.where(big, 0, delta))
    pack[end[big] - 2] = F.pack_delta_word(delta[big])
    wrowptr = np.zeros(n + 1, dtype=np.int64)
    wrowptr[1:] = np.cumsum(np.diff(rowptr) + np.bincount(rows[big], minlength=n))
    return PackedCSR(n=n, m=m, nnz=nnz, fmt=fmt, D=D, k_left=k_left,
                     n_words=int(pack.size), n_dummies=int(big.sum()), pack=pack,
                     wrowptr=wrowptr, row_exp=row_exp)


def word_rows(E: PackedCSR) -> np.ndarray:
    """The row of every word."""
    return np.repeat(np.arange(E.n, dtype=np.int64), np.diff(E.wrowptr))


def columns_after(E: PackedCSR) -> np.ndarray:
    """The running column after every word: the row's left offset plus the
    deltas of the row's words up to and including this one (the decode of
    sec. 4.4, row by row)."""
    _, d, _ = F.unpack_word(E.pack, E.D)
    r = word_rows(E)
    total = np.cumsum(d.astype(np.int64))
    before_row = np.concatenate([[0], total])[E.wrowptr[:-1]]  # deltas of earlier rows
    return left_offset(r, E.k_left) + total - before_row[r]


def spmv(E: PackedCSR, x: np.ndarray) -> np.ndarray:
    """y = A_q x in float64: for each row, walk its words from the left
    offset, add each delta to the column and, for flag-1 words, the decoded
    value times x at that column (sec. 4.4); FIX rows scaled by 2^e."""
    x = np.asarray(x, dtype=np.float64)
    flag, _, vb = F.unpack_word(E.pack, E.D)
    v = F.value_from_bits(vb, E.fmt, E.D)
    cols = columns_after(E)
    prod = np.where(flag == 1, v * x[np.where(flag == 1, cols, 0)] if E.m else 0.0, 0.0)
    y = np.zeros(E.n)
    np.add.at(y, word_rows(E), prod)
    if E.fmt == F.FMT_FIX:
        y = np.ldexp(y, E.row_exp)
    return y
