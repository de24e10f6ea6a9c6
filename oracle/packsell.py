"""PackSELL encoder, decoder and SpMV algorithm (oracle; test infrastructure).

The encoder takes the steps of sec. 4 in the paper's order:

E0  values rounded to float32 (the conversion in sec. 4.2.2 assumes a float).
E1  k_left = lower bandwidth = max(0, max over stored (i, j) of i - j),
    on the original row order.
E2  left offset per row, block-uniform (eq. 4):
    dfrak_i = floor(i/sigma)*sigma - k_left if k_left < floor(i/sigma)*sigma,
    else 0.
E3  delta encoding (eq. 2): walk each row with prev = dfrak_i; for each
    stored (j, v): d = j - prev; if d < 2^D emit a flag-1 word carrying v,
    else emit a dummy (flag 0, delta d) at the same column followed by the
    flag-1 word with delta 0 (sec. 4.3); prev = j.
E4  cnt_i = stored words of row i (nonzeros + dummies).
E5  SELL-C-sigma row sort (sec. 3, sec. 4.3): inside each window of sigma
    rows, a stable sort by cnt, descending (ties keep ascending row order);
    perm_i = original row - window start, for stored row i.
E6  slices of C stored rows; w_k = max cnt over the slice (rows past n count
    as 0); offset_0 = 0, offset_{k+1} = offset_k + C * w_k (in words).
E7  pack[offset_k + j*C + l] = word j of stored row k*C + l, or the all-zero
    padding word when j >= cnt (sec. 4.3).
E8  implicit mode keeps ``perm`` and produces y in the original order;
    explicit mode produces y in stored order (sec. 3).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import formats as F

PERM_EXPLICIT = 0
PERM_IMPLICIT = 1


@dataclasses.dataclass
class Encoded:
    n: int
    m: int
    nnz: int
    fmt: int
    D: int
    C: int
    sigma: int
    perm_mode: int
    k_left: int
    n_slices: int
    n_words: int
    n_dummies: int
    pack: np.ndarray  # uint32[n_words]
    offset: np.ndarray  # int64[n_slices + 1]
    perm: np.ndarray  # uint8/uint16[n] (local row in window), stored order
    stored_rows: np.ndarray  # int64[n]: original row of stored row i
    cnt: np.ndarray  # int64[n]: words of each ORIGINAL row
    row_exp: np.ndarray | None  # int64[n] FIX exponents, stored order


def k_left_of(rowptr: np.ndarray, col: np.ndarray, n: int) -> int:
    """E1: lower bandwidth (never negative)."""
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    if rows.size == 0:
        return 0
    return int(max(0, int(np.max(rows - col.astype(np.int64)))))


def left_offsets(n: int, sigma: int, k_left: int) -> np.ndarray:
    """E2 / eq. 4 for every row index 0..n-1."""
    blk = (np.arange(n, dtype=np.int64) // sigma) * sigma
    return np.where(k_left < blk, blk - k_left, 0)


def _check_csr(rowptr, col, n, m):
    if rowptr.shape != (n + 1,) or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise ValueError("bad rowptr")
    nnz = int(rowptr[-1])
    if col.shape != (nnz,):
        raise ValueError("bad col length")
    if nnz and (col.min() < 0 or col.max() >= m):
        raise ValueError("column out of range")
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    same_row = rows[1:] == rows[:-1]
    if np.any(same_row & (np.diff(col.astype(np.int64)) <= 0)):
        raise ValueError("columns must strictly increase within a row")


def encode(rowptr, col, val, n: int, m: int, fmt: int, D: int, C: int,
           sigma: int, perm_mode: int = PERM_IMPLICIT) -> Encoded:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    lo, hi = F.d_range(fmt)
    if not (lo <= D <= hi):
        raise ValueError("D out of range for the format")
    if C < 1 or C > 64 or (C & (C - 1)):
        raise ValueError("C must be a power of two in [1, 64]")
    if sigma < 1 or sigma > 65536:
        raise ValueError("sigma must be in [1, 65536]")
    _check_csr(rowptr, col, n, m)
    nnz = int(rowptr[-1])

    # E0
    v32 = np.asarray(val, dtype=np.float64).astype(np.float32)
    # E1, E2
    kl = k_left_of(rowptr, col, n)
    dfrak = left_offsets(n, sigma, kl)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    # E3: previous column of each entry (dfrak for the leftmost one)
    first = np.zeros(nnz, dtype=bool)
    first[rowptr[:-1][np.diff(rowptr) > 0]] = True
    prev = np.empty(nnz, dtype=np.int64)
    prev[1:] = col[:-1]
    prev[first] = dfrak[rows[first]]
    delta = col - prev
    assert np.all(delta >= 0)
    overflow = delta >= (1 << D)
    # value fields
    row_exp_orig = None
    if fmt == F.FMT_FP16:
        vbits = F.fp16_value_bits(v32)
    elif fmt == F.FMT_E8MY:
        vbits = F.e8my_value_bits(v32, D)
    else:
        absmax = np.zeros(n)
        if nnz:
            np.maximum.at(absmax, rows, np.abs(v32.astype(np.float64)))
        row_exp_orig = F.fix_row_exponent(absmax, D)
        vbits = F.fix_value_bits(v32, row_exp_orig[rows], D)
    # words in row-major order: a dummy (if any) then the value word
    n_dum = int(overflow.sum())
    words_per_entry = 1 + overflow.astype(np.int64)
    pos_end = np.cumsum(words_per_entry)  # exclusive end in row-major stream
    stream = np.empty(nnz + n_dum, dtype=np.uint32)
    val_pos = pos_end - 1
    stream[val_pos] = F.pack_value_word(vbits, np.where(overflow, 0, delta))
    dum_pos = val_pos[overflow] - 1
    stream[dum_pos] = F.pack_delta_word(delta[overflow])
    # E4
    cnt = np.diff(rowptr) + np.bincount(rows[overflow], minlength=n).astype(np.int64)
    stream_rowptr = np.zeros(n + 1, dtype=np.int64)
    stream_rowptr[1:] = np.cumsum(cnt)
    # E5: stable descending sort by cnt inside each sigma window
    win = np.arange(n, dtype=np.int64) // sigma
    stored_rows = np.lexsort((np.arange(n), -cnt, win)).astype(np.int64)
    perm_local = stored_rows - (stored_rows // sigma) * sigma
    perm_dtype = np.uint8 if sigma <= 256 else np.uint16
    # E6
    n_slices = (n + C - 1) // C
    cnt_stored = np.zeros(n_slices * C, dtype=np.int64)
    cnt_stored[:n] = cnt[stored_rows]
    widths = cnt_stored.reshape(n_slices, C).max(axis=1) if n_slices else np.zeros(0, np.int64)
    offset = np.zeros(n_slices + 1, dtype=np.int64)
    offset[1:] = np.cumsum(C * widths)
    n_words = int(offset[-1])
    # E7: scatter every row's words to its slice lane; the rest stays padding
    pack = np.zeros(n_words, dtype=np.uint32)
    stored_index = np.empty(n, dtype=np.int64)
    stored_index[stored_rows] = np.arange(n)
    w_row = np.repeat(np.arange(n, dtype=np.int64), cnt)  # original row per word
    j_in_row = np.arange(nnz + n_dum, dtype=np.int64) - stream_rowptr[w_row]
    si = stored_index[w_row]
    dest = offset[si // C] + j_in_row * C + (si % C)
    pack[dest] = stream
    row_exp = None
    if row_exp_orig is not None:
        row_exp = row_exp_orig[stored_rows]
    return Encoded(n=n, m=m, nnz=nnz, fmt=fmt, D=D, C=C, sigma=sigma,
                   perm_mode=perm_mode, k_left=kl, n_slices=n_slices,
                   n_words=n_words, n_dummies=n_dum, pack=pack, offset=offset,
                   perm=perm_local.astype(perm_dtype), stored_rows=stored_rows,
                   cnt=cnt, row_exp=row_exp)


def row_words(offset, n: int, C: int):
    """Word positions of every stored row, row after row (sec. 3): stored
    row i is lane l = i mod C of slice k = floor(i/C), and its word j < w_k
    sits at offset_k + j*C + l.  Returns (row, position, row start) with
    row start[i] the index of row i's first word in that listing."""
    i = np.arange(n, dtype=np.int64)
    k, l = i // C, i % C
    w = (offset[k + 1] - offset[k]) // C
    start = np.zeros(n + 1, dtype=np.int64)
    start[1:] = np.cumsum(w)
    row = np.repeat(i, w)
    j = np.arange(int(start[-1]), dtype=np.int64) - start[row]
    return row, offset[k[row]] + j * C + l[row], start


def row_columns(delta, row, start, left):
    """Column at every word: the row's left offset (eq. 4) plus the running
    sum of its deltas up to and including the word (sec. 4.4)."""
    run = np.cumsum(np.asarray(delta, dtype=np.int64))
    before = np.concatenate([[0], run])[start[:-1]]  # deltas of the rows before
    return left[row] + run - before[row]


def decode_rows(E: Encoded):
    """Every stored row's words, decoded (sec. 4.2.1, sec. 4.4).

    Stored row i sits in slice k = floor(i/C) at lane l = i mod C; its word
    j < w_k is pack[offset_k + j*C + l] (sec. 3).  Its columns are the left
    offset of eq. 4 plus the running sum of the row's deltas; a flag-1 word
    is an entry (decoded value, times 2^e_row for FIX), a flag-0 word only
    moves the column.  Returns, per word in row-major order (stored row,
    then j): stored row, word position, flag, column, value.
    """
    n = E.n
    row, pos, start = row_words(E.offset, n, E.C)
    flag, delta, vbits = F.unpack_word(E.pack[pos], E.D)
    col = row_columns(delta, row, start, left_offsets(n, E.sigma, E.k_left))
    val = np.where(flag == 1, F.value_from_bits(vbits, E.fmt, E.D), 0.0)
    if E.fmt == F.FMT_FIX:
        val = np.ldexp(val, E.row_exp[row])
    return row, pos, flag, col, val


def spmv_algorithm(E: Encoded, x: np.ndarray, return_trace: bool = False):
    """y = A_q x through the format (sec. 4.4): decode each stored row, then
    take its dot product with x over its flag-1 words, in float64.  The
    result goes to row floor(i/sigma)*sigma + perm_i (implicit mode) or to
    stored row i (explicit mode).  Flag-0 words read no x (a padding word's
    column may lie past m).

    With ``return_trace`` also returns the column and the value decoded at
    every word position (int64[n_words], float64[n_words]; phantom rows past
    n stay 0).
    """
    n = E.n
    x = np.asarray(x, dtype=np.float64)
    row, pos, flag, col, val = decode_rows(E)
    has = flag == 1
    prod = np.zeros(row.size)
    prod[has] = val[has] * x[col[has]]
    t = np.bincount(row, weights=prod, minlength=n)[:n] if n else np.zeros(0)
    y = np.zeros(n, dtype=np.float64)
    if E.perm_mode == PERM_IMPLICIT:
        i = np.arange(n, dtype=np.int64)
        y[(i // E.sigma) * E.sigma + E.perm.astype(np.int64)] = t
    else:
        y[:] = t
    if return_trace:
        cols = np.zeros(E.n_words, dtype=np.int64)
        vals = np.zeros(E.n_words, dtype=np.float64)
        cols[pos] = col
        if E.fmt == F.FMT_FIX:  # the trace holds the field value, unscaled
            vals[pos] = np.ldexp(val, -E.row_exp[row])
        else:
            vals[pos] = val
        return y, cols, vals
    return y


def decode_csr(E: Encoded):
    """Decoder: (rowptr, col, value) of A_q in the original row order from
    the encoded arrays only (the flag-1 words of each row, in word order)."""
    n = E.n
    row, _, flag, col, val = decode_rows(E)
    has = flag == 1
    i = np.arange(n, dtype=np.int64)
    orig = ((i // E.sigma) * E.sigma + E.perm.astype(np.int64))[row[has]]
    order = np.argsort(orig, kind="stable")  # keeps word order inside a row
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, orig + 1, 1)
    return np.cumsum(rowptr), col[has][order], val[has][order]


def quantized_values(rowptr, col, val, n: int, fmt: int, D: int) -> np.ndarray:
    """Values of A_q (float64) in CSR order: what a flag-1 word decodes to,
    times the row scale for FIX.  Computed from the quantisers directly,
    without building the format."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    v32 = np.asarray(val, dtype=np.float64).astype(np.float32)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    if fmt == F.FMT_FP16:
        return F.value_from_bits(F.fp16_value_bits(v32), fmt, D)
    if fmt == F.FMT_E8MY:
        return F.value_from_bits(F.e8my_value_bits(v32, D), fmt, D)
    absmax = np.zeros(n)
    if v32.size:
        np.maximum.at(absmax, rows, np.abs(v32.astype(np.float64)))
    e = F.fix_row_exponent(absmax, D)
    q = F.value_from_bits(F.fix_value_bits(v32, e[rows], D), fmt, D)
    return np.ldexp(q, e[rows])
