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


def spmv_algorithm(E: Encoded, x: np.ndarray, return_trace: bool = False):
    """The PackSELL SpMV of sec. 4.4, executed as written in float64.

    For every stored row i: c = dfrak_i (eq. 4); i' = floor(i/sigma)*sigma +
    perm_i; k = floor(i/C); l = i mod C; s = offset_k;
    w = (offset_{k+1} - s)/C; t = 0; for j < w: unpack pack[s + j*C + l] to
    (v, d); c += d; t += v * x_c.  Then y_{i'} = t (implicit mode) or
    y_i = t (explicit mode).  All rows advance together, one j at a time.

    Readings: flag-0 words carry value 0 and their product is skipped, so a
    padding word never reads x (its column can lie past m for empty rows);
    FIX rows multiply t by 2^e_row at the end.

    With ``return_trace`` also returns the column reconstructed at every word
    position (int64[n_words]) and every decoded value (float64[n_words]).
    """
    n, C, sigma = E.n, E.C, E.sigma
    x = np.asarray(x, dtype=np.float64)
    i = np.arange(n, dtype=np.int64)
    c = left_offsets(n, sigma, E.k_left)  # block-uniform, same for i and i'
    k = i // C
    l = i % C
    s = E.offset[k]
    w = (E.offset[k + 1] - s) // C
    t = np.zeros(n, dtype=np.float64)
    cols = np.zeros(E.n_words, dtype=np.int64) if return_trace else None
    vals = np.zeros(E.n_words, dtype=np.float64) if return_trace else None
    active = np.nonzero(w > 0)[0]
    j = 0
    while active.size:
        p_idx = s[active] + j * C + l[active]
        flag, d, vb = F.unpack_word(E.pack[p_idx], E.D)
        v = F.value_from_bits(vb, E.fmt, E.D)
        c[active] += d.astype(np.int64)
        has = flag == 1
        prod = np.zeros(active.size)
        prod[has] = v[has] * x[c[active][has]]
        t[active] += prod
        if return_trace:
            cols[p_idx] = c[active]
            vals[p_idx] = v
        j += 1
        active = active[w[active] > j]
    if E.fmt == F.FMT_FIX:
        t = np.ldexp(t, E.row_exp)
    y = np.zeros(n, dtype=np.float64)
    if E.perm_mode == PERM_IMPLICIT:
        y[(i // sigma) * sigma + E.perm.astype(np.int64)] = t
    else:
        y[:] = t
    if return_trace:
        # padding words of slices' phantom rows (>= n) decode as delta 0
        return y, cols, vals
    return y


def decode_csr(E: Encoded):
    """Decoder: recover (rowptr, col, value) of A_q in the original row order
    from the encoded arrays only, by replaying the word stream of every
    stored row (flag-1 words are entries, flag-0 words only move c)."""
    n, C, sigma = E.n, E.C, E.sigma
    i = np.arange(n, dtype=np.int64)
    orig = (i // sigma) * sigma + E.perm.astype(np.int64)
    c = left_offsets(n, sigma, E.k_left)
    k = i // C
    l = i % C
    s = E.offset[k]
    w = (E.offset[k + 1] - s) // C
    ent_r, ent_j, ent_c, ent_v = [], [], [], []
    active = np.nonzero(w > 0)[0]
    j = 0
    while active.size:
        flag, d, vb = F.unpack_word(E.pack[s[active] + j * C + l[active]], E.D)
        c[active] += d.astype(np.int64)
        has = flag == 1
        ent_r.append(orig[active][has])
        ent_j.append(np.full(int(has.sum()), j))
        ent_c.append(c[active][has])
        v = F.value_from_bits(vb[has], E.fmt, E.D)
        if E.fmt == F.FMT_FIX:
            v = np.ldexp(v, E.row_exp[active][has])
        ent_v.append(v)
        j += 1
        active = active[w[active] > j]
    if ent_r:
        r = np.concatenate(ent_r)
        jj = np.concatenate(ent_j)
        cc = np.concatenate(ent_c)
        vv = np.concatenate(ent_v)
    else:
        r = jj = cc = np.zeros(0, np.int64)
        vv = np.zeros(0)
    order = np.lexsort((jj, r))
    r, cc, vv = r[order], cc[order], vv[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    return np.cumsum(rowptr), cc, vv


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
