"""Sparse triangular solves on CSR-packed words, with level scheduling
(oracle; test infrastructure only, never called by the product path).

The paper names sparse triangular solves as another kernel that its
packing suits (sec. 6), since their implementations resemble SpMV.
Reading: L is lower triangular with every row holding its diagonal as its
last (largest-column) entry, or upper triangular (``upper``) with the
diagonal as every row's first entry; it is packed as CSR-based
delta-value words (oracle.packcsr), so the solve uses the quantised L_q:

  y_i = (b_i - sum_{j < i} (L_q)_ij y_j) / (L_q)_ii,   i = 0 .. n-1,

or, upper, the same sum over j > i with i running from n-1 down to 0.

A level schedule groups rows that can be solved together: level(i) = 0
for a row with no off-diagonal entries, else 1 + max level(j) over its
off-diagonal columns j.  Rows of one level depend only on rows of lower
levels.
"""
from __future__ import annotations

import numpy as np

from . import packcsr as PC
from . import packsell as P


def check_triangle(rowptr, col, n: int, upper: bool = False) -> None:
    """Every row non-empty; its diagonal the last entry (lower) or the
    first (upper)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    if np.any(np.diff(rowptr) <= 0):
        raise ValueError("every row needs its diagonal")
    diag = col[rowptr[:-1]] if upper else col[rowptr[1:] - 1]
    if np.any(diag != np.arange(n)):
        raise ValueError("each row's diagonal must be its first (upper) or last (lower) entry")


def off_diagonal(rowptr, col, i: int, upper: bool) -> np.ndarray:
    s, e = rowptr[i], rowptr[i + 1]
    return col[s + 1:e] if upper else col[s:e - 1]


def levels(rowptr, col, n: int, upper: bool = False) -> np.ndarray:
    """Level of every row, in dependency order (rows ascending for lower,
    descending for upper): the definition."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    check_triangle(rowptr, col, n, upper)
    lev = np.zeros(n, dtype=np.int64)
    for i in (range(n - 1, -1, -1) if upper else range(n)):
        deps = off_diagonal(rowptr, col, i, upper)
        lev[i] = 1 + int(lev[deps].max()) if deps.size else 0
    return lev


def level_schedule(lev: np.ndarray):
    """Rows sorted by level (ascending row order inside a level) and the
    level pointer: level l holds order[ptr[l]:ptr[l+1]]."""
    order = np.argsort(lev, kind="stable").astype(np.int64)
    counts = np.bincount(lev, minlength=int(lev.max()) + 1 if lev.size else 0)
    ptr = np.zeros(counts.size + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    return order, ptr


def quantised_lower(rowptr, col, val, n: int, fmt: int, D: int) -> np.ndarray:
    """Values of L_q in CSR order (what the packed words decode to)."""
    return P.quantized_values(rowptr, col, val, n, fmt, D)


def solve(E: PC.PackedCSR, b: np.ndarray, upper: bool = False) -> np.ndarray:
    """Substitution in float64 on the packed words, row by row (forward for
    lower, backward for upper): walk the row's words (columns as running
    sums of deltas from the left offset); every flag-1 word but the
    diagonal subtracts value * y[column]; the diagonal is the last word
    (lower) or the first flag-1 word (upper)."""
    from . import formats as F
    b = np.asarray(b, dtype=np.float64)
    flag, _, vb = F.unpack_word(E.pack, E.D)
    v = F.value_from_bits(vb, E.fmt, E.D)
    if E.fmt == F.FMT_FIX:
        v = np.ldexp(v, np.repeat(E.row_exp, np.diff(E.wrowptr)))
    cols = PC.columns_after(E)
    y = np.zeros(E.n)
    for i in (range(E.n - 1, -1, -1) if upper else range(E.n)):
        s, e = int(E.wrowptr[i]), int(E.wrowptr[i + 1])
        live = np.nonzero(flag[s:e] == 1)[0] + s
        dpos = live[0] if upper else e - 1
        if dpos != live[0 if upper else -1] or cols[dpos] != i:
            raise ValueError("the diagonal must be the row's first (upper) or last (lower) entry")
        off = live[live != dpos]
        acc = float(np.dot(v[off], y[cols[off]]))
        y[i] = (b[i] - acc) / v[dpos]
    return y
