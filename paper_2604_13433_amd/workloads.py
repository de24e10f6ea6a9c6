"""Seeded synthetic matrices and vectors (input recipes only).

This module generates the inputs that the GPU library, its tests, the
benchmark and the CPU oracle all consume.  It holds no PackSELL arithmetic:
no quantisation, delta encoding, packing or SpMV.  Everything is plain numpy
driven by ``numpy.random.default_rng(seed)`` so a (recipe, seed) pair always
produces the same bytes.

The paper measures on SuiteSparse matrices (sec. 5.1) and on HPCG-style
stencils (Table 2); neither collection is available here, so these recipes
stand in for them with the same structural traits:

* ``poisson2d``      -- 2D 5-point Poisson, diagonal 4, off-diagonals -1.
* ``stencil``        -- variable-coefficient 5/7/27-point stencils with one
  lognormal coefficient per undirected grid edge (ghost edges outside the
  domain included in the diagonal, so every interior row sums to zero and
  boundary rows are strictly diagonally dominant).  The 27-point variant is
  the variable-coefficient analogue of the HPCG matrices of Table 2.
* ``powerlaw``       -- irregular rows whose lengths follow a truncated power
  law, 90% of each row inside a +/-512 band and 10% uniform far columns
  (the high-RSD regime of sec. 5.1.1), values N(0,1) then row-sum scaled.
* ``batch``          -- many stencils of uneven size.
* ``convdiff3d``     -- a nonsymmetric convection-diffusion stencil, for the
  nested solver of sec. 5.2.1 (whose test set mixes SPD and nonsymmetric
  matrices).

Diagonal scalings used by the paper as workload preparation
(row-sum scaling G^-1 A of sec. 5.1.2, symmetric scaling of sec. 5.2) are
also here, since they define the inputs rather than the method.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np


@dataclasses.dataclass
class CSR:
    """Compressed sparse row matrix with strictly increasing columns per row."""

    n: int
    m: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz] (callers round to float32 where needed)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64[nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), self.row_lengths())

    def with_values(self, val: np.ndarray) -> "CSR":
        return CSR(self.n, self.m, self.rowptr, self.col, val, self.name)

    def dense(self) -> np.ndarray:
        """Dense float64 copy (tiny matrices only)."""
        a = np.zeros((self.n, self.m), dtype=np.float64)
        a[self.rows(), self.col.astype(np.int64)] = self.val
        return a


def csr_from_dense(a: np.ndarray, name: str = "") -> CSR:
    """CSR of the nonzero pattern of a dense array (tests only)."""
    a = np.asarray(a, dtype=np.float64)
    n, m = a.shape
    r, c = np.nonzero(a)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(n, m, rowptr, c.astype(np.int32), a[r, c].copy(), name)


def csr_from_triplets(n: int, m: int, rows, cols, vals, name: str = "") -> CSR:
    """CSR from (row, col, val) triplets with no duplicate (row, col) pairs."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        same = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if same.any():
            raise ValueError("duplicate (row, col) pair")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(n, m, rowptr, cols.astype(np.int32), vals, name)


# ---------------------------------------------------------------------------
# Structured stencils
# ---------------------------------------------------------------------------

def _stencil_offsets(ndim: int, kind: str):
    """Neighbour offsets (tuples of -1/0/1 per axis, axis 0 fastest)."""
    if kind == "star":
        offs = []
        for ax in range(ndim):
            for s in (-1, 1):
                o = [0] * ndim
                o[ax] = s
                offs.append(tuple(o))
        return offs
    if kind == "box":
        return [o for o in itertools.product((-1, 0, 1), repeat=ndim) if any(o)]
    raise ValueError(kind)


def _positive_half(offs):
    """One representative of each +/- pair: last nonzero component positive."""
    half = []
    for o in offs:
        nz = [v for v in o if v != 0]
        if nz[-1] > 0:
            half.append(o)
    return half


def stencil(dims, kind: str, seed: int | None, ln_sigma: float = 0.5,
            name: str = "") -> CSR:
    """Variable-coefficient stencil matrix on a Cartesian grid.

    ``dims`` are the grid extents with axis 0 varying fastest in the row
    numbering.  ``kind`` is "star" (5-point in 2D, 7-point in 3D) or "box"
    (9/27-point).  Every undirected edge between a grid point and a neighbour
    (including edges that leave the domain) draws kappa ~ lognormal(0,
    ln_sigma); a_ij = a_ji = -kappa for in-domain neighbours and a_ii is the
    sum of kappa over all of the point's edges.  With ``seed=None`` every
    kappa is 1 (constant coefficients).

    Draw order: for each positive-half offset, in the order produced by
    ``_positive_half``, one array of kappa over the grid extended by one
    point on each side, in C order of the reversed dims.
    """
    dims = tuple(int(d) for d in dims)
    ndim = len(dims)
    n = int(np.prod(dims))
    offs = _stencil_offsets(ndim, kind)
    half = _positive_half(offs)
    rng = np.random.default_rng(seed) if seed is not None else None
    ext = tuple(d + 2 for d in dims)
    # kappa[o][q + 1] is the coefficient of the edge (q, q + o).
    kappa = {}
    for o in half:
        if rng is None:
            kappa[o] = np.ones(ext[::-1], dtype=np.float64)
        else:
            kappa[o] = rng.lognormal(0.0, ln_sigma, size=ext[::-1])
    # grid coordinates of every row, arrays indexed [z, y, x] (axis 0 last)
    grids = np.meshgrid(*[np.arange(d) for d in dims[::-1]], indexing="ij")
    coords = [g.reshape(-1) for g in grids[::-1]]  # coords[ax][row]
    strides = [int(np.prod(dims[:ax])) for ax in range(ndim)]

    def edge_kappa(lower_coords, o):
        idx = tuple((lower_coords[ax] + 1) for ax in range(ndim))[::-1]
        return kappa[o][idx]

    diag = np.zeros(n, dtype=np.float64)
    entries = {}  # linear offset -> (value array, valid mask)
    for o in offs:
        if o in kappa:
            lower = coords
            k = edge_kappa(lower, o)
        else:
            neg = tuple(-v for v in o)
            lower = [coords[ax] + o[ax] for ax in range(ndim)]
            k = edge_kappa(lower, neg)
        diag += k
        valid = np.ones(n, dtype=bool)
        for ax in range(ndim):
            nb = coords[ax] + o[ax]
            valid &= (nb >= 0) & (nb < dims[ax])
        lin = sum(o[ax] * strides[ax] for ax in range(ndim))
        entries[lin] = (-k, valid)
    entries[0] = (diag, np.ones(n, dtype=bool))
    lins = sorted(entries)
    vals = np.stack([entries[l][0] for l in lins], axis=1)
    mask = np.stack([entries[l][1] for l in lins], axis=1)
    cols = np.arange(n, dtype=np.int64)[:, None] + np.asarray(lins, dtype=np.int64)[None, :]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(counts)
    return CSR(n, n, rowptr, cols[mask].astype(np.int32), vals[mask], name)


def convdiff3d(g: int, seed: int, wind=(1.0, 0.5, 0.25), ln_sigma: float = 0.5,
               name: str = "") -> CSR:
    """Nonsymmetric 3D convection-diffusion on a g^3 grid: the 7-point
    variable-coefficient diffusion of ``stencil`` (lognormal(0, ln_sigma)
    edge coefficients, seed ``seed``) plus first-order upwind convection
    with the constant velocity ``wind`` (one component per axis, >= 0, in
    units of the mean edge coefficient): each point adds wind[ax] to its
    diagonal and -wind[ax] to its lower neighbour along axis ax (dropped at
    the boundary).  A diagonally dominant M-matrix with a nonsymmetric
    pattern of values, a stand-in for the nonsymmetric problems the paper
    solves with F3R (sec. 5.2.1)."""
    a = stencil((g, g, g), "star", seed, ln_sigma)
    rows = a.rows()
    colv = a.col.astype(np.int64)
    val = a.val.copy()
    diag = rows == colv
    val[diag] += float(sum(wind))
    for ax, v in enumerate(wind):
        lower = rows - colv == g ** ax
        val[lower] -= v
    return CSR(a.n, a.m, a.rowptr, a.col, val, name or f"convdiff7_{g}")


def block_stencil(dims, dof: int, seed: int, name: str = "") -> CSR:
    """Vector (``dof`` unknowns per grid point) 27-point stencil: every
    unknown couples to all ``dof`` unknowns of each of its 27 neighbours
    (itself included), so a row holds up to 27 * dof entries in runs of
    3 * dof consecutive columns (unknowns numbered point-major).  Values are
    N(0, 1) with a dominant positive diagonal, then row-sum scaled.  A
    high-locality pattern of the kind the paper credits for small-D gains
    (sec. 5.1.2); an extra workload, not one of the five benchmark configs."""
    g = stencil(dims, "box", seed=None)
    rng = np.random.default_rng(seed)
    rows_p = g.rows()
    cols_p = g.col.astype(np.int64)
    # every point entry (p, q) becomes the dof x dof block (p*dof+a, q*dof+b)
    blk_a = np.arange(dof)[None, :, None]
    blk_b = np.arange(dof)[None, None, :]
    rr = np.broadcast_to(rows_p[:, None, None] * dof + blk_a, (rows_p.size, dof, dof)).reshape(-1)
    cc = np.broadcast_to(cols_p[:, None, None] * dof + blk_b, (rows_p.size, dof, dof)).reshape(-1)
    vals = rng.standard_normal(rr.size)
    diag = rr == cc
    vals[diag] = np.abs(vals[diag]) + 27 * dof
    n = g.n * dof
    a = csr_from_triplets(n, n, rr, cc, vals, name or f"block{dof}_27pt")
    return row_sum_scale(a)


def poisson2d(g: int) -> CSR:
    """2D 5-point Poisson on a g x g grid: diagonal 4, off-diagonals -1."""
    a = stencil((g, g), "star", seed=None, name=f"poisson2d_{g}")
    return a


def stencil_nnz(dims, kind: str) -> int:
    """Closed-form stored-entry count of ``stencil(dims, kind)``.

    box: prod(3 d - 2) (each axis contributes 3 d - 2 in-range (point,
    neighbour) pairs).  star: n + 2 * sum over axes of (d_ax - 1) * n / d_ax.
    """
    dims = [int(d) for d in dims]
    if kind == "box":
        return int(np.prod([3 * d - 2 for d in dims]))
    n = int(np.prod(dims))
    return n + sum(2 * (d - 1) * (n // d) for d in dims)


# ---------------------------------------------------------------------------
# Irregular power-law rows
# ---------------------------------------------------------------------------

def _sample_distinct(lo, size, k, rng):
    """For each row r draw k[r] distinct integers from [lo[r], lo[r]+size[r]).

    Uniform over k-subsets.  Rows that need more than half of their range
    (or whose range is small) give every candidate a random key and keep the
    k smallest.  The other rows oversample with replacement, drop repeats,
    assign random keys and keep the k smallest keys; rows that came up short
    are redrawn (each redraw succeeds with high probability because
    2k + 8 draws from at least 2k candidates leave >= k distinct ones).
    Returns (row_index, value) int64 arrays.
    """
    lo = np.asarray(lo, np.int64)
    size = np.asarray(size, np.int64)
    k = np.asarray(k, np.int64)
    assert np.all(k <= size)
    out_r, out_v = [], []
    dense = (k > 0) & ((2 * k > size) | (size <= 64))
    drows = np.nonzero(dense)[0]
    # dense rows, in chunks to bound memory
    chunk = max(1, 4_000_000 // max(1, int(size[drows].max()) if drows.size else 1))
    for s0 in range(0, drows.size, chunk):
        rows = drows[s0:s0 + chunk]
        sz = size[rows]
        rr = np.repeat(rows, sz)
        off = np.arange(rr.size) - np.repeat(np.cumsum(sz) - sz, sz)
        pri = rng.random(rr.size)
        order = np.argsort(rr + pri, kind="stable")  # by row, then priority
        rr, off = rr[order], off[order]
        start = np.cumsum(sz) - sz
        kk = k[rows]
        idx = np.repeat(start, kk) + (np.arange(kk.sum()) - np.repeat(np.cumsum(kk) - kk, kk))
        out_r.append(rr[idx])
        out_v.append(lo[rr[idx]] + off[idx])
    todo = np.nonzero((k > 0) & ~dense)[0]
    while todo.size:
        kk = k[todo]
        draw = np.minimum(size[todo], 2 * kk + 8)
        rr = np.repeat(todo, draw)
        vv = lo[rr] + (rng.random(rr.size) * size[rr]).astype(np.int64)
        key = rr * (int(size.max()) + 1) + (vv - lo[rr])
        key, first = np.unique(key, return_index=True)
        rr, vv = rr[first], vv[first]
        pri = rng.random(rr.size)
        order = np.argsort(rr + pri, kind="stable")  # by row, then priority
        rr, vv = rr[order], vv[order]
        starts = np.searchsorted(rr, todo)
        ends = np.searchsorted(rr, todo, side="right")
        have = ends - starts
        ok = have >= kk
        sel_rows = todo[ok]
        if sel_rows.size:
            s = starts[ok]
            n_take = kk[ok]
            idx = np.repeat(s, n_take) + (np.arange(n_take.sum()) -
                                          np.repeat(np.cumsum(n_take) - n_take, n_take))
            out_r.append(rr[idx])
            out_v.append(vv[idx])
        todo = todo[~ok]
    if not out_r:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(out_r), np.concatenate(out_v)


def powerlaw_lengths(n: int, alpha: float, l_min: float, l_max: int, rng) -> np.ndarray:
    """Row lengths floor(L), L with density proportional to L^-alpha on
    [l_min, l_max] (inverse-CDF sampling of the truncated Pareto law)."""
    a = alpha - 1.0
    u = rng.random(n)
    tail = (l_min / l_max) ** a
    x = l_min * (1.0 - u * (1.0 - tail)) ** (-1.0 / a)
    return np.clip(np.floor(x).astype(np.int64), 1, l_max)


def powerlaw(n: int, seed: int, alpha: float = 2.1, l_min: float = 5.614,
             l_max: int = 5000, band: int = 512, near_frac: float = 0.9,
             name: str = "") -> CSR:
    """Irregular n x n matrix with power-law row lengths.

    Row length L ~ floor(truncated power law) (alpha=2.1, l_min=5.614 gives
    mean ~30, median 10, max 5000).  round(near_frac * L) distinct columns
    (capped at the band size) come from [i - band, i + band] intersected with
    [0, n); the rest are distinct uniform columns outside that band.  Values
    are N(0, 1), then each row is divided by its absolute row sum (the
    G^-1 A scaling of sec. 5.1.2).
    """
    rng = np.random.default_rng(seed)
    L = powerlaw_lengths(n, alpha, l_min, l_max, rng)
    i = np.arange(n, dtype=np.int64)
    b_lo = np.maximum(i - band, 0)
    b_hi = np.minimum(i + band, n - 1)
    bsize = b_hi - b_lo + 1
    near = np.minimum(np.rint(near_frac * L).astype(np.int64), bsize)
    far = np.minimum(L - near, n - bsize)
    r1, c1 = _sample_distinct(b_lo, bsize, near, rng)
    # far columns: draw from [0, n - bsize) and skip over the band
    r2, u2 = _sample_distinct(np.zeros(n, np.int64), n - bsize, far, rng)
    c2 = np.where(u2 >= b_lo[r2], u2 + bsize[r2], u2)
    rows = np.concatenate([r1, r2])
    cols = np.concatenate([c1, c2])
    vals = rng.standard_normal(rows.size)
    a = csr_from_triplets(n, n, rows, cols, vals, name or f"powerlaw_{n}")
    return row_sum_scale(a)


# ---------------------------------------------------------------------------
# Workload preparation (sec. 5.1.2 and sec. 5.2 scalings)
# ---------------------------------------------------------------------------

def row_sum_scale(a: CSR) -> CSR:
    """G^-1 A with g_i = sum_j |a_ij| (rows with g_i = 0 left unchanged)."""
    g = np.zeros(a.n)
    np.add.at(g, a.rows(), np.abs(a.val))
    g[g == 0] = 1.0
    return a.with_values(a.val / g[a.rows()])


def symmetric_diag_scale(a: CSR) -> CSR:
    """Gbar^-1 A Gbar^-1 with gbar_i = sqrt(|a_ii|) (square matrices)."""
    rows = a.rows()
    colv = a.col.astype(np.int64)
    d = np.ones(a.n)
    on_diag = rows == colv
    d[rows[on_diag]] = np.sqrt(np.abs(a.val[on_diag]))
    d[d == 0] = 1.0
    return a.with_values(a.val / (d[rows] * d[colv]))


def ones_rhs(a: CSR) -> np.ndarray:
    """b = A * 1 (the row sums), so that x* = 1 solves A x = b."""
    b = np.zeros(a.n)
    np.add.at(b, a.rows(), a.val)
    return b


def to_f32(a: CSR) -> CSR:
    """Values rounded to float32 (round to nearest even) and back."""
    return a.with_values(a.val.astype(np.float32).astype(np.float64))


def uniform_vector(m: int, seed: int, k: int = 1, lo: float = -1.0,
                   hi: float = 1.0) -> np.ndarray:
    """float32 vector (k == 1) or row-major m x k block, U[lo, hi)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=(m, k) if k > 1 else m)
    return np.ascontiguousarray(x.astype(np.float32))


# ---------------------------------------------------------------------------
# The five benchmark workloads
# ---------------------------------------------------------------------------

def m1_poisson2d() -> CSR:
    """2D 5-point Poisson, 64 x 64 grid (n = 4096, nnz = 20,224)."""
    return poisson2d(64)


def m2_laplace3d(g: int = 128, seed: int = 2) -> CSR:
    """3D 7-point variable-coefficient Laplacian, g^3 grid, lognormal(0, 0.5)."""
    return stencil((g, g, g), "star", seed, 0.5, f"laplace7_{g}")


def m3_powerlaw(n: int = 1_000_000, seed: int = 4) -> CSR:
    return powerlaw(n, seed, name=f"powerlaw_{n}")


def m4_stencil27(g: int = 100, seed: int = 6) -> CSR:
    """SPD 27-point variable-coefficient stencil, g^3 grid, lognormal(0, 1)."""
    return stencil((g, g, g), "box", seed, 1.0, f"stencil27_{g}")


def m5_batch(count: int = 64, n_lo: int = 10_000, n_hi: int = 500_000,
             seed: int = 7) -> list[CSR]:
    """``count`` stencils, n log-uniform in [n_lo, n_hi], alternating a 2D
    5-point (g = round(sqrt n)) and a 3D 7-point (g = round(cbrt n)) grid,
    coefficients lognormal(0, 0.5), each with its own derived seed."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))
    mats = []
    for b, nb in enumerate(ns):
        if b % 2 == 0:
            g = max(2, int(round(math.sqrt(nb))))
            mats.append(stencil((g, g), "star", seed * 1000 + b, 0.5, f"b{b}_5pt_{g}"))
        else:
            g = max(2, int(round(nb ** (1.0 / 3.0))))
            mats.append(stencil((g, g, g), "star", seed * 1000 + b, 0.5, f"b{b}_7pt_{g}"))
    return mats
