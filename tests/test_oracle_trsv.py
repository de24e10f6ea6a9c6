"""Pins of the triangular-solve oracle (lower and upper): scipy's triangular solver on the
same quantised matrix, the residual of the solution, closed-form levels of
grid Laplacians (level = i + j (+ k) in natural order), a dense solve, and
the level property on random matrices."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from helpers import FMTS
from oracle import packcsr as PC
from oracle import trsv as TR
from paper_2604_13433_amd import workloads as W


def tril_of(a):
    """Lower triangle (with the diagonal) of a CSR matrix as a CSR."""
    M = sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m))
    L = sp.tril(M).tocsr()
    L.sort_indices()
    return W.csr_from_triplets(a.n, a.n, np.repeat(np.arange(a.n), np.diff(L.indptr)),
                               L.indices, L.data)


def random_lower(seed, n, per_row):
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = min(i, int(rng.integers(0, per_row + 1)))
        c = np.unique(np.concatenate([rng.integers(max(0, i - 50), i, size=k) if k else [],
                                      rng.integers(0, i, size=1) if i and rng.random() < 0.3 else []]))
        c = np.append(c.astype(np.int64), i)
        rows += [i] * c.size
        cols += list(c)
    vals = rng.standard_normal(len(rows))
    a = W.csr_from_triplets(n, n, rows, cols, vals)
    # a diagonal that dominates its row keeps the solve well conditioned
    last = a.rowptr[1:] - 1
    rs = np.add.reduceat(np.abs(a.val), a.rowptr[:-1])
    a.val[last] = np.where(np.arange(n) % 2, 1.0, -1.0) * (rs + 1.0)
    return a


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9), ("fix", 18)])
def test_solve_equals_scipy_on_the_quantised_matrix(fmt, D):
    a = random_lower(1, 400, 6)
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.n, FMTS[fmt], D)
    b = np.random.default_rng(2).uniform(-1, 1, a.n)
    y = TR.solve(E, b)
    q = TR.quantised_lower(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
    Lq = sp.csr_matrix((q, a.col, a.rowptr), shape=(a.n, a.n))
    ref = spl.spsolve_triangular(Lq, b, lower=True)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(Lq @ y - b)) <= 1e-12


def test_solve_equals_dense_solve_with_long_jumps():
    """Columns far to the left (dummies before the value word)."""
    n = 300
    rows, cols = [], []
    for i in range(n):
        c = sorted({0, i // 2, i}) if i else [0]
        rows += [i] * len(c)
        cols += c
    vals = np.where(np.array(rows) == np.array(cols), 4.0, -1.0)
    a = W.csr_from_triplets(n, n, rows, cols, vals)
    E = PC.encode(a.rowptr, a.col, a.val, n, n, FMTS["e8my"], 4)  # 2^4: many dummies
    assert E.n_dummies > 0
    b = np.arange(n, dtype=np.float64) / n
    dense = np.zeros((n, n))
    dense[a.rows(), a.col] = a.val
    assert np.max(np.abs(TR.solve(E, b) - np.linalg.solve(dense, b))) <= 1e-12


@pytest.mark.parametrize("dims", [(7, 9), (5, 6, 4)])
def test_levels_of_grid_laplacians(dims):
    """Natural order: a grid point depends on its lower neighbours along each
    axis, so its level is the sum of its coordinates."""
    a = tril_of(W.stencil(dims, "star", 1, 1.0, "lap"))
    lev = TR.levels(a.rowptr, a.col, a.n)
    idx = np.indices(dims[::-1]).reshape(len(dims), -1)  # slowest axis first
    assert np.array_equal(lev, idx.sum(axis=0))
    order, ptr = TR.level_schedule(lev)
    assert ptr.size == sum(dims) - len(dims) + 2
    assert np.array_equal(np.sort(order), np.arange(a.n))


def test_level_property_on_random_matrices():
    a = random_lower(3, 2000, 8)
    lev = TR.levels(a.rowptr, a.col, a.n)
    rows = a.rows()
    off = a.col != rows
    need = np.full(a.n, -1)
    np.maximum.at(need, rows[off], lev[a.col[off]])
    assert np.array_equal(lev, need + 1)
    order, ptr = TR.level_schedule(lev)
    for l in range(ptr.size - 1):
        rs = order[ptr[l]:ptr[l + 1]]
        assert np.all(lev[rs] == l) and np.all(np.diff(rs) > 0)


def test_rejects_a_row_without_its_diagonal():
    a = W.csr_from_triplets(3, 3, [0, 1, 2], [0, 0, 2], [1.0, 1.0, 1.0])
    with pytest.raises(ValueError):
        TR.levels(a.rowptr, a.col, 3)


def transpose_of(a):
    """The transpose as a CSR with sorted columns (upper when a is lower)."""
    M = sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m)).T.tocsr()
    M.sort_indices()
    return W.csr_from_triplets(a.m, a.n, np.repeat(np.arange(a.m), np.diff(M.indptr)),
                               M.indices, M.data)


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 6), ("fix", 18)])
def test_upper_solve_equals_scipy(fmt, D):
    u = transpose_of(random_lower(4, 400, 6))
    E = PC.encode(u.rowptr, u.col, u.val, u.n, u.n, FMTS[fmt], D)
    b = np.random.default_rng(3).uniform(-1, 1, u.n)
    y = TR.solve(E, b, upper=True)
    q = TR.quantised_lower(u.rowptr, u.col, u.val, u.n, FMTS[fmt], D)
    Uq = sp.csr_matrix((q, u.col, u.rowptr), shape=(u.n, u.n))
    ref = spl.spsolve_triangular(Uq, b, lower=False)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(Uq @ y - b)) <= 1e-12


def test_upper_levels_of_a_grid_laplacian():
    """Upper triangle in natural order: a point depends on its upper
    neighbours, so its level is the sum of its distances to the far
    corner."""
    dims = (6, 5, 4)
    a = W.stencil(dims, "star", 1, 1.0, "lap")
    M = sp.triu(sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m))).tocsr()
    M.sort_indices()
    u = W.csr_from_triplets(a.n, a.n, np.repeat(np.arange(a.n), np.diff(M.indptr)), M.indices,
                            M.data)
    lev = TR.levels(u.rowptr, u.col, u.n, upper=True)
    idx = np.indices(dims[::-1]).reshape(3, -1)
    far = np.array(dims[::-1])[:, None] - 1 - idx
    assert np.array_equal(lev, far.sum(axis=0))
    with pytest.raises(ValueError):
        TR.levels(u.rowptr, u.col, u.n, upper=False)  # the diagonal is not last
