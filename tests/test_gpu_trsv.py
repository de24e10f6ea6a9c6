"""GPU parity for the level-scheduled triangular solves (lower and upper) on
CSR-packed words (and their plain-CSR comparator).

The level schedule (row order and level pointer) must equal the oracle's
bit for bit.  Forward substitution in float32 is componentwise backward
stable: the computed y solves (L_q + dL) y = b with |dL| <= g_k |L_q|,
g_k = k u / (1 - k u), u = 2^-24 and k the longest row.  The tests check
exactly that bound, max_i |L_q y - b|_i / (|L_q| |y|)_i <= g_k, in float64
against the quantised matrix, and the distance to the oracle's float64
solution and to scipy's float64 triangular solve of the same L_q as sanity
bounds, at every size.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla
import torch

from helpers import FMTS
from oracle import packcsr as PC
from oracle import trsv as TR
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W
from test_oracle_trsv import random_lower, transpose_of, tril_of

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
U = 2.0 ** -24


def backward_error(a, q, y, b):
    Lq = sp.csr_matrix((q, a.col, a.rowptr), shape=(a.n, a.n))
    r = np.abs(Lq @ y - b)
    den = abs(Lq) @ np.abs(y)
    return float(np.max(r / np.maximum(den, 1e-300)))


def bound(a):
    k = int(np.max(np.diff(a.rowptr)))
    return k * U / (1 - k * U)


def check_solve(a, fmt, D, seed=0, check_oracle=True, upper=False):
    S = B.TriangularSolve(a.rowptr, a.col, a.val, a.n, fmt, D, DEV, upper=upper)
    order, ptr = TR.level_schedule(TR.levels(a.rowptr, a.col, a.n, upper))
    assert S.n_levels == ptr.size - 1
    assert np.array_equal(S.level_ptr[: ptr.size], ptr)
    assert np.array_equal(S.order.cpu().numpy()[: a.n].astype(np.int64), order)
    b = np.random.default_rng(seed).uniform(-1, 1, a.n).astype(np.float32)
    y = S(torch.from_numpy(b).to(DEV)).cpu().numpy().astype(np.float64)
    if fmt is None:
        q = a.val.astype(np.float32).astype(np.float64)
    else:
        q = TR.quantised_lower(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
    assert backward_error(a, q, y, b.astype(np.float64)) <= bound(a)
    Lq = sp.csr_matrix((q, a.col, a.rowptr), shape=(a.n, a.n))
    if a.n:
        ref = sla.spsolve_triangular(Lq, b.astype(np.float64), lower=not upper)
        assert np.max(np.abs(y - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    if check_oracle and fmt is not None:
        E = PC.encode(a.rowptr, a.col, a.val, a.n, a.n, FMTS[fmt], D)
        ref = TR.solve(E, b.astype(np.float64), upper)
        assert np.max(np.abs(y - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    return S, y


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9), ("e8my", 4), ("fix", 18), (None, 0)])
def test_random_lower(fmt, D):
    for seed, (n, per_row) in enumerate([(300, 6), (5000, 12)]):
        check_solve(random_lower(10 + seed, n, per_row), fmt, D, seed)


def test_grid_laplacian_64_levels_and_solve():
    a = tril_of(W.stencil((64, 64, 64), "star", 3, 0.5, "lap64"))
    S, _ = check_solve(a, "e8my", 12)
    assert S.n_levels == 3 * 63 + 1


def test_laplace3d_128_full_size():
    """The lower triangle of the 7-point 128^3 variable-coefficient Laplacian
    (lognormal(0, 0.5) edge coefficients, rounded to FP16): 382 levels,
    level l holding the points with i+j+k = l.  Checked against the oracle's
    float64 solve and scipy's on the same quantised L."""
    a = tril_of(W.m2_laplace3d(128))
    S, y = check_solve(a, "fp16", 15)
    assert S.n_levels == 382
    g = np.arange(128)
    s = (g[:, None, None] + g[None, :, None] + g[None, None, :]).ravel()
    assert np.array_equal(np.diff(S.level_ptr[:383]), np.bincount(s))


def test_edges():
    d = W.csr_from_triplets(50, 50, np.arange(50), np.arange(50), np.linspace(1, 3, 50))
    S = B.TriangularSolve(d.rowptr, d.col, d.val, 50, "e8my", 12, DEV)
    assert S.n_levels == 1
    b = torch.ones(50, device=DEV)
    qd = TR.quantised_lower(d.rowptr, d.col, d.val, 50, FMTS["e8my"], 12).astype(np.float32)
    assert np.array_equal(S(b).cpu().numpy(), (np.float32(1.0) / qd).astype(np.float32))
    e = W.csr_from_triplets(0, 0, [], [], [])
    S = B.TriangularSolve(e.rowptr, e.col, e.val, 0, "fp16", 15, DEV)
    assert S.n_levels == 0 and S(torch.zeros(0, device=DEV)).numel() == 0
    bad = W.csr_from_triplets(3, 3, [0, 1, 2], [0, 0, 2], [1.0, 1.0, 1.0])  # row 1: no diagonal
    with pytest.raises(B.PackSELLError):
        B.TriangularSolve(bad.rowptr, bad.col, bad.val, 3, "fp16", 15, DEV)
    up = W.csr_from_triplets(2, 2, [0, 0, 1], [0, 1, 1], [1.0, 1.0, 1.0])  # upper entry
    with pytest.raises(B.PackSELLError):
        B.TriangularSolve(up.rowptr, up.col, up.val, 2, "fp16", 15, DEV)


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 5), ("fix", 18), (None, 0)])
def test_random_upper(fmt, D):
    for seed, (n, per_row) in enumerate([(300, 6), (5000, 12)]):
        check_solve(transpose_of(random_lower(30 + seed, n, per_row)), fmt, D, seed, upper=True)


def test_grid_laplacian_64_upper():
    """Upper triangle of a 64^3 stencil: 190 levels, the grid walked from the
    far corner."""
    import scipy.sparse as sp

    a = W.stencil((64, 64, 64), "star", 3, 0.5, "lap64")
    M = sp.triu(sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m))).tocsr()
    M.sort_indices()
    u = W.csr_from_triplets(a.n, a.n, np.repeat(np.arange(a.n), np.diff(M.indptr)), M.indices,
                            M.data)
    S, _ = check_solve(u, "e8my", 12, upper=True)
    assert S.n_levels == 3 * 63 + 1
    with pytest.raises(B.PackSELLError):  # the diagonal is first, not last
        B.TriangularSolve(u.rowptr, u.col, u.val, u.n, "e8my", 12, DEV, upper=False)
