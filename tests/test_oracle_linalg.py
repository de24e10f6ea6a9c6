"""Pins for the oracle's float64 products, solvers and the input generators.

Pinned against: scipy.sparse products and dense numpy products (independent
library routines the oracle does not call), the dot-product identity of the
transpose, the linearity of y = A x in the values (central differences),
the closed-form solution x* = 1 of A x = A 1, CG equivalence of flexible CG
with an identity inner solve, and the nnz counts printed in Table 2.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import formats as F
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import workloads as W


def _sp(a):
    return sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m))


def test_csr_spmv_vs_scipy():
    rng = np.random.default_rng(0)
    a = W.powerlaw(3000, seed=11)
    x = rng.uniform(-1, 1, a.m)
    assert np.allclose(L.spmv(a.rowptr, a.col, a.val, x), _sp(a) @ x, rtol=1e-14, atol=1e-15)


def test_spmv_t_dense_and_dot_identity():
    rng = np.random.default_rng(1)
    d = (rng.random((50, 70)) < 0.1) * rng.standard_normal((50, 70))
    a = W.csr_from_dense(d)
    g = rng.standard_normal(50)
    x = rng.standard_normal(70)
    yt = L.spmv_t(a.rowptr, a.col, a.val, g, 70)
    assert np.allclose(yt, d.T @ g, rtol=1e-14, atol=1e-14)
    lhs = L.spmv(a.rowptr, a.col, a.val, x) @ g
    assert abs(lhs - x @ yt) <= 1e-12 * (np.abs(d) @ np.abs(x)) @ np.abs(g)


def test_grad_values_central_difference():
    rng = np.random.default_rng(2)
    d = (rng.random((20, 30)) < 0.2) * rng.standard_normal((20, 30))
    a = W.csr_from_dense(d)
    g = rng.standard_normal(20)
    x = rng.standard_normal(30)
    gv = L.grad_values(a.rowptr, a.col, g, x)
    h = 2.0 ** -10
    for e in range(0, a.nnz, 7):
        vp, vm = a.val.copy(), a.val.copy()
        vp[e] += h
        vm[e] -= h
        fd = (g @ L.spmv(a.rowptr, a.col, vp, x) - g @ L.spmv(a.rowptr, a.col, vm, x)) / (2 * h)
        assert abs(fd - gv[e]) <= 1e-10


def test_backward_error_zero_for_exact():
    a = W.m1_poisson2d()
    x = W.uniform_vector(a.m, 3).astype(np.float64)
    y = L.spmv(a.rowptr, a.col, a.val, x)
    assert L.backward_error(a.rowptr, a.col, a.val, x, y) == 0.0
    assert L.inf_norm(a.rowptr, a.val) == 8.0


def _small_spd(g=8, seed=6):
    a = W.symmetric_diag_scale(W.stencil((g, g, g), "box", seed, 1.0))
    return a, W.ones_rhs(a)


def test_cg_solves_ones():
    a, b = _small_spd()
    r = L.cg(a.rowptr, a.col, a.val, b, tol=1e-10)
    assert r.converged and r.rel_residual < 1e-10
    assert np.max(np.abs(r.x - 1)) < 1e-8
    ref = np.linalg.solve(a.dense(), b)
    assert np.allclose(r.x, ref, atol=1e-8)


def test_fcg_with_identity_inner_is_cg():
    a, b = _small_spd(6, 9)
    for k in (1, 3, 10):
        cg = L.cg(a.rowptr, a.col, a.val, b, tol=0.0, max_iter=k)
        fc = L.iocg(a.rowptr, a.col, a.val, a.val, b, m_in=0, tol=0.0,
                    max_outer=k, inner=lambda r: r.copy())
        assert cg.iterations == fc.iterations == k
        assert np.allclose(cg.x, fc.x, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("D", [9, 12])
def test_iocg_converges_with_quantised_inner(D):
    a, b = _small_spd(10, 4)
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, F.FMT_E8MY, D)
    r = L.iocg(a.rowptr, a.col, a.val, q, b, m_in=20, tol=1e-10)
    assert r.converged and r.rel_residual < 1e-10
    assert np.max(np.abs(r.x - 1)) < 1e-8


def test_inner_cg_many_steps_solves():
    a, b = _small_spd(5, 2)
    z = L.inner_cg(a.rowptr, a.col, a.val, b, m_in=400)
    assert np.allclose(z, 1.0, atol=1e-8)


# ---------------------------------------------------------------------------
# Generators (inputs shared by both sides)
# ---------------------------------------------------------------------------

def test_table2_hpcg_nnz_closed_form():
    # HPCG_x_y_z has n = 2^(x+y+z) rows of a 27-point stencil (Table 2)
    table2 = {(7, 7, 7): 55742968, (8, 7, 7): 111777784,
              (8, 8, 7): 224140792, (8, 8, 8): 449455096}
    for (x, y, z), nnz in table2.items():
        assert W.stencil_nnz((2 ** x, 2 ** y, 2 ** z), "box") == nnz


@pytest.mark.parametrize("dims,kind", [((7, 5, 4), "box"), ((6, 6, 6), "star"),
                                       ((9, 4), "star"), ((64, 64), "star")])
def test_stencil_generator(dims, kind):
    a = W.stencil(dims, kind, seed=3)
    assert a.nnz == W.stencil_nnz(dims, kind)
    d = a.dense()
    assert np.array_equal(d, d.T)
    assert np.linalg.eigvalsh(d).min() > 0
    # rows with every neighbour in the domain sum to zero; boundary rows keep
    # their ghost edges on the diagonal and are strictly dominant
    full = a.row_lengths() == a.row_lengths().max()
    rs = d.sum(1)
    assert np.all(np.abs(rs[full]) < 1e-12 * np.diag(d)[full])
    assert np.all(rs[~full] > 0)


def test_benchmark_sizes():
    assert W.m1_poisson2d().nnz == 20224
    assert W.stencil_nnz((128, 128, 128), "star") == 14581760
    assert W.stencil_nnz((100, 100, 100), "box") == 26463592


def test_generators_deterministic():
    a1 = W.stencil((5, 6, 7), "star", 2)
    a2 = W.stencil((5, 6, 7), "star", 2)
    assert np.array_equal(a1.val, a2.val) and np.array_equal(a1.col, a2.col)
    p1, p2 = W.powerlaw(2000, 4), W.powerlaw(2000, 4)
    assert np.array_equal(p1.col, p2.col) and np.array_equal(p1.val, p2.val)


def test_powerlaw_structure():
    a = W.powerlaw(20000, 4)
    rows = a.rows()
    c = a.col.astype(np.int64)
    same = rows[1:] == rows[:-1]
    assert np.all(np.diff(c)[same] > 0)
    near = np.abs(c - rows) <= 512
    L_ = a.row_lengths()
    # per row: round(0.9 L) band columns, capped at the band size
    i = np.arange(a.n)
    band = np.minimum(i + 512, a.n - 1) - np.maximum(i - 512, 0) + 1
    per_row = np.bincount(rows, weights=near, minlength=a.n)
    assert np.array_equal(per_row, np.minimum(np.rint(0.9 * L_), band))
    assert L_.max() <= 5000 and L_.min() >= 1
    # row-sum scaled
    s = np.add.reduceat(np.abs(a.val), a.rowptr[:-1])
    assert np.allclose(s, 1.0)
