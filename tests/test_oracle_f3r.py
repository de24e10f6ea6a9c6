"""Pins of the F3R oracle (nested flexible GMRES and Richardson, sec. 5.2.1),
each against something other than the oracle itself:

* GMRES optimality: after j steps with a fixed preconditioner M, the
  residual estimate and the true residual equal the least-squares minimum of
  ||r0 - A M k|| over the Krylov space K_j(A M, r0), found by brute force
  from an explicit Krylov basis;
* finite termination: a full cycle (m = n) solves a small system exactly
  (compared with numpy's dense solve);
* Richardson: the closed-form truncated Neumann series;
* nesting: with exact inner layers the outer layer converges in one step;
* end to end: F3R reaches the tolerance on SPD and nonsymmetric stencils and
  its x matches a direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from oracle import f3r as F3
from oracle import linalg as L
from paper_2604_13433_amd import workloads as W


def small_nonsym(n=40, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    A[np.abs(A) < 0.2] = 0.0
    np.fill_diagonal(A, 4 + rng.random(n))
    return A


def brute_min_residual(A, M, r0, j):
    """min over k in K_j(A M, r0) of ||r0 - A M k||, by least squares on an
    orthonormalised explicit Krylov basis."""
    K = [r0]
    for _ in range(j - 1):
        K.append(A @ (M @ K[-1]))
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    AMQ = A @ (M @ Q)
    c, *_ = np.linalg.lstsq(AMQ, r0, rcond=None)
    return float(np.linalg.norm(r0 - AMQ @ c))


@pytest.mark.parametrize("precond", ["identity", "fixed"])
def test_fgmres_steps_are_gmres_optimal(precond):
    A = small_nonsym()
    n = A.shape[0]
    rng = np.random.default_rng(1)
    M = np.eye(n) if precond == "identity" else np.diag(1 / np.diag(A)) + 0.01 * rng.random((n, n))
    r0 = rng.standard_normal(n)
    ar = F3._Arnoldi(r0, 12)
    for j in range(1, 13):
        est = ar.step(lambda v: A @ v, lambda v: M @ v)
        want = brute_min_residual(A, M, r0, j)
        assert est == pytest.approx(want, rel=1e-8, abs=1e-12)
        x = ar.update(np.zeros(n))
        assert np.linalg.norm(r0 - A @ x) == pytest.approx(want, rel=1e-8, abs=1e-12)


def test_full_cycle_solves_exactly():
    A = small_nonsym(30, 3)
    b = np.random.default_rng(4).standard_normal(30)
    x = F3.fgmres_cycle(lambda v: A @ v, lambda v: v, b, 30)
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-10


def test_happy_breakdown_on_the_identity():
    b = np.random.default_rng(5).standard_normal(10)
    ar = F3._Arnoldi(b, 5)
    est = ar.step(lambda v: v, lambda v: v)
    assert est == 0.0 and ar.done
    assert np.allclose(ar.update(np.zeros(10)), b)
    assert np.array_equal(F3.fgmres_cycle(lambda v: v, lambda v: v, np.zeros(4), 3), np.zeros(4))


@pytest.mark.parametrize("m,omega", [(1, 1.0), (2, 1.0), (3, 0.7), (5, 0.9)])
def test_richardson_is_the_truncated_neumann_series(m, omega):
    A = small_nonsym(20, 6) / 5.0
    r = np.random.default_rng(7).standard_normal(20)
    z = F3.richardson(lambda v: A @ v, r, m, omega)
    Tm = np.eye(20) - omega * A
    want = sum(omega * np.linalg.matrix_power(Tm, i) @ r for i in range(m))
    assert np.max(np.abs(z - want)) < 1e-12 * max(1.0, np.abs(want).max())


def _csr(a):
    return a.rowptr, a.col, a.val


def test_exact_inner_layers_converge_in_one_outer_step():
    a = W.symmetric_diag_scale(W.stencil((5, 5, 4), "box", 3, 1.0))
    b = W.ones_rhs(a)
    # an FGMRES(m2 = n) second layer on the same values is an exact solve
    p = F3.F3RParams(m1=10, m2=a.n, m3=2, m4=2)
    r = F3.f3r(*_csr(a), a.val, a.val, b, p, tol=1e-10)
    assert r.converged and r.outer_steps == 1 and r.cycles == 1
    assert np.max(np.abs(r.x - 1.0)) < 1e-8


@pytest.mark.parametrize("kind", ["spd", "nonsym"])
def test_f3r_converges_to_the_direct_solution(kind):
    if kind == "spd":
        a = W.symmetric_diag_scale(W.stencil((12, 12, 12), "box", 6, 1.0))
    else:
        a = W.symmetric_diag_scale(W.convdiff3d(12, 9, wind=(2.0, 1.0, 0.5)))
    b = np.random.default_rng(2).uniform(0, 1, a.n)
    As = sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.n))
    want = sla.spsolve(As.tocsc(), b)
    v32 = a.val.astype(np.float32).astype(np.float64)
    v16 = a.val.astype(np.float16).astype(np.float64)
    for vals in ((a.val, a.val), (v32, v16)):
        r = F3.f3r(*_csr(a), vals[0], vals[1], b, F3.F3RParams(), tol=1e-10)
        assert r.converged and r.rel_residual < 1e-10
        true = np.linalg.norm(b - L.spmv(a.rowptr, a.col, a.val, r.x)) / np.linalg.norm(b)
        assert true < 1e-10
        assert np.max(np.abs(r.x - want)) < 1e-7 * np.abs(want).max()
        # the estimate is monotone (GMRES minimises the residual in each cycle)
        h = np.array(r.history)
        assert np.all(np.diff(h) <= 1e-12)


def test_restarts_reach_the_tolerance():
    a = W.symmetric_diag_scale(W.convdiff3d(10, 4))
    b = W.ones_rhs(a)
    p = F3.F3RParams(m1=2, m2=2, m3=2, m4=1, omega=0.8)  # weak inner layers, short cycles
    r = F3.f3r(*_csr(a), a.val, a.val, b, p, tol=1e-10)
    assert r.converged and r.cycles > 1
    assert np.max(np.abs(r.x - 1.0)) < 1e-8
