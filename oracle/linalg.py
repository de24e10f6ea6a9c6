"""Float64 reference products and solvers (oracle; test infrastructure).

The PackSELL SpMV computes exactly y = A_q x up to the order of its
float32 accumulation, where A_q holds the quantised values at the stored
positions (dummies and padding contribute nothing).  The plain definition of
that product -- a float64 CSR SpMV over the quantised values -- is therefore
the reference the GPU results are compared with (eq. 1).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import native


def spmv(rowptr, col, val_q, x) -> np.ndarray:
    """y_i = sum over stored j of a_q[i, j] * x_j, float64 (eq. 1)."""
    return native.csr_spmv(rowptr, col, val_q, np.asarray(x, dtype=np.float64))


def spmv_multi(rowptr, col, val_q, X) -> np.ndarray:
    """Y = A_q X for a row-major m x k block, one column at a time."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        return spmv(rowptr, col, val_q, X)
    return np.stack([spmv(rowptr, col, val_q, X[:, r]) for r in range(X.shape[1])], axis=1)


def spmv_t(rowptr, col, val_q, g, m: int) -> np.ndarray:
    """y_j = sum over stored (i, j) of a_q[i, j] * g_i, float64."""
    return native.csr_spmv_t(rowptr, col, val_q, np.asarray(g, dtype=np.float64), m)


def grad_values(rowptr, col, g, x) -> np.ndarray:
    """d<g, A x>/d a_ij = g_i * x_j at every stored (i, j), CSR order."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    rows = np.repeat(np.arange(rowptr.size - 1, dtype=np.int64), np.diff(rowptr))
    return np.asarray(g, np.float64)[rows] * np.asarray(x, np.float64)[np.asarray(col, np.int64)]


def inf_norm(rowptr, val) -> float:
    """||A||_inf = max over rows of sum |a_ij|."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    a = np.abs(np.asarray(val, dtype=np.float64))
    if a.size == 0:
        return 0.0
    s = np.add.reduceat(a, rowptr[:-1].clip(max=a.size - 1))
    s[np.diff(rowptr) == 0] = 0.0
    return float(s.max()) if s.size else 0.0


def backward_error(rowptr, col, val, x, y) -> float:
    """||y - A x||_inf / (||A||_inf ||x||_inf) with the unquantised A (eq. 5)."""
    ax = spmv(rowptr, col, val, x)
    den = inf_norm(rowptr, val) * float(np.max(np.abs(x)))
    return float(np.max(np.abs(np.asarray(y, np.float64) - ax)) / den) if den else 0.0


def normalised_error(y, y_ref, rowptr, val_q, x) -> float:
    """||y - y_ref||_inf / (||A_q||_inf ||x||_inf): the parity measure."""
    den = inf_norm(rowptr, val_q) * float(np.max(np.abs(x)))
    err = float(np.max(np.abs(np.asarray(y, np.float64) - y_ref))) if np.size(y) else 0.0
    return err / den if den else err


# ---------------------------------------------------------------------------
# Solvers (sec. 5.2)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    iterations: int  # outer iterations (CG: iterations)
    inner_iterations: int
    rel_residual: float  # true ||b - A x||_2 / ||b||_2
    converged: bool
    history: list


def cg(rowptr, col, val, b, tol=1e-10, max_iter=10000) -> SolveResult:
    """Textbook conjugate gradients from x0 = 0 in float64.

    Applied to the symmetrically scaled matrix Gbar^-1 A Gbar^-1 (sec. 5.2),
    whose diagonal is one, so the Jacobi preconditioner is the identity and
    PCG reduces to CG.  Stops when ||b - A x||_2 / ||b||_2 < tol (eq. 6),
    judged on the recursively updated residual and confirmed on the true one.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    nb = np.sqrt(b @ b)
    hist = []
    it = 0
    while it < max_iter:
        q = spmv(rowptr, col, val, p)
        pq = p @ q
        if not pq > 0:
            break
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rr_new = r @ r
        it += 1
        hist.append(np.sqrt(rr_new) / nb)
        if np.sqrt(rr_new) / nb < tol:
            true = np.linalg.norm(b - spmv(rowptr, col, val, x)) / nb
            if true < tol:
                return SolveResult(x, it, 0, true, True, hist)
            r = b - spmv(rowptr, col, val, x)
            rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    true = np.linalg.norm(b - spmv(rowptr, col, val, x)) / nb
    return SolveResult(x, it, 0, true, bool(true < tol), hist)


def inner_cg(rowptr, col, val_q, r, m_in: int) -> np.ndarray:
    """Inner solve of the inner-outer CG: m_in CG iterations on A_q z = r
    from z = 0, on the normalised right-hand side r / ||r||, result scaled
    back by ||r||.  No convergence test; stops early only on breakdown
    (zero residual or non-positive curvature)."""
    nr = np.sqrt(r @ r)
    if nr == 0:
        return np.zeros_like(r)
    rin = r / nr
    z = np.zeros_like(r)
    res = rin.copy()
    p = res.copy()
    rr = res @ res
    for _ in range(m_in):
        q = spmv(rowptr, col, val_q, p)
        pq = p @ q
        if not pq > 0 or rr == 0:
            break
        alpha = rr / pq
        z += alpha * p
        res -= alpha * q
        rr_new = res @ res
        p = res + (rr_new / rr) * p
        rr = rr_new
    return z * nr


def iocg(rowptr, col, val_hi, val_q, b, m_in: int, tol=1e-10,
         max_outer=10000, inner=None) -> SolveResult:
    """Inner-outer CG (sec. 5.2.2): flexible CG (Notay) outer iteration in
    float64 on A, preconditioned by ``m_in`` inner CG iterations on the
    quantised A_q.  Outer step k:

        z_k = Inner(r_k)
        p_k = z_k - [(z_k, q_{k-1}) / (p_{k-1}, q_{k-1})] p_{k-1}   (k > 0)
        q_k = A p_k
        alpha_k = (p_k, r_k) / (p_k, q_k)
        x += alpha_k p_k ;  r -= alpha_k q_k

    (flexible CG truncated to one previous direction).  Stops when the
    updated residual passes ||r||/||b|| < tol and the true residual
    ||b - A x||/||b|| confirms it; otherwise the true residual replaces r.
    ``inner`` replaces the inner solve (a function of r) when given.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.sqrt(b @ b)
    p_prev = q_prev = None
    pq_prev = None
    hist = []
    k = 0
    while k < max_outer:
        z = inner(r) if inner is not None else inner_cg(rowptr, col, val_q, r, m_in)
        if p_prev is None:
            p = z
        else:
            p = z - ((z @ q_prev) / pq_prev) * p_prev
        q = spmv(rowptr, col, val_hi, p)
        pq = p @ q
        if not pq > 0:
            break
        alpha = (p @ r) / pq
        x += alpha * p
        r -= alpha * q
        k += 1
        rel = np.sqrt(r @ r) / nb
        hist.append(rel)
        if rel < tol:
            rt = b - spmv(rowptr, col, val_hi, x)
            true = np.sqrt(rt @ rt) / nb
            if true < tol:
                return SolveResult(x, k, k * m_in, true, True, hist)
            r = rt
        p_prev, q_prev, pq_prev = p, q, pq
    rt = b - spmv(rowptr, col, val_hi, x)
    true = np.sqrt(rt @ rt) / nb
    return SolveResult(x, k, k * m_in, true, bool(true < tol), hist)
