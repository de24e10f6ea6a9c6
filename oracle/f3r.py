"""F3R nested Krylov solver in float64 (oracle; test infrastructure only).

Sec. 5.2.1 describes F3R as four nested layers: three flexible GMRES
layers and an innermost preconditioned Richardson layer, each layer
preconditioning the one outside it; the two inner layers run their products
with FP16 matrix values.  The paper takes the layer parameters and the
preconditioner from other work; our reading (layer lengths, weight, the
identity preconditioner after symmetric scaling, sec. 5.2) is stated in
``F3RParams``.

Every layer here works in float64.  The layers' operators are passed in as
separate value arrays on one CSR structure, so the mixed-precision forms
are modelled by giving the inner layers the values their products use
(float32-rounded values for layer 2, FP16 values for layers 3 and 4).

Flexible GMRES follows the textbook algorithm (Saad, Iterative Methods for
Sparse Linear Systems, flexible GMRES): Arnoldi with modified Gram-Schmidt
on the products of the preconditioned vectors, Givens rotations on the
Hessenberg matrix, and the update x0 + Z y with y the least-squares
solution.  Richardson iterates z <- z + omega (r - A z) from z = 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import linalg


@dataclasses.dataclass
class F3RParams:
    """Layer lengths: m1 steps per restart cycle of the outer FGMRES, m2 and
    m3 steps of the two inner FGMRES layers (one cycle each, from zero, no
    convergence test), m4 Richardson iterations with weight omega."""
    m1: int = 100
    m2: int = 8
    m3: int = 4
    m4: int = 2
    omega: float = 1.0


@dataclasses.dataclass
class F3RResult:
    x: np.ndarray
    outer_steps: int      # Arnoldi steps of the outer layer, over all cycles
    cycles: int           # restart cycles of the outer layer
    rel_residual: float   # true ||b - A x|| / ||b|| with the outer values
    converged: bool
    history: list         # residual estimate after every outer step


def richardson(matvec, r, m: int, omega: float) -> np.ndarray:
    """m Richardson iterations z <- z + omega (r - A z) from z = 0 (the
    preconditioner inside the iteration is the identity)."""
    z = np.zeros_like(r)
    for _ in range(m):
        z = z + omega * (r - matvec(z))
    return z


class _Arnoldi:
    """One flexible GMRES cycle, one step at a time, from x0 with residual r0."""

    def __init__(self, r0: np.ndarray, m: int):
        self.beta = float(np.sqrt(r0 @ r0))
        self.m = m
        self.V = [r0 / self.beta] if self.beta > 0 else []
        self.Z = []
        self.H = np.zeros((m + 1, m))
        self.cs = np.zeros(m)
        self.sn = np.zeros(m)
        self.g = np.zeros(m + 1)
        self.g[0] = self.beta
        self.j = 0
        self.done = self.beta == 0  # happy breakdown or nothing to do

    def step(self, matvec, precond):
        j = self.j
        z = precond(self.V[j])
        w = matvec(z)
        for i in range(j + 1):  # modified Gram-Schmidt
            self.H[i, j] = w @ self.V[i]
            w = w - self.H[i, j] * self.V[i]
        h = float(np.sqrt(w @ w))
        self.H[j + 1, j] = h
        self.Z.append(z)
        self.V.append(w / h if h > 0 else np.zeros_like(w))
        # previous rotations on the new column, then a new one for h
        for i in range(j):
            a, b = self.H[i, j], self.H[i + 1, j]
            self.H[i, j] = self.cs[i] * a + self.sn[i] * b
            self.H[i + 1, j] = -self.sn[i] * a + self.cs[i] * b
        a, b = self.H[j, j], self.H[j + 1, j]
        d = np.hypot(a, b)
        c, s = (a / d, b / d) if d > 0 else (1.0, 0.0)
        self.cs[j], self.sn[j] = c, s
        self.H[j, j] = d
        self.H[j + 1, j] = 0.0
        self.g[j + 1] = -s * self.g[j]
        self.g[j] = c * self.g[j]
        self.j = j + 1
        if h == 0:
            self.done = True
        return abs(self.g[j + 1])

    def update(self, x0: np.ndarray) -> np.ndarray:
        """x0 + Z y, y solving the triangle R y = g over the steps taken
        (columns whose diagonal vanished contribute nothing)."""
        k = self.j
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            d = self.H[i, i]
            y[i] = (self.g[i] - self.H[i, i + 1:k] @ y[i + 1:k]) / d if d != 0 else 0.0
        x = x0.copy()
        for i in range(k):
            x = x + y[i] * self.Z[i]
        return x


def fgmres_cycle(matvec, precond, r: np.ndarray, m: int) -> np.ndarray:
    """One cycle of m flexible GMRES steps on A z = r from z = 0."""
    ar = _Arnoldi(r, m)
    while ar.j < m and not ar.done:
        ar.step(matvec, precond)
    return ar.update(np.zeros_like(r))


def f3r(rowptr, col, val1, val2, val3, b, params: F3RParams = F3RParams(),
        tol: float = 1e-10, max_cycles: int = 100) -> F3RResult:
    """Solve A x = b from x0 = 0 with F3R (sec. 5.2.1): the outer flexible
    GMRES(m1) on values ``val1`` (restarted until the true relative
    residual is below ``tol``, eq. 6), preconditioned by one FGMRES(m2)
    cycle on ``val2``, preconditioned by one FGMRES(m3) cycle on ``val3``,
    preconditioned by m4 Richardson iterations on ``val3``.

    The outer layer checks its residual estimate after every step; when it
    passes, or the cycle is full, it forms x and takes the true residual,
    stopping there if that passes too and restarting from it otherwise.
    """
    b = np.asarray(b, dtype=np.float64)
    A1 = lambda v: linalg.spmv(rowptr, col, val1, v)
    A2 = lambda v: linalg.spmv(rowptr, col, val2, v)
    A3 = lambda v: linalg.spmv(rowptr, col, val3, v)
    p = params
    layer4 = lambda r: richardson(A3, r, p.m4, p.omega)
    layer3 = lambda r: fgmres_cycle(A3, layer4, r, p.m3)
    layer2 = lambda r: fgmres_cycle(A2, layer3, r, p.m2)
    nb = float(np.sqrt(b @ b))
    x = np.zeros_like(b)
    r = b.copy()
    hist = []
    steps = cycles = 0
    true = float(np.sqrt(r @ r)) / nb if nb else 0.0
    while true >= tol and cycles < max_cycles:
        ar = _Arnoldi(r, p.m1)
        cycles += 1
        while ar.j < p.m1 and not ar.done:
            est = ar.step(A1, layer2) / nb
            steps += 1
            hist.append(est)
            if est < tol:
                break
        x = ar.update(x)
        r = b - A1(x)
        true = float(np.sqrt(r @ r)) / nb
    return F3RResult(x, steps, cycles, true, bool(true < tol), hist)
