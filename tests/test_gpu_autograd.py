"""GPU checks of the differentiable product (forward, grad_x, grad_values).

Reference gradients come from the oracle in float64 on the same quantised
values: grad_x = A_q^T g and grad_values = g_i x_j.  Finite differences
check both: y is linear in x, so a central difference with a large step is
exact up to float32 rounding; values are perturbed by steps that keep them
on the E8MY grid (the re-encoded word then holds exactly the perturbed value).
"""
import numpy as np
import pytest
import torch

from helpers import random_csr
from oracle import formats as F
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import autograd as AG
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def grid_values(a, D, seed):
    """Values already on the E8MY grid of D (so quantisation is exact)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(a.nnz).astype(np.float32)
    return F.e8my_value_bits(v, D).view(np.float32)


@pytest.mark.parametrize("adjoint", ["atomic", "transpose"])
@pytest.mark.parametrize("k", [1, 4])
def test_gradients_against_fp64_reference(k, adjoint):
    a = random_csr(11, 900, 700, per_row=12)
    D = 9
    vals = torch.tensor(grid_values(a, D, 1), device=DEV, requires_grad=True)
    lin = AG.PackSELLLinear(a.rowptr, a.col, vals, a.n, a.m, "e8my", D, adjoint=adjoint)
    assert (lin.transposed() is not None) == (adjoint == "transpose")
    X = W.uniform_vector(a.m, 2, k=k)
    G = W.uniform_vector(a.n, 3, k=k)
    x = torch.tensor(X, device=DEV, requires_grad=True)
    y = lin(x)
    (y * torch.tensor(G, device=DEV)).sum().backward()
    q = vals.detach().double().cpu().numpy()
    Gd, Xd = G.astype(np.float64).reshape(a.n, k), X.astype(np.float64).reshape(a.m, k)
    ref_gx = np.stack([L.spmv_t(a.rowptr, a.col, q, Gd[:, r], a.m) for r in range(k)], 1)
    ref_gv = sum(L.grad_values(a.rowptr, a.col, Gd[:, r], Xd[:, r]) for r in range(k))
    gx = x.grad.double().cpu().numpy().reshape(a.m, k)
    gv = vals.grad.double().cpu().numpy()
    colsum = np.bincount(a.col, weights=np.abs(q), minlength=a.m).max()
    assert np.max(np.abs(gx - ref_gx)) / (colsum * np.abs(Gd).max()) <= 1e-6
    assert np.max(np.abs(gv - ref_gv)) / (np.abs(Xd).max() * np.abs(Gd).max() * k) <= 1e-6
    ref_y = np.stack([L.spmv(a.rowptr, a.col, q, Xd[:, r]) for r in range(k)], 1)
    den = L.inf_norm(a.rowptr, q) * np.abs(Xd).max()
    assert np.max(np.abs(y.detach().double().cpu().numpy().reshape(a.n, k) - ref_y)) / den <= 1e-6


def test_finite_differences():
    a = random_csr(12, 400, 400, per_row=8)
    D = 9
    v0 = grid_values(a, D, 4)
    x = torch.tensor(W.uniform_vector(a.m, 5), device=DEV)
    g = torch.tensor(W.uniform_vector(a.n, 6), device=DEV)

    def f(vals_np, xx):
        vals = torch.tensor(vals_np, device=DEV)
        lin = AG.PackSELLLinear(a.rowptr, a.col, vals, a.n, a.m, "e8my", D)
        return float((lin(xx).double() * g.double()).sum())

    vals = torch.tensor(v0, device=DEV, requires_grad=True)
    xx = x.clone().requires_grad_(True)
    lin = AG.PackSELLLinear(a.rowptr, a.col, vals, a.n, a.m, "e8my", D)
    (lin(xx) * g).sum().backward()
    # x: y is linear in x, so a step of 1 is exact up to rounding
    for j in (0, 17, 123, 399):
        e = torch.zeros_like(x)
        e[j] = 1.0
        fd = (f(v0, x + e) - f(v0, x - e)) / 2.0
        assert abs(fd - float(xx.grad[j])) <= 1e-5 * (1 + abs(fd))
    # values: 16 units of the E8MY grid keep the perturbed value representable
    bits = v0.view(np.uint32)
    for e_i in (0, 55, 1000, a.nnz - 1):
        step = np.uint32(16 << (D + 1))
        vp, vm = bits.copy(), bits.copy()
        vp[e_i] = bits[e_i] + step
        vm[e_i] = bits[e_i] - step
        fp, fm = vp.view(np.float32), vm.view(np.float32)
        h = float(fp[e_i]) - float(v0[e_i])
        hm = float(v0[e_i]) - float(fm[e_i])
        if abs(h - hm) > 1e-12 * abs(h):  # crossed a binade: skip
            continue
        fd = (f(fp, x) - f(fm, x)) / (2 * h)
        assert abs(fd - float(vals.grad[e_i])) <= 1e-4 * (1 + abs(fd))


def test_transpose_adjoint_rejects_fix():
    a = random_csr(14, 50, 50, per_row=3)
    vals = torch.tensor(a.val.astype(np.float32), device=DEV)
    with pytest.raises(ValueError):
        AG.PackSELLLinear(a.rowptr, a.col, vals, a.n, a.m, "fix", 15, adjoint="transpose")


def test_reencodes_after_update():
    a = random_csr(13, 200, 200, per_row=5)
    vals = torch.tensor(grid_values(a, 9, 7), device=DEV)
    lin = AG.PackSELLLinear(a.rowptr, a.col, vals, a.n, a.m, "e8my", 9)
    x = torch.ones(a.m, device=DEV)
    y1 = lin(x).clone()
    with torch.no_grad():
        vals.mul_(2.0)
    y2 = lin(x)
    assert torch.allclose(y2, 2 * y1)
