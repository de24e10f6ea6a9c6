"""GPU parity for the solvers: float64 CG and inner-outer CG (sec. 5.2.2).

b = A 1 on a symmetrically scaled SPD stencil, so x* = 1 (closed form); the
oracle's CG / IO-CG run on the same inputs.  Error paths are forced from the
host (iteration limit, a negative definite matrix, b = 0), never on the GPU.
"""
import numpy as np
import pytest
import torch

from oracle import formats as F
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def system(g=24, seed=6, sign=1.0):
    a = W.symmetric_diag_scale(W.stencil((g, g, g), "box", seed, 1.0))
    a = a.with_values(sign * a.val)
    return a, W.ones_rhs(a)


def operators(a, fmt="e8my", D=9, C=64, sigma=256):
    hi = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float64, C, sigma, B.IMPLICIT, DEV)
    lo = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, C, sigma, B.IMPLICIT, DEV)
    return lo, hi


def test_fp64_cg_matches_oracle():
    a, b = system()
    _, hi = operators(a)
    x, info = B.pcg(None, hi, torch.from_numpy(b).to(DEV), tol=1e-10, max_outer=5000)
    x = x.cpu().numpy()
    ref = L.cg(a.rowptr, a.col, a.val, b, tol=1e-10)
    assert info["rel_residual"] < 1e-10
    true = np.linalg.norm(b - L.spmv(a.rowptr, a.col, a.val, x)) / np.linalg.norm(b)
    assert true < 1e-10
    assert np.max(np.abs(x - 1.0)) < 1e-7
    assert np.max(np.abs(x - ref.x)) < 1e-7
    # same arithmetic up to reduction order: iteration counts agree closely
    assert abs(info["outer_iterations"] - ref.iterations) <= max(3, ref.iterations // 50)


@pytest.mark.parametrize("fmt,D,m_in", [("e8my", 9, 20), ("e8my", 12, 50), ("fp16", 15, 20),
                                        ("fix", 15, 30)])
def test_iocg_converges(fmt, D, m_in):
    a, b = system(20, 4)
    lo, hi = operators(a, fmt, D)
    x, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), tol=1e-10, m_in=m_in, max_outer=500)
    x = x.cpu().numpy()
    assert info["rel_residual"] < 1e-10
    true = np.linalg.norm(b - L.spmv(a.rowptr, a.col, a.val, x)) / np.linalg.norm(b)
    assert true < 1e-10
    assert np.max(np.abs(x - 1.0)) < 1e-7
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n,
                           {"e8my": F.FMT_E8MY, "fp16": F.FMT_FP16, "fix": F.FMT_FIX}[fmt], D)
    ref = L.iocg(a.rowptr, a.col, a.val, q, b, m_in=m_in, tol=1e-10)
    assert ref.converged
    # the inner solve runs in float32 on the GPU and in float64 in the
    # oracle, so outer counts may differ slightly
    assert abs(info["outer_iterations"] - ref.iterations) <= max(2, ref.iterations // 3)
    assert info["inner_iterations"] <= info["outer_iterations"] * m_in


def test_iteration_limit_reports_not_converged():
    a, b = system(16, 5)
    lo, hi = operators(a)
    x, info = B.pcg(None, hi, torch.from_numpy(b).to(DEV), tol=1e-10, max_outer=3, check=False)
    assert info["status"] == B.ENOTCONV and info["outer_iterations"] == 3
    assert info["rel_residual"] > 1e-10
    x, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), tol=1e-12, m_in=2, max_outer=2,
                    check=False)
    assert info["status"] == B.ENOTCONV and info["outer_iterations"] == 2


def test_breakdown_on_negative_definite():
    a, b = system(12, 3, sign=-1.0)
    lo, hi = operators(a)
    _, info = B.pcg(None, hi, torch.from_numpy(b).to(DEV), tol=1e-10, max_outer=100, check=False)
    assert info["status"] == B.EBREAKDOWN
    _, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), tol=1e-10, m_in=5, max_outer=100,
                    check=False)
    assert info["status"] == B.EBREAKDOWN


def test_zero_rhs_and_exact_guess():
    a, b = system(10, 2)
    lo, hi = operators(a)
    x, info = B.pcg(lo, hi, torch.zeros(a.n, dtype=torch.float64, device=DEV), tol=1e-10)
    assert info["status"] == B.OK and float(x.abs().max()) == 0.0
    x0 = torch.ones(a.n, dtype=torch.float64, device=DEV)
    x, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), x0=x0, tol=1e-10)
    assert info["status"] == B.OK and info["outer_iterations"] == 0
    assert info["rel_residual"] < 1e-10


def test_rejects_explicit_order():
    a, b = system(8, 2)
    hi = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float64, 64, 256, B.EXPLICIT, DEV)
    with pytest.raises(B.PackSELLError) as e:
        B.pcg(None, hi, torch.from_numpy(b).to(DEV))
    assert e.value.status == B.EINVAL


def test_fp64_cg_on_64_bit_words():
    """Plain float64 CG with the operator given as 64-bit-word PackSELL
    (E11M37): it solves the system of the values it holds, so it is checked
    against the oracle's CG on those quantised values."""
    from oracle import packsell64 as P64

    a, b = system()
    D = 14
    hi = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e11my", D, 64, 256, B.IMPLICIT, DEV)
    x, info = B.pcg(None, hi, torch.from_numpy(b).to(DEV), tol=1e-10, max_outer=5000)
    x = x.cpu().numpy()
    q = P64.quantized(a.val, D)
    true = np.linalg.norm(b - L.spmv(a.rowptr, a.col, q, x)) / np.linalg.norm(b)
    assert info["rel_residual"] < 1e-10 and true < 1e-10
    ref = L.cg(a.rowptr, a.col, q, b, tol=1e-10)
    assert np.max(np.abs(x - ref.x)) < 1e-7
    assert abs(info["outer_iterations"] - ref.iterations) <= max(3, ref.iterations // 50)
    assert np.max(np.abs(x - 1.0)) < 1e-6  # the quantised system is within 2^-38 of A


@pytest.mark.parametrize("inner", [("e8my", 9), ("fp16", 15)])
def test_iocg_with_64_bit_outer_operator(inner):
    from oracle import packsell64 as P64

    a, b = system(20, 4)
    D = 14
    lo = B.encode(a.rowptr, a.col, a.val, a.n, a.m, inner[0], inner[1], 64, 256, B.IMPLICIT, DEV)
    hi = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e11my", D, 64, 256, B.IMPLICIT, DEV)
    x, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), tol=1e-10, m_in=20, max_outer=500)
    x = x.cpu().numpy()
    q_hi = P64.quantized(a.val, D)
    true = np.linalg.norm(b - L.spmv(a.rowptr, a.col, q_hi, x)) / np.linalg.norm(b)
    assert info["rel_residual"] < 1e-10 and true < 1e-10
    q_lo = P.quantized_values(a.rowptr, a.col, a.val, a.n,
                              {"e8my": F.FMT_E8MY, "fp16": F.FMT_FP16}[inner[0]], inner[1])
    ref = L.iocg(a.rowptr, a.col, q_hi, q_lo, b, m_in=20, tol=1e-10)
    assert ref.converged
    assert np.max(np.abs(x - ref.x)) < 1e-7
    assert abs(info["outer_iterations"] - ref.iterations) <= max(2, ref.iterations // 3)


@pytest.mark.parametrize("fmt,D", [("fix16", 7), ("fix16", 5), ("e5my", 4)])
def test_iocg_with_16_bit_inner_operator(fmt, D):
    """IO-CG with a 16-bit-word inner operator (int8 / int10 FIX16, E5M5):
    the solution and the outer iteration count follow the oracle's IO-CG on
    the same quantised inner values."""
    from oracle import packsell16 as P16

    a, b = system(20, 4)
    lo, hi = operators(a, fmt, D)
    x, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), tol=1e-10, m_in=20, max_outer=500)
    x = x.cpu().numpy()
    assert info["rel_residual"] < 1e-10
    true = np.linalg.norm(b - L.spmv(a.rowptr, a.col, a.val, x)) / np.linalg.norm(b)
    assert true < 1e-10
    q_lo = P16.quantized(a.rowptr, a.val, a.n, {"fix16": P16.FMT_FIX16, "e5my": P16.FMT_E5MY}[fmt],
                         D)
    ref = L.iocg(a.rowptr, a.col, a.val, q_lo, b, m_in=20, tol=1e-10)
    assert ref.converged
    assert np.max(np.abs(x - ref.x)) < 1e-7
    assert abs(info["outer_iterations"] - ref.iterations) <= max(2, ref.iterations // 3)


@pytest.fixture(scope="module")
def m4():
    """The 27-point 100^3 system (n = 10^6, 26.5 M nonzeros), symmetrically
    scaled, b = A 1, and the oracle's float64 CG on it."""
    a = W.symmetric_diag_scale(W.m4_stencil27())
    b = W.ones_rhs(a)
    return a, b, L.cg(a.rowptr, a.col, a.val, b, tol=1e-10)


def _true_residual(a, val, b, x):
    return np.linalg.norm(b - L.spmv(a.rowptr, a.col, val, x)) / np.linalg.norm(b)


def test_m4_full_size_fp64_cg(m4):
    a, b, ref = m4
    assert ref.converged
    _, hi = operators(a)
    x, info = B.pcg(None, hi, torch.from_numpy(b).to(DEV), tol=1e-10, max_outer=5000)
    x = x.cpu().numpy()
    assert info["rel_residual"] < 1e-10 and _true_residual(a, a.val, b, x) < 1e-10
    assert np.max(np.abs(x - ref.x)) < 1e-7 and np.max(np.abs(x - 1.0)) < 1e-7
    assert abs(info["outer_iterations"] - ref.iterations) <= max(3, ref.iterations // 50)


@pytest.mark.parametrize("outer", ["sell", "e11my"])
def test_m4_full_size_iocg_e8m8(m4, outer):
    """IO-CG with an E8M8 inner operator (D = 14, no dummies on this
    matrix) and m_in = 20; the float64 operator is FP64 SELL or 64-bit
    E11M37 words.  x, the outer and inner iteration counts and the true
    residual follow the oracle's inner-outer CG on the same quantised
    values."""
    from oracle import packsell64 as P64

    a, b, _ = m4
    lo = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 14, 64, 256, B.IMPLICIT, DEV)
    if outer == "sell":
        hi = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float64, 64, 256, B.IMPLICIT,
                           DEV)
        q_hi = a.val
    else:
        hi = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e11my", 14, 64, 256, B.IMPLICIT, DEV)
        q_hi = P64.quantized(a.val, 14)
    x, info = B.pcg(lo, hi, torch.from_numpy(b).to(DEV), tol=1e-10, m_in=20, max_outer=500)
    x = x.cpu().numpy()
    q_lo = P.quantized_values(a.rowptr, a.col, a.val, a.n, F.FMT_E8MY, 14)
    ref = L.iocg(a.rowptr, a.col, q_hi, q_lo, b, m_in=20, tol=1e-10)
    assert ref.converged
    assert info["rel_residual"] < 1e-10 and _true_residual(a, q_hi, b, x) < 1e-10
    assert np.max(np.abs(x - ref.x)) < 1e-7
    assert abs(info["outer_iterations"] - ref.iterations) <= max(2, ref.iterations // 3)
    # no inner breakdown on this matrix: every outer step runs its m_in inner steps
    assert info["inner_iterations"] == info["outer_iterations"] * 20
    assert ref.inner_iterations == ref.iterations * 20
