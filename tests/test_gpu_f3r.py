"""GPU parity for the F3R nested solver (sec. 5.2.1).

* FP64-F3R (every layer float64) against the oracle's float64 F3R on the
  same values: the solution, the outer step count and the true residual.
* The mixed-precision forms (float32 second layer, FP16 values in layers 3
  and 4) with half-value SELL and with FP16 PackSELL words: bit-identical
  solutions and step counts (the paper's "identical convergence"), and the
  oracle's F3R on the same float32 / FP16 values.
* Restart cycles, solves that repeat bit for bit, other 32-bit word formats
  in the inner layers, and the error paths (forced from the host).
"""
import numpy as np
import pytest
import torch

from oracle import f3r as F3
from oracle import formats as F
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def spd(g=16, seed=6):
    return W.symmetric_diag_scale(W.stencil((g, g, g), "box", seed, 1.0))


def nonsym(g=16, seed=9):
    return W.symmetric_diag_scale(W.convdiff3d(g, seed, wind=(2.0, 1.0, 0.5)))


def sell(a, dtype):
    return B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, dtype, 64, 256, B.IMPLICIT, DEV)


def packed(a, fmt="fp16", D=15):
    return B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, B.IMPLICIT, DEV)


def rhs(a, kind):
    if kind == "ones":
        return W.ones_rhs(a)
    return np.random.default_rng(a.n).uniform(0.0, 1.0, a.n)  # b ~ U[0, 1) as in sec. 5.2


def true_residual(a, b, x):
    return np.linalg.norm(b - L.spmv(a.rowptr, a.col, a.val, x)) / np.linalg.norm(b)


def v32(a):
    return a.val.astype(np.float32).astype(np.float64)


def v16(a):
    return P.quantized_values(a.rowptr, a.col, a.val, a.n, F.FMT_FP16, 15)


@pytest.mark.parametrize("make,kind", [(spd, "ones"), (nonsym, "uniform")])
def test_fp64_f3r_matches_oracle(make, kind):
    a = make()
    b = rhs(a, kind)
    x, info = B.f3r(sell(a, torch.float64), torch.from_numpy(b).to(DEV), tol=1e-10)
    x = x.cpu().numpy()
    ref = F3.f3r(a.rowptr, a.col, a.val, a.val, a.val, b, F3.F3RParams(), tol=1e-10)
    assert ref.converged
    assert info["rel_residual"] < 1e-10 and true_residual(a, b, x) < 1e-10
    assert np.max(np.abs(x - ref.x)) < 1e-8 * np.abs(ref.x).max()
    assert abs(info["outer_iterations"] - ref.outer_steps) <= 1
    assert info["inner_iterations"] == info["outer_iterations"] * 8


@pytest.mark.parametrize("make,kind", [(spd, "ones"), (nonsym, "uniform")])
def test_mixed_forms_identical_and_match_oracle(make, kind):
    a = make()
    b = rhs(a, kind)
    bd = torch.from_numpy(b).to(DEV)
    A1, A2 = sell(a, torch.float64), sell(a, torch.float32)
    xs, infs = B.f3r(A1, bd, A2, sell(a, torch.float16), tol=1e-10)
    xp, infp = B.f3r(A1, bd, A2, packed(a), tol=1e-10)
    # FP16 values embedded in the words: the same iterates bit for bit
    assert torch.equal(xs, xp)
    assert infs["outer_iterations"] == infp["outer_iterations"]
    assert infs["rel_residual"] == infp["rel_residual"]
    x = xp.cpu().numpy()
    assert infp["rel_residual"] < 1e-10 and true_residual(a, b, x) < 1e-10
    ref = F3.f3r(a.rowptr, a.col, a.val, v32(a), v16(a), b, F3.F3RParams(), tol=1e-10)
    assert ref.converged
    assert np.max(np.abs(x - ref.x)) < 1e-7 * np.abs(ref.x).max()
    # the inner layers run in float32 here and in float64 in the oracle
    assert abs(infp["outer_iterations"] - ref.outer_steps) <= 2


def test_solves_repeat_bit_for_bit():
    a = nonsym(12, 3)
    bd = torch.from_numpy(rhs(a, "uniform")).to(DEV)
    A1, A2, A3 = sell(a, torch.float64), sell(a, torch.float32), packed(a)
    x1, i1 = B.f3r(A1, bd, A2, A3, tol=1e-10)
    x2, i2 = B.f3r(A1, bd, A2, A3, tol=1e-10)
    assert torch.equal(x1, x2) and i1["outer_iterations"] == i2["outer_iterations"]
    y1, _ = B.f3r(A1, bd, tol=1e-10)
    y2, _ = B.f3r(A1, bd, tol=1e-10)
    assert torch.equal(y1, y2)
    # inner operators loaded with the resident cache policy: the same solve
    A3.cache_hint = B.CACHE_RESIDENT
    x3, _ = B.f3r(A1, bd, A2, A3, tol=1e-10)
    assert torch.equal(x1, x3)
    S3 = sell(a, torch.float16)
    z1, _ = B.f3r(A1, bd, A2, S3, tol=1e-10)
    S3.cache_hint = B.CACHE_RESIDENT
    z2, _ = B.f3r(A1, bd, A2, S3, tol=1e-10)
    assert torch.equal(z1, z2)


def test_restart_cycles_follow_the_oracle():
    """Short cycles and weak inner layers: several restarts, each confirmed
    on the true residual."""
    a = nonsym(10, 4)
    b = W.ones_rhs(a)
    prm = dict(m1=2, m2=2, m3=2, m4=1, omega=0.8)
    x, info = B.f3r(sell(a, torch.float64), torch.from_numpy(b).to(DEV), tol=1e-10, **prm)
    ref = F3.f3r(a.rowptr, a.col, a.val, a.val, a.val, b, F3.F3RParams(**prm), tol=1e-10)
    assert ref.converged and ref.cycles > 1
    x = x.cpu().numpy()
    assert info["rel_residual"] < 1e-10 and true_residual(a, b, x) < 1e-10
    assert np.max(np.abs(x - 1.0)) < 1e-8
    assert abs(info["outer_iterations"] - ref.outer_steps) <= 2


@pytest.mark.parametrize("fmt,D", [("e8my", 9), ("e8my", 12), ("fix", 15)])
def test_other_word_formats_in_the_inner_layers(fmt, D):
    a = spd(14, 2)
    b = W.ones_rhs(a)
    x, info = B.f3r(sell(a, torch.float64), torch.from_numpy(b).to(DEV), sell(a, torch.float32),
                    packed(a, fmt, D), tol=1e-10)
    x = x.cpu().numpy()
    assert info["rel_residual"] < 1e-10 and true_residual(a, b, x) < 1e-10
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n,
                           {"e8my": F.FMT_E8MY, "fix": F.FMT_FIX}[fmt], D)
    ref = F3.f3r(a.rowptr, a.col, a.val, v32(a), q, b, F3.F3RParams(), tol=1e-10)
    assert np.max(np.abs(x - ref.x)) < 1e-7
    assert abs(info["outer_iterations"] - ref.outer_steps) <= 2


def test_zero_rhs_exact_guess_and_limits():
    a = spd(8, 1)
    A1 = sell(a, torch.float64)
    x, info = B.f3r(A1, torch.zeros(a.n, dtype=torch.float64, device=DEV))
    assert info["status"] == B.OK and float(x.abs().max()) == 0.0
    b = torch.from_numpy(W.ones_rhs(a)).to(DEV)
    x, info = B.f3r(A1, b, x0=torch.ones(a.n, dtype=torch.float64, device=DEV))
    assert info["status"] == B.OK and info["outer_iterations"] == 0
    x, info = B.f3r(A1, b, tol=1e-14, m1=1, m2=1, m3=1, m4=1, max_cycles=2, check=False)
    assert info["status"] == B.ENOTCONV and info["outer_iterations"] == 2
    for bad in (dict(m1=0), dict(m2=33), dict(omega=0.0), dict(max_cycles=0)):
        with pytest.raises(B.PackSELLError) as e:
            B.f3r(A1, b, **bad)
        assert e.value.status == B.EINVAL
    with pytest.raises(B.PackSELLError) as e:  # explicit order is refused
        B.f3r(B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float64, 64, 256, B.EXPLICIT,
                            DEV), b)
    assert e.value.status == B.EINVAL


def test_workspace_too_small():
    import ctypes

    a = spd(6, 1)
    A1 = sell(a, torch.float64)
    b = torch.from_numpy(W.ones_rhs(a)).to(DEV)
    x = torch.zeros_like(b)
    prm = B.CF3RParams(10, 4, 2, 2, 1.0, 5, 0)
    need = ctypes.c_size_t()
    assert B.lib().pksell_f3r_workspace(a.n, 0, ctypes.byref(prm), ctypes.byref(need)) == B.OK
    ws = torch.empty(need.value - 1, dtype=torch.uint8, device=DEV)
    info = B.CPcgInfo()
    rc = B.lib().pksell_f3r(ctypes.byref(A1.desc), None, None, None, B._ptr(b), B._ptr(x), 1e-10,
                            ctypes.byref(prm), ctypes.byref(info), B._ptr(ws), need.value - 1,
                            B._stream(DEV))
    assert rc == B.EWORKSPACE


def test_mixed_forms_identical_on_m4_full_size():
    """The 27-point 100^3 system of the solver benchmark (n = 10^6): FP16
    SELL and FP16 PackSELL inner layers give the same solve bit for bit,
    and both reach a true residual below 1e-10 in float64."""
    a = W.symmetric_diag_scale(W.m4_stencil27())
    b = W.ones_rhs(a)
    bd = torch.from_numpy(b).to(DEV)
    A1 = sell(a, torch.float64)
    A2 = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, 64, 256, B.IMPLICIT, DEV,
                       paired=True)
    xs, infs = B.f3r(A1, bd, A2, sell(a, torch.float16), tol=1e-10)
    xp, infp = B.f3r(A1, bd, A2, packed(a), tol=1e-10)
    assert torch.equal(xs, xp) and infs["outer_iterations"] == infp["outer_iterations"]
    assert true_residual(a, b, xp.cpu().numpy()) < 1e-10
    assert float((xp - 1.0).abs().max()) < 1e-7


def test_mid_size_mixed_form_matches_oracle():
    """A 40^3 27-point system: the PackSELL form against the oracle's F3R
    on the same float32 (layer 2) and FP16 (layers 3-4) values."""
    a = spd(40, 5)
    b = rhs(a, "ones")
    bd = torch.from_numpy(b).to(DEV)
    x, info = B.f3r(sell(a, torch.float64), bd, sell(a, torch.float32), packed(a), tol=1e-10)
    x = x.cpu().numpy()
    ref = F3.f3r(a.rowptr, a.col, a.val, v32(a), v16(a), b, F3.F3RParams(), tol=1e-10)
    assert ref.converged
    assert info["rel_residual"] < 1e-10 and true_residual(a, b, x) < 1e-10
    assert np.max(np.abs(x - ref.x)) < 1e-7 * np.abs(ref.x).max()
    assert abs(info["outer_iterations"] - ref.outer_steps) <= 2
