"""GPU parity for 64-bit-word PackSELL (E11MY values, float64 products).

Words and offsets must equal the 64-bit oracle's bit for bit; products must
equal the oracle's float64 product on the same quantised values within
1e-13, normalised by ||A_q||_inf ||x||_inf (float64 accumulation, so the
bar is set by float64 rounding, not by the 1e-6 of the float32 products).
Every other product, adjoint and batched entry point, and the solvers'
inner (float32) operator, must reject 64-bit-word matrices; the solvers
take them only as the float64 operator (tests/test_gpu_pcg.py).
"""
import numpy as np
import pytest
import torch

from helpers import random_csr
from oracle import linalg as L
from oracle import packsell64 as P64
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL64 = 1e-13


def encode_both(a, D, C, sigma, mode=B.IMPLICIT):
    A = B.encode(a.rowptr, a.col, a.val.astype(np.float64), a.n, a.m, "e11my", D, C, sigma, mode,
                 DEV)
    E = P64.encode(a.rowptr, a.col, a.val, a.n, a.m, D, C, sigma,
                   P64.PERM_IMPLICIT if mode == B.IMPLICIT else P64.PERM_EXPLICIT)
    return A, E


def check_words(A, E):
    assert A.k_left == E.k_left and A.n_dummies == E.n_dummies and A.n_words == E.n_words
    assert np.array_equal(A.offset.cpu().numpy(), E.offset)
    assert np.array_equal(A.pack.cpu().numpy().view(np.uint64)[:A.n_words], E.pack)


def check_product(A, a, D, x, E, mode=B.IMPLICIT):
    y = B.spmv_f64(A, torch.from_numpy(x).to(DEV)).cpu().numpy()
    q = P64.quantized(a.val, D)
    ref = L.spmv(a.rowptr, a.col, q, x)
    if mode == B.EXPLICIT:
        ref = ref[E.stored_rows]
    den = L.inf_norm(a.rowptr, q) * float(np.abs(x).max())
    err = float(np.max(np.abs(y - ref))) / den if den else 0.0
    assert err <= TOL64, err


@pytest.mark.parametrize("D", [2, 9, 14, 30, 51])
@pytest.mark.parametrize("C,sigma", [(64, 256), (32, 1), (8, 65536), (64, 300)])
def test_random_words_and_product(D, C, sigma):
    for si, (n, m, dens) in enumerate([(37, 53, 0.2), (700, 650, 0.03), (2500, 3000, None)]):
        a = random_csr(40 + si, n, m, density=dens) if dens else random_csr(40 + si, n, m, per_row=11)
        A, E = encode_both(a, D, C, sigma)
        check_words(A, E)
        x = np.random.default_rng(si).uniform(-1, 1, a.m)
        check_product(A, a, D, x, E)


def test_explicit_order_and_values_of_every_scale():
    a = random_csr(50, 1200, 1100, per_row=8)
    rng = np.random.default_rng(3)
    a.val[:] = rng.standard_normal(a.nnz) * 10.0 ** rng.integers(-200, 200, a.nnz)
    A, E = encode_both(a, 12, 64, 4096, B.EXPLICIT)
    check_words(A, E)
    x = rng.uniform(-1, 1, a.m)
    check_product(A, a, 12, x, E, B.EXPLICIT)


def test_laplace3d_128_full_size():
    """The 7-point 128^3 Laplacian with D = 15 (E11M36): no dummies, the
    plane jump 16256 fits in 15 bits."""
    a = W.m2_laplace3d(128)
    A, E = encode_both(a, 15, 64, 256, B.EXPLICIT)
    check_words(A, E)
    assert A.n_dummies == 0
    x = W.uniform_vector(a.m, 3).astype(np.float64)
    check_product(A, a, 15, x, E, B.EXPLICIT)


def test_stencil27_full_size():
    """The scaled 27-point 100^3 system of the solver benchmark, D = 14."""
    a = W.symmetric_diag_scale(W.m4_stencil27())
    A, E = encode_both(a, 14, 64, 256)
    check_words(A, E)
    x = np.random.default_rng(5).uniform(-1, 1, a.m)
    check_product(A, a, 14, x, E)


def test_edges():
    empty = W.csr_from_triplets(0, 0, [], [], [])
    A = B.encode(empty.rowptr, empty.col, empty.val, 0, 0, "e11my", 9, 64, 256, B.IMPLICIT, DEV)
    assert B.spmv_f64(A, torch.zeros(0, dtype=torch.float64, device=DEV)).numel() == 0
    hollow = W.csr_from_triplets(50, 40, [3, 3, 49], [0, 39, 20], [1.0, -2.0, 0.5])
    A, E = encode_both(hollow, 5, 64, 256)
    check_words(A, E)
    x = np.arange(40, dtype=np.float64)
    y = B.spmv_f64(A, torch.from_numpy(x).to(DEV)).cpu().numpy()
    want = np.zeros(50)
    want[3], want[49] = 1.0 * 0 - 2.0 * 39, 0.5 * 20
    assert np.array_equal(y, want)


def test_other_entry_points_reject_64_bit_words():
    a = random_csr(51, 300, 300, per_row=5)
    A, _ = encode_both(a, 9, 64, 256)
    xf = torch.zeros(a.m, device=DEV)
    with pytest.raises(B.PackSELLError):
        B.spmv(A, xf)
    with pytest.raises(B.PackSELLError):
        B.spmv_t(A, torch.zeros(a.n, device=DEV))
    with pytest.raises(B.PackSELLError):
        B.BatchedSpMV([A], [xf], [torch.zeros(a.n, device=DEV)])
    with pytest.raises(B.PackSELLError):
        B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e11my", 9, 64, 256, B.IMPLICIT, DEV,
                 split_words=64)
    A32 = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 9, 64, 256, B.IMPLICIT, DEV)
    with pytest.raises(B.PackSELLError):
        B.spmv_f64(A32, torch.zeros(a.m, dtype=torch.float64, device=DEV))
    hi = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float64, 64, 256, B.IMPLICIT, DEV)
    with pytest.raises(B.PackSELLError):
        B.pcg(A, hi, torch.ones(a.n, dtype=torch.float64, device=DEV), tol=1e-8, m_in=5,
              max_outer=5)


@pytest.mark.parametrize("C,sigma,mode", [(64, 256, B.IMPLICIT), (64, 256, B.EXPLICIT),
                                          (16, 1, B.IMPLICIT)])
def test_multi_rhs(C, sigma, mode):
    """k right-hand sides (row-major x and y, passes of 4, 2 and 1 columns):
    every column within the float64 bar of the oracle's product and equal to
    the single-vector product of that column (both sum in word order)."""
    a = random_csr(44, 1800, 1700, per_row=10)
    A, E = encode_both(a, 11, C, sigma, mode)
    q = P64.quantized(a.val, 11)
    rng = np.random.default_rng(6)
    for k in (2, 3, 4, 5, 8, 13):
        X = rng.uniform(-1, 1, (a.m, k))
        Xd = torch.from_numpy(X).to(DEV)
        Y = B.spmv_f64(A, Xd)
        Yh = Y.cpu().numpy()
        den = L.inf_norm(a.rowptr, q) * float(np.abs(X).max())
        for r in range(k):
            ref = L.spmv(a.rowptr, a.col, q, X[:, r])
            if mode == B.EXPLICIT:
                ref = ref[E.stored_rows]
            assert float(np.max(np.abs(Yh[:, r] - ref))) / den <= TOL64, (k, r)
            assert torch.equal(Y[:, r], B.spmv_f64(A, Xd[:, r].contiguous())), (k, r)
