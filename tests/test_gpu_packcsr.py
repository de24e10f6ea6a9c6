"""GPU parity for CSR-packed matrices (PackSELL words stored row after row:
C = 1, sigma = 1) and their product balanced over chunks of words.

Words and the word row pointer must equal the CSR-packing oracle's bit for
bit, and the chunk plan (first owned row and anchor column per chunk) the
plan read off the oracle's word stream.  Products
must equal the oracle's float64 product on the same quantised values
within 1e-6, normalised by ||A_q||_inf ||x||_inf, and repeat bit for bit
(every sum has a fixed order).  At the power-law matrix's full size the
product is checked on sampled rows, each computed from the quantised values
of that row alone.
"""
import numpy as np
import pytest
import torch

from helpers import FMTS, SPMV_TOL, chunk_plan_from_words, random_csr
from oracle import linalg as L
from oracle import packcsr as PC
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def hollow(seed):
    """Empty rows at the start, in a run in the middle and at the end; long
    jumps (dummies); every 97th row 200 long."""
    rng = np.random.default_rng(seed)
    n, m = 3000, 70000
    rows, cols = [], []
    for i in range(n):
        if i < 5 or 1000 <= i < 1300 or i >= 2950 or rng.random() < 0.2:
            continue
        k = 200 if i % 97 == 0 else int(rng.integers(1, 12))
        c = np.unique(rng.integers(0, m, size=k))
        rows += [i] * c.size
        cols += list(c)
    return W.csr_from_triplets(n, m, rows, cols, rng.standard_normal(len(rows)))


def both(a, fmt, D, chunk):
    A = B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, chunk, DEV)
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D)
    return A, E


def check_layout(A, E, chunk):
    assert A.k_left == E.k_left and A.n_dummies == E.n_dummies and A.n_words == E.n_words
    assert np.array_equal(A.offset.cpu().numpy(), E.wrowptr)
    assert np.array_equal(A.pack.cpu().numpy().view(np.uint32)[: E.n_words], E.pack)
    if E.row_exp is not None:
        assert np.array_equal(A.row_exp.cpu().numpy()[: E.n].astype(np.int64), E.row_exp)
    lo, anchor = chunk_plan_from_words(E, chunk)
    assert A.desc.n_units == anchor.size
    if anchor.size:
        assert np.array_equal(A.t["units"].cpu().numpy().astype(np.int64), lo)
        assert np.array_equal(A.t["ckpt"].cpu().numpy().view(np.uint32).astype(np.int64), anchor)


def check_product(A, E, a, fmt, D, x):
    xt = torch.from_numpy(x.astype(np.float32)).to(DEV)
    y = B.spmv(A, xt)
    y2 = B.spmv(A, xt)
    assert torch.equal(y, y2)  # fixed summation order
    ref = PC.spmv(E, x.astype(np.float32).astype(np.float64))
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
    den = L.inf_norm(a.rowptr, q) * float(np.abs(x).max()) if a.m else 0.0
    err = float(np.max(np.abs(y.cpu().numpy().astype(np.float64) - ref))) if a.n else 0.0
    assert (err / den if den else err) <= SPMV_TOL, err
    return y


@pytest.mark.parametrize("chunk", [256, 512, 1024])
@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9), ("e8my", 3), ("fix", 20)])
def test_layout_plan_and_product(fmt, D, chunk):
    for si, a in enumerate([hollow(3), random_csr(4, 700, 650, density=0.03),
                            random_csr(5, 2500, 3000, per_row=11)]):
        A, E = both(a, fmt, D, chunk)
        check_layout(A, E, chunk)
        check_product(A, E, a, fmt, D, np.random.default_rng(si).uniform(-1, 1, a.m))


def test_rows_across_many_chunks_and_exact_fits():
    # one row over 16 chunks of 256 words, between empty rows
    a = W.csr_from_triplets(3, 50000, [1] * 4000, np.arange(0, 50000, 12)[:4000],
                            np.random.default_rng(1).standard_normal(4000))
    # rows of exactly 256 words: chunk edges on row starts
    n = 12
    b = W.csr_from_triplets(n, 256, np.repeat(np.arange(n), 256), np.tile(np.arange(256), n),
                            np.random.default_rng(2).standard_normal(256 * n))
    # a word count that is not a multiple of 4 (the last lane reads word by word)
    c = random_csr(6, 333, 500, per_row=7)
    for m in (a, b, c):
        A, E = both(m, "fp16", 15, 256)
        check_layout(A, E, 256)
        check_product(A, E, m, "fp16", 15, np.random.default_rng(3).uniform(-1, 1, m.m))


def test_edges():
    for n, m in ((0, 0), (70, 0), (70, 40)):
        a = W.csr_from_triplets(n, m, [], [], [])
        A = B.encode_packed_csr(a.rowptr, a.col, a.val, n, m, "fp16", 15, 512, DEV)
        assert A.n_words == 0 and A.desc.n_units == 0
        y = B.spmv(A, torch.ones(m, device=DEV), torch.full((n,), 7.0, device=DEV))
        assert not y.any()
    # k = 3 takes the one-row-slice product (no chunk plan): same values
    a = hollow(8)
    A, E = both(a, "e8my", 9, 512)
    x = np.random.default_rng(4).uniform(-1, 1, (a.m, 3))
    yk = B.spmv(A, torch.from_numpy(x.astype(np.float32)).to(DEV)).cpu().numpy()
    for j in range(3):
        ref = PC.spmv(E, x[:, j].astype(np.float32).astype(np.float64))
        q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS["e8my"], 9)
        den = L.inf_norm(a.rowptr, q) * float(np.abs(x[:, j]).max())
        assert float(np.max(np.abs(yk[:, j] - ref))) / den <= SPMV_TOL


def test_chunk_parameters_rejected():
    a = random_csr(7, 100, 100, per_row=4)
    for C, sigma, chunk in ((1, 2, 512), (1, 1, 384), (1, 1, 2048), (2, 1, 256)):
        with pytest.raises(B.PackSELLError):
            B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, C, sigma, B.EXPLICIT, DEV,
                     split_words=chunk)


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 12)])
def test_powerlaw_full_size_sampled_rows(fmt, D):
    """The 1M-row power-law matrix (row lengths 1..5000) with FP16 or E8M10
    words in 512-word chunks, as the benchmark runs it: words and plan
    against the oracle on the whole matrix, products on 3000 sampled rows."""
    a = W.m3_powerlaw()
    A = B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 512, DEV)
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D)
    check_layout(A, E, 512)
    x = W.uniform_vector(a.m, 9).astype(np.float64)
    y = B.spmv(A, torch.from_numpy(x.astype(np.float32)).to(DEV)).cpu().numpy()
    rng = np.random.default_rng(10)
    lens = np.diff(a.rowptr)
    rows = np.unique(np.concatenate([rng.integers(0, a.n, 2000), np.argsort(lens)[-1000:]]))
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
    den = L.inf_norm(a.rowptr, q) * float(np.abs(x).max())
    for r in rows:
        s, e = a.rowptr[r], a.rowptr[r + 1]
        ref = float(np.dot(q[s:e], x.astype(np.float32).astype(np.float64)[a.col[s:e]]))
        assert abs(float(y[r]) - ref) / den <= SPMV_TOL, r


def test_adjoint_and_value_gradients_on_packed_csr():
    """The adjoint A_q^T g and the value gradients g_i x_j run on the same
    one-row-slice words (the chunk plan is not used by them)."""
    import scipy.sparse as sp

    a = hollow(11)
    A, E = both(a, "e8my", 9, 512)
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS["e8my"], 9)
    rng = np.random.default_rng(12)
    g = rng.uniform(-1, 1, a.n).astype(np.float32)
    x = rng.uniform(-1, 1, a.m).astype(np.float32)
    yt = B.spmv_t(A, torch.from_numpy(g).to(DEV)).cpu().numpy().astype(np.float64)
    Aq = sp.csr_matrix((q, a.col, a.rowptr), shape=(a.n, a.m))
    ref = Aq.T @ g.astype(np.float64)
    colsum = float(np.max(abs(Aq).sum(axis=0)))
    assert np.max(np.abs(yt - ref)) / (colsum * np.abs(g).max()) <= SPMV_TOL
    rp = torch.from_numpy(a.rowptr).to(DEV)
    gv = B.grad_values(A, rp, torch.from_numpy(g).to(DEV), torch.from_numpy(x).to(DEV))
    want = (g[a.rows()] * x[a.col]).astype(np.float32)
    assert np.array_equal(gv.cpu().numpy()[: a.nnz], want)


@pytest.mark.parametrize("k", [2, 4])
@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("fix", 20)])
def test_several_right_hand_sides(fmt, D, k):
    """k = 2 and 4 run the chunk product on k columns at once (x m x k, y
    n x k, row-major): each column equals the oracle's product, and the
    result repeats bit for bit."""
    for si, a in enumerate([hollow(13), W.powerlaw(20_000, seed=2)]):
        A, E = both(a, fmt, D, 256)
        x = np.random.default_rng(20 + si).uniform(-1, 1, (a.m, k)).astype(np.float32)
        xt = torch.from_numpy(x).to(DEV)
        y = B.spmv(A, xt)
        assert torch.equal(y, B.spmv(A, xt))
        y = y.cpu().numpy().astype(np.float64)
        q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
        for j in range(k):
            ref = PC.spmv(E, x[:, j].astype(np.float64))
            den = L.inf_norm(a.rowptr, q) * float(np.abs(x[:, j]).max())
            assert float(np.max(np.abs(y[:, j] - ref))) / den <= SPMV_TOL, (si, j)


def test_four_columns_from_a_misaligned_view():
    """A k = 4 product whose x is a contiguous view starting 4 bytes into its
    storage cannot take the chunk kernel's 16-byte gathers: it runs the
    one-row-slice product instead, and still equals the oracle per column."""
    a = hollow(17)
    A, E = both(a, "fp16", 15, 512)
    x = np.random.default_rng(21).uniform(-1, 1, (a.m, 4)).astype(np.float32)
    store = torch.zeros(a.m * 4 + 1, dtype=torch.float32, device=DEV)
    store[1:] = torch.from_numpy(x.reshape(-1)).to(DEV)
    xv = store[1:].view(a.m, 4)
    assert xv.is_contiguous() and xv.data_ptr() % 16 != 0
    y = B.spmv(A, xv).cpu().numpy().astype(np.float64)
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS["fp16"], 15)
    for j in range(4):
        ref = PC.spmv(E, x[:, j].astype(np.float64))
        den = L.inf_norm(a.rowptr, q) * float(np.abs(x[:, j]).max())
        assert np.max(np.abs(y[:, j] - ref)) / den <= SPMV_TOL
