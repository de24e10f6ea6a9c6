"""GPU checks of the batched persistent product (many matrices, k RHS).

Each batched output must equal the single-matrix product bit for bit (the
same arithmetic in the same word order) and the oracle's float64 product
within 1e-6 (normalised).  Graph replays are checked against eager results
with the program's own eager work between replays.
"""
import numpy as np
import pytest
import torch

from helpers import SPMV_TOL, normalised_error, oracle_product
from oracle import formats as F
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def small_batch(count=10, seed=3):
    return W.m5_batch(count=count, n_lo=300, n_hi=40_000, seed=seed)


def encode_all(mats, D_of=lambda i: 9, fmt="e8my"):
    return [B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D_of(i), 64, 256, B.IMPLICIT, DEV)
            for i, a in enumerate(mats)]


@pytest.mark.parametrize("k", [1, 3, 8, 12, 32, 13, 64])
def test_batched_matches_single_and_oracle(k):
    mats = small_batch()
    enc = encode_all(mats, D_of=lambda i: [9, 12, 3][i % 3])
    xs = [torch.from_numpy(W.uniform_vector(a.m, 100 + i, k=k)).to(DEV) for i, a in enumerate(mats)]
    ys = [torch.full((a.n,) if k == 1 else (a.n, k), float("nan"), device=DEV) for a in mats]
    B.BatchedSpMV(enc, xs, ys)()
    torch.cuda.synchronize()
    for i, (a, A) in enumerate(zip(mats, enc)):
        single = B.spmv(A, xs[i])
        assert torch.equal(ys[i], single), i
        ref, q = oracle_product(a, F.FMT_E8MY, A.D, xs[i].cpu().numpy())
        assert normalised_error(ys[i].cpu().numpy(), ref, a, q, xs[i].cpu().numpy()) <= SPMV_TOL


def test_batched_fp16_and_fix():
    mats = small_batch(6, 5)
    for fmt, D in [("fp16", 15), ("fix", 15)]:
        enc = encode_all(mats, D_of=lambda i: D, fmt=fmt)
        xs = [torch.from_numpy(W.uniform_vector(a.m, i, k=8)).to(DEV) for i, a in enumerate(mats)]
        ys = [torch.empty((a.n, 8), device=DEV) for a in mats]
        B.BatchedSpMV(enc, xs, ys)()
        for i, A in enumerate(enc):
            assert torch.equal(ys[i], B.spmv(A, xs[i]))


def test_graph_replays_follow_inputs():
    mats = small_batch(8, 9)
    enc = encode_all(mats)
    xs = [torch.from_numpy(W.uniform_vector(a.m, i, k=8)).to(DEV) for i, a in enumerate(mats)]
    ys = [torch.empty((a.n, 8), device=DEV) for a in mats]
    bat = B.BatchedSpMV(enc, xs, ys).capture()
    for rep in range(4):
        with torch.no_grad():
            for x in xs:
                x.mul_(-1.5)  # eager work between replays
        bat.replay()
        torch.cuda.synchronize()
        for i, A in enumerate(enc):
            assert torch.equal(ys[i], B.spmv(A, xs[i])), (rep, i)


@pytest.mark.parametrize("k", [1, 8])
def test_batched_transpose(k):
    mats = small_batch(7, 11)
    enc = encode_all(mats)
    gs = [torch.from_numpy(W.uniform_vector(a.n, 50 + i, k=k)).to(DEV) for i, a in enumerate(mats)]
    outs = [torch.full((a.m,) if k == 1 else (a.m, k), 7.0, device=DEV) for a in mats]
    bat = B.BatchedSpMV(enc, gs, outs, transpose=True).capture()
    for rep in range(2):
        bat.replay()
        torch.cuda.synchronize()
        for i, (a, A) in enumerate(zip(mats, enc)):
            # the oracle's float64 A_q^T g on the same quantised values,
            # normalised by the largest column sum of |A_q| times max |g|
            q = P.quantized_values(a.rowptr, a.col, a.val, a.n, F.FMT_E8MY, A.D)
            g = gs[i].cpu().numpy().astype(np.float64).reshape(a.n, k)
            got = outs[i].cpu().numpy().astype(np.float64).reshape(a.m, k)
            colsum = float(np.bincount(a.col, weights=np.abs(q), minlength=a.m).max())
            for j in range(k):
                ref = L.spmv_t(a.rowptr, a.col, q, g[:, j], a.m)
                err = float(np.max(np.abs(got[:, j] - ref)))
                assert err <= SPMV_TOL * colsum * float(np.abs(g[:, j]).max()), (rep, i, j)


def test_m5_full_size_k8():
    """64 stencils, n log-uniform in [1e4, 5e5], E8M13, k = 8."""
    mats = W.m5_batch()
    enc = encode_all(mats)
    xs = [torch.from_numpy(W.uniform_vector(a.m, i, k=8)).to(DEV) for i, a in enumerate(mats)]
    ys = [torch.empty((a.n, 8), device=DEV) for a in mats]
    B.BatchedSpMV(enc, xs, ys).capture().replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for i in rng.choice(len(mats), 8, replace=False):
        a, A = mats[i], enc[i]
        x = xs[i].cpu().numpy()
        ref, q = oracle_product(a, F.FMT_E8MY, 9, x)
        assert normalised_error(ys[i].cpu().numpy(), ref, a, q, x) <= SPMV_TOL


def test_k1_two_slice_path_mixed_orders_and_empty():
    """k = 1 forward plans run the two-slice kernel over slice pairs: FP16,
    E8MY and FIX words, implicit and explicit row orders and an empty matrix
    in one batch, each output equal to its single-matrix product bit for
    bit; a transposed plan of the same batch keeps the persistent loop."""
    mats = small_batch(7, 11)
    mats.insert(3, W.csr_from_triplets(0, 0, [], [], []))
    for fmt, D in [("fp16", 15), ("e8my", 9), ("fix", 15)]:
        enc = [B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256,
                        B.EXPLICIT if i % 2 else B.IMPLICIT, DEV) for i, a in enumerate(mats)]
        xs = [torch.from_numpy(W.uniform_vector(a.m, 40 + i)).to(DEV) for i, a in enumerate(mats)]
        ys = [torch.full((a.n,), float("nan"), device=DEV) for a in mats]
        run = B.BatchedSpMV(enc, xs, ys)
        assert run.plan.pair_units == sum((A.desc.n_slices + 1) // 2 for A in enc)
        run()
        for i, A in enumerate(enc):
            assert torch.equal(ys[i], B.spmv(A, xs[i])), (fmt, i)
        tr = B.BatchedSpMV(enc, [torch.ones(a.n, device=DEV) for a in mats],
                           [torch.empty(a.m, device=DEV) for a in mats], transpose=True)
        assert tr.plan.pair_units == 0


def test_m5_full_size_k1():
    """64 stencils at k = 1 (the two-slice path): every output equal to the
    single-matrix product bit for bit, graph replay included."""
    mats = W.m5_batch()
    enc = encode_all(mats)
    xs = [torch.from_numpy(W.uniform_vector(a.m, i)).to(DEV) for i, a in enumerate(mats)]
    ys = [torch.empty(a.n, device=DEV) for a in mats]
    run = B.BatchedSpMV(enc, xs, ys).capture()
    run.replay()
    torch.cuda.synchronize()
    for i, A in enumerate(enc):
        assert torch.equal(ys[i], B.spmv(A, xs[i])), i
