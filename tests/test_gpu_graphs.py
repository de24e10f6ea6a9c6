"""Products captured in HIP graphs and replayed several times, with eager
work on the inputs (and outputs) between the replays; every replay must
equal the eager product of the same inputs, bit for bit (up to float32
rounding where atomics add in no fixed order).  The captured paths
zero their outputs with kernels, never with memset nodes: the transposed
batched plan, the atomic adjoint, split products (chunk sums combined by a
second kernel), 16-bit words, CSR-packed chunk products (cross-chunk rows
summed by a second kernel) and level-scheduled triangular solves (one
launch per level)."""
import numpy as np
import pytest
import torch

from helpers import random_csr
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
REPLAYS = 4


def replay_and_check(run, inputs, outputs, eager):
    """Capture ``run``; then, per replay, scale the inputs and scribble on
    the outputs eagerly, replay, and compare with ``eager()``."""
    run()  # warm up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(REPLAYS):
        with torch.no_grad():
            for x in inputs:
                x.mul_(-1.25).add_(0.5)
            for y in outputs:
                y.fill_(7.0)  # a replay must overwrite (or re-zero) every output
        g.replay()
        torch.cuda.synchronize()
        got = [y.clone() for y in outputs]
        want = eager()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a, b), (rep, i)


def test_batched_transpose_replays():
    mats = W.m5_batch(count=6, n_lo=300, n_hi=20_000, seed=4)
    enc = [B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 9, 64, 256, B.IMPLICIT, DEV)
           for a in mats]
    gs = [torch.from_numpy(W.uniform_vector(a.n, i, k=8)).to(DEV) for i, a in enumerate(mats)]
    outs = [torch.empty((a.m, 8), device=DEV) for a in mats]
    bat = B.BatchedSpMV(enc, gs, outs, transpose=True)

    def eager():
        return [B.spmv_t(A, g) for A, g in zip(enc, gs)]

    run = bat
    run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(REPLAYS):
        with torch.no_grad():
            for x in gs:
                x.mul_(-1.25).add_(0.5)
            for y in outs:
                y.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        ref = eager()
        for i, (o, r) in enumerate(zip(outs, ref)):
            # float32 atomics add in no fixed order: equal up to rounding
            den = float(r.abs().max()) + 1e-30
            assert float((o - r).abs().max()) / den <= 1e-5, (rep, i)


def test_spmv_t_replays():
    a = random_csr(21, 3000, 2600, per_row=9)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, DEV)
    g = torch.from_numpy(W.uniform_vector(a.n, 2)).to(DEV)
    y = torch.empty(a.m, device=DEV)
    run = lambda: B.spmv_t(A, g, y)
    run()
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        run()
    for rep in range(REPLAYS):
        with torch.no_grad():
            g.mul_(-1.25).add_(0.5)
            y.fill_(7.0)
        gr.replay()
        torch.cuda.synchronize()
        ref = B.spmv_t(A, g)
        den = float(ref.abs().max()) + 1e-30
        assert float((y - ref).abs().max()) / den <= 1e-5, rep


def test_split_product_replays():
    a = W.m3_powerlaw(n=20_000, seed=5)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 4096, B.IMPLICIT, DEV,
                 split_words=64)
    assert A.n_split_units > 0
    x = torch.from_numpy(W.uniform_vector(a.m, 4)).to(DEV)
    y = torch.empty(a.n, device=DEV)
    replay_and_check(lambda: B.spmv(A, x, y), [x], [y], lambda: [B.spmv(A, x)])


@pytest.mark.parametrize("fmt,D", [("e5my", 7), ("fix16", 9)])
def test_16_bit_words_replays(fmt, D):
    a = random_csr(22, 4000, 3500, per_row=10)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, B.IMPLICIT, DEV)
    x = torch.from_numpy(W.uniform_vector(a.m, 6)).to(DEV)
    y = torch.empty(a.n, device=DEV)
    replay_and_check(lambda: B.spmv(A, x, y), [x], [y], lambda: [B.spmv(A, x)])


def test_half_value_sell_replays():
    a = random_csr(23, 4000, 3500, per_row=10)
    S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float16, 64, 256, B.IMPLICIT, DEV)
    x = torch.from_numpy(W.uniform_vector(a.m, 7)).to(DEV)
    y = torch.empty(a.n, device=DEV)
    replay_and_check(lambda: B.sell_spmv(S, x, y), [x], [y], lambda: [B.sell_spmv(S, x)])


def test_packed_csr_product_replays():
    """The chunk-balanced product writes its cross-chunk pieces to the
    matrix's scratch and sums them in a second kernel: both in the graph."""
    a = W.m3_powerlaw(n=30_000, seed=6)
    A = B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 256, DEV)
    assert A.desc.n_units > 1
    x = torch.from_numpy(W.uniform_vector(a.m, 9)).to(DEV)
    y = torch.empty(a.n, device=DEV)
    replay_and_check(lambda: B.spmv(A, x, y), [x], [y], lambda: [B.spmv(A, x)])


def test_triangular_solve_replays():
    """One launch per level, all captured; y is scribbled on between replays."""
    import scipy.sparse as sp
    a = W.m2_laplace3d(24)
    L = sp.tril(sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.m))).tocsr()
    L.sort_indices()
    for fmt in ("fp16", None):
        S = B.TriangularSolve(L.indptr.astype(np.int64), L.indices.astype(np.int32), L.data, a.n,
                              fmt, 15, DEV)
        b = torch.from_numpy(W.uniform_vector(a.n, 10)).to(DEV)
        y = torch.empty(a.n, device=DEV)
        replay_and_check(lambda: S(b, y), [b], [y], lambda: [S(b)])
