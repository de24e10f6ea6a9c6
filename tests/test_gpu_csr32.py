"""GPU parity for the float32 CSR comparator balanced over entry chunks.

Its product must equal the oracle's float64 CSR product on the same
float32-rounded values within 1e-6, normalised by ||A||_inf ||x||_inf
(float32 sums in a different order), repeat bit for bit, and write 0 to
empty rows.  The plan (the first row starting in each chunk) must equal the
one read off the row pointer by a plain search.
"""
import numpy as np
import pytest
import torch

from helpers import SPMV_TOL, normalised_error, random_csr
from oracle import linalg as L
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def check(a, T, seed=0):
    A = B.csr32_encode(a.rowptr, a.col, a.val, a.n, a.m, T, DEV)
    nch = -(-a.nnz // T)
    assert A.n_chunks == nch
    lo = A.t["lo"].cpu().numpy().astype(np.int64)
    want = np.searchsorted(a.rowptr[:-1], np.arange(nch, dtype=np.int64) * T, side="left")
    assert np.array_equal(lo[:nch], want) and lo[nch] == a.n
    x = np.random.default_rng(seed).uniform(-1, 1, a.m).astype(np.float32)
    xd = torch.from_numpy(x).to(DEV)
    y = B.csr32_spmv(A, xd)
    v32 = a.val.astype(np.float32).astype(np.float64)
    ref = L.spmv(a.rowptr, a.col, v32, x.astype(np.float64))
    assert normalised_error(y.cpu().numpy(), ref, a, v32, x) <= SPMV_TOL
    assert torch.equal(y, B.csr32_spmv(A, xd))  # deterministic
    return A, y


@pytest.mark.parametrize("T", [256, 512, 1024])
def test_random(T):
    for si, (n, m, kw) in enumerate([(37, 53, dict(density=0.2)), (700, 650, dict(density=0.03)),
                                     (2500, 3000, dict(per_row=11)),
                                     (3000, 2000, dict(density=0.002))]):
        check(random_csr(80 + si, n, m, **kw), T, si)


def test_rows_across_many_chunks_and_empty_rows():
    """Rows of thousands of entries (each spans several chunks), rows that
    end exactly on a chunk boundary, and empty rows between them."""
    rng = np.random.default_rng(5)
    n, m = 400, 20000
    lens = rng.integers(0, 12, n)
    lens[::37] = 0
    lens[5], lens[77], lens[301] = 5000, 2300, 4096
    rows = np.repeat(np.arange(n), lens)
    cols = np.concatenate([np.sort(rng.choice(m, size=k, replace=False)) for k in lens])
    a = W.csr_from_triplets(n, m, rows, cols, rng.standard_normal(rows.size))
    for T in (256, 512, 1024):
        _, y = check(a, T, T)
        assert not y.cpu().numpy()[lens == 0].any()
    # a row ending exactly at a chunk boundary
    b = W.csr_from_triplets(3, 600, [0] * 512 + [1] * 3 + [2] * 509,
                            list(range(512)) + [1, 2, 3] + list(range(509)),
                            np.ones(1024))
    check(b, 512, 1)


def test_powerlaw():
    check(W.powerlaw(200_000, seed=7), 512, 3)


def test_powerlaw_1m_full_size():
    """The 1M-row power-law matrix at the benchmark's chunk size."""
    check(W.m3_powerlaw(), 512, 41)


def test_edges():
    empty = W.csr_from_triplets(0, 0, [], [], [])
    A = B.csr32_encode(empty.rowptr, empty.col, empty.val, 0, 0, 512, DEV)
    assert B.csr32_spmv(A, torch.zeros(0, device=DEV)).numel() == 0
    hollow = W.csr_from_triplets(70, 10, [], [], [])  # no entries: y = 0
    A = B.csr32_encode(hollow.rowptr, hollow.col, hollow.val, 70, 10, 256, DEV)
    assert not B.csr32_spmv(A, torch.ones(10, device=DEV), torch.ones(70, device=DEV)).any()
    a = random_csr(3, 50, 40, per_row=4)
    with pytest.raises(B.PackSELLError):
        B.csr32_encode(a.rowptr, a.col, a.val, a.n, a.m, 300, DEV)
