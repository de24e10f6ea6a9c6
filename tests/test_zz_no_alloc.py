"""pksell_spmv_static (the entry point that allocates nothing) against
pksell_spmv, through the C ABI.

Products that need scratch (CSR-packed words with a chunk plan, k = 1, 2
and 4; split wide slices, k = 1) take it from the library's per-GPU array;
they must equal pksell_spmv's results bit for bit (the same kernels in the
same order), on two calls in a row with the second matrix smaller, so the
second product runs over what the first left in the array.  A product that
needs no scratch runs as pksell_spmv.  A product needing more scratch than
the array holds is refused before any device work.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _x(m, k, seed):
    x = W.uniform_vector(m, seed, k)
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def _same(A, k, seed):
    x = _x(A.m, k, seed)
    want = B.spmv(A, x)
    y = torch.full_like(want, float("nan"))
    before = torch.cuda.memory_allocated(DEV)
    got = B.spmv_static(A, x, y)
    torch.cuda.synchronize(DEV)
    assert torch.cuda.memory_allocated(DEV) == before
    assert got.data_ptr() == y.data_ptr()
    assert torch.equal(got, want)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_chunk_plan_products_big_then_small(k):
    big = W.powerlaw(300_000, seed=31)
    small = W.powerlaw(20_000, seed=32)
    for a, chunk in ((big, 256), (small, 512)):
        A = B.encode_packed_csr(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, chunk, DEV)
        assert A.n_units > 0
        _same(A, k, 40 + k)


def test_split_slices_big_then_small():
    big = W.powerlaw(200_000, seed=33)
    small = W.powerlaw(15_000, seed=34)
    for a in (big, small):
        A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 9, 64, 65536, B.IMPLICIT, DEV,
                     split_words=128)
        assert A.n_split_units > 0
        _same(A, 1, 50)


def test_products_without_scratch():
    a = W.m2_laplace3d(g=24)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, DEV)
    _same(A, 1, 60)
    _same(A, 8, 61)


def test_refuses_more_scratch_than_the_array_holds():
    d = B.CMatrix()
    d.n, d.m, d.C, d.sigma, d.fmt, d.D = 1000, 1000, 1, 1, B.FP16, 15
    d.split_words, d.n_units = 256, 1 << 22  # (2k + 1) * n_units floats > 2^22
    rc = B.lib().pksell_spmv_static(ctypes.byref(d), None, None, 1, None)
    assert rc == B.ERANGE
    assert b"scratch" in B.lib().pksell_last_error()
