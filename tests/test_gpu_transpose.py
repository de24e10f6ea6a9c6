"""GPU checks of the device CSR transpose and the PackSELL copy of A^T.

The transposed CSR must equal the numpy transpose bit for bit (row order
kept inside every column), the words of the encoded A^T must equal the
oracle's encoding of that transpose, and the forward product on it must
equal the oracle's A_q^T g within 1e-6 (normalised by the largest absolute
column sum of A_q times ||g||_inf).
"""
import ctypes

import numpy as np
import pytest
import torch

from helpers import FMTS, SPMV_TOL, random_csr
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def np_transpose(a):
    rows = a.rows()
    order = np.lexsort((rows, a.col))  # by column, then row
    t_rowptr = np.zeros(a.m + 1, np.int64)
    t_rowptr[1:] = np.cumsum(np.bincount(a.col, minlength=a.m))
    return t_rowptr, rows[order].astype(np.int32), a.val[order]


@pytest.mark.parametrize("shape", [(1, 1, 1.0), (37, 53, 0.2), (700, 300, 0.03), (300, 900, None),
                                   (2000, 2000, None)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_csr_transpose_exact(shape, dtype):
    n, m, dens = shape
    a = random_csr(21, n, m, density=dens) if dens else random_csr(21, n, m, per_row=9)
    val = a.val.astype(dtype)
    tr, tc, tv = B.csr_transpose(a.rowptr, a.col, val, a.n, a.m, DEV)
    er, ec, ev = np_transpose(W.csr_from_triplets(a.n, a.m, a.rows(), a.col, val))
    assert np.array_equal(tr.cpu().numpy(), er)
    assert np.array_equal(tc.cpu().numpy(), ec)
    assert np.array_equal(tv.cpu().numpy(), ev.astype(dtype))


def test_csr_transpose_edges():
    # no entries; empty rows and columns; one dense row
    z = W.csr_from_triplets(5, 7, [], [], [])
    tr, tc, tv = B.csr_transpose(z.rowptr, z.col, z.val, 5, 7, DEV)
    assert np.array_equal(tr.cpu().numpy(), np.zeros(8, np.int64)) and tc.numel() == 0
    r = np.zeros(40, np.int64) + 3
    c = np.arange(40)
    a = W.csr_from_triplets(6, 50, r, c, np.arange(40, dtype=np.float64) + 1)
    tr, tc, tv = B.csr_transpose(a.rowptr, a.col, a.val, a.n, a.m, DEV)
    er, ec, ev = np_transpose(a)
    assert np.array_equal(tr.cpu().numpy(), er) and np.array_equal(tc.cpu().numpy(), ec)
    assert np.array_equal(tv.cpu().numpy(), ev)


def test_csr_transpose_rejects_malformed():
    a = random_csr(22, 30, 30, per_row=4)
    bad_col = a.col.copy()
    bad_col[5] = 30  # column out of range
    with pytest.raises(B.PackSELLError):
        B.csr_transpose(a.rowptr, bad_col, a.val, a.n, a.m, DEV)
    bad_rp = a.rowptr.copy()
    bad_rp[-1] += 3  # rowptr past nnz
    with pytest.raises(B.PackSELLError):
        B.csr_transpose(bad_rp, a.col, a.val, a.n, a.m, DEV)


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9), ("e8my", 2), ("e8my", 20)])
@pytest.mark.parametrize("C,sigma", [(64, 256), (32, 65536), (8, 3)])
def test_encoded_transpose_words_and_adjoint(fmt, D, C, sigma):
    a = random_csr(23, 1500, 1100, per_row=11)
    At = B.encode_transpose(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, C, sigma, B.IMPLICIT, DEV)
    tr, tc, tv = np_transpose(a)
    E = P.encode(tr, tc, tv, a.m, a.n, FMTS[fmt], D, C, sigma, P.PERM_IMPLICIT)
    assert At.n_words == E.n_words
    assert np.array_equal(At.pack.cpu().numpy().view(np.uint32)[:At.n_words], E.pack)
    g = W.uniform_vector(a.n, 7)
    yt = B.spmv(At, torch.from_numpy(g).to(DEV)).cpu().numpy()
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
    ref = L.spmv_t(a.rowptr, a.col, q, g, a.m)
    colsum = np.bincount(a.col, weights=np.abs(q), minlength=a.m).max()
    assert np.max(np.abs(yt - ref)) / (colsum * np.abs(g).max()) <= SPMV_TOL


def test_encode_transpose_rejects_fix():
    a = random_csr(24, 20, 20, per_row=3)
    with pytest.raises(ValueError):
        B.encode_transpose(a.rowptr, a.col, a.val, a.n, a.m, "fix", 15, device=DEV)


def test_symmetric_laplacian_transpose_equals_itself():
    """The 7-point Laplacian 128^3 is symmetric (one coefficient per
    undirected edge), so its transposed encoding must reproduce its own
    words bit for bit."""
    a = W.m2_laplace3d(128)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, DEV)
    At = B.encode_transpose(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, DEV)
    assert At.n_words == A.n_words
    assert torch.equal(At.pack[:At.n_words], A.pack[:A.n_words])
    assert torch.equal(At.offset, A.offset)


def test_powerlaw_adjoint_full_size():
    """n = 1,000,000 power-law rows: the transposed copy's product against
    the oracle's A_q^T g."""
    a = W.m3_powerlaw()
    At = B.encode_transpose(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 65536, B.IMPLICIT, DEV,
                            split_words=256)
    g = W.uniform_vector(a.n, 8)
    yt = B.spmv(At, torch.from_numpy(g).to(DEV)).cpu().numpy()
    q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS["fp16"], 15)
    ref = L.spmv_t(a.rowptr, a.col, q, g, a.m)
    colsum = np.bincount(a.col, weights=np.abs(q), minlength=a.m).max()
    assert np.max(np.abs(yt - ref)) / (colsum * np.abs(g).max()) <= SPMV_TOL


def test_csr_transpose_query_sizes():
    """The workspace holds the sorted keys, two index arrays, the row map and
    the sort's own scratch (the sort sizes its scratch from the device)."""
    ws = ctypes.c_size_t()
    assert B.lib().pksell_csr_transpose_query(1000, 800, 12345, ctypes.byref(ws)) == B.OK
    assert ws.value >= 4 * 4 * 12345
    assert B.lib().pksell_csr_transpose_query(0, 0, 0, ctypes.byref(ws)) == B.OK
