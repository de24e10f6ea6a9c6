"""GPU checks of wide-slice splitting for the single-vector product.

The unit and split tables must equal a host recount from the oracle's slice
offsets, the chunk checkpoints must equal the column the oracle's sec. 4.4
walk reaches before each chunk's first word (bit for bit), the words
themselves must not change, and the split product must agree with the
oracle's float64 product within 1e-6 (normalised).
"""
import numpy as np
import pytest
import torch

from helpers import FMTS, SPMV_TOL, normalised_error, oracle_product
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def skewed_csr(seed, n=3000, m=4000, long_rows=(0, 7, 100, 1500, 2999), long_len=1900):
    """Short rows (0..12 entries) plus a few very long ones, so some slices
    are many chunks wide and most are one unit."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = long_len if i in long_rows else int(rng.integers(0, 13))
        c = np.sort(rng.choice(m, size=min(k, m), replace=False))
        rows.append(np.full(c.size, i))
        cols.append(c)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    return W.csr_from_triplets(n, m, r, c, rng.standard_normal(r.size))


def expected_tables(offset, J):
    w = (offset[1:] - offset[:-1]) // 64
    units, splits, base = [], [], 0
    for k, wk in enumerate(w):
        if wk > J:
            ch = -(-int(wk) // J)
            units += [(k, c, ch, base) for c in range(ch)]
            splits.append((k, base, ch, 0))
            base += ch
        else:
            units.append((k, 0, 1, 0))
    return np.array(units, np.int64).reshape(-1, 4), np.array(splits, np.int64).reshape(-1, 4), base


def u32(t, count):
    return t.cpu().numpy().view(np.uint32)[:count].astype(np.int64)


def check_split(a, fmt, D, sigma, J, mode=B.IMPLICIT, seed=1):
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, sigma, mode, DEV, split_words=J)
    E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D, 64, sigma, mode)
    assert np.array_equal(A.pack.cpu().numpy().view(np.uint32)[:A.n_words], E.pack)
    units, splits, n_split_units = expected_tables(E.offset, J)
    assert (A.n_units, A.n_split_units, A.n_split_slices) == (len(units), n_split_units, len(splits))
    assert n_split_units > 0
    assert np.array_equal(u32(A.t["units"], 4 * len(units)).reshape(-1, 4), units)
    assert np.array_equal(u32(A.t["splits"], 4 * len(splits)).reshape(-1, 4), splits)
    # checkpoints: the column reached before word c*J of each lane
    x = W.uniform_vector(a.m, seed)
    _, cols, _ = P.spmv_algorithm(E, x, return_trace=True)
    ck = u32(A.t["ckpt"], 64 * n_split_units).reshape(-1, 64)
    left = P.left_offsets(a.n, sigma, E.k_left)
    for k, base, ch, _ in splits:
        for lane in range(64):
            t = k * 64 + lane
            if t >= a.n:
                continue
            assert ck[base, lane] == left[t]
            for c in range(1, ch):
                assert ck[base + c, lane] == cols[E.offset[k] + (c * J - 1) * 64 + lane], (k, c, lane)
    xt = torch.from_numpy(x).to(DEV)
    y = B.spmv(A, xt).cpu().numpy()
    ref, q = oracle_product(a, FMTS[fmt], D, x)
    if mode == B.EXPLICIT:
        ref = ref[E.stored_rows]
    assert normalised_error(y, ref, a, q, x) <= SPMV_TOL
    return A, y


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 13), ("e8my", 4), ("fix", 20)])
@pytest.mark.parametrize("J", [8, 64, 256])
def test_split_tables_ckpt_and_product(fmt, D, J):
    check_split(skewed_csr(2), fmt, D, 256, J)


@pytest.mark.parametrize("sigma,mode", [(1, B.IMPLICIT), (300, B.IMPLICIT), (65536, B.EXPLICIT),
                                        (4096, B.EXPLICIT)])
def test_split_sigma_and_modes(sigma, mode):
    check_split(skewed_csr(5, n=2500, m=2500), "e8my", 9, sigma, 64, mode)


def test_split_matches_unsplit_closely_and_is_deterministic():
    a = skewed_csr(8)
    x = torch.from_numpy(W.uniform_vector(a.m, 3)).to(DEV)
    A0 = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, DEV)
    A1 = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, DEV,
                  split_words=32)
    y0 = B.spmv(A0, x)
    y1 = B.spmv(A1, x)
    scale = float(y0.abs().max())
    assert float((y0 - y1).abs().max()) <= 1e-5 * scale
    for _ in range(3):
        assert torch.equal(B.spmv(A1, x), y1)
    # multi-vector products ignore the split tables
    X = torch.from_numpy(W.uniform_vector(a.m, 4, k=4)).to(DEV)
    assert torch.equal(B.spmv(A1, X), B.spmv(A0, X))


def test_split_off_when_no_slice_is_wide():
    a = skewed_csr(9, long_rows=())
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, DEV,
                 split_words=64)
    assert A.n_split_units == 0 and A.n_units == A.desc.n_slices
    assert "units" not in A.t
    x = torch.from_numpy(W.uniform_vector(a.m, 1)).to(DEV)
    A0 = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, DEV)
    assert torch.equal(B.spmv(A, x), B.spmv(A0, x))


def test_split_rejects_bad_words():
    a = skewed_csr(10, n=300, m=300, long_rows=(5,), long_len=200)
    for J, C in [(12, 64), (4, 64), (64, 32)]:
        with pytest.raises(B.PackSELLError):
            B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, C, 256, B.IMPLICIT, DEV,
                     split_words=J)


def test_m3_powerlaw_split_full_size():
    """n = 1,000,000 power-law rows (max 5000 entries), FP16, sigma = 65536,
    J = 256, against the oracle's full float64 product."""
    a = W.m3_powerlaw()
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 65536, B.IMPLICIT, DEV,
                 split_words=256)
    assert A.n_split_units > 0
    x = W.uniform_vector(a.m, 5)
    y = B.spmv(A, torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref, q = oracle_product(a, FMTS["fp16"], 15, x)
    assert normalised_error(y, ref, a, q, x) <= SPMV_TOL
