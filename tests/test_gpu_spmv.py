"""GPU parity: encoder words, decoded columns and SpMV against the oracle.

Encoded words, offsets, perm and decoded columns must match the oracle bit
for bit; products must agree with the oracle's float64 product on the same
quantised values within 1e-6, normalised by ||A_q||_inf ||x||_inf.
"""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

from helpers import FMTS, SPMV_TOL, normalised_error, oracle_product, random_csr
from oracle import formats as F
from oracle import linalg as L
from oracle import packsell as P
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def words(A):
    return A.pack.cpu().numpy().view(np.uint32)[:A.n_words]


def both(a, fmt, D, C, sigma, mode=B.IMPLICIT):
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, C, sigma, mode, DEV)
    E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D, C, sigma, mode)
    return A, E


def assert_same_encoding(A, E):
    assert A.k_left == E.k_left
    assert A.n_dummies == E.n_dummies
    assert A.n_words == E.n_words
    assert np.array_equal(A.offset.cpu().numpy(), E.offset)
    assert np.array_equal(words(A), E.pack)
    if A.perm is not None and A.n:
        assert np.array_equal(A.perm.cpu().numpy()[:A.n].astype(np.int64),
                              E.perm.astype(np.int64))
    if E.row_exp is not None and A.n:
        assert np.array_equal(A.row_exp.cpu().numpy()[:A.n].astype(np.int64), E.row_exp)


def check_spmv(A, a, fmt, D, x, mode, E):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    y = B.spmv(A, xt).cpu().numpy()
    ref, q = oracle_product(a, FMTS[fmt], D, x)
    if mode == B.EXPLICIT:
        ref = ref[E.stored_rows]
    err = normalised_error(y, ref, a, q, x)
    assert err <= SPMV_TOL, err
    return err


def test_fixture_4x8():
    with open(os.path.join(GOLD, "fixture_4x8_e8m20.json")) as f:
        fx = json.load(f)
    r, c, v = [], [], []
    for i, row in enumerate(fx["rows"]):
        for j, val in row:
            r.append(i), c.append(j), v.append(val)
    a = W.csr_from_triplets(fx["n"], fx["m"], r, c, v)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", 2, 2, 2, B.IMPLICIT, DEV)
    assert A.k_left == fx["k_left"] and A.n_dummies == fx["n_dummies"]
    assert list(A.offset.cpu().numpy()) == fx["offset"]
    assert [int(w) for w in words(A)] == [int(h, 16) for h in fx["pack"]]
    assert list(A.perm.cpu().numpy()[:4]) == fx["perm"]
    cols, _ = B.decode(A)
    assert list(cols.cpu().numpy()) == fx["decoded_columns"]
    y = B.spmv(A, torch.tensor(fx["x"], dtype=torch.float32, device=DEV)).cpu().numpy()
    assert list(y) == fx["y"]
    yt = B.spmv_t(A, torch.ones(4, dtype=torch.float32, device=DEV)).cpu().numpy()
    assert list(yt) == fx["At_ones"]


CASES = [("fp16", 15), ("e8my", 1), ("e8my", 2), ("e8my", 9), ("e8my", 12), ("e8my", 22),
         ("fix", 15), ("fix", 4)]
SHAPES = [(1, 1, 1.0), (37, 53, 0.2), (300, 280, 0.05), (1000, 777, None), (2500, 4000, None)]


@pytest.mark.parametrize("fmt,D", CASES)
@pytest.mark.parametrize("C,sigma", [(64, 256), (32, 256), (2, 2), (64, 1), (16, 4096), (8, 3)])
def test_random_parity(fmt, D, C, sigma):
    for si, (n, m, dens) in enumerate(SHAPES):
        a = random_csr(1000 * D + 7 * C + si, n, m, density=dens, per_row=None if dens else 9)
        x = W.uniform_vector(m, si + 1)
        for mode in (B.IMPLICIT, B.EXPLICIT):
            A, E = both(a, fmt, D, C, sigma, mode)
            assert_same_encoding(A, E)
            check_spmv(A, a, fmt, D, x, mode, E)
        # decoded columns and values, word by word (positions of real rows)
        _, tr_cols, tr_vals = P.spmv_algorithm(E, x, return_trace=True)
        cols, vals = B.decode(A)
        word_row = np.full(E.n_words, -1)
        for t in range(a.n):
            k, l = divmod(t, C)
            word_row[E.offset[k] + l:E.offset[k + 1]:C] = t
        live = word_row >= 0
        assert np.array_equal(cols.cpu().numpy()[live], tr_cols[live])
        dv = vals.cpu().numpy().astype(np.float64)[live]
        ref_v = tr_vals[live]
        if FMTS[fmt] == F.FMT_FIX:
            # the oracle trace holds the integer q; the decoder applies 2^e
            ref_v = np.ldexp(ref_v, E.row_exp[word_row[live]])
        assert np.array_equal(dv, ref_v)


@pytest.mark.parametrize("k", [2, 3, 4, 8, 12, 13, 16, 20, 32, 36, 64])
def test_multiple_rhs(k):
    a = random_csr(5, 700, 650, density=0.02)
    X = W.uniform_vector(a.m, 9, k=k)
    for fmt, D in [("fp16", 15), ("e8my", 9), ("fix", 15)]:
        A, E = both(a, fmt, D, 64, 256)
        Y = B.spmv(A, torch.from_numpy(X).to(DEV)).cpu().numpy()
        ref, q = oracle_product(a, FMTS[fmt], D, X)
        assert normalised_error(Y, ref, a, q, X) <= SPMV_TOL


@pytest.mark.parametrize("k", [8, 12, 20, 32, 64])
def test_lane_groups_equal_single_vector_products(k):
    """k a multiple of 4 (lane groups of 2..16 lanes per row): every column
    of the block product equals the one-vector product of that column bit
    for bit -- the same words, decoded values and FMA order."""
    a = random_csr(6, 1500, 1400, density=0.01)
    A, _ = both(a, "e8my", 9, 64, 256)
    X = torch.from_numpy(W.uniform_vector(a.m, 10, k=k)).to(DEV)
    Y = B.spmv(A, X)
    for r in range(k):
        assert torch.equal(Y[:, r], B.spmv(A, X[:, r].contiguous())), r


@pytest.mark.parametrize("k", [32, 64])
def test_lane_groups_wide_window(k):
    """A 96^3 7-point Laplacian (k_left = 9216, implicit order): at k = 32
    and 64 the x rows one sigma-block reads span several MiB.  Every column
    equals the one-vector product bit for bit, and the oracle's within the
    bar."""
    a = W.m2_laplace3d(96)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.IMPLICIT, DEV)
    assert A.k_left == 96 * 96
    X = torch.from_numpy(W.uniform_vector(a.m, 11, k=k)).to(DEV)
    Y = B.spmv(A, X)
    for r in (0, 1, 27, 28, 31, k - 1):
        assert torch.equal(Y[:, r], B.spmv(A, X[:, r].contiguous())), r
    cols = [0, 28, k - 1]
    ref, q = oracle_product(a, F.FMT_FP16, 15, X[:, cols].cpu().numpy())
    assert normalised_error(Y[:, cols].cpu().numpy(), ref, a, q, X[:, cols].cpu().numpy()) <= SPMV_TOL


def test_m1_poisson_fp16():
    a = W.m1_poisson2d()
    x = W.uniform_vector(a.m, 1)
    for C in (64, 32):
        A, E = both(a, "fp16", 15, C, 256)
        assert_same_encoding(A, E)
        assert A.n_dummies == 0 and A.k_left == 64
        check_spmv(A, a, "fp16", 15, x, B.IMPLICIT, E)


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9)])
def test_m2_laplace3d_full_size(fmt, D):
    """3D 7-point 128^3 (n = 2,097,152; nnz = 14,581,760) at the launch
    configuration the benchmark times (C = 64, sigma = 256, implicit)."""
    a = W.m2_laplace3d()
    x = W.uniform_vector(a.m, 3)
    A, E = both(a, fmt, D, 64, 256)
    assert_same_encoding(A, E)
    check_spmv(A, a, fmt, D, x, B.IMPLICIT, E)


def sell_values(val, dt):
    """The values a SELL matrix of value type dt holds, in float64: float32
    and half values are rounded from float32 (float64 input rounded to
    float32 first), ties to even."""
    if dt == torch.float64:
        return np.asarray(val, np.float64)
    v32 = np.asarray(val).astype(np.float32)
    return (v32.astype(np.float16) if dt == torch.float16 else v32).astype(np.float64)


@pytest.mark.parametrize("C", [64, 32])
def test_sell_fp32_fp64_fp16(C):
    a = random_csr(3, 3000, 2500, per_row=12)
    x = W.uniform_vector(a.m, 4)
    for dt in (torch.float32, torch.float64, torch.float16):
        vdt = torch.float64 if dt == torch.float64 else torch.float32  # vector dtype
        for mode in (B.IMPLICIT, B.EXPLICIT):
            S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, dt, C, 256, mode, DEV)
            assert S.value_dtype == dt and S.dtype == vdt
            y = B.sell_spmv(S, torch.from_numpy(x.astype(np.float64)).to(DEV, vdt)).cpu().numpy()
            vals = sell_values(a.val, dt)
            ref = L.spmv(a.rowptr, a.col, vals, x)
            if mode == B.EXPLICIT:
                # SELL sorts rows by nonzero count; PackSELL with deltas that
                # never overflow (D = 22 > log2 m) has the same counts
                E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, F.FMT_E8MY, 22, C, 256, mode)
                assert E.n_dummies == 0
                ref = ref[E.stored_rows]
            tol = 1e-14 if dt == torch.float64 else SPMV_TOL
            assert normalised_error(y, ref, a, vals, x) <= tol


def test_sell_fp16_matches_packsell_fp16_laplace3d_128():
    """SELL with half values holds the same values as the FP16 PackSELL
    words (both round float32 to binary16, ties to even) and sums them with
    the same fused multiply-adds in the same order, so on the 128^3
    Laplacian at the benchmark's launch configuration (C = 64, sigma = 256,
    explicit order) the two products are bit-identical (the equivalence
    behind the paper's identical convergence of its FP16 SELL and PackSELL
    solvers, sec. 5.2.1); both are checked against the oracle."""
    a = W.m2_laplace3d()
    x = W.uniform_vector(a.m, 3)
    xd = torch.from_numpy(x).to(DEV)
    S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float16, 64, 256, B.EXPLICIT, DEV)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 15, 64, 256, B.EXPLICIT, DEV)
    ys = B.sell_spmv(S, xd).cpu().numpy().astype(np.float64)
    yp = B.spmv(A, xd).cpu().numpy().astype(np.float64)
    vals = sell_values(a.val, torch.float16)
    E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, F.FMT_FP16, 15, 64, 256, P.PERM_EXPLICIT)
    ref = L.spmv(a.rowptr, a.col, vals, x)[E.stored_rows]
    assert normalised_error(ys, ref, a, vals, x) <= SPMV_TOL
    assert normalised_error(yp, ref, a, vals, x) <= SPMV_TOL
    assert np.array_equal(ys, yp)
    # implicit order (the solvers' layout) and the one-slice-per-wave kernels
    # (27 words per lane on the 27-point stencil) give identical results too
    for g, mode in ((W.m2_laplace3d(), B.IMPLICIT), (W.m4_stencil27(48), B.IMPLICIT),
                    (W.m4_stencil27(48), B.EXPLICIT)):
        xg = torch.from_numpy(W.uniform_vector(g.m, 4)).to(DEV)
        Sg = B.sell_encode(g.rowptr, g.col, g.val, g.n, g.m, torch.float16, 64, 256, mode, DEV)
        Ag = B.encode(g.rowptr, g.col, g.val, g.n, g.m, "fp16", 15, 64, 256, mode, DEV)
        assert torch.equal(B.sell_spmv(Sg, xg), B.spmv(Ag, xg)), (g.n, mode)
    # bytes: 6 per SELL slot (int32 column + half) against 4 per word
    assert S.n_slots == A.n_words


def test_spmv_t_and_grad_values():
    a = random_csr(8, 1200, 900, per_row=10)
    g = W.uniform_vector(a.n, 5)
    x = W.uniform_vector(a.m, 6)
    for fmt, D in [("fp16", 15), ("e8my", 9), ("e8my", 1), ("fix", 15)]:
        A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, B.IMPLICIT, DEV)
        q = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
        yt = B.spmv_t(A, torch.from_numpy(g).to(DEV)).cpu().numpy()
        ref = L.spmv_t(a.rowptr, a.col, q, g, a.m)
        # normalised by ||A_q^T||_inf ||g||_inf (largest absolute column sum)
        colsum = np.bincount(a.col, weights=np.abs(q), minlength=a.m).max()
        assert np.max(np.abs(yt - ref)) / (colsum * np.abs(g).max()) <= SPMV_TOL
        gv = B.grad_values(A, torch.from_numpy(a.rowptr).to(DEV), torch.from_numpy(g).to(DEV),
                           torch.from_numpy(x).to(DEV)).cpu().numpy()
        # one float32 product per entry: exact to the float32 rounding of g_i x_j
        assert np.array_equal(gv, (g[a.rows()] * x[a.col]).astype(np.float32))


def test_edge_shapes():
    # empty matrix, all-empty rows, one column, tall matrix with empty rows
    cases = [W.csr_from_triplets(0, 0, [], [], []),
             W.csr_from_triplets(100, 50, [], [], []),
             W.csr_from_triplets(70, 1, np.arange(0, 70, 3), np.zeros(24, int), np.ones(24)),
             W.csr_from_triplets(300, 5, [0, 1, 2, 3, 4], [0, 1, 2, 3, 4], [1., 2, 3, 4, 5])]
    for a in cases:
        x = W.uniform_vector(max(a.m, 1), 2)[:a.m]
        for fmt, D in [("fp16", 15), ("e8my", 3)]:
            for sigma in (1, 64):
                A, E = both(a, fmt, D, 64, sigma)
                assert_same_encoding(A, E)
                y = B.spmv(A, torch.from_numpy(x).to(DEV)).cpu().numpy()
                ref, q = oracle_product(a, FMTS[fmt], D, x)
                # at most one product per row: float32 rounding of the exact value
                assert np.array_equal(y, ref.astype(np.float32)), (a.n, a.m, fmt, sigma)


def test_errors_from_device_checks():
    a = W.csr_from_triplets(3, 5, [0, 0, 1], [1, 3, 2], [1.0, 2.0, 3.0])
    bad_order = a.col.copy()
    bad_order[[0, 1]] = bad_order[[1, 0]]
    with pytest.raises(B.PackSELLError) as e:
        B.encode(a.rowptr, bad_order, a.val, 3, 5, "fp16", 15, 64, 256, B.IMPLICIT, DEV)
    assert e.value.status == B.EINVAL
    with pytest.raises(B.PackSELLError):
        B.encode(a.rowptr, a.col, a.val, 3, 3, "fp16", 15, 64, 256, B.IMPLICIT, DEV)
    with pytest.raises(B.PackSELLError):
        B.encode(a.rowptr, a.col, np.array([1.0, np.inf, 2.0]), 3, 5, "fix", 15, 64, 256,
                 B.IMPLICIT, DEV)
    bad_rp = a.rowptr.copy()
    bad_rp[1] = 7
    with pytest.raises(B.PackSELLError):
        B.encode(bad_rp, a.col, a.val, 3, 5, "fp16", 15, 64, 256, B.IMPLICIT, DEV)


def test_float64_input_rounds_through_float32():
    # 1 + 2^-11 + 2^-40 rounds to float32 1 + 2^-11, a half-precision tie
    # that goes to even (1.0); a direct float64 -> half rounding would give
    # 1 + 2^-10.  The encoder must round float64 -> float32 -> format.
    v = np.array([1 + 2.0 ** -11 + 2.0 ** -40, -(1 + 3 * 2.0 ** -11 + 2.0 ** -40), 3.0])
    a = W.csr_from_triplets(3, 3, [0, 1, 2], [0, 1, 2], v)
    A, E = both(a, "fp16", 15, 64, 256)
    assert_same_encoding(A, E)
    assert int(words(A)[0]) >> 16 == 0x3C00
    A, E = both(a, "e8my", 13, 64, 256)
    assert_same_encoding(A, E)


@pytest.mark.parametrize("fmt,D,C,sigma", [("fp16", 15, 64, 4096), ("e8my", 12, 64, 65536),
                                           ("e8my", 2, 32, 256), ("fix", 15, 64, 1024)])
def test_powerlaw_parity(fmt, D, C, sigma):
    """Irregular power-law rows (the high-RSD regime): n = 200,000."""
    a = W.powerlaw(200_000, seed=4)
    x = W.uniform_vector(a.m, 5)
    A, E = both(a, fmt, D, C, sigma)
    assert_same_encoding(A, E)
    check_spmv(A, a, fmt, D, x, B.IMPLICIT, E)


def test_m3_powerlaw_full_size():
    """n = 1,000,000 power-law rows (mean 30, max 5000), FP16, sigma = 65536."""
    a = W.m3_powerlaw()
    x = W.uniform_vector(a.m, 5)
    A, E = both(a, "fp16", 15, 64, 65536)
    assert_same_encoding(A, E)
    check_spmv(A, a, "fp16", 15, x, B.IMPLICIT, E)


def test_every_word_slot_written():
    """The fill phase writes every slot of every slice: driven through the C
    ABI with ``pack`` pre-filled by a sentinel (0xDEADBEEF) that none of the
    oracle's words equals for these inputs, the words end equal to the
    oracle's."""
    a = random_csr(31, 2000, 1700, per_row=9)
    L_ = B.lib()
    for fmt, D in [("fp16", 15), ("e8my", 3), ("fix", 12)]:
        desc = B.CMatrix()
        ws_bytes = ctypes.c_size_t()
        B._check(L_.pksell_encode_query(a.n, a.m, a.nnz, 64, 256, D, B.FMT_BY_NAME[fmt],
                                        B.IMPLICIT, ctypes.byref(desc), ctypes.byref(ws_bytes)))
        t = {"offset": torch.empty(desc.n_slices + 1, dtype=torch.int64, device=DEV),
             "perm": torch.empty(a.n * desc.perm_bytes, dtype=torch.uint8, device=DEV)}
        ws = torch.empty(ws_bytes.value, dtype=torch.uint8, device=DEV)
        rp = torch.from_numpy(a.rowptr).to(DEV)
        cl = torch.from_numpy(a.col.astype(np.int32)).to(DEV)
        vl = torch.from_numpy(a.val.astype(np.float32)).to(DEV)
        M = B.PackSELLMatrix(desc, t, DEV)
        M._bind()
        st = B._stream(DEV)
        args = (B._ptr(rp), B._ptr(cl), B._ptr(vl), B.F32, ctypes.byref(desc), B._ptr(ws),
                ws_bytes.value, st)
        B._check(L_.pksell_encode(*args))  # analyse
        t["pack"] = torch.full((desc.n_words,), -0x21524111, dtype=torch.int32, device=DEV)
        if fmt == "fix":
            t["row_exp"] = torch.full((a.n,), 0x7777, dtype=torch.int16, device=DEV)
        M._bind()
        B._check(L_.pksell_encode(*args))  # fill
        torch.cuda.synchronize()
        E = P.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D, 64, 256)
        assert not np.any(E.pack == 0xDEADBEEF)  # the sentinel is not a real word here
        got = words(M)
        assert np.array_equal(got, E.pack)
        if fmt == "fix":
            assert np.array_equal(M.row_exp.cpu().numpy().astype(np.int64), E.row_exp)


def test_save_and_load_roundtrip(tmp_path):
    a = random_csr(32, 900, 800, per_row=7)
    x = torch.from_numpy(W.uniform_vector(a.m, 2)).to(DEV)
    for fmt, D, split in [("e8my", 9, 0), ("fix", 15, 0), ("fp16", 15, 8)]:
        A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, B.IMPLICIT, DEV,
                     split_words=split)
        path = str(tmp_path / f"m_{fmt}.npz")
        A.save(path)
        A2 = B.PackSELLMatrix.load(path, DEV)
        assert A2.n_words == A.n_words and A2.k_left == A.k_left and A2.D == A.D
        assert torch.equal(A2.pack, A.pack)
        assert torch.equal(B.spmv(A2, x), B.spmv(A, x))


@pytest.mark.parametrize("C", [64, 16])
def test_sell_paired_slots_equal_plain_sell(C):
    """SELL with the float32 value beside its column in one 8-byte slot holds
    the same values in the same order as plain float32 SELL, so products are
    bit-identical; also against the oracle, on random rows and on the 128^3
    Laplacian (two slices per wave), both row orders."""
    for a in (random_csr(13, 3000, 2500, per_row=12), W.m2_laplace3d(64)):
        x = torch.from_numpy(W.uniform_vector(a.m, 14)).to(DEV)
        for mode in (B.IMPLICIT, B.EXPLICIT):
            S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, C, 256, mode, DEV)
            Sp = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, torch.float32, C, 256, mode, DEV,
                               paired=True)
            assert Sp.paired and Sp.n_slots == S.n_slots
            assert Sp.bytes_per_spmv() == S.bytes_per_spmv()
            yp = B.sell_spmv(Sp, x)
            assert torch.equal(yp, B.sell_spmv(S, x))
            if mode == B.IMPLICIT:
                vals = sell_values(a.val, torch.float32)
                ref = L.spmv(a.rowptr, a.col, vals, x.cpu().numpy())
                assert normalised_error(yp.cpu().numpy(), ref, a, vals, x.cpu().numpy()) <= SPMV_TOL


@pytest.mark.parametrize("stencil", ["laplace7_48", "stencil27_24"])
def test_cache_hint_resident_same_results(stencil):
    """cache_hint RESIDENT changes only the load policy of the single-vector
    products: the 7-point matrix runs the two-slice kernels, the 27-point
    one the one-slice-per-wave kernels.  PackSELL (FP16, E8M13, FIX; both
    row orders) and SELL (float32, paired, half values) products equal the
    streaming ones bit for bit, and the oracle's within the bar."""
    a = W.m2_laplace3d(48) if stencil == "laplace7_48" else W.m4_stencil27(24, seed=3)
    x = W.uniform_vector(a.m, 5)
    xt = torch.from_numpy(x).to(DEV)
    for fmt, D in (("fp16", 15), ("e8my", 9), ("fix", 15)):
        for mode in (B.IMPLICIT, B.EXPLICIT):
            A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 64, 256, mode, DEV)
            assert A.cache_hint == B.CACHE_STREAM
            y0 = B.spmv(A, xt)
            A.cache_hint = B.CACHE_RESIDENT
            y1 = B.spmv(A, xt)
            assert torch.equal(y0, y1), (fmt, mode)
            if mode == B.IMPLICIT:
                ref, q = oracle_product(a, FMTS[fmt], D, x)
                assert normalised_error(y1.cpu().numpy(), ref, a, q, x) <= SPMV_TOL
    for dt, paired in ((torch.float32, False), (torch.float32, True), (torch.float16, False)):
        S = B.sell_encode(a.rowptr, a.col, a.val, a.n, a.m, dt, 64, 256, B.IMPLICIT, DEV,
                          paired=paired)
        y0 = B.sell_spmv(S, xt)
        S.cache_hint = B.CACHE_RESIDENT
        assert torch.equal(y0, B.sell_spmv(S, xt)), (dt, paired)
