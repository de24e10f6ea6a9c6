"""Pins of the CSR-based packing oracle, each against something other than
the oracle itself: the PackSELL oracle at C = 1 and sigma = 1 (one-row
slices hold a row's words contiguously with no padding), a loop-by-loop
encoder and dense products.  The expected chunk plan of the GPU tests
(tests/helpers.py, read off the oracle's word stream) is checked here
against a plan found by walking rows word by word, and on closed-form
cases."""
import numpy as np
import pytest

from helpers import FMTS, chunk_plan_from_words, random_csr
from oracle import formats as F
from oracle import packcsr as PC
from oracle import packsell as P
from paper_2604_13433_amd import workloads as W


def hollow(seed=3):
    """Empty rows at the start, in runs in the middle and at the end, long
    jumps (dummies) and a few long rows."""
    rng = np.random.default_rng(seed)
    n, m = 400, 70000
    rows, cols = [], []
    for i in range(n):
        if i < 5 or 100 <= i < 130 or i >= 390 or rng.random() < 0.2:
            continue
        k = 200 if i % 97 == 0 else int(rng.integers(1, 12))
        c = np.unique(rng.integers(0, m, size=k))
        rows += [i] * c.size
        cols += list(c)
    return W.csr_from_triplets(n, m, rows, cols, rng.standard_normal(len(rows)))


CASES = [lambda: random_csr(1, 300, 250, density=0.04), lambda: random_csr(2, 90, 4000, per_row=7),
         hollow]


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9), ("e8my", 3), ("fix", 20)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_equals_packsell_with_one_row_slices(fmt, D, case):
    a = CASES[case]()
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D)
    S = P.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D, 1, 1, P.PERM_EXPLICIT)
    assert E.k_left == S.k_left and E.n_dummies == S.n_dummies and E.n_words == S.n_words
    assert np.array_equal(E.pack, S.pack)
    assert np.array_equal(E.wrowptr, S.offset)
    if fmt == "fix":
        assert np.array_equal(E.row_exp, S.row_exp)


def brute_force(a, fmt, D):
    """Row by row, entry by entry, from the format description alone."""
    k_left = 0
    for i in range(a.n):
        for e in range(a.rowptr[i], a.rowptr[i + 1]):
            k_left = max(k_left, i - int(a.col[e]))
    v32 = np.asarray(a.val, np.float64).astype(np.float32)
    if fmt == F.FMT_FIX:
        bits = np.zeros(a.nnz, np.uint32)
        for i in range(a.n):
            s, e = a.rowptr[i], a.rowptr[i + 1]
            mx = float(np.abs(v32[s:e].astype(np.float64)).max()) if e > s else 0.0
            ex = F.fix_row_exponent(np.array([mx]), D)
            bits[s:e] = F.fix_value_bits(v32[s:e], np.repeat(ex, e - s), D)
    elif fmt == F.FMT_FP16:
        bits = F.fp16_value_bits(v32)
    else:
        bits = F.e8my_value_bits(v32, D)
    words, wrowptr = [], [0]
    for i in range(a.n):
        prev = i - k_left if k_left < i else 0
        for e in range(a.rowptr[i], a.rowptr[i + 1]):
            d = int(a.col[e]) - prev
            if d >= (1 << D):
                words.append(d << 1)
                d = 0
            words.append(int(bits[e]) | (d << 1) | 1)
            prev = int(a.col[e])
        wrowptr.append(len(words))
    return np.array(words, np.uint32), np.array(wrowptr), k_left


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 5), ("fix", 12)])
def test_encoder_against_brute_force(fmt, D):
    a = hollow(7)
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D)
    words, wrowptr, k_left = brute_force(a, FMTS[fmt], D)
    assert E.k_left == k_left
    assert np.array_equal(E.pack, words) and np.array_equal(E.wrowptr, wrowptr)


@pytest.mark.parametrize("fmt,D", [("fp16", 15), ("e8my", 9), ("fix", 20)])
def test_spmv_equals_dense_product(fmt, D):
    a = hollow(5)
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.m, FMTS[fmt], D)
    x = np.random.default_rng(0).uniform(-1, 1, a.m)
    A = np.zeros((a.n, a.m))
    A[a.rows(), a.col] = P.quantized_values(a.rowptr, a.col, a.val, a.n, FMTS[fmt], D)
    ref = A @ x
    assert np.max(np.abs(PC.spmv(E, x) - ref)) <= 1e-13 * np.abs(A).sum(1).max()


def plan_by_walking(E, T):
    """lo by a linear scan over rows; anchor by walking the row that holds
    word c*T from its first word, adding deltas one word at a time."""
    n_chunks = -(-E.n_words // T)
    lo, anchor = [], []
    for c in range(n_chunks):
        p = c * T
        r = 0
        while r < E.n and E.wrowptr[r] < p:
            r += 1
        lo.append(r)
        owner = max(i for i in range(E.n) if E.wrowptr[i] <= p < E.wrowptr[i + 1])
        run = owner - E.k_left if E.k_left < owner else 0
        for q in range(E.wrowptr[owner], p):
            w = int(E.pack[q])
            run += ((w >> 1) & ((1 << E.D) - 1)) if w & 1 else (w >> 1)
        anchor.append(run)
    lo.append(E.n)
    return np.array(lo), np.array(anchor)


@pytest.mark.parametrize("T", [64, 128, 512])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_chunk_plan_against_walking(T, case):
    a = CASES[case]()
    E = PC.encode(a.rowptr, a.col, a.val, a.n, a.m, F.FMT_E8MY, 9)
    lo, anchor = chunk_plan_from_words(E, T)
    wlo, wanchor = plan_by_walking(E, T)
    assert np.array_equal(lo, wlo) and np.array_equal(anchor, wanchor)
    # every row is owned by exactly one chunk: rows lo[c]..lo[c+1]-1 start in
    # chunk c (the last chunk also takes the empty rows at the stream's end)
    for c in range(len(lo) - 1):
        starts = E.wrowptr[lo[c]:lo[c + 1]]
        assert np.all(starts >= c * T)
        if c + 1 < len(lo) - 1:
            assert np.all(starts < (c + 1) * T)


def test_chunk_plan_special_cases():
    # chunk boundaries on row starts: rows of exactly 64 words
    n = 10
    rows = np.repeat(np.arange(n), 64)
    cols = np.tile(np.arange(64), n)
    a = W.csr_from_triplets(n, 64, rows, cols, np.ones(rows.size))
    E = PC.encode(a.rowptr, a.col, a.val, n, 64, F.FMT_FP16, 15)
    lo, anchor = chunk_plan_from_words(E, 128)
    assert list(lo) == [0, 2, 4, 6, 8, 10]
    assert list(anchor) == [0, 0, 0, 0, 0]  # k_left = 9: left offsets 0 up to row 9
    # one row across many chunks: anchors are that row's running column
    a = W.csr_from_triplets(3, 5000, [1] * 1000, np.arange(0, 5000, 5), np.ones(1000))
    E = PC.encode(a.rowptr, a.col, a.val, 3, 5000, F.FMT_FP16, 15)
    lo, anchor = chunk_plan_from_words(E, 64)
    assert list(lo) == [0] + [2] * 15 + [3]
    assert list(anchor) == [0] + [5 * 64 * c - 5 for c in range(1, 16)]
    # no words at all: no chunks, lo = [n]
    a = W.csr_from_triplets(4, 9, [], [], [])
    E = PC.encode(a.rowptr, a.col, a.val, 4, 9, F.FMT_FP16, 15)
    lo, anchor = chunk_plan_from_words(E, 64)
    assert list(lo) == [4] and anchor.size == 0
