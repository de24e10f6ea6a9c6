"""Pins of the 64-bit-word PackSELL oracle (E11MY values, sec. 4.2.1 layout
with W = 64), each against something other than the oracle itself: an
integer rounding rule on the FP64 bit pattern, exact rational rounding,
hand-derived words, closed-form ties, a brute-force loop encoder and dense
products."""
import struct
from fractions import Fraction

import numpy as np
import pytest

from helpers import random_csr
from oracle import packsell64 as P64
from paper_2604_13433_amd import workloads as W


def bits_of(v: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def float_of(b: int) -> float:
    return struct.unpack("<d", struct.pack("<Q", b))[0]


def integer_rule(v: float, D: int) -> int:
    """Round-half-away on the magnitude bits: add half a unit of the kept
    precision and clear the dropped bits; past the largest finite value the
    result is infinity (the carry reaches the exponent field's all-ones)."""
    b = bits_of(v)
    sign, mag = b & (1 << 63), b & ((1 << 63) - 1)
    mag = (mag + (1 << D)) & ~((1 << (D + 1)) - 1)
    if mag >= 0x7FF0000000000000:
        mag = 0x7FF0000000000000
    return sign | mag


@pytest.mark.parametrize("D", [1, 2, 9, 14, 20, 29, 40, 50, 51])
def test_e11my_equals_integer_rule(D):
    rng = np.random.default_rng(D)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-300, 300, 2000),
                        [1.0, -1.0, 3.0, 1e308, -1.7976931348623157e308, 2.0 ** -1022]])
    got = P64.e11my_value_bits(v, D)
    want = np.array([integer_rule(float(x), D) for x in v], dtype=np.uint64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("D", [3, 17, 33])
def test_e11my_exact_rational_rounding(D):
    """q = round_half_away(v * 2^k) / 2^k with k such that q keeps 52 - D
    significant bits, in exact rational arithmetic."""
    rng = np.random.default_rng(100 + D)
    for v in rng.standard_normal(300) * 1e3:
        fv = Fraction(float(v))
        e = int(np.frexp(float(v))[1])  # |v| = f 2^e, 1/2 <= f < 1
        k = (52 - D) - e
        t = fv * (Fraction(2) ** k)
        r = (abs(t) + Fraction(1, 2)).__floor__() * (1 if t >= 0 else -1)
        q = Fraction(r) / (Fraction(2) ** k)
        got = float_of(int(P64.e11my_value_bits(np.array([v]), D)[0]))
        assert Fraction(got) == q


def test_e11my_closed_form_ties_and_specials():
    q = lambda v, D: float_of(int(P64.e11my_value_bits(np.array([v]), D)[0]))
    # D = 51: no explicit mantissa bits, values round to powers of two
    assert q(1.5, 51) == 2.0 and q(-1.5, 51) == -2.0 and q(1.25, 51) == 1.0
    assert q(1.75, 51) == 2.0 and q(3.0, 51) == 4.0
    # D = 50: one mantissa bit; 1.25 is a tie between 1.0 and 1.5 -> away
    assert q(1.25, 50) == 1.5 and q(-1.25, 50) == -1.5 and q(1.2, 50) == 1.0
    # specials
    assert q(0.0, 9) == 0.0 and np.signbit(q(-0.0, 9))
    assert q(np.inf, 9) == np.inf and q(-np.inf, 9) == -np.inf
    assert int(P64.e11my_value_bits(np.array([np.nan]), 9)[0]) == 0x7FF8000000000000
    assert q(1.7976931348623157e308, 1) == np.inf  # rounds past the largest finite value
    # subnormals on the grid 2^(D + 1 - 1074), ties away from zero
    tiny = 2.0 ** -1074
    assert q(3 * tiny, 1) == 4 * tiny and q(2 * tiny, 1) == 4 * tiny and q(tiny, 1) == 0.0
    assert q(5 * tiny, 2) == 8 * tiny and q(3 * tiny, 2) == 0.0


def test_hand_packed_words():
    """Sec. 4.2.1 layout with W = 64, words written out by hand."""
    # value 1.0 (FP64 0x3FF0000000000000), D = 20, delta 5: | 5 << 1 | 1
    assert int(P64.pack_value_word(P64.e11my_value_bits(np.array([1.0]), 20), 5)[0]) == \
        0x3FF000000000000B
    # value -2.5 (0xC004000000000000), D = 3, delta 7: | 14 | 1
    assert int(P64.pack_value_word(P64.e11my_value_bits(np.array([-2.5]), 3), 7)[0]) == \
        0xC00400000000000F
    # dummy with delta 2^40: the whole upper 63 bits hold the delta
    assert int(P64.pack_delta_word(np.array([1 << 40]))[0]) == 0x20000000000
    flag, d, vb = P64.unpack_word(np.array([0xC00400000000000F, 0x20000000000, 0], np.uint64), 3)
    assert list(flag) == [1, 0, 0] and list(d) == [7, 1 << 40, 0]
    assert int(vb[0]) == 0xC004000000000000 and int(vb[1]) == 0 and int(vb[2]) == 0


def brute_force_encode(a, D, C, sigma, implicit=True):
    """A loop-by-loop encoder written from the format description alone:
    row offsets (eq. 4), deltas, dummies, sigma-window sort by word count,
    slice widths, column-major words."""
    n = a.n
    k_left = 0
    for i in range(n):
        for e in range(a.rowptr[i], a.rowptr[i + 1]):
            k_left = max(k_left, i - int(a.col[e]))
    words_of = []
    for i in range(n):
        blk = (i // sigma) * sigma
        prev = blk - k_left if k_left < blk else 0
        ws = []
        for e in range(a.rowptr[i], a.rowptr[i + 1]):
            c = int(a.col[e])
            d = c - prev
            vb = integer_rule(float(a.val[e]), D) if np.isfinite(a.val[e]) else None
            if d >= (1 << D):
                ws.append(d << 1)
                d = 0
            ws.append(vb | (d << 1) | 1)
            prev = c
        words_of.append(ws)
    order = []
    for b0 in range(0, n, sigma):
        rows = list(range(b0, min(b0 + sigma, n)))
        rows.sort(key=lambda r: (-len(words_of[r]), r))
        order += rows
    n_slices = -(-n // C)
    pack, offset = [], [0]
    for k in range(n_slices):
        lanes = [order[t] if t < n else None for t in range(k * C, k * C + C)]
        w = max(len(words_of[r]) if r is not None else 0 for r in lanes)
        for j in range(w):
            for r in lanes:
                ws = words_of[r] if r is not None else []
                pack.append(ws[j] if j < len(ws) else 0)
        offset.append(len(pack))
    return np.array(pack, dtype=np.uint64), np.array(offset), order, k_left


@pytest.mark.parametrize("D,C,sigma", [(3, 4, 8), (9, 8, 3), (20, 2, 2), (51, 16, 64), (1, 4, 1)])
def test_encoder_against_brute_force(D, C, sigma):
    a = random_csr(7 + D, 90, 120, density=0.06)
    E = P64.encode(a.rowptr, a.col, a.val, a.n, a.m, D, C, sigma)
    pack, offset, order, k_left = brute_force_encode(a, D, C, sigma)
    assert E.k_left == k_left
    assert np.array_equal(E.offset, offset)
    assert np.array_equal(E.pack, pack)
    assert list(E.stored_rows) == order


@pytest.mark.parametrize("D", [2, 12, 30])
@pytest.mark.parametrize("mode", [P64.PERM_IMPLICIT, P64.PERM_EXPLICIT])
def test_spmv_equals_dense_product_of_quantised_values(D, mode):
    a = random_csr(3, 300, 250, density=0.04)
    E = P64.encode(a.rowptr, a.col, a.val, a.n, a.m, D, 8, 32, mode)
    x = np.random.default_rng(1).uniform(-1, 1, a.m)
    A = np.zeros((a.n, a.m))
    A[a.rows(), a.col] = P64.quantized(a.val, D)
    ref = A @ x
    if mode == P64.PERM_EXPLICIT:
        ref = ref[E.stored_rows]
    y = P64.spmv(E, x)
    assert np.max(np.abs(y - ref)) <= 1e-13 * (np.abs(A).sum(1).max() * np.abs(x).max())
    # flag-1 words are the nonzeros, flag-0 words the dummies and padding
    flag, d, _ = P64.unpack_word(E.pack, D)
    assert int(flag.sum()) == a.nnz
    assert int(((flag == 0) & (d > 0)).sum()) == E.n_dummies


def test_dummies_are_the_large_deltas():
    """A 7-point 16^3 stencil: a plane jump is 256 - 16 = 240 columns, so
    D = 7 (deltas below 128) needs a dummy at every row's z-neighbour jumps
    and D = 8 needs none past the first word."""
    a = W.m2_laplace3d(16)
    e7 = P64.encode(a.rowptr, a.col, a.val, a.n, a.m, 7, 64, 256)
    e8 = P64.encode(a.rowptr, a.col, a.val, a.n, a.m, 8, 64, 256)
    assert e7.n_dummies > e8.n_dummies
    assert e7.n_words > e8.n_words
