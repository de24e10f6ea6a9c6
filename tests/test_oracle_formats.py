"""Pins for the oracle's value formats and word codec (CPU only).

Each test checks the oracle against something other than itself: words packed
by hand (tests/golden/words.json), Python's own binary16 packing, an integer
closed form of the E8MY rounding, the paper's scaling form of the same
rounding, an exhaustive nearest-value search over small E8MY grids, closed-form
half-way cases of the FIX rounding, and error bounds.
"""
import json
import os
import struct

import numpy as np
import pytest

from oracle import formats as F

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FMT = {"fp16": F.FMT_FP16, "e8my": F.FMT_E8MY, "fix": F.FMT_FIX}


def _words():
    with open(os.path.join(GOLD, "words.json")) as f:
        return json.load(f)["words"]


@pytest.mark.parametrize("w", _words(), ids=lambda w: w["what"])
def test_hand_packed_words(w):
    fmt, D, word = FMT[w["fmt"]], w["D"], int(w["word"], 16)
    if w["value"] is None:
        packed = int(F.pack_delta_word(np.array([w["delta"]]))[0])
    else:
        v = np.array([w["value"]], dtype=np.float32)
        vb = F.fp16_value_bits(v) if fmt == F.FMT_FP16 else F.e8my_value_bits(v, D)
        packed = int(F.pack_value_word(vb, np.array([w["delta"]]))[0])
    assert packed == word, hex(packed)
    flag, delta, vb = F.unpack_word(np.array([word], dtype=np.uint32), D)
    assert int(delta[0]) == w["delta"]
    assert int(flag[0]) == (0 if w["value"] is None else 1)
    if w["value"] is None:
        assert int(vb[0]) == 0
    else:
        got = F.value_from_bits(vb, fmt, D)[0]
        q = np.float32(w["value"])
        if fmt == F.FMT_FP16:
            assert got == float(np.float16(q))
        else:
            # E8MY examples are chosen so the decoded value is the rounded one
            assert abs(got - float(q)) <= 2.0 ** (-(22 - D) - 1) * abs(float(q))


def test_unpack_roundtrip_all_D():
    rng = np.random.default_rng(0)
    for D in range(1, 31):
        V = 31 - D
        vfield = (rng.integers(0, 2 ** V, 2000, dtype=np.uint64) << np.uint64(D + 1)).astype(np.uint32)
        d = rng.integers(0, 2 ** D, 2000).astype(np.uint64)
        p = F.pack_value_word(vfield, d)
        flag, dd, vb = F.unpack_word(p, D)
        assert np.all(flag == 1) and np.array_equal(dd, d.astype(np.uint32))
        assert np.array_equal(vb, vfield)
        big = rng.integers(0, 2 ** 31, 2000).astype(np.uint64)
        flag, dd, vb = F.unpack_word(F.pack_delta_word(big), D)
        assert np.all(flag == 0) and np.array_equal(dd, big.astype(np.uint32))
        assert np.all(vb == 0)


def test_padding_word_decodes_to_nothing():
    for D in (1, 9, 15, 22, 30):
        flag, d, vb = F.unpack_word(np.zeros(1, np.uint32), D)
        assert int(flag[0]) == 0 and int(d[0]) == 0 and int(vb[0]) == 0


def _edge_floats():
    vals = [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.0, 65520.0, -65520.0, 1e6,
            2.0 ** -14, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -26,
            1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 6.1e-5, 5.96e-8, np.inf, -np.inf]
    return np.array(vals, dtype=np.float32)


def test_fp16_matches_struct_binary16():
    rng = np.random.default_rng(1)
    mags = 2.0 ** rng.uniform(-30, 17, 20000)
    v = np.concatenate([_edge_floats(),
                        (mags * rng.choice([-1, 1], mags.size)).astype(np.float32)])
    got = F.fp16_value_bits(v) >> np.uint32(16)
    for a, b in zip(v, got):
        assert F.fp16_value_bits_scalar(float(a)) >> 16 == int(b), float(a)
    # ties round to even
    assert int(F.fp16_value_bits(np.float32([1 + 2.0 ** -11]))[0]) >> 16 == 0x3C00
    assert int(F.fp16_value_bits(np.float32([1 + 3 * 2.0 ** -11]))[0]) >> 16 == 0x3C02
    assert int(F.fp16_value_bits(np.float32([np.nan]))[0]) >> 16 == 0x7E00


def _e8my_integer_rule(v32, D):
    """Independent closed form: round the magnitude bits to a multiple of
    2^(D+1) with ties away from zero, saturating to infinity."""
    b = np.asarray(v32, np.float32).view(np.uint32).astype(np.uint64)
    sign = b & np.uint64(0x80000000)
    mag = b & np.uint64(0x7FFFFFFF)
    r = (mag + np.uint64(1 << D)) & np.uint64(~((1 << (D + 1)) - 1) & 0xFFFFFFFF)
    r = np.minimum(r, np.uint64(0x7F800000))
    return (sign | r).astype(np.uint32)


@pytest.mark.parametrize("D", list(range(1, 23)))
def test_e8my_equals_integer_rule(D):
    rng = np.random.default_rng(D)
    bits = rng.integers(0x00800000, 0x7F800000, 20000, dtype=np.uint64).astype(np.uint32)
    bits |= (rng.integers(0, 2, bits.size).astype(np.uint32) << np.uint32(31))
    # exact ties and near-ties on random mantissas
    ties = (bits & np.uint32(~((1 << (D + 1)) - 1) & 0xFFFFFFFF)) | np.uint32(1 << D)
    subn = rng.integers(1, 0x00800000, 3000, dtype=np.uint64).astype(np.uint32)
    top = np.array([0x7F7FFFFF, 0xFF7FFFFF, 0x7F7FF000, 0x00800000, 0x00000001,
                    0x007FFFFF], dtype=np.uint32)
    allb = np.concatenate([bits, ties, ties - np.uint32(1), subn, top])
    v = allb.view(np.float32)
    assert np.array_equal(F.e8my_value_bits(v, D), _e8my_integer_rule(v, D))


@pytest.mark.parametrize("D", [1, 2, 9, 12, 22])
def test_e8my_error_bound(D):
    rng = np.random.default_rng(100 + D)
    v = (2.0 ** rng.uniform(-100, 100, 20000) * rng.choice([-1, 1], 20000)).astype(np.float32)
    q = F.e8my_value_bits(v, D).view(np.float32).astype(np.float64)
    Y = 22 - D
    assert np.all(np.abs(q - v) <= 2.0 ** -(Y + 1) * np.abs(v.astype(np.float64)))


def test_e8my_specials():
    v = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 3.4028235e38], dtype=np.float32)
    b = F.e8my_value_bits(v, 9)
    assert list(b[:4]) == [0, 0x80000000, 0x7F800000, 0xFF800000]
    assert b[4] == 0x7FC00000
    assert b[5] == 0x7F800000  # the largest float rounds past the top: infinity


@pytest.mark.parametrize("D", [1, 7, 15, 24, 29])
def test_fix_quantiser_bounds(D):
    V = 31 - D
    rng = np.random.default_rng(D)
    rows = rng.standard_normal((50, 40)) * 2.0 ** rng.uniform(-20, 20, (50, 1))
    v = rows.astype(np.float32)
    e = F.fix_row_exponent(np.abs(v.astype(np.float64)).max(axis=1), D)
    lim = 2 ** (V - 1) - 1
    for r in range(v.shape[0]):
        vb = F.fix_value_bits(v[r], np.full(v.shape[1], e[r]), D)
        q = F.value_from_bits(vb, F.FMT_FIX, D)
        assert np.all(np.abs(q) <= lim)
        # the largest magnitude lands in the top binade of the V-bit range
        assert np.abs(q).max() >= 2 ** (V - 2)
        unclamped = np.abs(np.ldexp(v[r].astype(np.float64), -int(e[r]))) < lim
        err = np.abs(np.ldexp(q, int(e[r])) - v[r])
        assert np.all(err[unclamped] <= 2.0 ** (int(e[r]) - 1))


def test_fix_exact_grid_values():
    D = 15  # FIX16
    v = np.array([3.0, -5.0, 0.25, 1024.0, 0.0], dtype=np.float32)
    e = F.fix_row_exponent(np.array([1024.0]), D)[0]
    q = F.value_from_bits(F.fix_value_bits(v, np.full(v.size, e), D), F.FMT_FIX, D)
    assert np.array_equal(np.ldexp(q, int(e)), v.astype(np.float64))


def _e8my_by_scaling(v32, D):
    """The conversion of sec. 4.2.2 as the paper states it, for normal
    inputs: with |v| = f 2^e (1/2 <= f < 1), round v to a multiple of
    2^(e - 24 + D + 1), ties away from zero (C's round), then clear the low
    D + 1 bits.  A different route from the oracle's neighbour search."""
    v = np.asarray(v32, np.float32).astype(np.float64)
    _, e = np.frexp(v)
    scale = np.ldexp(1.0, e - 24 + D + 1)
    t = v / scale
    r = np.sign(t) * np.floor(np.abs(t) + 0.5) * scale
    with np.errstate(over="ignore"):
        b = r.astype(np.float32).view(np.uint32)
    return b & np.uint32((0xFFFFFFFF << (D + 1)) & 0xFFFFFFFF)


@pytest.mark.parametrize("D", [1, 2, 5, 9, 12, 13, 15, 20, 22])
def test_e8my_equals_paper_scaling_steps(D):
    rng = np.random.default_rng(300 + D)
    bits = rng.integers(0x00800000, 0x7F800000, 20000, dtype=np.uint64).astype(np.uint32)
    bits |= (rng.integers(0, 2, bits.size).astype(np.uint32) << np.uint32(31))
    ties = (bits & np.uint32((0xFFFFFFFF << (D + 1)) & 0xFFFFFFFF)) | np.uint32(1 << D)
    v = np.concatenate([bits, ties, ties + np.uint32(1)]).view(np.float32)
    assert np.array_equal(F.e8my_value_bits(v, D), _e8my_by_scaling(v, D))


@pytest.mark.parametrize("D", [18, 20, 21, 22])
def test_e8my_brute_force_nearest(D):
    """Y = 22 - D <= 4: list every positive E8MY value with exponent in
    [-6, 6] (2^Y per binade), and take the nearest one by exhaustive search,
    ties to the larger magnitude."""
    Y = 22 - D
    grid = sorted({(1 + k / 2 ** Y) * 2.0 ** e for e in range(-6, 7) for k in range(2 ** Y)})
    grid = np.array(grid)
    rng = np.random.default_rng(D)
    v = (2.0 ** rng.uniform(-6, 6.9, 3000)).astype(np.float32)
    mids = ((grid[1:] + grid[:-1]) / 2).astype(np.float32)  # exact ties (Y small)
    v = np.concatenate([v, mids, grid.astype(np.float32)])
    v = v[(v >= 2.0 ** -6) & (v <= grid[-1])]
    a = v.astype(np.float64)
    dist = np.abs(a[:, None] - grid[None, :])
    best = dist.min(axis=1, keepdims=True)
    want = np.where(dist == best, grid[None, :], -np.inf).max(axis=1)  # tie: larger
    got = F.e8my_value_bits(v, D).view(np.float32).astype(np.float64)
    assert np.array_equal(got, want)
    got_neg = F.e8my_value_bits(-v, D).view(np.float32).astype(np.float64)
    assert np.array_equal(got_neg, -want)


@pytest.mark.parametrize("D,M", [(25, 20.0), (15, 20000.0), (25, 20.0 * 2.0 ** -10)])
def test_fix_ties_round_away_from_zero(D, M):
    """Half-way cases: with the row maximum M the row exponent makes
    v / 2^e_row land exactly on +-0.5, +-1.5, +-2.5, +-3.5; ties go away
    from zero (round-half-even would give 0, 2, 2, 4)."""
    e = int(F.fix_row_exponent(np.array([M]), D)[0])
    t = np.array([0.5, -0.5, 1.5, -1.5, 2.5, -2.5, 3.5, -3.5])
    v = np.ldexp(t, e).astype(np.float32)
    q = F.value_from_bits(F.fix_value_bits(v, np.full(v.size, e), D), F.FMT_FIX, D)
    assert list(q) == [1, -1, 2, -2, 3, -3, 4, -4]
