"""Pins of the 16-bit-word PackSELL oracle (E5MY and FIX16 values, sec. 4.2.1
layout with W = 16, dummy chains), each against something other than the
oracle itself: an integer rounding rule on every finite binary16 input, a
brute-force nearest-value search over the whole E5MY grid, closed-form
ties, the 32-bit FIX oracle with the same field width, hand-packed words, a
loop-by-loop encoder and dense products."""
import numpy as np
import pytest

from helpers import random_csr
from oracle import formats as F
from oracle import packsell16 as P16
from paper_2604_13433_amd import workloads as W


def integer_rule16(h: np.ndarray, D: int) -> np.ndarray:
    """Round-half-away on the binary16 magnitude bits: add half a unit of the
    kept precision and clear the dropped bits; a carry into the all-ones
    exponent gives infinity."""
    h = np.asarray(h, np.uint32)
    sign, mag = h & 0x8000, h & 0x7FFF
    mag = (mag + (1 << D)) & np.uint32(0xFFFF & ~((1 << (D + 1)) - 1))
    mag = np.where(mag >= 0x7C00, 0x7C00, mag)
    return (sign | mag).astype(np.uint16)


@pytest.mark.parametrize("D", range(1, 9))
def test_e5my_on_every_binary16_value(D):
    """Every finite binary16 number is a float32 input whose E5MY value must
    follow the integer rule on its own bits."""
    h = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    finite = (h & 0x7C00) != 0x7C00
    h = h[finite]
    v = h.view(np.float16).astype(np.float32)
    assert np.array_equal(P16.e5my_value_bits(v, D), integer_rule16(h, D))


def e5my_grid(D: int) -> np.ndarray:
    """All finite non-negative E5MY values, ascending (patterns with the low
    D + 1 bits zero)."""
    pats = np.arange(0, 0x7C00, 1 << (D + 1), dtype=np.uint32).astype(np.uint16)
    return np.sort(pats.view(np.float16).astype(np.float64))


@pytest.mark.parametrize("D", [1, 4, 7, 8])
def test_e5my_is_the_nearest_grid_value(D):
    """Brute force: the nearest E5MY value by search over the whole grid,
    ties to the larger magnitude, past the top half-step infinity."""
    rng = np.random.default_rng(D)
    grid = e5my_grid(D)
    top_half = grid[-1] + (grid[-1] - grid[-2]) / 2
    v = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-9, 6, 3000),
                        (grid[1:] + grid[:-1])[::37] / 2])  # exact midpoints
    v = v.astype(np.float32)
    got = P16.e5my_value_bits(v, D).view(np.float16).astype(np.float64)
    for x, g in zip(v.astype(np.float64), got):
        a = abs(x)
        if a >= top_half:
            want = np.inf
        else:
            dist = np.abs(grid - a)
            best = np.nonzero(dist == dist.min())[0]
            want = grid[best.max()]  # ties away from zero
        assert g == np.copysign(want, x), (x, g, want)


def test_e5my_closed_form_ties_and_specials():
    q = lambda v, D: float(P16.e5my_value_bits(np.array([v], np.float32), D).view(np.float16)[0])
    # D = 7 is E5M2: 1.0, 1.25, 1.5, 1.75 per binade
    assert q(1.125, 7) == 1.25 and q(-1.125, 7) == -1.25 and q(1.1, 7) == 1.0
    assert q(1.875, 7) == 2.0 and q(3.0, 7) == 3.0
    # largest finite E5M2 is 57344; the midpoint to 65536 rounds away (inf)
    assert q(57344.0, 7) == 57344.0 and q(61439.0, 7) == 57344.0
    assert q(61440.0, 7) == np.inf and q(-61440.0, 7) == -np.inf
    # subnormal grid 2^(D + 1 - 24): at D = 7 the step is 2^-16
    s = 2.0 ** -16
    assert q(1.5 * s, 7) == 2 * s and q(0.5 * s, 7) == s and q(0.49 * s, 7) == 0.0
    assert q(0.0, 7) == 0.0 and np.signbit(q(-0.0, 7))
    assert q(np.inf, 3) == np.inf and q(-np.inf, 3) == -np.inf
    assert int(P16.e5my_value_bits(np.array([np.nan], np.float32), 5)[0]) == 0x7E00
    # D = 7 values fit 8 bits: the low byte of every field is zero
    v = np.random.default_rng(0).standard_normal(500).astype(np.float32)
    assert np.all(P16.e5my_value_bits(v, 7) & 0xFF == 0)


@pytest.mark.parametrize("D", [1, 7, 13])
def test_fix16_reduces_to_fix_with_the_same_field_width(D):
    """FIX16 with delta width D has V = 15 - D value bits, as 32-bit FIX with
    delta width D + 16: the same exponents, the same integers."""
    rng = np.random.default_rng(D)
    M = np.abs(rng.standard_normal(200)) * 10.0 ** rng.integers(-20, 20, 200)
    M[:3] = 0.0
    e16 = P16.fix16_row_exponent(M, D)
    assert np.array_equal(e16, F.fix_row_exponent(M, D + 16))
    v = (rng.standard_normal(200) * M).astype(np.float32)
    got = P16.fix16_value_bits(v, e16, D)
    want = (F.fix_value_bits(v, e16, D + 16) >> np.uint32(16)).astype(np.uint16)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("D,M", [(7, 100.0), (7, 100.0 * 2.0 ** -12), (3, 1000.0)])
def test_fix16_ties_round_away_from_zero(D, M):
    """Half-way cases: v / 2^e_row = +-0.5, +-1.5, +-2.5, +-3.5 must give
    +-1, +-2, +-3, +-4 (round-half-even would give 0, 2, 2, 4); D = 7 is the
    int8 field."""
    e = int(P16.fix16_row_exponent(np.array([M]), D)[0])
    t = np.array([0.5, -0.5, 1.5, -1.5, 2.5, -2.5, 3.5, -3.5])
    v = np.ldexp(t, e).astype(np.float32)
    q = P16.value_from_bits(P16.fix16_value_bits(v, np.full(v.size, e), D), P16.FMT_FIX16, D)
    assert list(q) == [1, -1, 2, -2, 3, -3, 4, -4]


def test_hand_packed_words():
    """Sec. 4.2.1 layout with W = 16, written out by hand."""
    # E5M2 value 1.5 (binary16 0x3E00), D = 7, delta 5: 0x3E00 | 5 << 1 | 1
    vb = P16.e5my_value_bits(np.array([1.5], np.float32), 7)
    assert int(P16.pack_value_word(vb, 5)[0]) == 0x3E0B
    # a dummy with delta 2^15 - 1 is 0xFFFE
    assert int(P16.pack_delta_word(np.array([32767]))[0]) == 0xFFFE
    flag, d, b = P16.unpack_word(np.array([0x3E0B, 0xFFFE, 0], np.uint16), 7)
    assert list(flag) == [1, 0, 0] and list(d) == [5, 32767, 0]
    assert int(b[0]) == 0x3E00 and int(b[1]) == 0 and int(b[2]) == 0
    # FIX16 at D = 7: q = -3 as an int8 field in the upper byte
    e = np.array([0])
    assert int(P16.fix16_value_bits(np.array([-3.0], np.float32), e, 7)[0]) == 0xFD00
    with pytest.raises(OverflowError):
        P16.pack_delta_word(np.array([32768]))


def test_dummy_chain_counts():
    D = 7
    d = np.array([0, 127, 128, 32767, 32768, 65534, 65535, 100000])
    assert list(P16.dummies_for(d, D)) == [0, 0, 1, 1, 2, 2, 3, 4]


def brute_force_encode(a, fmt, D, C, sigma):
    """Loop-by-loop, from the format description alone: eq. 4 offsets,
    deltas, dummy chains, sigma-window sort, slice widths, column-major
    16-bit words."""
    n = a.n
    k_left = 0
    for i in range(n):
        for e in range(a.rowptr[i], a.rowptr[i + 1]):
            k_left = max(k_left, i - int(a.col[e]))
    bits, _ = P16.value_field(a.val, a.rowptr, fmt, D, n)
    words_of = []
    for i in range(n):
        blk = (i // sigma) * sigma
        prev = blk - k_left if k_left < blk else 0
        ws = []
        for e in range(a.rowptr[i], a.rowptr[i + 1]):
            c = int(a.col[e])
            d = c - prev
            if d >= (1 << D):
                while d > 0:
                    step = min(d, 32767)
                    ws.append(step << 1)
                    d -= step
            ws.append(int(bits[e]) | (d << 1) | 1)
            prev = c
        words_of.append(ws)
    order = []
    for b0 in range(0, n, sigma):
        rows = list(range(b0, min(b0 + sigma, n)))
        rows.sort(key=lambda r: (-len(words_of[r]), r))
        order += rows
    pack, offset = [], [0]
    for k in range(-(-n // C)):
        lanes = [order[t] if t < n else None for t in range(k * C, k * C + C)]
        w = max(len(words_of[r]) if r is not None else 0 for r in lanes)
        for j in range(w):
            for r in lanes:
                ws = words_of[r] if r is not None else []
                pack.append(ws[j] if j < len(ws) else 0)
        offset.append(len(pack))
    return np.array(pack, dtype=np.uint16), np.array(offset), order, k_left


@pytest.mark.parametrize("fmt,D,C,sigma", [(P16.FMT_E5MY, 7, 4, 8), (P16.FMT_E5MY, 2, 8, 3),
                                           (P16.FMT_FIX16, 7, 2, 2), (P16.FMT_FIX16, 13, 16, 64),
                                           (P16.FMT_E5MY, 8, 4, 1)])
def test_encoder_against_brute_force(fmt, D, C, sigma):
    a = random_csr(7 + D, 90, 120, density=0.06)
    E = P16.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, C, sigma)
    pack, offset, order, k_left = brute_force_encode(a, fmt, D, C, sigma)
    assert E.k_left == k_left
    assert np.array_equal(E.offset, offset)
    assert np.array_equal(E.pack, pack)
    assert list(E.stored_rows) == order


def test_long_dummy_chains_against_brute_force():
    """Columns up to 2^17 apart: chains of up to five dummies."""
    rng = np.random.default_rng(11)
    n, m = 40, 150000
    rows, cols = [], []
    for i in range(n):
        c = np.sort(rng.choice(m, size=rng.integers(0, 6), replace=False))
        rows += [i] * c.size
        cols += list(c)
    a = W.csr_from_triplets(n, m, rows, cols, rng.standard_normal(len(rows)))
    E = P16.encode(a.rowptr, a.col, a.val, a.n, a.m, P16.FMT_E5MY, 6, 4, 8)
    pack, offset, order, _ = brute_force_encode(a, P16.FMT_E5MY, 6, 4, 8)
    assert np.array_equal(E.pack, pack) and np.array_equal(E.offset, offset)
    flag, d, _ = P16.unpack_word(E.pack, 6)
    assert E.n_dummies > n  # several chains of two or more


@pytest.mark.parametrize("fmt,D", [(P16.FMT_E5MY, 3), (P16.FMT_E5MY, 7), (P16.FMT_FIX16, 7),
                                   (P16.FMT_FIX16, 2)])
@pytest.mark.parametrize("mode", [P16.PERM_IMPLICIT, P16.PERM_EXPLICIT])
def test_spmv_equals_dense_product_of_quantised_values(fmt, D, mode):
    a = random_csr(3, 300, 250, density=0.04)
    E = P16.encode(a.rowptr, a.col, a.val, a.n, a.m, fmt, D, 8, 32, mode)
    x = np.random.default_rng(1).uniform(-1, 1, a.m)
    A = np.zeros((a.n, a.m))
    A[a.rows(), a.col] = P16.quantized(a.rowptr, a.val, a.n, fmt, D)
    ref = A @ x
    if mode == P16.PERM_EXPLICIT:
        ref = ref[E.stored_rows]
    y = P16.spmv(E, x)
    assert np.max(np.abs(y - ref)) <= 1e-13 * (np.abs(A).sum(1).max() * np.abs(x).max())
    flag, d, _ = P16.unpack_word(E.pack, D)
    assert int(flag.sum()) == a.nnz
    assert int(((flag == 0) & (d > 0)).sum()) == E.n_dummies


def test_laplacian_words_per_row():
    """7-point 16^3 stencil with D = 7: plane jumps of 256 - 16 = 240 need one
    dummy each (two per interior row), line jumps of 15 none."""
    a = W.m2_laplace3d(16)
    E = P16.encode(a.rowptr, a.col, a.val, a.n, a.m, P16.FMT_E5MY, 7, 64, 256)
    flag, d, _ = P16.unpack_word(E.pack, 7)
    assert int(flag.sum()) == a.nnz
    interior = 14 ** 3
    assert E.n_dummies >= 2 * interior
