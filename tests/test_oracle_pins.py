"""Pins for the CPU oracle: every expected value here comes from something
other than the oracle itself -- closed forms, the paper's worked example,
Python's exact integer and rational arithmetic, ``math.fsum`` (correctly
rounded), numpy's own float16 decoding, and brute force on tiny inputs.
"""
import math
import random
from fractions import Fraction
from itertools import permutations

import numpy as np
import pytest

import oracle
from conftest import read_golden

M32 = 2 ** 32
SIZES = [0, 1, 2, 7, 31, 64, 65, 1023, 1025, 100_003]


def _u32(v):
    return v % M32


# ---------------------------------------------------------------- integers

@pytest.mark.parametrize("n", SIZES + [2 ** 20 + 7])
def test_int_sum_closed_form(n):
    # sum_{i=1..n} i = n(n+1)/2, wrapping modulo 2^32 (Algorithm 1, + wraps)
    x = np.arange(1, n + 1, dtype=np.uint64).astype(np.uint32)
    assert oracle.reduce(x, "sum", "uint32") == _u32(n * (n + 1) // 2)
    assert oracle.reduce(x.view(np.int32), "sum", "int32") == _u32(n * (n + 1) // 2)


@pytest.mark.parametrize("n", SIZES)
def test_int_sum_coverage_all_ones(n):
    assert oracle.reduce(np.ones(n, np.int32), "sum", "int32") == n


def test_int_sum_shuffled_signed():
    rng = np.random.default_rng(5)
    x = rng.integers(-1000, 1000, size=50_000, endpoint=True).astype(np.int32)
    expect = _u32(sum(int(v) for v in x))
    assert oracle.reduce(x, "sum", "int32") == expect
    assert oracle.reduce(rng.permutation(x), "sum", "int32") == expect


def _xor_prefix(m):
    # xor of 0..m: m, 1, m+1, 0 for m mod 4 = 0, 1, 2, 3
    return [m, 1, m + 1, 0][m % 4] if m >= 0 else 0


@pytest.mark.parametrize("n", SIZES + [2 ** 20 + 7])
def test_xor_closed_form(n):
    x = np.arange(n, dtype=np.uint32)
    assert oracle.reduce(x, "xor", "uint32") == _xor_prefix(n - 1)


@pytest.mark.parametrize("dtype", ["int32", "uint32"])
def test_and_or_planted_bits(dtype):
    rng = np.random.default_rng(11)
    n = 4096
    allones = np.full(n, 0xFFFFFFFF, np.uint32)
    cleared = 0
    for bit in rng.choice(32, size=9, replace=False):
        allones[rng.integers(0, n)] &= ~np.uint32(1 << int(bit))
        cleared |= 1 << int(bit)
    assert oracle.reduce(allones.view(np.dtype(dtype)), "and", dtype) == (0xFFFFFFFF & ~cleared)
    zeros = np.zeros(n, np.uint32)
    planted = 0
    for bit in rng.choice(32, size=7, replace=False):
        zeros[rng.integers(0, n)] |= np.uint32(1 << int(bit))
        planted |= 1 << int(bit)
    assert oracle.reduce(zeros.view(np.dtype(dtype)), "or", dtype) == planted


@pytest.mark.parametrize("n", [1, 2, 31, 1025, 65_537])
def test_int_min_max_permutation(n):
    rng = np.random.default_rng(n)
    base = -(n // 2)
    x = (rng.permutation(n) + base).astype(np.int32)
    assert oracle.reduce(x, "min", "int32") == _u32(base)
    assert oracle.reduce(x, "max", "int32") == _u32(base + n - 1)
    # unsigned interpretation of the same bits: negatives are huge
    u = x.view(np.uint32)
    assert oracle.reduce(u, "min", "uint32") == min(int(v) for v in u)
    assert oracle.reduce(u, "max", "uint32") == max(int(v) for v in u)


def test_int_min_planted_extreme():
    rng = np.random.default_rng(3)
    x = rng.integers(-1000, 1000, size=10_000).astype(np.int32)
    at = 4321
    x[at] = -2 ** 31
    assert oracle.reduce(x, "min", "int32") == _u32(-2 ** 31)
    x[at] = 2 ** 31 - 1
    assert oracle.reduce(x, "max", "int32") == 2 ** 31 - 1


def test_int_prod():
    assert oracle.reduce(np.ones(1000, np.int32), "prod", "int32") == 1
    x = np.ones(1000, np.int32)
    x[417] = 3
    assert oracle.reduce(x, "prod", "int32") == 3
    rng = np.random.default_rng(17)
    odd = (rng.integers(0, 2 ** 31, size=20_000, dtype=np.uint64) * 2 + 1).astype(np.uint32)
    expect = 1
    for v in odd:
        expect = (expect * int(v)) % M32
    assert oracle.reduce(odd, "prod", "uint32") == expect
    signed = rng.integers(-1000, 1000, size=200).astype(np.int32)
    expect = 1
    for v in signed:
        expect = (expect * int(v)) % M32
    assert oracle.reduce(signed, "prod", "int32") == expect


def test_int_brute_force_all_orders():
    rng = np.random.default_rng(23)
    x = rng.integers(-2 ** 31, 2 ** 31, size=6).astype(np.int32)
    for op in ["sum", "prod", "min", "max", "and", "or", "xor"]:
        results = {oracle.reduce(np.array(p, np.int32), op, "int32") for p in permutations(x)}
        assert len(results) == 1, op


# ------------------------------------------------ 16-bit bit patterns (and/or/xor on float16, bfloat16)

@pytest.mark.parametrize("dtype", ["float16", "bfloat16"])
def test_bitwise_16bit_planted_bits(dtype):
    # and over all-ones patterns with planted cleared bits gives exactly the
    # bits never cleared; or over zeros with planted set bits gives the plants
    rng = np.random.default_rng(41)
    n = 5000
    allones = np.full(n, 0xFFFF, np.uint16)
    cleared = 0
    for bit in rng.choice(16, size=6, replace=False):
        allones[rng.integers(0, n)] &= np.uint16(~(1 << int(bit)) & 0xFFFF)
        cleared |= 1 << int(bit)
    assert oracle.reduce(allones, "and", dtype) == 0xFFFF & ~cleared
    zeros = np.zeros(n, np.uint16)
    planted = 0
    for bit in rng.choice(16, size=5, replace=False):
        zeros[rng.integers(0, n)] |= np.uint16(1 << int(bit))
        planted |= 1 << int(bit)
    assert oracle.reduce(zeros, "or", dtype) == planted
    # the neutral elements are 16 bits wide
    assert oracle.identity("and", dtype) == 0xFFFF
    assert oracle.identity("or", dtype) == 0 and oracle.identity("xor", dtype) == 0


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 1000, 65_536])
def test_bitwise_16bit_xor_closed_form(n):
    x = np.arange(n, dtype=np.uint32).astype(np.uint16)
    assert oracle.reduce(x, "xor", "float16") == _xor_prefix(n - 1)
    assert oracle.reduce(x, "xor", "bfloat16") == _xor_prefix(n - 1)


def test_bitwise_16bit_vs_python_ints():
    import functools
    import operator
    rng = np.random.default_rng(42)
    x = rng.integers(0, 1 << 16, size=3001).astype(np.uint16)
    ints = [int(v) for v in x]
    for op, f, ident in (("and", operator.and_, 0xFFFF), ("or", operator.or_, 0), ("xor", operator.xor, 0)):
        expect = functools.reduce(f, ints, ident)
        assert oracle.reduce(x, op, "bfloat16") == expect
        # running values (scan), inclusive and exclusive, and per segment
        run = list(__import__("itertools").accumulate(ints, f))
        inc = oracle.scan(x, op, "float16")
        exc = oracle.scan(x, op, "float16", exclusive=True)
        assert inc.tolist() == run
        assert exc.tolist() == [ident] + run[:-1]
        off = np.array([0, 0, 17, 1000, 1000, 3001])
        seg = oracle.segmented(x, off, op, "bfloat16")
        for s in range(5):
            assert int(seg[s]) == functools.reduce(f, ints[off[s]:off[s + 1]], ident), (op, s)


def test_bitwise_16bit_scan_xor_closed_form():
    # xor scan of 0..n-1 as 16-bit patterns: position i holds xor(0..i)
    n = 4099
    x = np.arange(n, dtype=np.uint16)
    inc = oracle.scan(x, "xor", "bfloat16")
    assert all(int(inc[i]) == _xor_prefix(i) for i in range(n))


def test_identities():
    # neutral elements: value of the reduction over no elements
    assert oracle.identity("sum", "int32") == 0
    assert oracle.identity("prod", "uint32") == 1
    assert oracle.identity("min", "int32") == 2 ** 31 - 1
    assert oracle.identity("max", "int32") == _u32(-2 ** 31)
    assert oracle.identity("min", "uint32") == M32 - 1
    assert oracle.identity("max", "uint32") == 0
    assert oracle.identity("and", "uint32") == M32 - 1
    assert oracle.identity("min", "float32") == math.inf  # the listing's INFINITY init
    assert oracle.identity("max", "float64") == -math.inf
    assert oracle.identity("sum", "float16") == 0.0
    assert oracle.identity("prod", "bfloat16") == 1.0


# ---------------------------------------------------------------- decoding

def test_decode_every_float16_pattern():
    bits = np.arange(2 ** 16, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)  # numpy's own decoding
    got = np.array([oracle.load_float(bits, i, "float16") for i in range(2 ** 16)])
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.array_equal(np.signbit(got[~nan]), np.signbit(ref[~nan]))


def test_decode_every_bfloat16_pattern():
    bits = np.arange(2 ** 16, dtype=np.uint16)
    ref = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    got = np.array([oracle.load_float(bits, i, "bfloat16") for i in range(2 ** 16)])
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


# ---------------------------------------------------------------- float sums

def test_paper_footnote_example():
    rows = {r[0]: r[1:] for r in read_golden("footnote_example.txt")}
    vals = [float(int(v)) if v.lstrip("-").isdigit() and len(v) > 4 else float(v) for v in rows["values"]]
    exact = float(rows["exact"][0])
    assert vals[1] == 4.0 ** 50
    x = np.array(vals)
    assert oracle.exact_sum(x)[0] == exact
    # every evaluation order of plain double addition gives one of the listed values
    allowed = {float(v) for v in rows["float_results"]}
    for p in permutations(vals):
        assert (p[0] + p[1]) + p[2] in allowed
    assert oracle.exact_sum(x.astype(np.float32), "float32")[0] == exact


@pytest.mark.parametrize("n", [0, 1, 2, 100, 5792])
def test_float_sum_integers_exact(n):
    # 0 + 1 + ... + (n-1) is exactly representable in fp32 for n <= 5792
    x = np.arange(n, dtype=np.float32)
    assert oracle.exact_sum(x, "float32")[0] == n * (n - 1) / 2


def test_float_sum_pairs_cancel():
    rng = np.random.default_rng(8)
    v = rng.uniform(-1e30, 1e30, size=5000)
    x = rng.permutation(np.concatenate([v, -v]))
    assert oracle.exact_sum(x)[0] == 0.0


@pytest.mark.parametrize("n", [1, 10, 1000, 2 ** 20])
def test_float_sum_vs_fsum(n):
    rng = np.random.default_rng(n + 1)
    x64 = rng.uniform(-1, 1, size=n) * np.exp2(rng.integers(-60, 60, size=n))
    assert oracle.exact_sum(x64)[0] == math.fsum(x64)
    x32 = rng.uniform(-1, 1, size=n).astype(np.float32)
    assert oracle.exact_sum(x32, "float32")[0] == math.fsum(x32.astype(np.float64))
    s, a = oracle.exact_sum(x32, "float32")
    assert a == math.fsum(np.abs(x32.astype(np.float64)))


def test_float_sum_vs_fraction_adversarial():
    rng = random.Random(99)
    for trial in range(200):
        n = rng.randint(1, 12)
        vals = []
        for _ in range(n):
            e = rng.choice([-1074, -1060, -1022, -500, -40, 0, 52, 300, 1000])
            vals.append(rng.choice([-1, 1]) * rng.randint(1, 2 ** 53 - 1) * 2.0 ** (e - 52 if e > -1022 else -1074))
        vals = [v for v in vals if math.isfinite(v)]
        exact = sum((Fraction(v) for v in vals), Fraction(0))
        assert oracle.exact_sum(np.array(vals, np.float64))[0] == float(exact), (trial, vals)


def test_float_sum_ties_to_even():
    ulp = 2.0 ** -52
    # 1 + 2^-53 lies halfway between 1 and 1 + 2^-52: rounds to 1 (even)
    assert oracle.exact_sum(np.array([1.0, 2.0 ** -53]))[0] == 1.0
    # (1 + 2^-52) + 2^-53 is halfway to 1 + 2^-51: rounds up to the even one
    assert oracle.exact_sum(np.array([1.0 + ulp, 2.0 ** -53]))[0] == 1.0 + 2 * ulp
    # a tiny extra bit breaks the tie upwards
    assert oracle.exact_sum(np.array([1.0, 2.0 ** -53, 2.0 ** -1074]))[0] == 1.0 + ulp


def test_float_sum_specials():
    big = np.finfo(np.float64).max
    assert oracle.exact_sum(np.array([big, big]))[0] == math.inf
    assert oracle.exact_sum(np.array([big, big, -big]))[0] == big  # exact: no intermediate overflow
    assert math.isnan(oracle.exact_sum(np.array([1.0, math.nan]))[0])
    assert math.isnan(oracle.exact_sum(np.array([math.inf, -math.inf]))[0])
    assert oracle.exact_sum(np.array([math.inf, 1.0]))[0] == math.inf
    assert oracle.exact_sum(np.array([2.0 ** -1074, 2.0 ** -1074]))[0] == 2.0 ** -1073


@pytest.mark.parametrize("dtype", ["float16", "bfloat16"])
def test_half_sums_vs_fraction(dtype):
    rng = np.random.default_rng(4)
    bits = rng.integers(0, 2 ** 16, size=3000, dtype=np.uint16)
    if dtype == "float16":
        dec = bits.view(np.float16).astype(np.float64)
    else:
        dec = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    keep = np.isfinite(dec)
    bits, dec = bits[keep], dec[keep]
    exact = sum((Fraction(float(v)) for v in dec), Fraction(0))
    assert oracle.exact_sum(bits, dtype)[0] == float(exact)


# ---------------------------------------------------------------- float products

def test_prod_powers_of_two_exact():
    rng = np.random.default_rng(12)
    e = rng.integers(-30, 30, size=4000)
    e[-1] = -int(e[:-1].sum()) % 61 - 30
    x = np.exp2(e.astype(np.float64))
    assert oracle.reduce(x, "prod") == 2.0 ** int(e.sum())
    x32 = x.astype(np.float32)
    assert oracle.reduce(x32, "prod", "float32") == 2.0 ** int(e.sum())


def test_prod_vs_fraction():
    rng = np.random.default_rng(13)
    for _ in range(100):
        n = int(rng.integers(1, 30))
        x = rng.uniform(0.5, 2.0, size=n) * rng.choice([-1.0, 1.0], size=n)
        exact = Fraction(1)
        for v in x:
            exact *= Fraction(float(v))
        got = oracle.reduce(x, "prod")
        # double-double keeps ~104 bits: the result is the correctly rounded
        # product, or off by one ulp in a near-tie case
        assert abs(Fraction(got) - exact) <= Fraction(math.ulp(float(exact)))


def test_prod_zero_and_sign():
    assert oracle.reduce(np.array([2.0, 0.0, 5.0]), "prod") == 0.0
    assert oracle.reduce(np.array([-2.0, 3.0]), "prod") == -6.0


# IEEE 754: the sign of a product (zeros and infinities included) is the
# exclusive-or of the factors' signs; inf * 0 is NaN.  Python's own float
# multiplication is IEEE binary64, so math.prod of a few exactly
# representable factors is the expected value, sign bit included.
SIGNED_ZERO_CASES = [
    [-0.0], [0.0], [-2.0, 0.0], [-0.0, 2.0], [-0.0, -2.0], [0.0, -0.0], [-0.0, -0.0],
    [3.0, -0.0, 5.0, -1.0], [-1.0, 0.0, -1.0, -0.0, 7.0], [-math.inf, 2.0], [math.inf, -0.5, -4.0],
    [math.inf, 0.0], [-0.0, math.inf], [1e300, 1e300], [-1e300, 1e300], [1e-300, -1e-300],
]


def _same_bits(a, b):
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b and math.copysign(1.0, a) == math.copysign(1.0, b)


@pytest.mark.parametrize("vals", SIGNED_ZERO_CASES, ids=lambda v: ",".join(map(repr, v)))
def test_prod_signed_zero_and_infinity(vals):
    expect = math.prod(vals)
    got = oracle.reduce(np.array(vals, np.float64), "prod")
    assert _same_bits(got, expect), (vals, got, expect)
    if all(v == 0 or math.isinf(v) or abs(v) in (0.5, 1.0, 2.0, 3.0, 4.0, 5.0, 7.0) for v in vals):
        # the same factors stored as float32, float16 and bfloat16 (all exact)
        f32 = np.array(vals, np.float32)
        assert _same_bits(oracle.reduce(f32, "prod", "float32"), expect)
        assert _same_bits(oracle.reduce(f32.astype(np.float16), "prod", "float16"), expect)
        bf = (f32.view(np.uint32) >> 16).astype(np.uint16)
        assert _same_bits(oracle.reduce(bf, "prod", "bfloat16"), expect)
    # running products carry the same signs, and so does every segment
    run = oracle.scan(np.array(vals, np.float64), "prod", "float64")
    for i in range(len(vals)):
        assert _same_bits(run[i], math.prod(vals[: i + 1])), (vals, i)
    seg = oracle.segmented(np.array(vals * 2, np.float64), np.array([0, len(vals), 2 * len(vals)]), "prod")
    assert _same_bits(seg[0], expect) and _same_bits(seg[1], expect)


# ---------------------------------------------------------------- float min / max

@pytest.mark.parametrize("n", [1, 33, 4097, 2 ** 16 + 3])
def test_float_minmax_permutation(n):
    rng = np.random.default_rng(n)
    x = rng.permutation(n).astype(np.float32) - np.float32(n // 3)
    assert oracle.reduce(x, "min", "float32") == -(n // 3)
    assert oracle.reduce(x, "max", "float32") == n - 1 - n // 3
    h = x.astype(np.float64)
    assert oracle.reduce(h, "max") == n - 1 - n // 3


def test_float_minmax_nan_and_signed_zero():
    v, at = oracle.argextreme(np.array([1.0, math.nan, 5.0, math.nan]), "max", "float64")
    assert math.isnan(v) and at == 1
    v, at = oracle.argextreme(np.array([1.0, math.nan, -5.0]), "min", "float64")
    assert math.isnan(v) and at == 1
    v, at = oracle.argextreme(np.array([-0.0, 0.0, -0.0], np.float32), "max", "float32")
    assert v == 0 and not math.copysign(1, v) < 0 and at == 1
    v, at = oracle.argextreme(np.array([0.0, -0.0, 0.0], np.float32), "min", "float32")
    assert v == 0 and math.copysign(1, v) < 0 and at == 1
    v, at = oracle.argextreme(np.array([-math.inf, -math.inf]), "max", "float64")
    assert v == -math.inf and at == 0


def test_float_minmax_lowest_index_on_ties():
    x = np.array([0.5, 3.0, 2.0, 3.0, 3.0], np.float32)
    assert oracle.argextreme(x, "max", "float32") == (3.0, 1)
    x = np.array([0.5, -3.0, 2.0, -3.0], np.float32)
    assert oracle.argextreme(x, "min", "float32") == (-3.0, 1)


def test_float_minmax_half_dtypes_vs_numpy():
    rng = np.random.default_rng(21)
    h = rng.uniform(-100, 100, size=5000).astype(np.float16)
    assert oracle.reduce(h.view(np.uint16), "max", "float16") == float(h.max())
    assert oracle.reduce(h.view(np.uint16), "min", "float16") == float(h.min())


# ---------------------------------------------------------------- segmented

def test_segmented_reduces_to_plain_and_identity():
    rng = np.random.default_rng(31)
    x = rng.uniform(-1, 1, 10_000).astype(np.float32)
    off = np.array([0, 10_000], np.int64)
    assert oracle.segmented(x, off, "sum")[0] == math.fsum(x.astype(np.float64))
    off = np.array([0, 0, 5, 5, 10_000, 10_000], np.int64)
    out = oracle.segmented(x, off, "max")
    assert out[0] == -math.inf and out[2] == -math.inf and out[4] == -math.inf
    assert out[1] == float(x[:5].max()) and out[3] == float(x[5:].max())
    out = oracle.segmented(x.view(np.uint32), off, "and", "uint32")
    assert out[0] == M32 - 1


def test_segmented_vs_fsum_per_segment():
    rng = np.random.default_rng(32)
    lens = rng.integers(0, 300, size=200)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    x = rng.uniform(-1, 1, int(off[-1])).astype(np.float32)
    out = oracle.segmented(x, off, "sum")
    for s in range(200):
        assert out[s] == math.fsum(x[off[s]:off[s + 1]].astype(np.float64))
    xi = rng.integers(-1000, 1000, int(off[-1])).astype(np.int32)
    outi = oracle.segmented(xi, off, "sum", "int32")
    for s in range(200):
        assert outi[s] == _u32(sum(int(v) for v in xi[off[s]:off[s + 1]]))


# ---------------------------------------------------------------- row-wise

def test_row_forward_and_grad_sum_max():
    rng = np.random.default_rng(41)
    x = rng.standard_normal((5, 300)).astype(np.float32)
    x[2, 17] = x[2, 250] = x[2, 100] = 9.0  # tie: lowest index 17
    g = rng.standard_normal(5)
    y, idx, _ = oracle.row_forward(x, "max")
    assert idx[2] == 17 and y[2] == 9.0
    for r in range(5):
        assert idx[r] == int(np.argmax(x[r]))  # numpy argmax: first occurrence
    gm = oracle.row_grad(x, "max", g)
    expect = np.zeros_like(gm)
    expect[np.arange(5), idx] = g
    assert np.array_equal(gm, expect)
    gs = oracle.row_grad(x, "sum", g)
    assert np.array_equal(gs, np.repeat(g[:, None], 300, axis=1))
    ys, _, _ = oracle.row_forward(x, "sum")
    for r in range(5):
        assert ys[r] == math.fsum(x[r].astype(np.float64))
    yn, idn, _ = oracle.row_forward(-x, "min")
    assert np.array_equal(idn, idx) and np.array_equal(yn, -y)


def test_row_grad_prod_vs_fraction_with_zeros():
    rng = np.random.default_rng(43)
    x = rng.uniform(0.5, 1.5, size=(4, 9)).astype(np.float32)
    x[1, 3] = 0.0                  # one zero
    x[2, 1] = x[2, 7] = 0.0        # two zeros
    g = np.array([1.0, -2.0, 3.0, 0.5])
    grad = oracle.row_grad(x, "prod", g)
    for r in range(4):
        for j in range(9):
            exact = Fraction(float(g[r]))
            for i in range(9):
                if i != j:
                    exact *= Fraction(float(x[r, i]))
            assert abs(Fraction(grad[r, j]) - exact) <= Fraction(math.ulp(float(exact)) if exact else 0)
    assert np.all(grad[2] == 0.0)
    assert np.count_nonzero(grad[1]) == 1 and grad[1, 3] != 0
    _, _, z = oracle.row_forward(x, "prod")
    assert list(z) == [0, 1, 2, 0]


def test_row_grad_prod_central_difference():
    # the product is linear in each coordinate, so a central difference is
    # exact up to rounding
    rng = np.random.default_rng(44)
    x = rng.uniform(0.99, 1.01, size=(2, 64)).astype(np.float32)
    g = np.ones(2)
    grad = oracle.row_grad(x, "prod", g)
    h = 2.0 ** -12
    for r in range(2):
        row = x[r].astype(np.float64)
        for j in range(0, 64, 7):
            up, dn = row.copy(), row.copy()
            up[j] += h
            dn[j] -= h
            fd = (np.prod(up) - np.prod(dn)) / (2 * h)
            assert abs(fd - grad[r, j]) <= 1e-9 * abs(grad[r, j])


# ---------------------------------------------------------------- 64-bit integers

M64 = 2 ** 64


@pytest.mark.parametrize("n", [0, 1, 5, 1023, 100_003])
def test_int64_sum_and_xor_closed_forms(n):
    base = 2 ** 40  # values beyond 32 bits
    x = (np.arange(1, n + 1, dtype=np.uint64) + np.uint64(base))
    assert oracle.reduce(x, "sum", "uint64") == (n * (n + 1) // 2 + n * base) % M64
    assert oracle.reduce(x.view(np.int64), "sum", "int64") == (n * (n + 1) // 2 + n * base) % M64
    y = np.arange(n, dtype=np.uint64)
    assert oracle.reduce(y, "xor", "uint64") == _xor_prefix(n - 1)


def test_int64_min_max_signed_vs_unsigned():
    rng = np.random.default_rng(64)
    x = rng.integers(-2 ** 62, 2 ** 62, size=20_000, dtype=np.int64)
    x[123] = -2 ** 63
    x[777] = 2 ** 63 - 1
    assert oracle.reduce(x, "min", "int64") == (-2 ** 63) % M64
    assert oracle.reduce(x, "max", "int64") == 2 ** 63 - 1
    u = x.view(np.uint64)
    assert oracle.reduce(u, "min", "uint64") == min(int(v) for v in u)
    assert oracle.reduce(u, "max", "uint64") == max(int(v) for v in u)


def test_int64_prod_and_bitwise_vs_python():
    rng = np.random.default_rng(65)
    odd = rng.integers(0, 2 ** 62, size=5000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    expect = 1
    for v in odd:
        expect = (expect * int(v)) % M64
    assert oracle.reduce(odd, "prod", "uint64") == expect
    a = 0xFFFFFFFFFFFFFFFF
    o = 0
    for v in odd[:300]:
        a &= int(v)
        o |= int(v)
    assert oracle.reduce(odd[:300], "and", "uint64") == a
    assert oracle.reduce(odd[:300], "or", "uint64") == o


@pytest.mark.parametrize("dtype", ["int32", "uint32", "int64", "uint64"])
def test_int_argextreme_lowest_index(dtype):
    rng = np.random.default_rng(66)
    x = rng.integers(0, 1000, size=10_000).astype(dtype)
    x[[70, 9000, 4000]] = 5000   # ties for max: lowest index 70
    x[[6000, 30]] = np.array(0, dtype=dtype) if dtype.startswith("u") else -7  # min ties
    vals = [int(v) for v in x]
    for op, f in (("max", max), ("min", min)):
        v, at = oracle.argextreme(x, op, dtype)
        width = 32 if dtype.endswith("32") else 64
        assert v == f(vals) % (2 ** width)
        assert at == vals.index(f(vals))
    assert oracle.argextreme(np.zeros(0, dtype=dtype), "max", dtype)[1] == -1


def test_segmented_int64_vs_python():
    rng = np.random.default_rng(67)
    lens = rng.integers(0, 200, size=100)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    x = rng.integers(-2 ** 62, 2 ** 62, size=int(off[-1]), dtype=np.int64)
    out = oracle.segmented(x, off, "sum", "int64")
    for s in range(100):
        assert int(out[s]) == sum(int(v) for v in x[off[s]:off[s + 1]]) % M64


# ---------------------------------------------------------------- scans
# The scan is the prefix form of the reduction: out[i] reduces x[0..i]
# (inclusive) or x[0..i) (exclusive), restarting at segment heads.

@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 4097, 100_003])
def test_scan_int_sum_closed_form(n):
    # prefix sums of 1..n are k(k+1)/2 (mod 2^32); the exclusive form is shifted by one
    x = np.arange(1, n + 1, dtype=np.uint64).astype(np.uint32)
    k = np.arange(1, n + 1, dtype=np.uint64)
    inc = oracle.scan(x, "sum", "uint32")
    exc = oracle.scan(x, "sum", "uint32", exclusive=True)
    assert np.array_equal(inc, (k * (k + 1) // 2) % M32)
    assert np.array_equal(exc, ((k - 1) * k // 2) % M32)


def test_scan_xor_closed_form():
    n = 5000
    x = np.arange(n, dtype=np.uint32)
    inc = oracle.scan(x, "xor", "uint32")
    assert [int(v) for v in inc] == [_xor_prefix(i) for i in range(n)]
    exc = oracle.scan(x, "xor", "uint32", exclusive=True)
    assert [int(v) for v in exc] == [_xor_prefix(i - 1) for i in range(n)]


@pytest.mark.parametrize("dtype", ["int32", "uint32", "int64", "uint64"])
def test_scan_int_vs_numpy_accumulate(dtype):
    # numpy's cumulative sum / product / extrema / bitwise accumulations, with
    # Python integers reducing modulo the width for + and x
    rng = np.random.default_rng(11)
    width = 32 if "32" in dtype else 64
    signed = dtype.startswith("int")
    n = 3000
    x = rng.integers(-1000 if signed else 0, 1000, size=n, endpoint=True).astype(dtype)
    bits = x.view(np.uint32 if width == 32 else np.uint64).astype(np.uint64)
    mask = (1 << width) - 1
    ref_sum = np.array([v & mask for v in np.cumsum([int(v) for v in x], dtype=object)], dtype=np.uint64)
    assert np.array_equal(oracle.scan(x, "sum", dtype), ref_sum)
    ref_max = np.maximum.accumulate(x).view(bits.dtype if width == 64 else np.uint32).astype(np.uint64)
    ref_min = np.minimum.accumulate(x).view(bits.dtype if width == 64 else np.uint32).astype(np.uint64)
    assert np.array_equal(oracle.scan(x, "max", dtype), ref_max)
    assert np.array_equal(oracle.scan(x, "min", dtype), ref_min)
    for op, uf in (("and", np.bitwise_and), ("or", np.bitwise_or), ("xor", np.bitwise_xor)):
        assert np.array_equal(oracle.scan(x, op, dtype), uf.accumulate(bits)), op
    odd = (rng.integers(0, 1 << 30, size=200) * 2 + 1).astype(dtype)
    run, ref = 1, []
    for v in odd:
        run = (run * int(v)) & mask
        ref.append(run)
    assert np.array_equal(oracle.scan(odd, "prod", dtype), np.array(ref, dtype=np.uint64))


def test_scan_paper_example_exact():
    # Section 1.1's example: 1.5 + 4^50 - 4^50.  The exact prefix sums are 1.5,
    # 4^50 + 1.5 (which rounds to 4^50) and 1.5, not the 0 a double fold gives.
    x = np.array([1.5, 4.0 ** 50, -(4.0 ** 50)])
    assert list(oracle.scan(x, "sum", "float64")) == [1.5, 4.0 ** 50, 1.5]
    assert list(oracle.scan(x, "sum", "float64", exclusive=True)) == [0.0, 1.5, 4.0 ** 50]


def test_scan_float_sum_vs_fsum_prefixes():
    rng = np.random.default_rng(12)
    x = (rng.uniform(-1, 1, 2000) * np.exp2(rng.integers(-30, 30, 2000))).astype(np.float32)
    out = oracle.scan(x, "sum", "float32")
    xs = [float(v) for v in x]
    for i in list(range(0, 2000, 97)) + [1999]:
        assert out[i] == math.fsum(xs[: i + 1]), i
    exc = oracle.scan(x, "sum", "float32", exclusive=True)
    assert exc[0] == 0.0 and all(exc[i] == math.fsum(xs[:i]) for i in range(1, 2000, 131))


def test_scan_float_prod_and_minmax():
    # powers of two multiply exactly; running extrema match numpy's accumulate
    rng = np.random.default_rng(13)
    k = rng.integers(-3, 4, size=300)
    x = np.exp2(k).astype(np.float32)
    assert np.array_equal(oracle.scan(x, "prod", "float32"), np.exp2(np.cumsum(k)).astype(np.float64))
    y = rng.standard_normal(500).astype(np.float32)
    assert np.array_equal(oracle.scan(y, "max", "float32"), np.maximum.accumulate(y).astype(np.float64))
    assert np.array_equal(oracle.scan(y, "min", "float32", exclusive=True)[1:],
                          np.minimum.accumulate(y)[:-1].astype(np.float64))
    assert oracle.scan(y, "min", "float32", exclusive=True)[0] == math.inf
    # a NaN makes every later running extreme NaN (IEEE 754-2019 maximum)
    y[200] = np.nan
    m = oracle.scan(y, "max", "float32")
    assert not np.isnan(m[:200]).any() and np.isnan(m[200:]).all()


def test_scan_half_dtypes_vs_numpy_decoding():
    rng = np.random.default_rng(14)
    h = rng.standard_normal(400).astype(np.float16)
    vals = h.astype(np.float64)
    assert np.array_equal(oracle.scan(h, "max", "float16"), np.maximum.accumulate(vals))
    out = oracle.scan(h, "sum", "float16")
    assert out[-1] == math.fsum(vals.tolist())
    b = (rng.standard_normal(400).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    bvals = (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.array_equal(oracle.scan(b, "min", "bfloat16"), np.minimum.accumulate(bvals))


def test_scan_segments_position_in_segment():
    # x = all ones: the inclusive sum at i is i - head(i) + 1, the exclusive one
    # i - head(i), where head(i) is the last run start <= i (position 0 counts)
    rng = np.random.default_rng(15)
    n = 5000
    heads = np.sort(rng.choice(np.arange(-5, n + 5), size=300))
    heads = np.concatenate([heads, heads[:20]])  # duplicates: empty segments
    heads.sort()
    inc = oracle.scan(np.ones(n, np.int32), "sum", "int32", heads=heads)
    exc = oracle.scan(np.ones(n, np.int32), "sum", "int32", exclusive=True, heads=heads)
    starts = sorted({0} | {int(h) for h in heads if 0 <= h < n})
    last = np.zeros(n, np.int64)
    for s in starts:
        last[s:] = s
    pos = np.arange(n) - last
    assert np.array_equal(inc, pos + 1) and np.array_equal(exc, pos)


def test_scan_segments_end_values_match_segment_reduction():
    # the last inclusive value of each nonempty segment is that segment's
    # reduction (computed by the separate segmented fold)
    rng = np.random.default_rng(16)
    lengths = rng.integers(0, 50, size=200)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    x = rng.integers(-2**31, 2**31, size=int(off[-1])).astype(np.int32)
    for op in ("sum", "max", "xor"):
        inc = oracle.scan(x, op, "int32", heads=off)
        red = oracle.segmented(x, off, op, "int32")
        for s in range(200):
            if lengths[s]:
                assert inc[off[s + 1] - 1] == red[s]


def test_scan_rejects_decreasing_heads():
    with pytest.raises(ValueError):
        oracle.scan(np.ones(10, np.int32), "sum", "int32", heads=np.array([5, 2]))


# ------------------------------------------------- timing baseline (Algorithm 1)

@pytest.mark.parametrize("threads", [1, 2, 3, 8])
@pytest.mark.parametrize("n", [0, 1, 2, 7, 1023, 100_003])
def test_fold_sum_f32_closed_form(n, threads):
    # integers 0..n-1 held exactly in float32 and in the double accumulator:
    # every split gives n(n-1)/2 exactly, also with more threads than elements
    x = np.arange(n, dtype=np.float32)
    assert oracle.fold_sum_f32(x, threads) == n * (n - 1) // 2


@pytest.mark.parametrize("threads", [1, 5])
def test_fold_sum_f32_within_double_fold_bound(threads):
    # a left fold in double over n values is within (n - 1) 2^-53 sum|x| of the
    # exact sum (math.fsum is correctly rounded); the chunked fold adds T - 1
    # more additions, within the same bound
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, 200_001).astype(np.float32)
    exact = math.fsum(x.astype(np.float64))
    bound = (x.size + threads) * 2.0 ** -53 * float(np.abs(x.astype(np.float64)).sum())
    assert abs(oracle.fold_sum_f32(x, threads) - exact) <= bound


def test_fold_sum_f32_rejects_bad_thread_counts():
    with pytest.raises(ValueError):
        oracle.fold_sum_f32(np.ones(4, np.float32), 0)
    with pytest.raises(ValueError):
        oracle.fold_sum_f32(np.ones(4, np.float32), 257)
