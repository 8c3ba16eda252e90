"""Plain reduction: HIP path (through the C ABI) against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
from helpers import INTS, TORCH, check_against_oracle, gpu_available, same_float, to_gpu, value_of, bits_of
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402

OPS = ["sum", "prod", "min", "max", "and", "or", "xor"]
SWEEP_N = [1, 31, 1023, 1025, 2 ** 20 + 7]


def _run(x_np, op, dtype, pad=0, compensated=False):
    x = to_gpu(x_np, dtype, pad_front=pad)
    print(f"[plain] op={op} dtype={dtype} n={x_np.size} pad={pad}", flush=True)
    out = rd.reduce_compensated(x) if compensated else rd.reduce(x, op)
    torch.cuda.synchronize()
    abs_sum = None
    if op == "sum" and dtype not in INTS:
        ref, abs_sum = oracle.exact_sum(x_np, dtype)
    else:
        ref = oracle.reduce(x_np, op, dtype)
    check_against_oracle(out, ref, x_np, op, dtype, abs_sum, compensated)
    return out


@pytest.mark.parametrize("op,dtype", [("sum", "float32"), ("max", "float32"), ("sum", "int32"),
                                      ("xor", "int32"), ("min", "int32")])
def test_plain_small_workload(op, dtype):
    # 2^20 elements, the cache-resident workload
    x = W.plain(2 ** 20, dtype, op, config=0)
    _run(x, op, dtype)


@pytest.mark.parametrize("dtype", ["int32", "uint32", "float32", "float64", "int64", "uint64"])
@pytest.mark.parametrize("op", OPS)
def test_plain_sweep(op, dtype):
    for n in SWEEP_N:
        x = W.plain(n, dtype, op, config=1, salt=n)
        _run(x, op, dtype)


@pytest.mark.parametrize("dtype", ["float16", "bfloat16"])
@pytest.mark.parametrize("op", OPS)
def test_plain_half_dtypes(op, dtype):
    for n in [1, 7, 8, 9, 1025, 300_001]:
        x = W.plain(n, dtype, op, config=1, salt=n)
        _run(x, op, dtype)


@pytest.mark.parametrize("dtype", ["int32", "uint32", "float32", "float64", "float16", "bfloat16", "int64"])
@pytest.mark.parametrize("op", ["sum", "max", "xor"])
def test_plain_misaligned_base(op, dtype):
    for pad in (1, 2, 3):
        for n in (5, 1000, 65_537):
            x = W.plain(n, dtype, op, config=1, salt=pad * 7 + n)
            _run(x, op, dtype, pad=pad)


@pytest.mark.parametrize("dtype", ["int32", "uint32", "float32", "float64", "float16", "bfloat16", "int64", "uint64"])
@pytest.mark.parametrize("op", OPS)
def test_plain_empty_is_identity(op, dtype):
    x = np.zeros(0, dtype=W.STORAGE[dtype])
    _run(x, op, dtype)


def test_int_prod_odd_supplement():
    for dtype in INTS:
        x = W.odd_int_supplement(2 ** 20 + 7, dtype)
        _run(x, "prod", dtype)


def test_float_specials():
    nan, inf = math.nan, math.inf
    cases = [
        (np.array([1.0, nan, -5.0, 2.0], np.float32), "max"),
        (np.array([1.0, nan, -5.0, 2.0], np.float32), "min"),
        (np.array([-0.0, 0.0, -0.0], np.float32), "max"),
        (np.array([0.0, -0.0, 0.0], np.float32), "min"),
        (np.array([-inf, -inf], np.float64), "max"),
        (np.array([inf, 1.0], np.float32), "sum"),
    ]
    for x, op in cases:
        dtype = str(x.dtype)
        out = rd.reduce(to_gpu(x, dtype), op)
        torch.cuda.synchronize()
        if op == "sum":
            assert value_of(out) == math.inf
        else:
            assert same_float(value_of(out), oracle.reduce(x, op, dtype)), (x, op)
    # NaN far into a long array, every lane layout
    for at in (0, 5, 4095, 1_000_003):
        x = W.plain(2 ** 20 + 9, "float32", "max", salt=at)
        x[at] = np.float32(nan)
        assert math.isnan(value_of(rd.reduce(to_gpu(x, "float32"), "max")))
        assert math.isnan(value_of(rd.reduce(to_gpu(x, "float32"), "min")))


def test_paper_footnote_example_on_gpu():
    # 1.5 + 4^50 - 4^50: a plain float sum gives 0 or 1.5; compensated gives 1.5
    x = np.array([1.5, 4.0 ** 50, -(4.0 ** 50)], np.float32)
    plain = value_of(rd.reduce(to_gpu(x, "float32"), "sum"))
    assert plain in (0.0, 1.5)
    comp = value_of(rd.reduce_compensated(to_gpu(x, "float32")))
    assert comp == 1.5


def test_coverage_all_ones_every_config():
    # every element is read exactly once, for every launch shape
    n = 3 * 2 ** 20 + 13
    x = np.ones(n, np.int32)
    xg = to_gpu(x, "int32")
    xs = to_gpu(x, "int32", pad_front=1)
    try:
        for block in (64, 256, 1024):
            for unroll in (1, 2, 4, 8, 16):
                for bpc in (1, 3, 8):
                    for nt in (0, 1):
                        for layout in (0, 1, 2):
                            cfg = dict(block=block, unroll=unroll, blocks_per_cu=bpc, nontemporal=nt,
                                       layout=layout)
                            rd.config_force("plain", cfg)
                            assert bits_of(rd.reduce(xg, "sum")) == n, cfg
                            assert bits_of(rd.reduce(xs, "sum")) == n, cfg
    finally:
        rd.config_force("plain", None)


@pytest.mark.parametrize("dtype", ["int64", "float16", "bfloat16", "float64"])
def test_coverage_all_ones_every_config_2_and_8_byte(dtype):
    # the same coverage pin for 2- and 8-byte elements (8 and 2 per 16-byte
    # load): a sum of ones is exact here (float16/bfloat16 accumulate in
    # float32, exact below 2^24), so any skipped or repeated element shows
    n = 3 * 2 ** 20 + 13
    x = W.to_storage(np.ones(n), dtype) if dtype in ("float16", "bfloat16") else np.ones(n, W.STORAGE[dtype])
    xg = to_gpu(x, dtype)
    xs = to_gpu(x, dtype, pad_front=1)
    try:
        for block in (64, 256, 1024):
            for unroll in (1, 2, 4, 8, 16):
                for bpc in (1, 3, 8):
                    for nt in (0, 1):
                        for layout in (0, 1, 2):
                            cfg = dict(block=block, unroll=unroll, blocks_per_cu=bpc, nontemporal=nt,
                                       layout=layout)
                            rd.config_force("plain", cfg)
                            for t in (xg, xs):
                                out = rd.reduce(t, "sum")
                                got = bits_of(out) if dtype == "int64" else value_of(out)
                                assert got == n, (dtype, cfg)
    finally:
        rd.config_force("plain", None)


# Production launch shapes: n = 2^24 + 7 falls in the same launch-table row
# as the benchmark's 2^28 (log2 buckets 24..62) at an eighth of the data, so
# every (op, dtype) runs the exact kernel instantiation and grid the large
# inputs use.
PRODUCTION_N = 2 ** 24 + 7
ALL_DTYPES = ["int32", "uint32", "float32", "float64", "float16", "bfloat16", "int64", "uint64"]


@pytest.mark.parametrize("dtype", ALL_DTYPES)
@pytest.mark.parametrize("op", OPS)
def test_plain_production_shape(op, dtype):
    assert rd.config_get("plain", TORCH[dtype], op, PRODUCTION_N) == rd.config_get("plain", TORCH[dtype], op, 2 ** 28)
    if op == "prod" and dtype in INTS:
        x = W.odd_int_supplement(PRODUCTION_N, dtype, salt=24)  # a nonzero product mod 2^k
    else:
        x = W.plain(PRODUCTION_N, dtype, op, config=1, salt=24)
    _run(x, op, dtype)


@pytest.mark.parametrize("dtype", ["float32", "float16", "bfloat16"])
def test_compensated_production_shape(dtype):
    t = TORCH[dtype]
    assert rd.config_get("compensated", t, "sum", PRODUCTION_N) == rd.config_get("compensated", t, "sum", 2 ** 28)
    x = W.plain(PRODUCTION_N, dtype, "sum", config=1, salt=24)
    _run(x, "sum", dtype, compensated=True)


def test_config_invariance_int_results():
    x = W.plain(2 ** 20 + 7, "int32", "xor", salt=3)
    ref = oracle.reduce(x, "xor", "int32")
    xg = to_gpu(x, "int32")
    try:
        for block, unroll in [(64, 1), (128, 16), (512, 4), (1024, 8)]:
            rd.config_force("plain", dict(block=block, unroll=unroll, blocks_per_cu=4, nontemporal=0))
            assert bits_of(rd.reduce(xg, "xor")) == ref
    finally:
        rd.config_force("plain", None)


def test_float_sum_deterministic():
    x = to_gpu(W.plain(2 ** 22 + 3, "float32", "sum", salt=9), "float32")
    first = bits_of(rd.reduce(x, "sum"))
    for _ in range(10):
        assert bits_of(rd.reduce(x, "sum")) == first


def test_permutation_invariance_ints_and_minmax():
    rng = np.random.default_rng(5)
    x = W.plain(100_003, "int32", "sum", salt=5)
    xp = rng.permutation(x)
    for op in ("sum", "min", "max", "xor", "and", "or"):
        assert bits_of(rd.reduce(to_gpu(x, "int32"), op)) == bits_of(rd.reduce(to_gpu(xp, "int32"), op))
    f = W.plain(100_003, "float32", "max", salt=5)
    fp = rng.permutation(f)
    for op in ("min", "max"):
        assert bits_of(rd.reduce(to_gpu(f, "float32"), op)) == bits_of(rd.reduce(to_gpu(fp, "float32"), op))


@pytest.mark.parametrize("op,dtype", [("sum", "float32"), ("max", "float32"), ("xor", "int32"),
                                      ("min", "int32")])
def test_full_size_2_28(op, dtype):
    # the benchmarked size, in the launch configuration the benchmark uses
    n = 2 ** 28
    x = W.plain(n, dtype, op, config=1, salt=28)
    _run(x, op, dtype)


def test_explicit_workspace_and_stream():
    ws = rd.Workspace()
    s = torch.cuda.Stream()
    x = W.plain(2 ** 20, "float32", "sum", config=0)
    xg = to_gpu(x, "float32")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out = rd.reduce(xg, "sum", workspace=ws)
    s.synchronize()
    ref, a = oracle.exact_sum(x)
    assert abs(value_of(out) - ref) <= 2.0 ** -20 * a
    ws.close()


@pytest.mark.parametrize("dtype", ["float32", "float64", "float16", "bfloat16"])
def test_float_prod_powers_of_two_exact(dtype):
    # ones with planted powers of two: every partial product is an exact power
    # of two, so any grouping gives the exact product (bit-exact coverage pin)
    rng = np.random.default_rng(77)
    for n in (1, 33, 4099, 2 ** 20 + 5):
        e = np.zeros(n, np.int64)
        at = rng.choice(n, size=min(n, 60), replace=False)
        e[at] = rng.choice([-3, -2, -1, 1, 2, 3], size=at.size)
        x = W.to_storage(np.exp2(e.astype(np.float64)), dtype)
        out = rd.reduce(to_gpu(x, dtype), "prod")
        expect = 2.0 ** int(e.sum())
        assert oracle.reduce(x, "prod", dtype) == expect
        assert value_of(out) == expect, (dtype, n)


@pytest.mark.parametrize("dtype", ["int32", "float32"])
def test_paper_design_baselines(dtype):
    # the paper's own designs (two-stage; unrolled with the barrier-free tree)
    for n in (0, 1, 63, 1025, 5_533_214):
        x_np = W.plain(n, dtype, "sum", config=0, salt=n)
        x = to_gpu(x_np, dtype)
        if dtype == "int32":
            ref = oracle.reduce(x_np, "sum", dtype)
        else:
            ref, abs_sum = oracle.exact_sum(x_np)
        for variant, unrolls in ((0, [1]), (1, [1, 2, 3, 4, 5, 6, 7, 8, 16])):
            for f in unrolls:
                out = rd.reduce_paper_design(x, variant, f)
                if dtype == "int32":
                    assert bits_of(out) == ref, (n, variant, f)
                else:
                    assert abs(value_of(out) - ref) <= 2.0 ** -20 * abs_sum, (n, variant, f)
