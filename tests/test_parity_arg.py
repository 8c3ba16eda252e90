"""Arg-reduction (min/max and the lowest index attaining it) against the oracle."""
import math

import numpy as np
import pytest

import oracle
from helpers import INTS, bits_of, gpu_available, same_float, to_gpu, value_of
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402

DTYPES = ["int32", "uint32", "int64", "uint64", "float32", "float64", "float16", "bfloat16"]


def check(x_np, op, dtype, pad=0):
    print(f"[arg] op={op} dtype={dtype} n={x_np.size} pad={pad}", flush=True)
    val, idx = rd.argreduce(to_gpu(x_np, dtype, pad_front=pad), op)
    torch.cuda.synchronize()
    ref_v, ref_i = oracle.argextreme(x_np, op, dtype)
    assert int(idx.item()) == ref_i, (op, dtype, x_np.size, int(idx.item()), ref_i)
    if dtype in INTS:
        assert bits_of(val) == ref_v, (op, dtype)
    else:
        assert same_float(value_of(val), ref_v), (op, dtype, value_of(val), ref_v)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["min", "max"])
def test_arg_random_with_ties(op, dtype):
    rng = np.random.default_rng(DTYPES.index(dtype) * 2 + (op == "max"))
    for n in (1, 7, 9, 1025, 100_003, 2 ** 20 + 7):
        x = W.plain(n, dtype, op, config=1, salt=n)
        if n > 10:
            ext_at = np.sort(rng.choice(n, size=4, replace=False))
            ext = x.max() if op == "max" else x.min()
            x[ext_at] = ext  # ties: the lowest of these (or an earlier natural one) wins
        check(x, op, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_arg_empty_and_misaligned(dtype):
    for op in ("min", "max"):
        val, idx = rd.argreduce(to_gpu(np.zeros(0, W.STORAGE[dtype]), dtype), op)
        assert int(idx.item()) == -1
        x = W.plain(65_537, dtype, op, config=1, salt=3)
        for pad in (1, 2, 3):
            check(x, op, dtype, pad=pad)


@pytest.mark.parametrize("dtype", ["float32", "float64", "float16", "bfloat16"])
def test_arg_float_specials(dtype):
    n = 300_001
    base = W.plain(n, dtype, "max", config=1, salt=1)
    nan = W.to_storage(np.array([math.nan]), dtype)[0]
    for at in (0, 5, 4095, 299_999):
        x = base.copy()
        x[at] = nan
        x[min(at + 17, n - 1)] = nan
        check(x, "max", dtype)
        check(x, "min", dtype)
    z = W.to_storage(np.array([-0.0, 0.0, -0.0, 0.0]), dtype)
    check(z, "max", dtype)
    check(z, "min", dtype)
    neg_inf = W.to_storage(np.full(5000, -math.inf), dtype)
    check(neg_inf, "max", dtype)  # all equal to max's neutral element: index 0
    pos_inf = W.to_storage(np.full(5000, math.inf), dtype)
    check(pos_inf, "min", dtype)


@pytest.mark.parametrize("dtype", INTS)
def test_arg_int_neutral_values(dtype):
    info = np.iinfo(W.STORAGE[dtype])
    check(np.full(4099, info.min, W.STORAGE[dtype]), "max", dtype)
    check(np.full(4099, info.max, W.STORAGE[dtype]), "min", dtype)
    x = np.full(70_001, info.min, W.STORAGE[dtype])
    x[[900, 70_000]] = info.max
    check(x, "max", dtype)
    check(x, "min", dtype)


def test_arg_full_size():
    x = W.plain(2 ** 28, "float32", "max", config=1, salt=28)
    x[[123_456_789, 200_000_000]] = np.float32(2.0)
    check(x, "max", "float32")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["min", "max"])
def test_arg_production_shape(op, dtype):
    # n = 2^24 + 7 selects the launch-table row the 2^28 inputs use
    n = 2 ** 24 + 7
    t = {"int32": torch.int32, "uint32": torch.uint32, "int64": torch.int64, "uint64": torch.uint64,
         "float32": torch.float32, "float64": torch.float64, "float16": torch.float16,
         "bfloat16": torch.bfloat16}[dtype]
    assert rd.config_get("plain", t, op, n) == rd.config_get("plain", t, op, 2 ** 28)
    x = W.plain(n, dtype, op, config=1, salt=24)
    rng = np.random.default_rng(24 + DTYPES.index(dtype))
    ext_at = np.sort(rng.choice(n, size=3, replace=False))
    x[ext_at] = x.max() if op == "max" else x.min()  # ties: the lowest index wins
    check(x, op, dtype)
