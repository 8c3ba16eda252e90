"""Precision experiment: plain (float32-accumulated) and compensated sums of
bfloat16 / float16 / float32 data sets against the exact oracle."""
import math

import numpy as np
import pytest

import oracle
from helpers import gpu_available, to_gpu, value_of
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402


@pytest.mark.parametrize("kind", W.PRECISION_SETS)
@pytest.mark.parametrize("dtype", ["bfloat16", "float16", "float32"])
def test_precision_sets(dtype, kind):
    n = 2 ** 24 + 5
    x_np = W.precision(n, dtype, kind)
    exact, abs_sum = oracle.exact_sum(x_np, dtype)
    x = to_gpu(x_np, dtype)
    plain = value_of(rd.reduce(x, "sum"))
    comp = value_of(rd.reduce_compensated(x))
    print(f"[precision] {dtype} {kind}: exact={exact!r} sum|x|={abs_sum!r} "
          f"plain_err={abs(plain - exact) / abs_sum:.3e} comp_err={abs(comp - exact) / abs_sum:.3e}", flush=True)
    assert abs(plain - exact) <= 2.0 ** -20 * abs_sum
    assert abs(comp - exact) <= 2.0 ** -40 * abs_sum


def test_compensated_recovers_cancellation_exactly_small():
    # the footnote example repeated with absorbing magnitudes interleaved
    vals = []
    for k in range(0, 51, 5):
        vals += [4.0 ** k, 1.5, -(4.0 ** k), 0.25]
    x_np = np.array(vals, np.float32)
    exact, _ = oracle.exact_sum(x_np)
    assert value_of(rd.reduce_compensated(to_gpu(x_np, "float32"))) == exact


@pytest.mark.parametrize("dtype", ["float32", "float16", "bfloat16"])
def test_compensated_edges(dtype):
    for n in (0, 1, 7, 9, 1025, 300_001):
        x_np = W.precision(n, dtype, "logu", salt=n)
        exact, abs_sum = oracle.exact_sum(x_np, dtype)
        for pad in (0, 1):
            got = value_of(rd.reduce_compensated(to_gpu(x_np, dtype, pad_front=pad)))
            assert abs(got - exact) <= 2.0 ** -40 * abs_sum, (n, pad, got, exact)
