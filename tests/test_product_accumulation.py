"""Why float products accumulate in float64 (CPU only, numpy and the oracle).

The benchmark's product data are float32 values uniform in [0.999, 1.001].  A
float32 product of such factors stays close to 1.0, where the exact product of
two factors often lies half-way between two float32 neighbours up to a tiny
second-order term of one sign, so round-to-nearest breaks those near-ties in
one direction: the rounding errors are biased, and they add up with the number
of multiplications instead of cancelling.  The reduction kernel folds its
input into G x B x U x V independent slots (grid-stride, 2^21 slots for float32
at the benchmark's launch shape: 512 work-groups of 512 work-items, U = 2,
V = 4) and then multiplies the slots in a tree; emulating that order in numpy
float32 shows the drift is far beyond the rounding-walk bound
|ln(p / p_exact)| <= 8 sqrt(n) u + 4 u (u = 2^-24) that float32 accumulation
would have to meet, while float64 accumulation (what the kernels do) is within
(n - 1) 2^-53 of the exact product, as the GPU parity tests require.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1710_07358_amd import workloads as W

U32 = 2.0 ** -24


def _slot_fold_then_tree(x: np.ndarray, slots: int, dtype) -> float:
    """Slot s folds x[s], x[s + slots], ... in order (the grid-stride walk),
    then the slots multiply pairwise (a tree), all in `dtype`."""
    m = x.reshape(-1, slots).astype(dtype)
    acc = np.ones(slots, dtype)
    for j in range(m.shape[0]):
        acc *= m[j]
    while acc.size > 1:
        acc = acc[0::2] * acc[1::2]
    return float(acc[0])


@pytest.mark.parametrize("n", [2 ** 22, 2 ** 24])
def test_float32_product_accumulation_misses_the_rounding_walk_bound(n):
    x = W.plain(n, "float32", "prod", config=1, salt=28)
    exact = oracle.reduce(x, "prod", "float32")  # double-double left fold
    slots = 2 ** 21
    p32 = _slot_fold_then_tree(x, slots, np.float32)
    walk_bound = 8 * math.sqrt(n) * U32 + 4 * U32
    assert abs(math.log(p32 / exact)) > 2 * walk_bound, (p32, exact)
    # float64 accumulation in the same order meets the worst-case product bound
    p64 = _slot_fold_then_tree(x, slots, np.float64)
    assert abs(p64 - exact) <= (n - 1) * 2.0 ** -53 * abs(exact)
