"""Scan (inclusive / exclusive, plain and segmented): HIP path against the CPU oracle.

Tolerances for float sums follow from the arithmetic of the kernel: a term
reaches an output through at most V - 1 (lane total) + 7 (DPP scan) + U - 1
(pieces) + 1 + 15 (earlier wavefronts) + 1 + 1 (tile prefix, rounding to the
accumulator) + V (the lane's running fold) = 2V + U + 24 roundings, each
bounded by u times the running sum of |x| (u = 2^-24 for float32, float16 and
bfloat16 data, which accumulate in float32; 2^-53 for float64).  With V <= 8
and U <= 8 that is at most 48, so |out - exact| <= 48 u sum|x| over the prefix
(tile prefixes travel in float64 and add far less).  The tests hold float32,
float16 and bfloat16 sums to the float-sum bar 2^-20 sum|x| (tighter than
48 u = 2^-18.4), float64 sums to 48 u.  Products accumulate in float64:
any product tree of k factors is within (k-1) 2^-53 of the exact product,
plus one float32 rounding of the output.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import as_oracle_array, abs_storage, gpu_available, to_gpu, INTS, BITWISE
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402

DTYPES = ["int32", "uint32", "float32", "float64", "float16", "bfloat16", "int64", "uint64"]
OPS = ["sum", "prod", "min", "max", "and", "or", "xor"]
SALT = 7  # scan inputs: their own seeds


def data(n, dtype, op, salt=0):
    if op == "prod" and dtype in INTS:
        return W.odd_int_supplement(n, dtype, salt=SALT + salt)
    return W.plain(n, dtype, op, config=1, salt=SALT + salt)


def check_scan(x_np, op, dtype, out, exclusive, heads=None):
    got = as_oracle_array(out, dtype, op)
    ref = oracle.scan(x_np, op, dtype, exclusive=exclusive, heads=heads)
    assert got.shape == ref.shape
    if dtype in INTS or op in BITWISE:
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"{op}/{dtype} excl={exclusive}: {bad.size} differ, first at {bad[:5]}: " \
                              f"got {got[bad[:5]]}, oracle {ref[bad[:5]]}"
        return
    if op in ("min", "max"):
        both_nan = np.isnan(got) & np.isnan(ref)
        same = (got == ref) & (np.signbit(got) == np.signbit(ref))
        bad = np.nonzero(~(both_nan | same))[0]
        assert bad.size == 0, f"{op}/{dtype}: {bad.size} differ, first at {bad[:5]}"
        return
    if op == "sum":
        u = 2.0 ** -53 if dtype == "float64" else 2.0 ** -24
        scale = oracle.scan(abs_storage(x_np, dtype), "sum", dtype, exclusive=exclusive, heads=heads)
        # the float-sum bar (2^-20 sum|x| over the prefix), or the kernel's
        # own worst-case bound 48u sum|x| where that is tighter (float64)
        tol = min(2.0 ** -20, 48 * u)
        err = np.abs(got - ref)
        bad = np.nonzero(err > tol * scale)[0]
        assert bad.size == 0, f"sum/{dtype}: {bad.size} beyond {tol:.3g} sum|x|, first at {bad[:5]}: " \
                              f"got {got[bad[:5]]}, exact {ref[bad[:5]]}"
        return
    # products: k factors in the prefix (position inside the run)
    n = x_np.size
    start = np.zeros(n, dtype=np.int64)
    if heads is not None:
        h = np.asarray(heads, dtype=np.int64)
        h = h[(h >= 0) & (h < n)]
        start[h] = np.arange(n)[h]
        start = np.maximum.accumulate(start)
    k = np.arange(n) - start + (0 if exclusive else 1)
    out_u = 0.0 if dtype == "float64" else 2.0 ** -24
    bound = np.maximum(k - 1, 0) * 2.0 ** -53 * 1.001 + out_u
    ref_out = ref if dtype == "float64" else ref.astype(np.float32).astype(np.float64)
    special = (ref_out == 0) | np.isinf(ref_out) | np.isnan(ref_out)
    # zeros and infinities carry the xor of the factors' signs; NaN stays NaN
    same = (np.isnan(got) & np.isnan(ref_out)) | ((got == ref_out) & (np.signbit(got) == np.signbit(ref_out)))
    bad = np.nonzero(special & ~same)[0]
    assert bad.size == 0, f"prod/{dtype}: {bad.size} zero/inf/NaN results differ, first at {bad[:5]}"
    ok = np.abs(got - ref) <= bound * np.abs(ref)
    assert np.all(ok | special), f"prod/{dtype}"


def run_scan(x_np, op, dtype, exclusive, heads=None, pad=0, inplace=False):
    print(f"[scan] op={op} dtype={dtype} n={x_np.size} excl={exclusive} "
          f"heads={None if heads is None else len(heads)} pad={pad} inplace={inplace}", flush=True)
    x = to_gpu(x_np, dtype, pad_front=pad)
    offs = None if heads is None else torch.from_numpy(np.ascontiguousarray(heads, dtype=np.int64)).cuda()
    out = rd.scan(x, op, exclusive=exclusive, offsets=offs, out=x if inplace else None)
    torch.cuda.synchronize()
    check_scan(x_np, op, dtype, out, exclusive, heads)
    return out


@pytest.mark.parametrize("exclusive", [False, True])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_scan_every_op_and_dtype(dtype, op, exclusive):
    # 100,003 elements: 13 to 49 tiles depending on the element size, ragged end
    run_scan(data(100_003, dtype, op), op, dtype, exclusive)


@pytest.mark.parametrize("n", [1, 2, 31, 63, 64, 65, 1023, 4095, 4096, 4097, 8191, 12_289])
@pytest.mark.parametrize("dtype,op", [("float32", "sum"), ("int32", "sum"), ("float32", "max"), ("uint64", "xor")])
def test_scan_small_and_tile_edges(n, dtype, op):
    x = data(n, dtype, op, salt=n)
    run_scan(x, op, dtype, False)
    run_scan(x, op, dtype, True)


@pytest.mark.parametrize("block,unroll", [(64, 4), (64, 8), (256, 4), (1024, 8)])
def test_scan_tree_levels(block, unroll):
    # 64-wide work-groups make float32 tiles of 64 x unroll x 4 elements:
    # 8,400,000 elements are 8,203 (unroll 4) or 4,102 (unroll 8) tiles, so the
    # tree of 8-wide groups has five levels (8^4 = 4,096 tiles) and its top
    # level is partly filled
    cfg = {"block": block, "unroll": unroll, "blocks_per_cu": 4, "nontemporal": 1, "layout": 0}
    rd.config_force("scan", cfg)
    rd.config_force("segmented_scan", cfg)
    try:
        x = data(8_400_000, "int32", "sum")
        run_scan(x, "sum", "int32", False)
        run_scan(x, "sum", "int32", True)
        heads = np.arange(0, 8_400_000, 77_777, dtype=np.int64)
        run_scan(x, "sum", "int32", False, heads=heads)
        f = data(300_007, "float32", "sum")
        run_scan(f, "sum", "float32", False)
    finally:
        rd.config_force("scan", None)
        rd.config_force("segmented_scan", None)


def test_scan_one_work_group_and_wide_grid():
    # one persistent work-group walks every tile; then more groups than tiles
    for bpc in (1, 16):
        rd.config_force("scan", {"block": 256, "unroll": 4, "blocks_per_cu": bpc, "nontemporal": 0, "layout": 0})
        try:
            x = data(70_001, "int32", "sum")
            run_scan(x, "sum", "int32", False)
        finally:
            rd.config_force("scan", None)
    # a grid of one: force one compute unit's worth is not possible from here;
    # a one-tile input runs on a single work-group
    run_scan(data(100, "float32", "sum"), "sum", "float32", False)


@pytest.mark.parametrize("dtype,op", [("float32", "sum"), ("int32", "xor"), ("bfloat16", "max"), ("float64", "prod")])
def test_scan_unaligned_and_in_place(dtype, op):
    x = data(50_001, dtype, op)
    run_scan(x, op, dtype, False, pad=1)   # misaligned start: element-wise path everywhere
    run_scan(x, op, dtype, True, pad=3)
    run_scan(x, op, dtype, False, inplace=True)


def test_scan_deterministic_float_sums():
    x_np = data(1 << 22, "float32", "sum")
    x = to_gpu(x_np, "float32")
    a = rd.scan(x, "sum").clone()
    for _ in range(3):
        torch.randn(1 << 20, device="cuda").sum()  # unrelated work in between
        b = rd.scan(x, "sum")
        torch.cuda.synchronize()
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    check_scan(x_np, "sum", "float32", a, False)


def _mixed_offsets(rng, n_target, nseg):
    kinds = rng.integers(0, 5, size=nseg)
    lens = np.where(kinds == 0, 0, np.where(kinds == 1, 1, np.where(kinds == 2, rng.integers(2, 70, nseg),
                    np.where(kinds == 3, rng.integers(70, 3000, nseg), rng.integers(3000, 20_000, nseg)))))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return off[: np.searchsorted(off, n_target) + 1]


@pytest.mark.parametrize("exclusive", [False, True])
@pytest.mark.parametrize("op", ["sum", "prod", "max", "xor"])
@pytest.mark.parametrize("dtype", DTYPES)
def test_segmented_scan(dtype, op, exclusive):
    rng = np.random.default_rng(W.seed(3, op, dtype, SALT))
    off = _mixed_offsets(rng, 150_000, 400)
    n = int(off[-1])
    run_scan(data(n, dtype, op, salt=1), op, dtype, exclusive, heads=off)


def test_segmented_scan_lognormal_lengths():
    lens = W.segment_lengths(nseg=256, median=64.0, salt=SALT)
    off = W.offsets_from_lengths(lens)
    n = int(off[-1])
    for op in ("sum", "max"):
        run_scan(W.segmented_values(n, op, salt=SALT), op, "float32", False, heads=off)


def test_segmented_scan_heads_outside_and_degenerate():
    x = data(30_000, "int32", "sum")
    # offsets that start late, end early, repeat, and leave the range
    heads = np.array([-5, 0, 0, 17, 4096, 4096, 4097, 12_000, 29_999, 30_000, 40_000], dtype=np.int64)
    run_scan(x, "sum", "int32", False, heads=heads)
    run_scan(x, "sum", "int32", True, heads=heads)
    # every element its own segment
    run_scan(x[:9000], "max", "int32", False, heads=np.arange(9001, dtype=np.int64))
    # no offsets at all: the plain scan
    run_scan(x, "xor", "int32", False, heads=np.zeros(0, dtype=np.int64))
    # one segment covering everything
    run_scan(x, "sum", "int32", False, heads=np.array([0, 30_000], dtype=np.int64))


def test_scan_graph_replay():
    x_np = data(200_000, "float32", "sum")
    x = to_gpu(x_np, "float32")
    off_np = _mixed_offsets(np.random.default_rng(5), 200_000, 300)
    offs = torch.from_numpy(off_np).cuda()
    xi_np = data(200_000, "int32", "sum")
    xi = to_gpu(xi_np, "int32")
    ws = rd.Workspace()
    eager = rd.scan(x, "sum", workspace=ws).clone()
    eager_seg = rd.scan(xi, "sum", offsets=offs, workspace=ws).clone()
    out = torch.empty_like(eager)
    out_seg = torch.empty_like(eager_seg)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            rd.scan(x, "sum", out=out, workspace=ws)
            rd.scan(xi, "sum", offsets=offs, out=out_seg, workspace=ws)
    for rep in range(4):
        out.zero_()
        out_seg.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), eager.view(torch.int32)), rep
        assert torch.equal(out_seg, eager_seg), rep
        rd.scan(x, "max", workspace=ws)  # eager launches between replays advance the epoch too
        torch.cuda.synchronize()
    check_scan(x_np, "sum", "float32", eager, False)
    check_scan(xi_np, "sum", "int32", eager_seg, False, heads=off_np)


def test_scan_full_size_int32_and_sampled_float32():
    # the benchmark's size: 2^28 elements
    n = 1 << 28
    xi_np = W.plain(n, "int32", "sum", config=1, salt=SALT)
    got = rd.scan(to_gpu(xi_np, "int32"), "sum")
    torch.cuda.synchronize()
    check_scan(xi_np, "sum", "int32", got, False)
    del got
    xf_np = W.plain(n, "float32", "sum", config=1, salt=SALT)
    out = rd.scan(to_gpu(xf_np, "float32"), "sum")
    torch.cuda.synchronize()
    for i in (4095, 4096 * 64 + 5, (1 << 27) + 12_345, n - 1):
        ref, asum = oracle.exact_sum(xf_np[: i + 1], "float32")
        got_i = float(out[i].item())
        assert abs(got_i - ref) <= 2.0 ** -20 * asum, (i, got_i, ref)
