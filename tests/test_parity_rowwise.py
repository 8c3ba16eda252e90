"""Row-wise forward and hand-written backward: HIP path against the CPU
oracle's definitions, FP64 finite differences, and the autograd Function."""
import math

import numpy as np
import pytest

import oracle
from helpers import gpu_available, same_float
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402

OPS = ["sum", "max", "min", "prod"]
SHAPES = [(1, 1), (3, 5), (7, 4099), (2, 16384), (5, 16385), (4, 40_000), (3, 65_536 + 3)]


def prod_grad_ok(got, ref):
    # NaN and infinite entries (IEEE products of the other entries, e.g.
    # 0 x inf) must match exactly; finite ones within 2^-12 |ref| plus a floor
    # relative to the row's largest finite gradient
    nan_r, inf_r = np.isnan(ref), np.isinf(ref)
    if not (np.array_equal(np.isnan(got), nan_r) and np.array_equal(np.isinf(got), inf_r)
            and np.array_equal(got[inf_r], ref[inf_r])):
        return False
    fin = ~(nan_r | inf_r)
    r = np.where(fin, ref, 0.0)
    g = np.where(fin, got, 0.0)
    scale = np.max(np.abs(r), axis=1, keepdims=True)
    return bool(np.all(np.abs(g - r) <= 2.0 ** -12 * np.abs(r) + 2.0 ** -40 * scale))


def check_forward(x_np, op, y, saved):
    yref, idx, z = oracle.row_forward(x_np, op)
    got = y.cpu().numpy().astype(np.float64)
    if op == "sum":
        for r in range(x_np.shape[0]):
            _, a = oracle.exact_sum(x_np[r])
            assert abs(got[r] - yref[r]) <= 2.0 ** -20 * a, (r, got[r], yref[r])
    elif op in ("max", "min"):
        assert np.array_equal(got, yref, equal_nan=True), (got, yref)
        real = ~np.isnan(yref)
        assert np.array_equal(np.signbit(got[real]), np.signbit(yref[real]))  # -0 < +0
        gidx = saved[: 8 * x_np.shape[0]].cpu().view(torch.int64).numpy()
        assert np.array_equal(gidx, idx)
    else:
        for r in range(x_np.shape[0]):
            ref32 = float(np.float32(yref[r]))  # the float32 output rounds once
            if ref32 == 0.0 or math.isinf(ref32) or math.isnan(ref32):
                # a zero keeps its sign (the xor of every factor's sign)
                assert same_float(got[r], ref32), (r, got[r], yref[r])
            else:
                n = x_np.shape[1]
                bound = (n - 1) * 2.0 ** -53 * 1.001 + 2.0 ** -24
                assert abs(got[r] - yref[r]) <= bound * abs(yref[r]), (r, got[r], yref[r])


def check_backward(x_np, op, g_np, grad):
    ref = oracle.row_grad(x_np, op, g_np.astype(np.float64))
    got = grad.cpu().numpy().astype(np.float64)
    if op in ("sum", "max", "min"):
        assert np.array_equal(got, ref.astype(np.float32).astype(np.float64))
    else:
        assert prod_grad_ok(got, ref), float(np.max(np.abs(got - ref) / (np.abs(ref) + 1e-300)))


def run_rows(x_np, op, g_np=None, pad=False):
    rows, cols = x_np.shape
    print(f"[rowwise] op={op} shape={x_np.shape} pad={pad}", flush=True)
    if pad:  # rows not 16-byte aligned: view into a larger buffer
        big = torch.empty(rows * cols + 1, dtype=torch.float32, device="cuda")
        x = big[1:].view(rows, cols)
        x.copy_(torch.from_numpy(x_np))
    else:
        x = torch.from_numpy(x_np).cuda()
    y, saved = rd.rowreduce_forward(x, op)
    torch.cuda.synchronize()
    check_forward(x_np, op, y, saved)
    if g_np is None:
        g_np = np.linspace(-2.0, 3.0, rows).astype(np.float32)
    grad = rd.rowreduce_backward(x, torch.from_numpy(g_np).cuda(), saved, op)
    torch.cuda.synchronize()
    check_backward(x_np, op, g_np, grad)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("shape", SHAPES)
def test_rowwise_shapes(op, shape):
    rows, cols = shape
    rng = np.random.default_rng(rows * 1000 + cols)
    if op == "prod":
        x = rng.uniform(0.99, 1.01, size=shape).astype(np.float32)
    else:
        x = rng.standard_normal(shape).astype(np.float32)
    run_rows(x, op)
    run_rows(x, op, pad=True)


@pytest.mark.parametrize("op", OPS)
def test_rowwise_every_step_width(op):
    # The forward walks a row in steps of 1024 x S columns (whole steps
    # pipelined, one ragged step guarded); the launch table may pick any S.
    # Widths: below one step, one whole step, whole steps plus one column, and
    # a product chunk (16,384 columns) plus a ragged remainder.
    rng = np.random.default_rng(31)
    try:
        for S in (1, 2, 4, 8):
            rd.config_force("rowwise", dict(block=256, unroll=S, blocks_per_cu=2, nontemporal=S % 2, layout=0))
            for cols in (1000, 1024 * S, 3 * 1024 * S + 1, 16384 + 1024 * S + 7):
                shape = (3, cols)
                x = (rng.uniform(0.99, 1.01, size=shape) if op == "prod" else rng.standard_normal(shape)).astype(np.float32)
                if op == "prod":
                    x[1, cols // 2] = 0.0  # one zero: the backward's single-zero rule
                run_rows(x, op)
                run_rows(x, op, pad=True)
    finally:
        rd.config_force("rowwise", None)


@pytest.mark.parametrize("op", ["max", "min"])
def test_rowwise_ties_lowest_index(op):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 50_000)).astype(np.float32)
    ext = np.float32(9.0 if op == "max" else -9.0)
    x[0, [17, 49_999]] = ext
    x[1, [40_000, 3, 16_384]] = ext        # lowest index 3, across chunks
    x[2, :] = ext                         # all equal -> column 0
    x[3, [16_383, 16_384]] = ext          # chunk boundary
    x[4, [0, 1]] = ext
    x[5, 7] = np.float32("nan")           # NaN wins, first NaN
    x[5, 9] = np.float32("nan")
    run_rows(x, op)


def test_rowwise_signed_zero_extremes():
    x = np.array([[-0.0, 0.0, -0.0, 0.0], [0.0, -0.0, 0.0, -0.0]], np.float32)
    run_rows(x, "max")
    run_rows(x, "min")


@pytest.mark.parametrize("op", OPS)
def test_rowwise_empty_rows(op):
    # cols = 0: every row reduces to the neutral element (max/min: column -1)
    for rows in (1, 5, 3000):
        x = np.zeros((rows, 0), np.float32)
        y, saved = rd.rowreduce_forward(torch.empty((rows, 0), device="cuda"), op)
        torch.cuda.synchronize()
        ident = {"sum": 0.0, "max": -math.inf, "min": math.inf, "prod": 1.0}[op]
        assert np.all(y.cpu().numpy() == ident), (op, rows)
        check_forward(x, op, y, saved)
        grad = rd.rowreduce_backward(torch.empty((rows, 0), device="cuda"),
                                     torch.ones(rows, device="cuda"), saved, op)
        assert tuple(grad.shape) == (rows, 0)


def test_rowwise_prod_signed_zeros():
    # IEEE: the sign of a product is the xor of its factors' signs, zeros
    # included; 0 x inf is NaN (Section 1.1's x combiner on floats)
    rows = [[-0.0, 2.0, 3.0], [-0.0, -2.0, 1.0], [0.0, -2.0, 1.0], [-0.0, -0.0, 5.0], [0.0, -0.0, 1.0],
            [math.inf, 0.0, 1.0], [-0.0, 1.0, 1.0], [2.0, -0.0, -1.0]]
    x = np.array(rows, np.float32)
    run_rows(x, "prod")
    y, _ = rd.rowreduce_forward(torch.from_numpy(x).cuda(), "prod")
    got = y.cpu().numpy()
    for r, row in enumerate(rows):
        expect = math.prod(row)
        if math.isnan(expect):
            assert math.isnan(got[r]), r
        else:
            assert got[r] == expect and math.copysign(1.0, got[r]) == math.copysign(1.0, expect), (r, got[r])
    # the same rows spread over a long row: zeros far apart, in different chunks
    wide = np.ones((4, 40_000), np.float32)
    wide[0, [3, 30_000]] = [-0.0, -0.0]
    wide[1, [17_000]] = -0.0
    wide[1, 39_999] = -1.0
    wide[2, [0, 16_384, 39_999]] = [-0.0, 0.0, -0.0]
    wide[3, [20_000]] = -0.0
    wide[3, [5]] = -3.0
    run_rows(wide, "prod")


def test_rowwise_prod_zero_counts():
    rng = np.random.default_rng(5)
    x = rng.uniform(0.95, 1.05, size=(6, 40_000)).astype(np.float32)
    x[1, 12_345] = 0.0                      # one zero
    x[2, [5, 39_999]] = 0.0                 # two zeros
    x[3, 16_384] = 0.0                      # one zero at a chunk start
    x[4, :] = 0.0                           # all zeros
    x[5, [0]] = -0.0                        # one negative zero
    run_rows(x, "prod")


@pytest.mark.parametrize("op", ["sum", "max", "prod"])
def test_rowwise_finite_differences_slice(op):
    # FP64 central differences of the exact function on a 64 x 1024 slice
    x = W.rowwise(64, 1024, op, salt=11)
    g = np.random.default_rng(1).standard_normal(64).astype(np.float32)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    y = rd.rowreduce(xt, op)
    y.backward(torch.from_numpy(g).cuda())
    grad = xt.grad.cpu().numpy().astype(np.float64)
    x64 = x.astype(np.float64)
    f = {"sum": np.sum, "max": np.max, "prod": np.prod}[op]
    h = 2.0 ** -12
    rng = np.random.default_rng(2)
    checked = 0
    for r in range(64):
        cols = rng.choice(1024, size=16, replace=False)
        if op == "max":
            cols = np.append(cols, int(np.argmax(x64[r])))
        for j in cols:
            if op == "max":
                others = np.delete(x64[r], j)
                gap = abs(x64[r, j] - np.max(others))
                if gap < 2 * h:  # a tie within the step: one-sided slopes differ
                    continue
            up, dn = x64[r].copy(), x64[r].copy()
            up[j] += h
            dn[j] -= h
            fd = g[r] * (f(up) - f(dn)) / (2 * h)
            tol = 2.0 ** -12 * abs(fd) + 1e-6 * abs(g[r]) * (abs(f(x64[r])) if op == "prod" else 1.0)
            assert abs(grad[r, j] - fd) <= tol, (op, r, j, grad[r, j], fd)
            checked += 1
    assert checked > 500


def test_rowwise_autograd_matches_kernels():
    x = W.rowwise(16, 5000, "max", salt=2)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    g = torch.linspace(-1, 1, 16, device="cuda")
    rd.rowreduce(xt, "max").backward(g)
    y, saved = rd.rowreduce_forward(torch.from_numpy(x).cuda(), "max")
    direct = rd.rowreduce_backward(torch.from_numpy(x).cuda(), g, saved, "max")
    assert torch.equal(xt.grad, direct)


def test_rowwise_prod_supplement_no_zero_rows():
    # rows without zeros take the prefix/suffix-scan path at full width
    x = W.rowwise(8, 262_144, "prod", salt=7)
    x[x == 0] = np.float32(1.0)
    x[5, 1000] = 0.0  # and one row with a single zero
    run_rows(x, "prod")


@pytest.mark.parametrize("op", ["sum", "max", "prod"])
def test_rowwise_full_shape_sampled_rows(op):
    rows, cols = 4096, 262_144
    x_np = W.rowwise(rows, cols, op)
    x = torch.from_numpy(x_np).cuda()
    g_np = np.random.default_rng(4).standard_normal(rows).astype(np.float32)
    y, saved = rd.rowreduce_forward(x, op)
    grad = rd.rowreduce_backward(x, torch.from_numpy(g_np).cuda(), saved, op)
    torch.cuda.synchronize()
    sample = [0, 1, rows - 1] + list(np.random.default_rng(9).choice(rows, 6, replace=False))
    if op == "max":
        sample += list(W.tie_rows(rows, cols, op)[:4])
    sample = sorted(set(int(s) for s in sample))
    ysub = y[sample]
    if op in ("max", "min"):
        full_idx = saved[: 8 * rows].view(torch.int64)
        sub_saved = full_idx[sample].contiguous().view(torch.uint8)
    else:
        sub_saved = None
    xs = x_np[sample]
    check_forward(xs, op, ysub, sub_saved if sub_saved is not None else saved)
    check_backward(xs, op, g_np[sample], grad[sample])
    del x, grad
    torch.cuda.empty_cache()


def _mixed_prod_rows(rows, cols, salt):
    # every other row holds one zero (fill kernel), the others none (the
    # exclusive-product kernel, which runs on the library's side stream)
    x = W.rowwise(rows, cols, "prod", salt=salt)
    x[x == 0] = np.float32(1.0)
    x[::2, (77 + salt) % cols] = 0.0
    return x


def test_rowwise_prod_graph_replay_with_side_stream():
    # forward and backward captured in one graph: the backward's fork to the
    # side stream and its join back are captured with it; replays with new
    # data, eager work between them
    rows, cols = 12, 40_000
    g_np = np.linspace(-2.0, 3.0, rows).astype(np.float32)
    g = torch.from_numpy(g_np).cuda()
    x = torch.empty(rows, cols, dtype=torch.float32, device="cuda")
    x.copy_(torch.from_numpy(_mixed_prod_rows(rows, cols, 0)))
    y, saved = rd.rowreduce_forward(x, "prod")  # eager calls before capture
    rd.rowreduce_backward(x, g, saved, "prod")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            yg, sg = rd.rowreduce_forward(x, "prod")
            gg = rd.rowreduce_backward(x, g, sg, "prod")
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        x_np = _mixed_prod_rows(rows, cols, rep + 1)
        print(f"[rowwise] graph replay {rep}", flush=True)
        x.copy_(torch.from_numpy(x_np))
        graph.replay()
        torch.cuda.synchronize()
        check_forward(x_np, "prod", yg, sg)
        check_backward(x_np, "prod", g_np, gg)
        rd.reduce(x.view(-1), "sum")
        torch.cuda.synchronize()


def test_rowwise_prod_backward_two_caller_streams():
    # two callers on two streams share the side stream: each call's join waits
    # for its own exclusive-product launch
    rows, cols = 10, 70_000
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    xs = [_mixed_prod_rows(rows, cols, 5), _mixed_prod_rows(rows, cols, 6)]
    gs = [np.linspace(-1.0, 1.0, rows).astype(np.float32), np.linspace(2.0, -3.0, rows).astype(np.float32)]
    xt = [torch.from_numpy(a).cuda() for a in xs]
    gt = [torch.from_numpy(a).cuda() for a in gs]
    torch.cuda.synchronize()
    grads = []
    for i, st in enumerate(streams):
        with torch.cuda.stream(st):
            _, saved = rd.rowreduce_forward(xt[i], "prod")
            grads.append(rd.rowreduce_backward(xt[i], gt[i], saved, "prod"))
    torch.cuda.synchronize()
    for i in range(2):
        check_backward(xs[i], "prod", gs[i], grads[i])


@pytest.mark.parametrize("op", ["sum", "max", "prod"])
def test_rowwise_backward_fill_over_several_launches(op):
    # 2^22 + 3 one-column rows: more (row, tile) work-groups than one fill
    # launch takes (2^22), so the fill runs as two launches, the second
    # starting at a nonzero row
    rows, cols = (1 << 22) + 3, 1
    rng = np.random.default_rng(11)
    x_np = rng.standard_normal((rows, cols)).astype(np.float32)
    if op == "prod":
        x_np[::3] = 0.0  # rows with a zero (fill) among zero-free rows (exclusive products)
    g_np = rng.standard_normal(rows).astype(np.float32)
    print(f"[rowwise] fill over several launches op={op} rows={rows}", flush=True)
    x = torch.from_numpy(x_np).cuda()
    _, saved = rd.rowreduce_forward(x, op)
    grad = rd.rowreduce_backward(x, torch.from_numpy(g_np).cuda(), saved, op)
    torch.cuda.synchronize()
    check_backward(x_np, op, g_np, grad)
