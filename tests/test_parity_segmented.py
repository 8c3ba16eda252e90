"""Segmented reduction (one persistent launch): HIP path against the CPU oracle."""
import math
import zlib

import numpy as np
import pytest

import oracle
from helpers import gpu_available, to_gpu, same_float
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402


def _gpu_out_as_oracle(out: torch.Tensor, dtype: str, op: str) -> np.ndarray:
    """GPU segment results in the oracle's representation (uint64 bits or float64)."""
    o = out.cpu()
    if dtype in ("int32", "uint32", "int64", "uint64") or op in ("and", "or", "xor"):
        size = o.element_size()
        view = {2: torch.int16, 4: torch.int32, 8: torch.int64}[size]
        v = o.view(view).numpy().astype(np.int64)
        if size < 8:
            v = v % (1 << (8 * size))
            return v.astype(np.uint64)
        return o.view(torch.int64).numpy().view(np.uint64)
    return o.to(torch.float64).numpy()


def check_segments(x_np, off, op, dtype, out):
    got = _gpu_out_as_oracle(out, dtype, op)
    ref = oracle.segmented(x_np, off, op, dtype)
    nseg = len(off) - 1
    if dtype in ("int32", "uint32", "int64", "uint64") or op in ("and", "or", "xor"):
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"{op}/{dtype}: {bad.size} segments differ, first {bad[:5]}"
        return
    if op in ("min", "max"):
        for s in range(nseg):
            assert same_float(float(got[s]), float(ref[s])), (op, dtype, s, got[s], ref[s])
        return
    if op == "sum":
        for s in range(nseg):
            a, b = int(off[s]), int(off[s + 1])
            _, asum = oracle.exact_sum(x_np[a:b], dtype)
            assert abs(got[s] - ref[s]) <= 2.0 ** -20 * asum, (s, got[s], ref[s])
        return
    if op == "prod":
        for s in range(nseg):
            n = int(off[s + 1] - off[s])
            bound = max(n - 1, 0) * 2.0 ** -53 * 1.001 + (0.0 if dtype == "float64" else 2.0 ** -24)
            ref_out = ref[s] if dtype == "float64" else float(np.float32(ref[s]))
            if ref_out == 0.0 or math.isinf(ref_out) or math.isnan(ref_out):
                assert same_float(float(got[s]), ref_out), (s, got[s], ref[s])
            else:
                assert abs(got[s] - ref[s]) <= bound * abs(ref[s]), (s, got[s], ref[s])


def run(x_np, off, op, dtype, pad=0):
    print(f"[segmented] op={op} dtype={dtype} nseg={len(off) - 1} n={int(off[-1])} pad={pad}", flush=True)
    x = to_gpu(x_np, dtype, pad_front=pad)
    offs = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).cuda()
    out = rd.segmented(x, offs, op)
    torch.cuda.synchronize()
    check_segments(x_np, off, op, dtype, out)
    return out


def mixed_lengths(rng, nseg, big=40_000):
    kinds = rng.integers(0, 5, size=nseg)
    lens = np.where(kinds == 0, 0, np.where(kinds == 1, 1, np.where(kinds == 2, rng.integers(2, 70, nseg),
                    np.where(kinds == 3, rng.integers(70, 3000, nseg), rng.integers(3000, big, nseg)))))
    return lens.astype(np.int64)


@pytest.mark.parametrize("dtype", ["int32", "uint32", "float32", "float64", "float16", "bfloat16", "int64", "uint64"])
@pytest.mark.parametrize("op", ["sum", "prod", "min", "max", "and", "or", "xor"])
def test_segmented_mixed_lengths(op, dtype):
    rng = np.random.default_rng(zlib.crc32(f"{op}/{dtype}".encode()))
    lens = mixed_lengths(rng, 700)
    off = W.offsets_from_lengths(lens)
    x = W.plain(int(off[-1]), dtype, op, config=1, salt=17)
    run(x, off, op, dtype)


@pytest.mark.parametrize("dtype", ["int32", "float32", "float64", "bfloat16"])
def test_segmented_edge_layouts(dtype):
    op = "sum"
    n = 300_007
    x = W.plain(n, dtype, op, config=1, salt=5)
    cases = {
        "one segment": np.array([0, n]),
        "all empty": np.array([0, 0, 0, 0]),
        "empty ends": np.array([0, 0, 0, 5, n, n, n]),
        "offset start and end": np.array([3, 17, 1000, n - 9]),
        "length one": np.arange(0, 5001),
        "one long then many short": np.concatenate([[0], np.arange(200_000, n + 1, 7), [n]]),
    }
    for name, off in cases.items():
        off = np.unique(off) if name not in ("all empty", "empty ends") else off
        print(name, flush=True)
        run(x, off.astype(np.int64), op, dtype)
        run(x, off.astype(np.int64), "max" if dtype != "int32" else "xor", dtype)
    # misaligned base pointer
    run(x, np.array([0, 11, 4000, n]), op, dtype, pad=1)


def test_segmented_single_segment_equals_plain():
    x_np = W.plain(2 ** 22 + 3, "float32", "sum", salt=8)
    x = to_gpu(x_np, "float32")
    seg = rd.segmented(x, torch.tensor([0, x_np.size], dtype=torch.int64, device="cuda"), "max")
    plain = rd.reduce(x, "max")
    assert seg.item() == plain.item() == oracle.reduce(x_np, "max", "float32")


@pytest.mark.parametrize("block", [64, 1024])
def test_segmented_one_segment_over_every_work_group(block):
    # every wavefront's piece crosses its range: the pieces combine per
    # work-group (1 or 16 wavefronts) and then across all work-groups
    x_np = W.plain(2 ** 23 + 5, "int32", "sum", salt=11)
    off = np.array([0, x_np.size], np.int64)
    try:
        rd.config_force("segmented", dict(block=block, unroll=2, blocks_per_cu=2, nontemporal=1, layout=0))
        run(x_np, off, "sum", "int32")
        run(x_np, np.array([0, 3, x_np.size - 2, x_np.size], np.int64), "xor", "int32")
    finally:
        rd.config_force("segmented", None)


@pytest.mark.parametrize("block,unroll,windows", [(64, 2, 70_000), (512, 2, 70_000), (1024, 2, 70_000),
                                                   (256, 4, 20_000)])
def test_segmented_window_boundaries(block, unroll, windows):
    # Segment ends on, just before and just after the edges of windows (64 x U
    # vectors, dealt round-robin to a work-group's wavefronts) and of rounds
    # (one window per wavefront), over enough data that every work-group runs
    # several batches: covers a wavefront carrying a segment's elements from
    # one of its windows to its next, and the in-order join of window pieces.
    wb = block // 64
    win = 64 * unroll * 4  # int32 / float32 elements per window
    rng = np.random.default_rng(block + unroll)
    base = [win, win - 1, 1, win + 1, wb * win, wb * win - 1, 2, wb * win + 1, (wb + 1) * win, 3 * win - 5, 0, 7,
            (wb - 1) * win + 3 if wb > 1 else 5, 64 * wb * win + 11]
    lens = []
    while sum(lens) < windows * win:  # 70,000 windows: > 256 per work-group, several join batches
        lens.extend(base[i] for i in rng.permutation(len(base)))
        lens.extend(int(v) for v in rng.integers(0, 3 * win, 20))
    off = W.offsets_from_lengths(np.array(lens, np.int64))
    x_np = W.plain(int(off[-1]), "int32", "sum", salt=21)
    xf = W.segmented_values(int(off[-1]), "sum", salt=22)
    try:
        rd.config_force("segmented", dict(block=block, unroll=unroll, blocks_per_cu=1, nontemporal=1, layout=0))
        run(x_np, off, "sum", "int32")
        run(x_np, off, "xor", "int32", pad=1)
        run(xf, off, "sum", "float32", pad=3)
    finally:
        rd.config_force("segmented", None)


def test_segmented_long_segments_span_many_wavefronts():
    lens = np.array([1, 2 ** 22, 5, 2 ** 22 - 1, 3, 2 ** 21 + 17], np.int64)
    off = W.offsets_from_lengths(lens)
    for op in ("sum", "max", "min"):
        x = W.segmented_values(int(off[-1]), op, salt=3)
        run(x, off, op, "float32")
    xi = W.plain(int(off[-1]), "int32", "sum", salt=4)
    run(xi, off, "sum", "int32")
    run(xi, off, "xor", "int32")


def test_segmented_every_config_identical_int_results():
    rng = np.random.default_rng(12)
    lens = mixed_lengths(rng, 3000)
    off = W.offsets_from_lengths(lens)
    x_np = W.plain(int(off[-1]), "int32", "sum", salt=9)
    ref = oracle.segmented(x_np, off, "sum", "int32")
    x = to_gpu(x_np, "int32")
    offs = torch.from_numpy(off).cuda()
    try:
        for block in (64, 256, 1024):
            for unroll in (2, 4, 8):
                for bpc in (1, 3, 8):
                    rd.config_force("segmented", dict(block=block, unroll=unroll, blocks_per_cu=bpc,
                                                      nontemporal=bpc % 2, layout=0))
                    got = rd.segmented(x, offs, "sum").cpu().view(torch.int32).numpy().astype(np.int64) % 2 ** 32
                    assert np.array_equal(got.astype(np.uint64), ref), (block, unroll, bpc)
    finally:
        rd.config_force("segmented", None)


def test_segmented_deterministic():
    lens = W.segment_lengths(nseg=4096, salt=2)
    off = W.offsets_from_lengths(lens)
    x = to_gpu(W.segmented_values(int(off[-1]), "sum", salt=2), "float32")
    offs = torch.from_numpy(off).cuda()
    first = rd.segmented(x, offs, "sum").cpu()
    for _ in range(5):
        assert torch.equal(rd.segmented(x, offs, "sum").cpu().view(torch.int32), first.view(torch.int32))


def test_segmented_graph_replay_with_new_data():
    lens = W.segment_lengths(nseg=2048, salt=6)
    off = W.offsets_from_lengths(lens)
    n = int(off[-1])
    offs = torch.from_numpy(off).cuda()
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    out = torch.empty(len(lens), dtype=torch.float32, device="cuda")
    ws = rd.Workspace()
    x.copy_(torch.from_numpy(W.segmented_values(n, "max", salt=100)))
    rd.segmented(x, offs, "max", out=out, workspace=ws)  # eager call before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            rd.segmented(x, offs, "max", out=out, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        x_np = W.segmented_values(n, "max", salt=200 + rep)
        x.copy_(torch.from_numpy(x_np))
        graph.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        assert np.array_equal(got, oracle.segmented(x_np, off, "max")), rep
        # eager work between replays
        rd.reduce(x, "sum")
    ws.close()


def test_segmented_capture_needs_a_workspace_or_prior_call():
    off = torch.tensor([0, 4, 8], dtype=torch.int64, device="cuda")
    x = torch.ones(8, device="cuda")
    s = torch.cuda.Stream()  # fresh stream: no default workspace yet
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with pytest.raises(RuntimeError, match="CAPTURE"):
            with torch.cuda.graph(graph, stream=s):
                rd.segmented(x, off, "sum")
    torch.cuda.synchronize()


@pytest.mark.parametrize("op", ["sum", "max"])
def test_segmented_full_workload(op):
    # 65,536 log-normal segments (median 1024), about 2^28 float32 elements
    lens = W.segment_lengths()
    off = W.offsets_from_lengths(lens)
    x_np = W.segmented_values(int(off[-1]), op)
    x = to_gpu(x_np, "float32")
    out = rd.segmented(x, torch.from_numpy(off).cuda(), op)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.segmented(x_np, off, op)
    if op == "max":
        assert np.array_equal(got, ref)
    else:
        # per-segment bound 2^-20 * sum|x|: check on all segments via sums of |x| by prefix sums
        absx = np.abs(x_np.astype(np.float64))
        csum = np.concatenate([[0.0], np.cumsum(absx)])
        abs_seg = csum[off[1:]] - csum[off[:-1]]
        err = np.abs(got - ref)
        assert np.all(err <= 2.0 ** -20 * abs_seg * (1 + 1e-9) + 1e-300), float(np.max(err / np.maximum(abs_seg, 1e-300)))
