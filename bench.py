#!/usr/bin/env python3
"""Benchmark of the MI355X parallel reduction (one JSON line on stdout).

Headline: float32 sum over n = 2^28 elements (1 GiB, uniform(-1, 1), seeded),
one launch of the plain kernel per step, inputs resident in HBM.  Bandwidth
counts the input bytes once, in decimal GB/s -- the convention of the
execution-time table of Section 4 (5,533,214 x 4 B / 0.249780 ms = 88.6 GB/s).

Also measured (outside the timed headline loop) and reported in the same line:
* segmented: 65,536 log-normal segments (~2^28 float32) for + and max, one
  persistent launch per step, captured in a HIP graph and replayed; its time
  per algorithmic byte relative to the plain kernel's;
* row-wise forward + backward over a 4096 x 262144 float32 matrix for +, max
  and x, time per algorithmic byte relative to the plain kernel's;
* the compensated sum at 2^28;
* the precision table: plain and compensated sums of 2^28 bf16/fp16/fp32
  values (uniform, log-uniform random-sign, +-4^k cancellation) against the
  exact sum;
* per_launch: median and minimum of per-launch event times of the headline;
* cpu_baseline: the CPU oracle's Algorithm 1 left fold of the same 2^28 input,
  one thread and every usable core, each the median of 5 runs, with the core
  count and CPU model; the exact long-accumulator sum's time is reported as
  the cost of correctness;
* paper_context: the Section 4 execution times quoted with their hardware,
  beside this GPU's times at the same n.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-secondary] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "GB/s & % of HBM peak, fp32 sum n=2^28; batched/fwd+bwd vs plain at tol"


def gbps(nbytes: float, seconds: float) -> float:
    """Decimal GB/s of nbytes moved in seconds."""
    return nbytes / seconds / 1e9


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_launches(fn, steps: int, warmup: int, torch) -> float:
    """Average seconds per call of fn() measured with HIP events on the
    current stream (the stream every launch goes to)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3 / steps


def time_each(fn, reps: int, warmup: int, torch) -> list:
    """Seconds of each of `reps` calls of fn(), every call bracketed by its own
    pair of HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) / 1e3 for a, b in ev]


def launch_stats(fn, reps: int, warmup: int, torch) -> dict:
    """Median and minimum of per-launch event times (ms)."""
    ts = sorted(time_each(fn, reps, warmup, torch))
    return {"median_ms": round(ts[len(ts) // 2] * 1e3, 5), "min_ms": round(ts[0] * 1e3, 5), "reps": reps}


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model}


def cpu_fold_baseline(oracle, x_np, runs: int = 5) -> dict:
    """Algorithm 1's left fold of the headline input on the host: one thread,
    then every usable core (contiguous chunks, partials added in chunk order;
    capped by OMP_NUM_THREADS where set), each the median of `runs` runs."""
    info = cpu_info()
    threads = info["usable_cores"]
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    threads = min(threads, 256)
    nbytes = x_np.nbytes

    def median_time(t):
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.fold_sum_f32(x_np, t)
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[runs // 2]

    t1 = median_time(1)
    tn = median_time(threads)
    return {"value": round(gbps(nbytes, t1), 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the full workload ({x_np.size} float32): Algorithm 1 left fold in double, "
                      f"median of {runs} runs",
            "seconds": round(t1, 4),
            "all_cores": {"value": round(gbps(nbytes, tn), 4), "unit": "GB/s", "cores": threads,
                          "seconds": round(tn, 4), "median_of": runs,
                          "note": "contiguous chunk per thread, partial sums added in chunk order"},
            **info}


# The paper's own execution times for this path (Section 4 tables), quoted with
# their hardware as context: one vector of 5,533,214 elements, + as combiner;
# GB/s counts the input bytes once (decimal).
PAPER_SECTION4 = {
    "workload": "one vector of 5,533,214 int32/float32 elements, sum (Section 4)",
    "rows": [
        {"variant": "two-stage reduction (Catanzaro), F=1", "ms": 0.249780, "GBps": 88.61, "pct_of_peak": 26.63,
         "hardware": "OpenCL GPU (model not named in the text), CodeXL profiler, mean of 5 runs"},
        {"variant": "unrolled step 1, F=8", "ms": 0.089490, "GBps": 247.32, "pct_of_peak": 74.32,
         "hardware": "same OpenCL GPU"},
        {"variant": "unrolled step 1, F=16", "ms": 0.088160, "GBps": 251.05, "pct_of_peak": 75.44,
         "hardware": "same OpenCL GPU"},
        {"variant": "Harris kernel 7 (CUDA)", "ms": 0.17766, "GBps": 124.6,
         "hardware": "NVIDIA Tesla C2075"},
        {"variant": "unrolled step 1, CUDA, F=8", "ms": 0.17867, "GBps": 123.9,
         "hardware": "NVIDIA Tesla C2075"},
    ],
}


def bench_segmented(rd, W, oracle, torch, np, steps, warmup, plain_s_per_byte, launch_loop=True):
    lens = W.segment_lengths()
    off = W.offsets_from_lengths(lens)
    n = int(off[-1])
    nseg = len(lens)
    dev = torch.device("cuda")
    res = {"segments": nseg, "elements": n, "lengths": "lognormal median 1024 sigma 1.6651 clip [1, 2^22]"}
    algo_bytes = 4 * n + 8 * (nseg + 1) + 4 * nseg
    offs = torch.from_numpy(off).to(dev)
    rng = np.random.default_rng(7)
    sample = np.unique(np.concatenate([rng.integers(0, nseg, 200), [int(np.argmax(lens))]]))
    for op in ("sum", "max"):
        x_np = W.segmented_values(n, op)
        x = torch.from_numpy(x_np).to(dev)
        out = torch.empty(nseg, dtype=torch.float32, device=dev)
        ws = rd.Workspace()
        rd.segmented(x, offs, op, out=out, workspace=ws)
        torch.cuda.synchronize()
        eager = time_launches(lambda: rd.segmented(x, offs, op, out=out, workspace=ws), steps, warmup, torch)
        # captured once, replayed
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                rd.segmented(x, offs, op, out=out, workspace=ws)
        torch.cuda.current_stream().wait_stream(s)
        replay = time_launches(graph.replay, steps, warmup, torch)
        got = out.cpu().numpy().astype(np.float64)
        worst = 0.0
        for sidx in sample:
            a, b = int(off[sidx]), int(off[sidx + 1])
            seg = x_np[a:b]
            if op == "sum":
                ref, asum = oracle.exact_sum(seg)
                err = abs(got[sidx] - ref) / max(asum, 1e-300)
                worst = max(worst, err)
                assert err <= 2.0 ** -20, (sidx, got[sidx], ref)
            else:
                assert got[sidx] == oracle.reduce(seg, "max", "float32"), sidx
        t = min(eager, replay)
        per_seg = None
        if op == "sum" and launch_loop:
            # baseline: one plain launch per segment (65,536 launches), eager and graph-captured
            outs = torch.empty(nseg, dtype=torch.float32, device=dev)
            views = [x[int(off[i]):int(off[i + 1])] for i in range(nseg)]

            def one_per_segment():
                for i in range(nseg):
                    rd.reduce(views[i], "sum", out=outs[i], workspace=ws)

            one_per_segment()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            one_per_segment()
            torch.cuda.synchronize()
            t_loop = time.perf_counter() - t0
            g2 = torch.cuda.CUDAGraph()
            s2 = torch.cuda.Stream()
            s2.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s2):
                with torch.cuda.graph(g2, stream=s2):
                    one_per_segment()
            torch.cuda.current_stream().wait_stream(s2)
            t_g2 = time_launches(g2.replay, 3, 1, torch)
            got_ps = outs.cpu().numpy().astype(np.float64)
            for sidx in sample:  # the baseline must be right too
                ref, asum = oracle.exact_sum(x_np[int(off[sidx]):int(off[sidx + 1])])
                assert abs(got_ps[sidx] - ref) <= 2.0 ** -20 * asum, sidx
            per_seg = {"launches": nseg, "ms_eager_host_loop": round(t_loop * 1e3, 2),
                       "ms_graph_replay": round(t_g2 * 1e3, 3),
                       "single_launch_speedup_vs_graph": round(t_g2 / t, 1)}
            del g2
        res[op] = {"ms": round(t * 1e3, 4), "ms_eager": round(eager * 1e3, 4), "ms_graph": round(replay * 1e3, 4),
                   "one_launch_per_segment": per_seg,
                   "GBps": round(gbps(algo_bytes, t), 1),
                   "per_byte_vs_plain": round((t / algo_bytes) / plain_s_per_byte, 4),
                   "checked_segments": int(len(sample)),
                   "max_err_over_abs_sum": worst if op == "sum" else 0.0}
        del graph
        ws.close()
    res["algorithmic_bytes"] = algo_bytes
    return res


def bench_precision(rd, W, oracle, torch, n):
    """Error of the float32-accumulated and the compensated sum against the
    exact sum, for each stored dtype and data set (2^28 elements)."""
    dev = torch.device("cuda")
    res = {}
    for dtype in ("bfloat16", "float16", "float32"):
        for kind in W.PRECISION_SETS:
            x_np = W.precision(n, dtype, kind)
            exact, abs_sum = oracle.exact_sum(x_np, dtype)
            if dtype == "float32":
                x = torch.from_numpy(x_np).to(dev)
            else:
                x = torch.from_numpy(x_np.view(np.int16)).to(dev).view(
                    torch.bfloat16 if dtype == "bfloat16" else torch.float16)
            plain = float(rd.reduce(x, "sum").item())
            comp = float(rd.reduce_compensated(x).item())
            ep, ec = abs(plain - exact), abs(comp - exact)
            res[f"{dtype}/{kind}"] = {
                "exact": exact, "sum_abs": abs_sum,
                "plain_err_over_sum_abs": ep / abs_sum, "comp_err_over_sum_abs": ec / abs_sum,
                "plain_err_over_exact": ep / abs(exact) if exact else None,
                "comp_err_over_exact": ec / abs(exact) if exact else None,
                "plain_pass_2^-20": ep <= 2.0 ** -20 * abs_sum, "comp_pass_2^-40": ec <= 2.0 ** -40 * abs_sum}
            log(f"precision {dtype}/{kind}: plain {ep / abs_sum:.3e}  compensated {ec / abs_sum:.3e}")
            del x, x_np
    return res


def bench_rowwise(rd, torch, steps, warmup, plain_s_per_byte):
    """Row-wise forward and backward over a 4096 x 262144 float32 matrix.

    sum, max: normal(0, 1).  prod: uniform(0.99, 1.01) with exact zeros at rate
    1e-4 (about 26 per row, so the gradient is write-only almost everywhere).
    prod_z0: the same values with no zero, every row taking the full-width
    exclusive-product gradient (reads x, writes grad: the dense 8 B/element
    case).  prod_z01: alternate rows hold exactly one zero (write-only rows)."""
    rows, cols = 4096, 262144
    dev = torch.device("cuda")
    gen = torch.Generator(device=dev)
    res = {"shape": [rows, cols]}
    n = rows * cols
    for case in ("sum", "max", "prod", "prod_z0", "prod_z01"):
        op = case.split("_")[0]
        gen.manual_seed(171007358 + 4000 + {"sum": 0, "max": 30, "prod": 10, "prod_z0": 11, "prod_z01": 12}[case])
        if op == "prod":
            x = torch.rand(rows, cols, device=dev, generator=gen) * 0.02 + 0.99
            if case == "prod":
                x[torch.rand(rows, cols, device=dev, generator=gen) < 1e-4] = 0.0
            elif case == "prod_z01":
                at = torch.randint(0, cols, (rows // 2,), device=dev, generator=gen)
                x[torch.arange(1, rows, 2, device=dev), at] = 0.0
        else:
            x = torch.randn(rows, cols, device=dev, generator=gen)
        g = torch.randn(rows, device=dev, generator=gen)
        y, saved = rd.rowreduce_forward(x, op)
        torch.cuda.synchronize()
        t_f = time_launches(lambda: rd.rowreduce_forward(x, op), steps, warmup, torch)
        t_b = time_launches(lambda: rd.rowreduce_backward(x, g, saved, op), steps, warmup, torch)
        fwd_bytes = 4 * n
        row = {}
        if op == "prod":
            zeros = (x == 0).sum(dim=1)
            dense_rows = int((zeros == 0).sum().item())
            bwd_bytes = 4 * n + 4 * dense_rows * cols  # write all; read x for zero-free rows
            row["zero_free_rows"] = dense_rows
            row["bwd_dense_8B_per_elem_GBps"] = round(gbps(8 * n, t_b), 1)
        else:
            bwd_bytes = 4 * n
        t = t_f + t_b
        row.update({"fwd_ms": round(t_f * 1e3, 4), "bwd_ms": round(t_b * 1e3, 4),
                    "fwd_GBps": round(gbps(fwd_bytes, t_f), 1), "bwd_GBps": round(gbps(bwd_bytes, t_b), 1),
                    "bwd_bytes": bwd_bytes,
                    "fwd_per_byte_vs_plain": round((t_f / fwd_bytes) / plain_s_per_byte, 4),
                    "bwd_per_byte_vs_plain": round((t_b / bwd_bytes) / plain_s_per_byte, 4),
                    "per_byte_vs_plain": round((t / (fwd_bytes + bwd_bytes)) / plain_s_per_byte, 4)})
        res[case] = row
        del x, y, saved, g
        torch.cuda.empty_cache()
    return res


def bench_scan(rd, W, oracle, torch, np, steps, warmup, plain_s_per_byte):
    """Inclusive float32 sum scan at n = 2^28 (reads 1 GiB, writes 1 GiB), its
    segmented form over the log-normal segments, and torch.cumsum beside it."""
    dev = torch.device("cuda")
    n = 2 ** 28
    x_np = W.plain(n, "float32", "sum", config=1, salt=7)
    x = torch.from_numpy(x_np).to(dev)
    out = torch.empty_like(x)
    t = time_launches(lambda: rd.scan(x, "sum", out=out), steps, warmup, torch)
    nbytes = 8 * n
    res = {"n": n, "ms": round(t * 1e3, 4), "GBps": round(gbps(nbytes, t), 1),
           "per_byte_vs_plain": round((t / nbytes) / plain_s_per_byte, 4),
           "config": rd.config_get("scan", torch.float32, "sum", n)}
    worst = 0.0
    for i in (4095, (1 << 27) + 12_345, n - 1):
        ref, asum = oracle.exact_sum(x_np[: i + 1])
        worst = max(worst, abs(float(out[i].item()) - ref) / asum)
    res["sampled_err_over_abs_sum"] = worst
    res["pass"] = worst <= 2.0 ** -20
    tc = time_launches(lambda: torch.cumsum(x, 0, out=out), steps, warmup, torch)
    res["torch_cumsum_ms"] = round(tc * 1e3, 4)
    res["torch_cumsum_GBps"] = round(gbps(nbytes, tc), 1)
    del x, out
    torch.cuda.empty_cache()
    lens = W.segment_lengths()
    off_np = W.offsets_from_lengths(lens)
    m = int(off_np[-1])
    xs_np = W.segmented_values(m, "sum")
    xs = torch.from_numpy(xs_np).to(dev)
    offs = torch.from_numpy(off_np).to(dev)
    outs = torch.empty_like(xs)
    ts = time_launches(lambda: rd.scan(xs, "sum", out=outs, offsets=offs), steps, warmup, torch)
    sbytes = 8 * m + 8 * off_np.size
    seg = {"segments": int(lens.size), "elements": m, "ms": round(ts * 1e3, 4), "GBps": round(gbps(sbytes, ts), 1),
           "per_byte_vs_plain": round((ts / sbytes) / plain_s_per_byte, 4)}
    worst = 0.0
    for s_ in (0, 1, lens.size // 2, lens.size - 1):
        a, b = int(off_np[s_]), int(off_np[s_ + 1])
        if b > a:
            ref, asum = oracle.exact_sum(xs_np[a:b])
            worst = max(worst, abs(float(outs[b - 1].item()) - ref) / max(asum, 1e-300))
    seg["sampled_err_over_abs_sum"] = worst
    seg["pass"] = worst <= 2.0 ** -20
    res["segmented"] = seg
    del xs, outs, offs
    torch.cuda.empty_cache()
    return res


def bench_argreduce(rd, torch, x, steps, warmup):
    """Maximum and the lowest index attaining it over the 2^28 float32 input,
    checked against torch (value equal to the maximum, no earlier index
    holding it)."""
    t = time_launches(lambda: rd.argreduce(x, "max"), steps, warmup, torch)
    tv, ti = rd.argreduce(x, "max")
    v, i = float(tv.item()), int(ti.item())
    ok = v == float(x.max().item()) and float(x[i].item()) == v and not bool((x[:i] == v).any().item())
    return {"op": "max", "ms": round(t * 1e3, 4), "GBps": round(gbps(4 * x.numel(), t), 1), "index": i,
            "pass": ok}


def bench_shard(rd, torch, steps, warmup):
    """One GPU's share of the 8-way sharded headline: 2^25 float32 (128 MiB).
    It fits the 256 MB MALL, so the cold figure rotates over 4 such buffers
    (512 MiB); the hot figure re-reads one buffer."""
    dev = torch.device("cuda")
    n = 2 ** 25
    bufs = [torch.rand(n, device=dev) for _ in range(4)]
    out = torch.empty((), device=dev)
    t_hot = time_launches(lambda: rd.reduce(bufs[0], "sum", out=out), steps, warmup, torch)
    state = {"i": 0}

    def rotate():
        state["i"] = (state["i"] + 1) % 4
        rd.reduce(bufs[state["i"]], "sum", out=out)

    t_cold = time_launches(rotate, 4 * steps, warmup, torch)
    res = {"n": n, "cold_ms": round(t_cold * 1e3, 5), "cold_GBps": round(gbps(4 * n, t_cold), 1),
           "hot_ms": round(t_hot * 1e3, 5), "hot_GBps": round(gbps(4 * n, t_hot), 1)}
    del bufs
    torch.cuda.empty_cache()
    return res


def bench_paper_designs(rd, torch, steps, warmup):
    """The paper's two designs (Section 2.3 two-stage; Section 3 unrolled F
    times with the barrier-free tree) beside this library's kernel, float32
    sum, at the paper's n = 5,533,214 and at 2^28."""
    dev = torch.device("cuda")
    res = {}
    for n in (5_533_214, 2 ** 28):
        gen = torch.Generator(device=dev)
        gen.manual_seed(171007358 + 5000)
        x = torch.rand(n, device=dev, generator=gen) * 2 - 1
        out = torch.empty((), device=dev)
        row = {}
        t = time_launches(lambda: rd.reduce(x, "sum", out=out), steps, warmup, torch)
        row["library"] = {"ms": round(t * 1e3, 5), "GBps": round(gbps(4 * n, t), 1)}
        t = time_launches(lambda: rd.reduce_paper_design(x, 0, 1, out=out), steps, warmup, torch)
        row["two_stage"] = {"ms": round(t * 1e3, 5), "GBps": round(gbps(4 * n, t), 1)}
        for f in (1, 2, 4, 8, 16):
            t = time_launches(lambda: rd.reduce_paper_design(x, 1, f, out=out), steps, warmup, torch)
            row[f"unrolled_F{f}"] = {"ms": round(t * 1e3, 5), "GBps": round(gbps(4 * n, t), 1)}
        res[str(n)] = row
        del x
        torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------- HBM traffic

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_reduce_kernel_f32_sum_2p28.txt")
KERNEL_SOURCES = ["paper_1710_07358_amd/csrc/rd_device.hpp", "paper_1710_07358_amd/csrc/reduce_plain.hpp",
                  "paper_1710_07358_amd/csrc/k_f32_plain.hip"]


def kernel_fingerprint(launch: dict) -> str:
    """Hash of the headline kernel's sources and launch shape: counters taken
    for another version of either do not describe this one."""
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    h.update(json.dumps(launch, sort_keys=True).encode())
    return h.hexdigest()[:16]


def read_traffic(launch: dict):
    """HBM bytes per launch from the committed counter summary, or None when
    it was taken for a different kernel build or launch shape."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(None, 1) for line in f if line.strip() and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("fingerprint", "").strip() != kernel_fingerprint(launch):
        return None
    return float(kv["hbm_bytes_per_launch"])


def _pmc_rows(directory: str):
    import csv
    import glob

    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def summarize_pmc(fetch_dir: str, write_dir: str, calib_bytes: int) -> str:
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch) into HBM bytes per launch of the reduce kernel, each counter
    scaled by what it reads for a device copy of calib_bytes."""
    def per_kernel(rows, counter):
        sums = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            key = "reduce" if "reduce_kernel" in r["Kernel_Name"] else (
                "copy" if ("copy" in r["Kernel_Name"].lower() or "elementwise" in r["Kernel_Name"]) else None)
            if key:
                sums.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: sorted(v)[len(v) // 2] for k, v in sums.items()}  # median per dispatch

    fetch = per_kernel(_pmc_rows(fetch_dir), "FETCH_SIZE")
    write = per_kernel(_pmc_rows(write_dir), "WRITE_SIZE")
    kib = calib_bytes / 1024.0
    s_fetch = kib / fetch["copy"]
    s_write = kib / write["copy"]
    reduce_bytes = (fetch["reduce"] * s_fetch + write["reduce"] * s_write) * 1024.0
    return (f"reduce_fetch_kib {fetch['reduce']:.1f}\nreduce_write_kib {write['reduce']:.1f}\n"
            f"copy_fetch_kib {fetch['copy']:.1f}\ncopy_write_kib {write['copy']:.1f}\n"
            f"calibration_copy_bytes {calib_bytes}\nscale_fetch {s_fetch:.5f}\nscale_write {s_write:.5f}\n"
            f"hbm_bytes_per_launch {reduce_bytes:.0f}\nalgorithmic_bytes_per_launch {4 * 2 ** 28}\n")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-secondary", action="store_true", help="headline kernel only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision error table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device copy of the 1 GiB input (counter calibration)")
    ap.add_argument("--only", choices=["compensated", "segmented", "rowwise", "scan", "paper_designs", "shard",
                                       "argreduce"],
                    default=None,
                    help="run one secondary workload alone (for profiling) and print its results")
    ap.add_argument("--no-launch-loop", action="store_true",
                    help="skip the one-launch-per-segment baseline (65,536 launches; for counter runs)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM-traffic summary of two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        import torch  # noqa: F401  (binding import needs it)

        import paper_1710_07358_amd as rd

        launch = rd.config_get("plain", torch.float32, "sum", 2 ** 28)
        sys.stdout.write(summarize_pmc(*args.summarize_pmc, calib_bytes=4 * 2 ** 28))
        print(f"fingerprint {kernel_fingerprint(launch)}")
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              "the reduction's multi-GPU form is not part of this library", file=sys.stderr)
        return 2

    import torch

    import paper_1710_07358_amd as rd
    from paper_1710_07358_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = 2 ** 28
    if args.only:
        import oracle  # the sections check sampled results against the CPU oracle

        xp = torch.from_numpy(W.plain(n, "float32", "sum", config=1, salt=28)).to(dev)
        outp = torch.empty((), dtype=torch.float32, device=dev)
        plain_spb = time_launches(lambda: rd.reduce(xp, "sum", out=outp), 20, 3, torch) / (4 * n)
        del xp
        torch.cuda.empty_cache()
        if args.only == "scan":
            res = bench_scan(rd, W, oracle, torch, np, args.steps, args.warmup, plain_spb)
        elif args.only == "segmented":
            res = bench_segmented(rd, W, oracle, torch, np, args.steps, args.warmup, plain_spb,
                                  launch_loop=not args.no_launch_loop)
        elif args.only == "rowwise":
            res = bench_rowwise(rd, torch, args.steps, args.warmup, plain_spb)
        elif args.only == "paper_designs":
            res = bench_paper_designs(rd, torch, args.steps, args.warmup)
        elif args.only == "shard":
            res = bench_shard(rd, torch, args.steps, args.warmup)
        elif args.only == "argreduce":
            xa = torch.from_numpy(W.plain(n, "float32", "sum", config=1, salt=28)).to(dev)
            res = bench_argreduce(rd, torch, xa, args.steps, args.warmup)
        else:
            x = torch.from_numpy(W.plain(n, "float32", "sum", config=1, salt=28)).to(dev)
            outc = torch.empty((), dtype=torch.float64, device=dev)
            tc = time_launches(lambda: rd.reduce_compensated(x, out=outc), args.steps, args.warmup, torch)
            res = {"ms": round(tc * 1e3, 4), "GBps": round(gbps(4 * n, tc), 1)}
        print(json.dumps({"only": args.only, "result": res}), flush=True)
        return 0
    log("generating input")
    x_np = W.plain(n, "float32", "sum", config=1, salt=28)
    x = torch.from_numpy(x_np).to(dev)
    out = torch.empty((), dtype=torch.float32, device=dev)
    cfg = rd.config_get("plain", torch.float32, "sum", n)
    log(f"timing plain fp32 sum n=2^28 config={cfg}")
    t = time_launches(lambda: rd.reduce(x, "sum", out=out), args.steps, args.warmup, torch)
    nbytes = 4 * n
    achieved = gbps(nbytes, t)
    per_launch = launch_stats(lambda: rd.reduce(x, "sum", out=out), max(20, args.steps), 1, torch)
    got = float(out.item())
    if args.calibrate_copy:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del y

    import oracle  # CPU oracle: correctness check and the cpu_baseline leg

    check = {}
    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle's Algorithm 1 fold on the same input")
        cpu = cpu_fold_baseline(oracle, x_np)
        t0 = time.perf_counter()
        ref, abs_sum = oracle.exact_sum(x_np)
        t_exact = time.perf_counter() - t0
        cpu["correctness_cost_s"] = round(t_exact, 3)  # the exact long-accumulator sum, one thread
        err = abs(got - ref)
        check = {"exact": ref, "gpu": got, "abs_err": err, "abs_sum": abs_sum,
                 "err_over_abs_sum": err / abs_sum, "tol": "2^-20*sum|x|",
                 "pass": err <= 2.0 ** -20 * abs_sum}

    secondary = {}
    if not args.no_secondary:
        plain_spb = t / nbytes
        tsum = time_launches(lambda: torch.sum(x), args.steps, args.warmup, torch)
        secondary["torch_sum"] = {"ms": round(tsum * 1e3, 4), "GBps": round(gbps(nbytes, tsum), 1)}
        log("compensated sum")
        outc = torch.empty((), dtype=torch.float64, device=dev)
        tc = time_launches(lambda: rd.reduce_compensated(x, out=outc), args.steps, args.warmup, torch)
        secondary["compensated"] = {"ms": round(tc * 1e3, 4), "GBps": round(gbps(nbytes, tc), 1)}
        if check:
            ec = abs(float(outc.item()) - check["exact"])
            secondary["compensated"].update({"abs_err": ec, "err_over_abs_sum": ec / check["abs_sum"],
                                             "pass": ec <= 2.0 ** -40 * check["abs_sum"]})
        log("arg-reduction")
        secondary["argreduce"] = bench_argreduce(rd, torch, x, args.steps, args.warmup)
        del x
        torch.cuda.empty_cache()
        log("segmented")
        secondary["segmented"] = bench_segmented(rd, W, oracle, torch, np, max(args.steps // 2, 5),
                                                 args.warmup, plain_spb)
        log("row-wise forward + backward")
        secondary["rowwise"] = bench_rowwise(rd, torch, max(args.steps // 5, 3), 2, plain_spb)
        log("scan")
        secondary["scan"] = bench_scan(rd, W, oracle, torch, np, max(args.steps // 5, 5), 2, plain_spb)
        log("one GPU's shard")
        secondary["shard_2p25"] = bench_shard(rd, torch, args.steps, args.warmup)
        log("the paper's designs")
        secondary["paper_designs"] = bench_paper_designs(rd, torch, max(args.steps // 5, 5), 2)
        if not args.no_precision:
            log("precision sets")
            secondary["precision"] = bench_precision(rd, W, oracle, torch, n)

    line = {
        "metric": METRIC,
        "value": round(achieved, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain float32 sum, n=2^28 (1 GiB) uniform(-1,1), seeded PCG64",
                   "global_batch": n, "seq_len": 1, "parallelism": "single GPU",
                   "launch": cfg},
        "pct_hbm_peak": round(100.0 * achieved / HBM_PEAK_GBPS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": read_traffic(cfg),
                     "kernel": "reduce_kernel<F32 sum>", "bytes_per_launch": nbytes,
                     "avg_launch_ms": round(t * 1e3, 5)},
        "per_launch": per_launch,
        "cpu_baseline": cpu,
        "paper_context": dict(PAPER_SECTION4, mi355x_same_n=secondary.get("paper_designs", {}).get("5533214")),
        "check": check,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
