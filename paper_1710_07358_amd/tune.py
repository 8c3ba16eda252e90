"""Autotuner for the launch table of librd (block, unroll, blocks per CU,
non-temporal loads, chunk order), per (kind, element size, op class, size
bucket, for the plain, compensated, segmented, row-wise and scan kernels), plus
the unroll sweep that mirrors Section 4's execution-time table.

Each candidate is forced through ``rd_config_force`` and timed with HIP
events on the launching stream (median of repeated timed batches).  The
search is coordinate descent from the built-in default: one parameter at a
time over its allowed values, keeping the fastest, for two passes.

Usage (on a GPU):
    python -m paper_1710_07358_amd.tune --out paper_1710_07358_amd/tuned_gfx950.txt
    python -m paper_1710_07358_amd.tune --unroll-sweep
"""
from __future__ import annotations

import argparse
import statistics
import sys
import time

import numpy as np
import torch

from . import api as rd

# representative size per log2(n) bucket of the built-in table
BUCKETS = [(0, 17, 1 << 16), (18, 23, 1 << 22), (24, 62, 1 << 28)]
DTYPE_OF_SIZE = {2: torch.bfloat16, 4: torch.float32, 8: torch.float64}
OPS_OF_CLASS = {0: "sum", 1: "max", 2: "xor"}
SPACE = {
    "plain": {"block": [256, 512, 1024], "unroll": [1, 2, 4, 8, 16], "blocks_per_cu": [1, 2, 4, 8],
              "nontemporal": [0, 1], "layout": [0, 1, 2]},
    "compensated": {"block": [256, 512, 1024], "unroll": [1, 2, 4, 8, 16], "blocks_per_cu": [1, 2, 4],
                    "nontemporal": [0, 1], "layout": [0, 1, 2]},
    "segmented": {"block": [256, 512, 1024], "unroll": [2, 4, 8], "blocks_per_cu": [1, 2, 4, 8],
                  "nontemporal": [0, 1], "layout": [0]},
    "rowwise": {"block": [256], "unroll": [1, 2, 4, 8], "blocks_per_cu": [1, 2, 4, 8],
                "nontemporal": [0, 1], "layout": [0]},
    "rowwise_bwd": {"block": [256], "unroll": [1, 2, 4, 8], "blocks_per_cu": [1, 2, 4, 8],
                    "nontemporal": [0, 1], "layout": [0]},
    # scans: tile = block x unroll x 16 bytes; layout does not apply
    "scan": {"block": [256, 512, 1024], "unroll": [4, 8], "blocks_per_cu": [1, 2, 3, 4],
             "nontemporal": [0, 1], "layout": [0]},
    "segmented_scan": {"block": [256, 512, 1024], "unroll": [4, 8], "blocks_per_cu": [1, 2, 3, 4],
                       "nontemporal": [0, 1], "layout": [0]},
}
KIND_ID = {"plain": 0, "compensated": 1, "segmented": 2, "rowwise": 3, "rowwise_bwd": 4, "scan": 5,
           "segmented_scan": 6}


def time_call(fn, reps: int = 20, batches: int = 3, warm_s: float = 0.05) -> float:
    """Median seconds per call over `batches` timed batches of `reps` calls."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(batches):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) / 1e3 / reps)
    return statistics.median(out)


def _valid(kind: str, cfg: dict) -> bool:
    return cfg["block"] * cfg["blocks_per_cu"] <= 4096


def descend(kind: str, start: dict, run, passes: int = 2, log=None, space: dict | None = None,
            timer=None) -> tuple[dict, float]:
    """Coordinate descent over `space` (default SPACE[kind]) from `start`;
    timer(run) (default time_call) times the forced call."""
    space = SPACE[kind] if space is None else space
    timer = time_call if timer is None else timer
    best = dict(start)
    rd.config_force(kind, best)
    best_t = timer(run)
    for _ in range(passes):
        for key, values in space.items():
            for v in values:
                if v == best[key]:
                    continue
                cand = dict(best, **{key: v})
                if not _valid(kind, cand):
                    continue
                rd.config_force(kind, cand)
                t = timer(run)
                if log:
                    log(f"  {kind} {cand} {t * 1e6:.1f} us")
                if t < best_t:
                    best, best_t = cand, t
    rd.config_force(kind, None)
    return best, best_t


def _case_runner(kind: str, esize: int, opclass: int, n: int, dev):
    dtype = DTYPE_OF_SIZE[esize]
    op = OPS_OF_CLASS[opclass]
    if kind == "segmented":
        from . import workloads as W
        off = W.offsets_from_lengths(W.segment_lengths())
        total, nseg = int(off[-1]), len(off) - 1
        x = (torch.rand(total, device=dev) * 2 - 1).to(dtype)
        offs = torch.from_numpy(off).to(dev)
        out = torch.empty(nseg, dtype=rd.out_dtype(dtype, op), device=dev)
        return (lambda: rd.segmented(x, offs, op, out=out)), total * esize
    if kind in ("rowwise", "rowwise_bwd"):
        rows, cols = 4096, 262144
        rop = {0: "sum", 1: "max", 2: "prod"}[opclass]
        if rop == "prod":  # the benchmark's product rows: factors near 1, zeros at rate 1e-4
            x = torch.rand(rows, cols, device=dev) * 0.02 + 0.99
            x[torch.rand(rows, cols, device=dev) < 1e-4] = 0.0
        else:
            x = torch.randn(rows, cols, device=dev)
        if kind == "rowwise":
            return (lambda: rd.rowreduce_forward(x, rop)), rows * cols * 4
        g = torch.randn(rows, device=dev)
        _, saved = rd.rowreduce_forward(x, rop)
        return (lambda: rd.rowreduce_backward(x, g, saved, rop)), rows * cols * 4
    if kind == "plain":
        if dtype.is_floating_point:
            x = torch.rand(n, device=dev).to(dtype)
        else:
            x = torch.randint(-1000, 1000, (n,), device=dev, dtype=dtype)
        out = torch.empty((), dtype=rd.out_dtype(dtype, op), device=dev)
        return (lambda: rd.reduce(x, op, out=out)), n * esize
    if kind == "compensated":
        x = torch.rand(n, device=dev).to(dtype)
        out = torch.empty((), dtype=torch.float64, device=dev)
        return (lambda: rd.reduce_compensated(x, out=out)), n * esize
    if kind in ("scan", "segmented_scan"):
        if dtype.is_floating_point:
            x = torch.rand(n, device=dev).to(dtype)
        else:
            x = torch.randint(-1000, 1000, (n,), device=dev, dtype=dtype)
        out = torch.empty(n, dtype=rd.out_dtype(dtype, op), device=dev)
        if kind == "scan":
            return (lambda: rd.scan(x, op, out=out)), n * (esize + out.element_size())
        from . import workloads as W
        off = W.offsets_from_lengths(W.segment_lengths())
        offs = torch.from_numpy(np.minimum(off, n)).to(dev)
        return (lambda: rd.scan(x, op, out=out, offsets=offs)), n * (esize + out.element_size())
    raise ValueError(kind)


TABLE_HEADER = "# kind esize opclass log2n_lo log2n_hi block unroll blocks_per_cu nontemporal layout"


def table_line(kind: str, esize: int, opclass: int, lo: int, hi: int, cfg: dict) -> str:
    """One entry of the launch table in the format rd_tune_load reads."""
    return (f"{KIND_ID[kind]} {esize} {opclass} {lo} {hi} {cfg['block']} {cfg['unroll']} "
            f"{cfg['blocks_per_cu']} {cfg['nontemporal']} {cfg['layout']}")


def tune_table(kinds, esizes, log) -> list[str]:
    dev = torch.device("cuda", torch.cuda.current_device())
    lines = [TABLE_HEADER]
    for kind in kinds:
        row_kind = kind in ("rowwise", "rowwise_bwd")
        for esize in esizes:
            if kind == "compensated" and esize == 8:
                continue
            if row_kind and esize != 4:
                continue  # row-wise kernels are float32 only
            for opclass in (0, 1, 2):
                if kind == "compensated" and opclass != 0:
                    continue

                if esize == 2 and opclass == 2:
                    continue  # 16-bit bitwise: keep defaults
                # the segmented, row-wise and scan launches are planned for one size bucket
                buckets = [(0, 62, 1 << 28)] if kind in ("segmented", "rowwise", "rowwise_bwd", "scan",
                                                         "segmented_scan") else BUCKETS
                for lo, hi, n in buckets:
                    run, nbytes = _case_runner(kind, esize, opclass, n, dev)
                    cls_op = "prod" if (row_kind and opclass == 2) else OPS_OF_CLASS[opclass]
                    start = rd.config_get(kind, DTYPE_OF_SIZE[esize], cls_op, n)
                    start["block"] = 256 if row_kind else start["block"]
                    best, t = descend(kind, start, run)
                    log(f"{kind} esize={esize} opclass={opclass} n=2^{n.bit_length() - 1}: {best} "
                        f"{t * 1e6:.1f} us {nbytes / t / 1e9:.0f} GB/s")
                    lines.append(table_line(kind, esize, opclass, lo, hi, best))
                    del run
                    torch.cuda.empty_cache()
    return lines


def unroll_sweep(n: int, log) -> list[dict]:
    """Time the plain float32 sum for U = 1, 2, 4, 8, 16 with the rest of the
    tuned configuration fixed (the MI355X analogue of Section 4's table)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    x = torch.rand(n, device=dev) * 2 - 1
    out = torch.empty((), device=dev)
    base = rd.config_get("plain", torch.float32, "sum", n)
    rows = []
    for u in (1, 2, 4, 8, 16):
        rd.config_force("plain", dict(base, unroll=u))
        t = time_call(lambda: rd.reduce(x, "sum", out=out), reps=50)
        rows.append({"unroll": u, "ms": t * 1e3, "GBps": 4 * n / t / 1e9})
    rd.config_force("plain", None)
    t1 = rows[0]["ms"]
    for r in rows:
        r["speedup"] = t1 / r["ms"]
        r["usage_pct"] = 100 * r["GBps"] / 8000.0
        log(f"U={r['unroll']:2d}  {r['ms']:.5f} ms  {r['speedup']:.3f}x  {r['GBps']:.1f} GB/s  {r['usage_pct']:.2f}%")
    return rows


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="write the tuned table here")
    ap.add_argument("--kinds", default="plain,compensated,segmented,rowwise,rowwise_bwd,scan,segmented_scan")
    ap.add_argument("--esizes", default="2,4,8")
    ap.add_argument("--unroll-sweep", action="store_true")
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    if args.unroll_sweep:
        for n in (5_533_214, 1 << 28):
            log(f"unroll sweep, float32 sum, n={n}")
            unroll_sweep(n, log)
        return 0
    lines = tune_table(args.kinds.split(","), [int(e) for e in args.esizes.split(",")], log)
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    else:
        sys.stdout.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
