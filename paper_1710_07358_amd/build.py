"""Build librd.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Every source under csrc/ is compiled in parallel into _build/, then linked
into paper_1710_07358_amd/librd.so.  HIP device code is built with packed
FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librd.so")
ARCH = os.environ.get("RD_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags() -> list[str]:
    return ["-O3", "-fPIC", "-std=c++17", "-Wall", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *_flags(), "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), *_flags(), "-x", "hip", "-c", src, "-o", obj]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"  # the host pass does not know the device feature
    msgs = [l for l in (proc.stdout + proc.stderr).splitlines() if l.strip() and noise not in l]
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
    if msgs:
        print("\n".join(msgs), file=sys.stderr)
    return obj


def build(jobs: int | None = None) -> str:
    """Compile every HIP/C++ source and link librd.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    # objects no current source produces (an older source layout) are removed,
    # so _build/ holds exactly what is linked
    wanted = {os.path.basename(src) + ".o" for src in srcs}
    for f in os.listdir(BUILD):
        if f.endswith(".o") and f not in wanted:
            os.remove(os.path.join(BUILD, f))
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
