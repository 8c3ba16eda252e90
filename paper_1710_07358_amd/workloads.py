"""Seeded synthetic inputs for the reduction workloads.

This module only draws random numbers and lays them out; it contains none of
the reduction's arithmetic, so both the GPU tests and the CPU oracle can take
their inputs from it.  Every generator is numpy ``PCG64`` seeded as
``171007358 + 1000*config + 10*op + dtype`` (plus an optional salt), so a
result row names its inputs by (config, op, dtype, n).

Workloads (the paper measures synthetic vectors only, Section 4):

* config 0 -- plain, n = 2^20: fp32 uniform(-1, 1) for + and max, int32
  uniform in [-2^20, 2^20] for +, xor and min;
* config 1 -- operator/dtype sweep: ints uniform over the full range for
  and/or/xor, in [-1000, 1000] for +/min/max/x (uint32: [0, 1000]); floats
  uniform(-1, 1), and uniform(0.999, 1.001) for x;
* config 2 -- precision sets (uniform[0,1], random-sign log-uniform
  magnitudes, and interleaved +-4^k cancellation pairs) stored as
  bf16/fp16/fp32;
* config 3 -- 65,536 segments with log-normal lengths (median 1024);
* config 4 -- a row-wise matrix with injected ties (max) or zeros (product).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 171007358
OP_INDEX = {"sum": 0, "prod": 1, "min": 2, "max": 3, "and": 4, "or": 5, "xor": 6}
DTYPE_INDEX = {"int32": 0, "uint32": 1, "float32": 2, "float64": 3, "float16": 4, "bfloat16": 5,
               "int64": 6, "uint64": 7}
BITWISE = ("and", "or", "xor")
# numpy storage type of each dtype (bf16 and fp16 travel as uint16 bit patterns)
STORAGE = {"int32": np.int32, "uint32": np.uint32, "float32": np.float32,
           "float64": np.float64, "float16": np.uint16, "bfloat16": np.uint16,
           "int64": np.int64, "uint64": np.uint64}
ELEM_BYTES = {"int32": 4, "uint32": 4, "float32": 4, "float64": 8, "float16": 2, "bfloat16": 2,
              "int64": 8, "uint64": 8}

# log-normal sigma giving mean length 4 x median: 1024 * exp(s^2/2) = 4096
SEGMENT_SIGMA = math.sqrt(2.0 * math.log(4.0))


def seed(config: int, op: str, dtype: str, salt: int = 0) -> int:
    return BASE_SEED + 1000 * config + 10 * OP_INDEX[op] + DTYPE_INDEX[dtype] + 100003 * salt


def generator(config: int, op: str, dtype: str, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed(config, op, dtype, salt)))


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returns uint16 bits."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def to_storage(values: np.ndarray, dtype: str) -> np.ndarray:
    """Store float64/float32 draws in the given float dtype (rounding to nearest)."""
    if dtype == "float32":
        return np.asarray(values, dtype=np.float32)
    if dtype == "float64":
        return np.asarray(values, dtype=np.float64)
    if dtype == "float16":
        return np.asarray(values, dtype=np.float16).view(np.uint16)
    if dtype == "bfloat16":
        return f32_to_bf16_bits(np.asarray(values, dtype=np.float32))
    raise ValueError(dtype)


def _uniform_f32(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    out = rng.random(n, dtype=np.float32)
    out *= np.float32(hi - lo)
    out += np.float32(lo)
    return out


def plain(n: int, dtype: str, op: str, config: int = 1, salt: int = 0) -> np.ndarray:
    """Input vector for the plain reduction (configs 0 and 1)."""
    rng = generator(config, op, dtype, salt)
    if config == 0:
        if dtype == "float32":
            return _uniform_f32(rng, n, -1.0, 1.0)
        if dtype == "int32":
            return rng.integers(-(2 ** 20), 2 ** 20, size=n, endpoint=True, dtype=np.int32)
    if dtype == "int32":
        if op in BITWISE:
            return rng.integers(-(2 ** 31), 2 ** 31, size=n, dtype=np.int64).astype(np.int32)
        return rng.integers(-1000, 1000, size=n, endpoint=True, dtype=np.int32)
    if dtype == "uint32":
        if op in BITWISE:
            return rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        return rng.integers(0, 1000, size=n, endpoint=True, dtype=np.uint32)
    if dtype == "int64":
        if op in BITWISE:
            return rng.integers(0, 2 ** 64 - 1, size=n, dtype=np.uint64, endpoint=True).view(np.int64)
        return rng.integers(-1000, 1000, size=n, endpoint=True, dtype=np.int64)
    if dtype == "uint64":
        if op in BITWISE:
            return rng.integers(0, 2 ** 64 - 1, size=n, dtype=np.uint64, endpoint=True)
        return rng.integers(0, 1000, size=n, endpoint=True, dtype=np.uint64)
    if op in BITWISE:  # raw bit patterns of float data: use ordinary float draws
        lo, hi = -1.0, 1.0
    elif op == "prod":
        lo, hi = 0.999, 1.001
    else:
        lo, hi = -1.0, 1.0
    if dtype == "float64":
        return rng.uniform(lo, hi, size=n)
    return to_storage(_uniform_f32(rng, n, lo, hi), dtype)


def odd_int_supplement(n: int, dtype: str, salt: int = 0) -> np.ndarray:
    """Odd 32-bit integers: units modulo 2^32, so an integer product stays nonzero."""
    rng = generator(1, "prod", dtype, salt + 7)
    if dtype in ("int64", "uint64"):
        v = rng.integers(0, 2 ** 63, size=n, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        return v.view(np.int64) if dtype == "int64" else v
    v = rng.integers(0, 2 ** 31, size=n, dtype=np.uint64) * 2 + 1
    return v.astype(np.uint32).view(np.int32 if dtype == "int32" else np.uint32)


PRECISION_SETS = ("uniform", "logu", "cancel")


def precision(n: int, dtype: str, kind: str, salt: int = 0) -> np.ndarray:
    """Config 2 data sets, stored in dtype (float32 / float16 / bfloat16).

    uniform: U[0, 1].  logu: random sign times 2^U(-40, 40) (float16: 2^U(-14, 15)).
    cancel: blocks [+4^k, u, -4^k, v] with k uniform in 0..50 (float16: 0..7)
    and u, v uniform in [0, 2] -- the footnote example of Section 1.1 at scale.
    """
    rng = generator(2, "sum", dtype, salt + 1 + PRECISION_SETS.index(kind))
    if kind == "uniform":
        v = rng.random(n, dtype=np.float32)
    elif kind == "logu":
        lo, hi = (-14.0, 15.0) if dtype == "float16" else (-40.0, 40.0)
        mag = np.exp2(rng.uniform(lo, hi, size=n))
        sign = np.where(rng.integers(0, 2, size=n, dtype=np.int8) == 1, 1.0, -1.0)
        v = sign * mag
    elif kind == "cancel":
        kmax = 7 if dtype == "float16" else 50
        blocks = (n + 3) // 4
        k = rng.integers(0, kmax, size=blocks, endpoint=True)
        big = np.power(4.0, k)
        small = rng.uniform(0.0, 2.0, size=(blocks, 2))
        v = np.empty((blocks, 4), np.float64)
        v[:, 0] = big
        v[:, 1] = small[:, 0]
        v[:, 2] = -big
        v[:, 3] = small[:, 1]
        v = v.reshape(-1)[:n]
    else:
        raise ValueError(kind)
    return to_storage(v, dtype)


def segment_lengths(nseg: int = 65536, median: float = 1024.0, sigma: float = SEGMENT_SIGMA,
                    lo: int = 1, hi: int = 2 ** 22, salt: int = 0) -> np.ndarray:
    """Config 3 segment lengths: clip(round(exp(N(ln median, sigma^2))), lo, hi)."""
    rng = generator(3, "sum", "float32", salt)
    raw = np.exp(rng.normal(math.log(median), sigma, size=nseg))
    return np.clip(np.rint(raw), lo, hi).astype(np.int64)


def offsets_from_lengths(lengths: np.ndarray) -> np.ndarray:
    """Exclusive prefix of the lengths, nseg + 1 entries starting at 0 (layout, not reduction)."""
    off = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def segmented_values(n: int, op: str, salt: int = 0) -> np.ndarray:
    rng = generator(3, op, "float32", salt + 1)
    return _uniform_f32(rng, n, -1.0, 1.0)


def rowwise(rows: int, cols: int, op: str, salt: int = 0, row0: int = 0) -> np.ndarray:
    """Config 4 matrix (float32, row-major).

    sum/max: N(0, 1).  max additionally copies the row maximum to 1-3 other
    positions (at least one before the original) in 1% of the rows.
    prod: U(0.99, 1.01) with exact zeros at rate 1e-4.
    Rows are generated independently from (salt, row index), so any row
    range [row0, row0 + rows) can be produced on its own.
    """
    out = np.empty((rows, cols), np.float32)
    for i in range(rows):
        r = row0 + i
        rng = np.random.Generator(np.random.PCG64([seed(4, op, "float32", salt), r]))
        if op == "prod":
            row = _uniform_f32(rng, cols, 0.99, 1.01)
            zmask = rng.random(cols) < 1e-4
            row[zmask] = 0.0
        else:
            row = rng.standard_normal(cols, dtype=np.float32)
            if op in ("max", "min") and rng.random() < 0.01 and cols > 1:
                at = int(np.argmax(row) if op == "max" else np.argmin(row))
                copies = int(rng.integers(1, 3, endpoint=True))
                targets = set()
                if at > 0:
                    targets.add(int(rng.integers(0, at)))
                while len(targets) < min(copies, cols - 1):
                    t = int(rng.integers(0, cols))
                    if t != at:
                        targets.add(t)
                row[list(targets)] = row[at]
        out[i] = row
    return out


def tie_rows(rows: int, cols: int, op: str, salt: int = 0) -> np.ndarray:
    """Indices of rows of ``rowwise`` that received duplicated extremes."""
    hit = []
    for r in range(rows):
        rng = np.random.Generator(np.random.PCG64([seed(4, op, "float32", salt), r]))
        rng.standard_normal(cols, dtype=np.float32)
        if rng.random() < 0.01:
            hit.append(r)
    return np.array(hit, np.int64)
