"""CPU oracle for the parallel reduction -- TEST INFRASTRUCTURE ONLY.

This package is the correctness reference for the GPU library.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
it; the product path never does, and it imports nothing from the product.

It wraps ``oracle.c`` (plain C, built with gcc, no fast-math) through ctypes:

* integer and bitwise ops: the left fold of Algorithm 1 (Section 1.1) with the
  combiner swapped, wrapping modulo 2^32 for + and x;
* float sums: the exact sum of the stored values, rounded once to double;
* float products: a double-double left fold;
* float min/max: IEEE 754-2019 minimum/maximum (NaN wins, -0 < +0), with the
  lowest attaining index;
* segmented and row-wise forms, and row-wise gradients;
* scans (the prefix form of the reduction), plain or restarted at segment
  heads;
* a timing baseline (not a correctness source): Algorithm 1's float32 left
  fold accumulated in double, on one thread or over several threads.

Arrays are numpy arrays on the host.  bfloat16 data travels as ``uint16``
bit patterns with ``dtype="bfloat16"``; float16 may be ``np.float16`` or
``uint16`` bits with ``dtype="float16"``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OPS = {"sum": 0, "prod": 1, "min": 2, "max": 3, "and": 4, "or": 5, "xor": 6}
DTYPES = {"int32": 0, "uint32": 1, "float32": 2, "float64": 3, "float16": 4, "bfloat16": 5,
          "int64": 6, "uint64": 7}
INT_DTYPES = ("int32", "uint32", "int64", "uint64")
FLOAT_DTYPES = ("float32", "float64", "float16", "bfloat16")
BITWISE = ("and", "or", "xor")
_STORAGE = {"int32": np.int32, "uint32": np.uint32, "float32": np.float32,
            "float64": np.float64, "float16": np.uint16, "bfloat16": np.uint16,
            "int64": np.int64, "uint64": np.uint64}

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(LIB_PATH)
        i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_fold_u32.argtypes = [vp, i64, ci, ci, ctypes.POINTER(ctypes.c_uint32)]
        lib.orc_fold_u64.argtypes = [vp, i64, ci, ci, ctypes.POINTER(ctypes.c_uint64)]
        lib.orc_argext_int.argtypes = [vp, i64, ci, ci, ci, ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_int64)]
        lib.orc_fold_u16.argtypes = [vp, i64, ci, ctypes.POINTER(ctypes.c_uint16)]
        lib.orc_load_float.argtypes = [vp, i64, ci]
        lib.orc_load_float.restype = ctypes.c_double
        lib.orc_exact_sum.argtypes = [vp, i64, ci, dp, dp]
        lib.orc_prod.argtypes = [vp, i64, ci, dp]
        lib.orc_minmax.argtypes = [vp, i64, ci, ci, dp, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_segmented.argtypes = [vp, vp, i64, ci, ci, vp]
        lib.orc_scan.argtypes = [vp, i64, ci, ci, ci, vp, i64, vp]
        lib.orc_row_forward.argtypes = [vp, i64, i64, ci, vp, vp, vp]
        lib.orc_row_grad.argtypes = [vp, i64, i64, ci, vp, vp]
        lib.orc_fold_sum_f32.argtypes = [vp, i64, ci, dp]
        for f in (lib.orc_fold_u32, lib.orc_fold_u64, lib.orc_fold_u16, lib.orc_argext_int, lib.orc_exact_sum,
                  lib.orc_prod, lib.orc_minmax, lib.orc_segmented, lib.orc_scan, lib.orc_row_forward,
                  lib.orc_row_grad, lib.orc_fold_sum_f32):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _storage(x: np.ndarray, dtype: str) -> np.ndarray:
    want = _STORAGE[dtype]
    if dtype == "float16" and x.dtype == np.float16:
        x = x.view(np.uint16)
    if x.dtype != want:
        raise TypeError(f"oracle: array of {x.dtype} does not hold {dtype} data")
    return np.ascontiguousarray(x)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle: {what} returned {rc}")


def identity(op: str, dtype: str):
    """Neutral element of op for dtype: the value of a reduction over no elements."""
    x = np.zeros(0, dtype=_STORAGE[dtype])
    return reduce(x, op, dtype)


def reduce(x: np.ndarray, op: str, dtype: str | None = None):
    """x0 (op) x1 (op) ... (op) x(n-1) for a 1-D host array.

    Returns a Python int holding the unsigned bit pattern for integer dtypes
    and for bitwise ops on float dtypes (32/64/16 bits wide as stored), and a
    Python float otherwise (exact-then-rounded sum, double-double product,
    exact min/max).
    """
    dtype = dtype or str(x.dtype)
    x = _storage(np.ravel(x), dtype)
    lib, n = _load(), x.size
    if dtype in ("int32", "uint32") or (dtype == "float32" and op in BITWISE):
        out = ctypes.c_uint32()
        _check(lib.orc_fold_u32(_ptr(x), n, OPS[op], int(dtype == "int32"), ctypes.byref(out)), op)
        return out.value
    if dtype in ("int64", "uint64") or (dtype == "float64" and op in BITWISE):
        out64 = ctypes.c_uint64()
        _check(lib.orc_fold_u64(_ptr(x), n, OPS[op], int(dtype == "int64"), ctypes.byref(out64)), op)
        return out64.value
    if op in BITWISE:
        out16 = ctypes.c_uint16()
        _check(lib.orc_fold_u16(_ptr(x), n, OPS[op], ctypes.byref(out16)), op)
        return out16.value
    d = ctypes.c_double()
    if op == "sum":
        _check(lib.orc_exact_sum(_ptr(x), n, DTYPES[dtype], ctypes.byref(d), None), op)
    elif op == "prod":
        _check(lib.orc_prod(_ptr(x), n, DTYPES[dtype], ctypes.byref(d)), op)
    elif op in ("min", "max"):
        _check(lib.orc_minmax(_ptr(x), n, DTYPES[dtype], int(op == "max"), ctypes.byref(d), None), op)
    else:
        raise ValueError(op)
    return d.value


def exact_sum(x: np.ndarray, dtype: str | None = None) -> tuple[float, float]:
    """(sum, sum of |x|) of the stored float values, each exact then rounded once."""
    dtype = dtype or str(x.dtype)
    x = _storage(np.ravel(x), dtype)
    s, a = ctypes.c_double(), ctypes.c_double()
    _check(_load().orc_exact_sum(_ptr(x), x.size, DTYPES[dtype], ctypes.byref(s), ctypes.byref(a)), "sum")
    return s.value, a.value


def argextreme(x: np.ndarray, op: str, dtype: str | None = None) -> tuple:
    """(min or max value, lowest index attaining it; -1 when empty).

    Integer dtypes report the value as its unsigned bit pattern."""
    dtype = dtype or str(x.dtype)
    x = _storage(np.ravel(x), dtype)
    if dtype in INT_DTYPES:
        v, at = ctypes.c_uint64(), ctypes.c_int64()
        width = 32 if dtype in ("int32", "uint32") else 64
        _check(_load().orc_argext_int(_ptr(x), x.size, width, int(dtype.startswith("int")), int(op == "max"),
                                      ctypes.byref(v), ctypes.byref(at)), op)
        return v.value, at.value
    d, at = ctypes.c_double(), ctypes.c_int64()
    _check(_load().orc_minmax(_ptr(x), x.size, DTYPES[dtype], int(op == "max"),
                              ctypes.byref(d), ctypes.byref(at)), op)
    return d.value, at.value


def load_float(x: np.ndarray, i: int, dtype: str) -> float:
    """Exact double value of stored element i of a float array."""
    x = _storage(np.ravel(x), dtype)
    return _load().orc_load_float(_ptr(x), int(i), DTYPES[dtype])


def segmented(x: np.ndarray, offsets: np.ndarray, op: str, dtype: str | None = None) -> np.ndarray:
    """out[s] = reduce(x[offsets[s]:offsets[s+1]], op).

    float64 results for float data with sum/prod/min/max, else uint64 bit
    patterns (zero-extended)."""
    dtype = dtype or str(x.dtype)
    x = _storage(np.ravel(x), dtype)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = offsets.size - 1
    as_bits = dtype in INT_DTYPES or op in BITWISE
    out = np.empty(max(nseg, 0), dtype=np.uint64 if as_bits else np.float64)
    _check(_load().orc_segmented(_ptr(x), _ptr(offsets), nseg, DTYPES[dtype], OPS[op], _ptr(out)),
           "segmented")
    return out


def scan(x: np.ndarray, op: str, dtype: str | None = None, exclusive: bool = False,
         heads: np.ndarray | None = None) -> np.ndarray:
    """Inclusive (or exclusive) scan: out[i] = x[r] (op) ... (op) x[i] over i's run.

    Runs start at position 0 and at every position in ``heads`` (nondecreasing;
    CSR segment offsets give the per-segment scan).  float64 results for float
    data with sum/prod/min/max, else uint64 bit patterns (zero-extended)."""
    dtype = dtype or str(x.dtype)
    x = _storage(np.ravel(x), dtype)
    h = np.ascontiguousarray(np.zeros(0) if heads is None else heads, dtype=np.int64)
    as_bits = dtype in INT_DTYPES or op in BITWISE
    out = np.empty(x.size, dtype=np.uint64 if as_bits else np.float64)
    _check(_load().orc_scan(_ptr(x), x.size, DTYPES[dtype], OPS[op], int(bool(exclusive)),
                            _ptr(h), h.size, _ptr(out)), "scan")
    return out


def row_forward(x: np.ndarray, op: str):
    """Row-wise reduction of a float32 matrix: (y float64[rows], idx int64[rows], zeros int64[rows])."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    rows, cols = x.shape
    y = np.empty(rows, np.float64)
    idx = np.empty(rows, np.int64)
    z = np.empty(rows, np.int64)
    _check(_load().orc_row_forward(_ptr(x), rows, cols, OPS[op], _ptr(y), _ptr(idx), _ptr(z)),
           "row_forward")
    return y, idx, z


def row_grad(x: np.ndarray, op: str, g: np.ndarray) -> np.ndarray:
    """Gradient of the row-wise reduction given the upstream gradient g[rows] (float64 [rows, cols])."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    rows, cols = x.shape
    g = np.ascontiguousarray(g, dtype=np.float64)
    grad = np.empty((rows, cols), np.float64)
    _check(_load().orc_row_grad(_ptr(x), rows, cols, OPS[op], _ptr(g), _ptr(grad)), "row_grad")
    return grad


def fold_sum_f32(x: np.ndarray, threads: int = 1) -> float:
    """Algorithm 1's left fold of a float32 array in double: the CPU timing
    baseline.  With threads > 1, contiguous chunks fold on their own threads
    and the partial sums add in chunk order."""
    x = _storage(np.ravel(x), "float32")
    d = ctypes.c_double()
    _check(_load().orc_fold_sum_f32(_ptr(x), x.size, int(threads), ctypes.byref(d)), "fold_sum_f32")
    return d.value
