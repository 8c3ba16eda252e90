"""Shared test plumbing: moving seeded numpy inputs to the GPU and reading
GPU results back in the form the oracle reports them.  No reduction
arithmetic lives here."""
from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

FLOAT = ("float32", "float64", "float16", "bfloat16")
BITWISE = ("and", "or", "xor")
TORCH = {"int32": torch.int32, "uint32": torch.uint32, "float32": torch.float32,
         "float64": torch.float64, "float16": torch.float16, "bfloat16": torch.bfloat16,
         "int64": torch.int64, "uint64": torch.uint64}
INTS = ("int32", "uint32", "int64", "uint64")


def gpu_available() -> bool:
    return torch.cuda.is_available()


def to_gpu(a: np.ndarray, dtype: str, pad_front: int = 0) -> torch.Tensor:
    """Device tensor holding the bits of a (numpy storage of dtype), optionally
    placed pad_front elements into a larger allocation (misaligned start)."""
    a = np.ascontiguousarray(a)
    if dtype in ("float16", "bfloat16"):
        host = torch.from_numpy(a.view(np.int16).copy()).view(TORCH[dtype])
    elif dtype == "uint32":
        host = torch.from_numpy(a.view(np.int32).copy()).view(torch.uint32)
    elif dtype == "uint64":
        host = torch.from_numpy(a.view(np.int64).copy()).view(torch.uint64)
    else:
        host = torch.from_numpy(a.copy())
    if pad_front:
        big = torch.empty(a.size + pad_front, dtype=host.dtype, device="cuda")
        dev = big[pad_front:]
        dev.copy_(host.to("cuda"))
        return dev
    return host.to("cuda")


def bits_of(t: torch.Tensor) -> int:
    """Unsigned bit pattern of a 0-d device tensor."""
    t = t.detach().reshape(1).cpu()
    size = t.element_size()
    view = {2: torch.int16, 4: torch.int32, 8: torch.int64}[size]
    v = int(t.view(view).item())
    return v % (1 << (8 * size))


def value_of(t: torch.Tensor) -> float:
    return float(t.detach().reshape(1).cpu().to(torch.float64).item())


def same_float(a: float, b: float) -> bool:
    """Bit-level agreement for min/max: equal values, same zero sign, or both NaN."""
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b and math.copysign(1.0, a) == math.copysign(1.0, b)


def check_against_oracle(gpu_out: torch.Tensor, ref, x: np.ndarray, op: str, dtype: str,
                         abs_sum: float | None = None, compensated: bool = False):
    """Assert the GPU result matches the oracle to the bar for (op, dtype)."""
    n = x.size
    if dtype in INTS or op in BITWISE:
        got = bits_of(gpu_out)
        assert got == ref, f"{op}/{dtype} n={n}: got {got:#x}, oracle {ref:#x}"
        return
    got = value_of(gpu_out)
    if op in ("min", "max"):
        assert same_float(got, ref), f"{op}/{dtype} n={n}: got {got!r}, oracle {ref!r}"
    elif op == "sum":
        tol = (2.0 ** -40 if compensated else 2.0 ** -20) * abs_sum
        assert abs(got - ref) <= tol, f"sum/{dtype} n={n}: got {got!r}, exact {ref!r}, tol {tol!r}"
    elif op == "prod":
        # Float products accumulate in float64 whatever the input dtype: any
        # product tree of n factors is within (1+2^-53)^(n-1) - 1 of the exact
        # product, then float32 outputs add one rounding (2^-24).
        out_u = 0.0 if dtype == "float64" else 2.0 ** -24
        bound = (max(n - 1, 0) * 2.0 ** -53) * 1.001 + out_u
        ref_out = ref if dtype == "float64" else float(np.float32(ref))  # output range
        if ref_out == 0.0 or math.isinf(ref_out) or math.isnan(ref_out):
            # zeros and infinities compare with their sign (IEEE: the xor of the factors' signs)
            assert same_float(got, ref_out), f"prod/{dtype} n={n}: got {got!r}, oracle {ref!r}"
        else:
            assert abs(got - ref) <= bound * abs(ref), f"prod/{dtype} n={n}: got {got!r}, oracle {ref!r}"
    else:
        raise ValueError(op)


def as_oracle_array(out: torch.Tensor, dtype: str, op: str) -> np.ndarray:
    """GPU results in the oracle's array representation: uint64 bit patterns
    for integer dtypes and bitwise ops, float64 values otherwise."""
    o = out.detach().reshape(-1).cpu()
    if dtype in INTS or op in BITWISE:
        size = o.element_size()
        view = {2: torch.int16, 4: torch.int32, 8: torch.int64}[size]
        v = o.view(view).numpy()
        if size < 8:
            return (v.astype(np.int64) % (1 << (8 * size))).astype(np.uint64)
        return v.view(np.uint64)
    return o.to(torch.float64).numpy()


def abs_storage(x: np.ndarray, dtype: str) -> np.ndarray:
    """|x| in x's storage (sign bit cleared; float16/bfloat16 are uint16 bits)."""
    if dtype in ("float16", "bfloat16"):
        return (x.view(np.uint16) & np.uint16(0x7FFF)).astype(np.uint16)
    return np.abs(x)
