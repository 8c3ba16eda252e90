"""rd_reduce_noalloc (the allocation-free variant of rd_reduce) against
rd_reduce through the C ABI: same kernels and launch table, so the results
must be bitwise identical, checked on two calls in a row, the second with a
smaller input, plus the oracle's parity bar on both.  Run last: it shares the
library's per-GPU scratch array with nothing else in the suite."""
import ctypes
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

from paper_1710_07358_amd import _native as N  # noqa: E402
from paper_1710_07358_amd import api as rd  # noqa: E402

TORCH = {"int32": torch.int32, "uint32": torch.uint32, "float32": torch.float32, "float64": torch.float64,
         "int64": torch.int64, "uint64": torch.uint64, "float16": torch.float16, "bfloat16": torch.bfloat16}

# (dtype, op, first n, second n): the first size selects the launch table's
# largest-input row (the most work-groups), the second a smaller one
CASES = [
    ("float32", "sum", 2 ** 24 + 7, 1_000_003),
    ("int32", "xor", 2 ** 24 + 7, 31),
    ("uint32", "min", 2 ** 20 + 7, 1025),
    ("float64", "prod", 2 ** 24 + 7, 2 ** 20 + 7),
    ("int64", "sum", 2 ** 20 + 7, 1),
    ("bfloat16", "max", 2 ** 24 + 7, 4099),
    ("float16", "sum", 2 ** 20 + 7, 0),
]


def _device(x_np, dtype):
    if dtype in ("float16", "bfloat16"):
        return torch.from_numpy(x_np.view(np.int16)).cuda().view(TORCH[dtype])
    return torch.from_numpy(x_np).cuda()


def _call(fn_name, x, n, dtype, op):
    lib = N.lib()
    out = torch.empty((), dtype=rd.out_dtype(TORCH[dtype], op), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    args = [x.data_ptr() if n else None, n, rd.DTYPES[TORCH[dtype]], rd.OPS[op], out.data_ptr()]
    if fn_name == "rd_reduce":
        args.append(None)  # default workspace
    N.check(getattr(lib, fn_name)(*args, stream))
    return out


def _bits(t):
    return t.view(torch.int16 if t.element_size() == 2 else (torch.int32 if t.element_size() == 4 else torch.int64)).item()


def _oracle_ok(got_t, x_np, dtype, op):
    ref = oracle.reduce(x_np, op, dtype)
    if isinstance(ref, int):  # integers and bitwise: bit-exact
        width = 8 * got_t.element_size()
        return (_bits(got_t) % (1 << width)) == ref
    got = float(got_t.float().item() if got_t.dtype in (torch.float16, torch.bfloat16) else got_t.item())
    if op == "sum":
        exact, abs_sum = oracle.exact_sum(x_np, dtype)
        return abs(got - exact) <= 2.0 ** -20 * abs_sum
    if op == "prod":
        n = x_np.size
        out_u = 2.0 ** -53 if dtype == "float64" else 2.0 ** -24
        return abs(got - ref) <= ((n - 1) * 2.0 ** -53 * 1.001 + out_u) * abs(ref)
    return same_float(got, ref)  # min/max: bit-exact


@pytest.mark.parametrize("dtype,op,n1,n2", CASES)
def test_noalloc_matches_rd_reduce_twice_then_smaller(dtype, op, n1, n2):
    print(f"[noalloc] {dtype} {op} n={n1} then n={n2}", flush=True)
    for salt, n in ((1, n1), (2, n2)):
        x_np = W.plain(n, dtype, op, config=1, salt=salt)
        x = _device(x_np, dtype)
        want = _call("rd_reduce", x, n, dtype, op)
        got = _call("rd_reduce_noalloc", x, n, dtype, op)
        torch.cuda.synchronize()
        assert _bits(got) == _bits(want), (dtype, op, n, got.item(), want.item())
        assert _oracle_ok(got, x_np, dtype, op), (dtype, op, n, got.item())


def test_noalloc_repeated_calls_on_one_stream():
    # back-to-back calls without synchronising: each re-arms the shared array
    # before its reduction, on the same stream
    xs = [W.plain(n, "float32", "sum", config=1, salt=10 + i) for i, n in enumerate((3_000_001, 17, 2 ** 22))]
    dev = [torch.from_numpy(a).cuda() for a in xs]
    outs = [_call("rd_reduce_noalloc", d, d.numel(), "float32", "sum") for d in dev]
    wants = [_call("rd_reduce", d, d.numel(), "float32", "sum") for d in dev]
    torch.cuda.synchronize()
    for o, w, a in zip(outs, wants, xs):
        assert _bits(o) == _bits(w)
        exact, abs_sum = oracle.exact_sum(a)
        assert abs(o.item() - exact) <= 2.0 ** -20 * abs_sum


def test_noalloc_binding_and_empty_input():
    x = torch.arange(1, 1001, dtype=torch.int32, device="cuda")
    assert rd.reduce_noalloc(x, "sum").item() == 500_500
    assert rd.reduce_noalloc(x, "sum", n=10).item() == 55
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    assert rd.reduce_noalloc(e, "min").item() == math.inf
    assert rd.reduce_noalloc(e, "prod").item() == 1.0


def test_noalloc_rejects_bad_arguments():
    lib = N.lib()
    x = torch.ones(8, device="cuda")
    out = torch.empty((), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert lib.rd_reduce_noalloc(x.data_ptr(), -1, N.RD_F32, N.RD_SUM, out.data_ptr(), s) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_noalloc(x.data_ptr() + 2, 4, N.RD_F32, N.RD_SUM, out.data_ptr(), s) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_noalloc(x.data_ptr(), 4, N.RD_F32, N.RD_SUM, None, s) == N.RD_ERR_INVALID_ARG
