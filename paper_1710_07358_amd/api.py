"""PyTorch-facing binding of librd (include/rd.h), same operations and names.

Torch provides device memory and streams only: each call checks the tensors,
passes their device pointers and the current HIP stream to the C ABI, and
returns tensors the kernels wrote.  Calls are asynchronous on
``torch.cuda.current_stream()``.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as N

DTYPES = {torch.int32: N.RD_I32, torch.uint32: N.RD_U32, torch.float32: N.RD_F32,
          torch.float64: N.RD_F64, torch.float16: N.RD_F16, torch.bfloat16: N.RD_BF16,
          torch.int64: N.RD_I64, torch.uint64: N.RD_U64}
TORCH_DTYPE = {v: k for k, v in DTYPES.items()}
OPS = {"sum": N.RD_SUM, "prod": N.RD_PROD, "min": N.RD_MIN, "max": N.RD_MAX,
       "and": N.RD_AND, "or": N.RD_OR, "xor": N.RD_XOR}
KINDS = {"plain": N.RD_KIND_PLAIN, "compensated": N.RD_KIND_COMPENSATED,
         "segmented": N.RD_KIND_SEGMENTED, "rowwise": N.RD_KIND_ROWWISE,
         "rowwise_bwd": N.RD_KIND_ROWWISE_BWD, "scan": N.RD_KIND_SCAN,
         "segmented_scan": N.RD_KIND_SEGMENTED_SCAN}


def _dt(t: torch.Tensor) -> int:
    try:
        return DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}") from None


def _op(op: str) -> int:
    try:
        return OPS[op]
    except KeyError:
        raise ValueError(f"unknown op {op!r}; expected one of {sorted(OPS)}") from None


def _dev_tensor(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a tensor on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ws(workspace) -> int | None:
    return None if workspace is None else workspace.handle


def out_dtype(dtype: torch.dtype, op: str) -> torch.dtype:
    """Output dtype of reduce/segmented for (dtype, op)."""
    out = ctypes.c_int()
    N.check(N.lib().rd_out_dtype(DTYPES[dtype], _op(op), ctypes.byref(out)))
    return TORCH_DTYPE[out.value]


class Workspace:
    """Explicit workspace (partials + completion counters) for one stream."""

    def __init__(self, device: int | torch.device | None = None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        h = ctypes.c_void_p()
        N.check(N.lib().rd_workspace_create(ctypes.byref(h), dev.index))
        self.handle = h.value

    def reset(self, stream=None) -> None:
        s = stream.cuda_stream if stream is not None else _stream(self.device)
        N.check(N.lib().rd_workspace_reset(self.handle, s))

    def close(self) -> None:
        if self.handle:
            N.check(N.lib().rd_workspace_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_status(workspace: "Workspace | None" = None) -> int:
    """Wait-status bits (RD_WAIT_GRID = 1, RD_WAIT_SCAN = 2) of one workspace,
    or of every workspace of the current device; reading clears them.
    Synchronises the device."""
    flags = ctypes.c_uint(0)
    N.check(N.lib().rd_workspace_status(_ws(workspace), ctypes.byref(flags)))
    return int(flags.value)


def debug_force_wait_timeout(on: bool) -> None:
    """Failure-path test hook: while on, reduce() and scan() launches run one
    bounded wait out (their results are then unspecified)."""
    N.check(N.lib().rd_debug_force_wait_timeout(1 if on else 0))


def reduce(x: torch.Tensor, op: str, out: torch.Tensor | None = None, workspace: Workspace | None = None,
           n: int | None = None) -> torch.Tensor:
    """x[0] (op) ... (op) x[n-1] over a contiguous device tensor (0-d result).

    n defaults to x.numel(); a smaller n reduces a prefix."""
    x = _dev_tensor(x, "x")
    count = x.numel() if n is None else int(n)
    if count > x.numel():
        raise ValueError("n exceeds x.numel()")
    odt = out_dtype(x.dtype, op)
    if out is None:
        out = torch.empty((), dtype=odt, device=x.device)
    elif out.dtype != odt or not out.is_cuda:
        raise ValueError(f"out must be a {odt} tensor on the GPU")
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_reduce(x.data_ptr() if count else None, count, _dt(x), _op(op),
                                  out.data_ptr(), _ws(workspace), _stream(x.device)))
    return out


def reduce_noalloc(x: torch.Tensor, op: str, out: torch.Tensor | None = None, n: int | None = None) -> torch.Tensor:
    """reduce() without a workspace: the library's fixed per-GPU scratch array
    carries the grid stage, and the call allocates no device memory (pass
    `out` as well to keep the whole call allocation-free).  Calls that may
    overlap on one GPU race."""
    x = _dev_tensor(x, "x")
    count = x.numel() if n is None else int(n)
    if count > x.numel():
        raise ValueError("n exceeds x.numel()")
    odt = out_dtype(x.dtype, op)
    if out is None:
        out = torch.empty((), dtype=odt, device=x.device)
    elif out.dtype != odt or not out.is_cuda:
        raise ValueError(f"out must be a {odt} tensor on the GPU")
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_reduce_noalloc(x.data_ptr() if count else None, count, _dt(x), _op(op),
                                          out.data_ptr(), _stream(x.device)))
    return out


def reduce_compensated(x: torch.Tensor, out: torch.Tensor | None = None,
                       workspace: Workspace | None = None) -> torch.Tensor:
    """Compensated (two-sum) sum of float32/float16/bfloat16 data, float64 result."""
    x = _dev_tensor(x, "x")
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=x.device)
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_reduce_compensated(x.data_ptr() if x.numel() else None, x.numel(), _dt(x),
                                              out.data_ptr(), _ws(workspace), _stream(x.device)))
    return out


def argreduce(x: torch.Tensor, op: str, workspace: Workspace | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """(min or max value, lowest index attaining it) of a contiguous device tensor."""
    x = _dev_tensor(x, "x")
    if op not in ("min", "max"):
        raise ValueError("argreduce: op must be 'min' or 'max'")
    value = torch.empty((), dtype=x.dtype, device=x.device)
    index = torch.empty((), dtype=torch.int64, device=x.device)
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_argreduce(x.data_ptr() if x.numel() else None, x.numel(), _dt(x), _op(op),
                                     value.data_ptr(), index.data_ptr(), _ws(workspace), _stream(x.device)))
    return value, index


def reduce_paper_design(x: torch.Tensor, variant: int, unroll: int = 1, out: torch.Tensor | None = None,
                        workspace: Workspace | None = None) -> torch.Tensor:
    """Sum by one of the paper's own designs (variant 0: two-stage; 1: unrolled
    F times with the barrier-free tree), int32 or float32, for comparison."""
    x = _dev_tensor(x, "x")
    if out is None:
        out = torch.empty((), dtype=x.dtype, device=x.device)
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_reduce_paper_design(x.data_ptr() if x.numel() else None, x.numel(), _dt(x), int(variant),
                                               int(unroll), out.data_ptr(), _ws(workspace), _stream(x.device)))
    return out


def segmented(x: torch.Tensor, offsets: torch.Tensor, op: str, out: torch.Tensor | None = None,
              workspace: Workspace | None = None) -> torch.Tensor:
    """out[s] = reduce(x[offsets[s]:offsets[s+1]], op) for every segment, one launch."""
    x = _dev_tensor(x, "x")
    offsets = _dev_tensor(offsets, "offsets")
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.numel() < 1:
        raise ValueError("offsets must be a 1-D int64 tensor with nseg + 1 entries")
    nseg = offsets.numel() - 1
    odt = out_dtype(x.dtype, op)
    if out is None:
        out = torch.empty(nseg, dtype=odt, device=x.device)
    elif out.dtype != odt or out.numel() < nseg:
        raise ValueError(f"out must hold {nseg} elements of {odt}")
    if nseg == 0:
        return out
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_segmented_reduce(x.data_ptr(), offsets.data_ptr(), nseg, _dt(x), _op(op),
                                            out.data_ptr(), _ws(workspace), _stream(x.device)))
    return out


def scan(x: torch.Tensor, op: str, exclusive: bool = False, out: torch.Tensor | None = None,
         offsets: torch.Tensor | None = None, workspace: Workspace | None = None) -> torch.Tensor:
    """Inclusive (or exclusive) scan of a contiguous device tensor, one pass.

    out[i] = x[0] (op) ... (op) x[i] (exclusive: up to x[i-1]).  With CSR
    ``offsets`` (int64, nseg + 1 entries) the scan restarts at every segment
    start.  ``out`` may be ``x`` when the output dtype equals x's dtype."""
    x = _dev_tensor(x, "x")
    odt = out_dtype(x.dtype, op)
    if out is None:
        out = torch.empty(x.shape, dtype=odt, device=x.device)
    elif out.dtype != odt or out.numel() != x.numel() or not out.is_cuda or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {odt} GPU tensor of {x.numel()} elements")
    if x.numel() == 0:
        return out
    with torch.cuda.device(x.device):
        if offsets is None:
            N.check(N.lib().rd_scan(x.data_ptr(), x.numel(), _dt(x), _op(op), int(bool(exclusive)),
                                    out.data_ptr(), _ws(workspace), _stream(x.device)))
        else:
            offsets = _dev_tensor(offsets, "offsets")
            if offsets.dtype != torch.int64 or offsets.dim() != 1:
                raise ValueError("offsets must be a 1-D int64 tensor")
            N.check(N.lib().rd_segmented_scan(x.data_ptr(), x.numel(),
                                              offsets.data_ptr() if offsets.numel() else None,
                                              offsets.numel(), _dt(x), _op(op), int(bool(exclusive)),
                                              out.data_ptr(), _ws(workspace), _stream(x.device)))
    return out


def saved_bytes(op: str, rows: int, cols: int) -> int:
    return int(N.lib().rd_saved_bytes(_op(op), rows, cols))


def rowreduce_forward(x: torch.Tensor, op: str) -> tuple[torch.Tensor, torch.Tensor]:
    """Row-wise reduction of a float32 [rows, cols] tensor: (y[rows], saved state)."""
    x = _dev_tensor(x, "x")
    if x.dim() != 2 or x.dtype != torch.float32:
        raise ValueError("x must be a 2-D float32 tensor")
    rows, cols = x.shape
    y = torch.empty(rows, dtype=torch.float32, device=x.device)
    saved = torch.empty(max(saved_bytes(op, rows, cols), 8), dtype=torch.uint8, device=x.device)
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_rowreduce_fwd(x.data_ptr() if x.numel() else None, rows, cols, N.RD_F32, _op(op),
                                         y.data_ptr(), saved.data_ptr(), _stream(x.device)))
    return y, saved


def rowreduce_backward(x: torch.Tensor, g: torch.Tensor, saved: torch.Tensor, op: str) -> torch.Tensor:
    """Gradient of the row-wise reduction for upstream gradient g[rows]."""
    x = _dev_tensor(x, "x")
    g = _dev_tensor(g.to(torch.float32), "g")
    rows, cols = x.shape
    grad = torch.empty((rows, cols), dtype=torch.float32, device=x.device)
    if grad.numel() == 0:
        return grad
    with torch.cuda.device(x.device):
        N.check(N.lib().rd_rowreduce_bwd(x.data_ptr(), g.data_ptr(), saved.data_ptr(), rows, cols, N.RD_F32,
                                         _op(op), grad.data_ptr(), _stream(x.device)))
    return grad


class RowReduce(torch.autograd.Function):
    """y[r] = reduce(x[r, :], op) with hand-written backward kernels.

    max/min send the gradient to the LOWEST index attaining the extreme;
    prod uses zero-safe exclusive products (no division)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, op: str):
        y, saved = rowreduce_forward(x.contiguous(), op)
        ctx.op = op
        ctx.save_for_backward(x, saved)
        return y

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        x, saved = ctx.saved_tensors
        return rowreduce_backward(x.contiguous(), g.contiguous(), saved, ctx.op), None


def rowreduce(x: torch.Tensor, op: str) -> torch.Tensor:
    return RowReduce.apply(x, op)


def config_get(kind: str, dtype: torch.dtype, op: str, n: int) -> dict:
    c = N.RdConfig()
    N.check(N.lib().rd_config_get(KINDS[kind], DTYPES[dtype], _op(op), int(n), ctypes.byref(c)))
    return {"block": c.block, "unroll": c.unroll, "blocks_per_cu": c.blocks_per_cu,
            "nontemporal": c.nontemporal, "layout": c.layout}


def config_force(kind: str, cfg: dict | None) -> None:
    if cfg is None:
        N.check(N.lib().rd_config_force(KINDS[kind], None))
        return
    c = N.RdConfig(cfg["block"], cfg["unroll"], cfg["blocks_per_cu"], int(cfg.get("nontemporal", 0)),
                   int(cfg.get("layout", 0)))
    N.check(N.lib().rd_config_force(KINDS[kind], ctypes.byref(c)))


def tune_load(path: str | None) -> None:
    N.check(N.lib().rd_tune_load(path.encode() if path else None))
