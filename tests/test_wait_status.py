"""The bounded waits inside the kernels report a wait that ran out.

Stage 2 of Section 2.3 (one work-group combines every work-group's partial)
and the scan's tile prefixes run inside one launch here, so work-groups wait
for values others publish.  Every such wait is bounded; a wait that runs out
sets a status word the host reads with rd_workspace_status.  The failure path
is forced from the host with a test hook that adds one wait for a slot that
nothing publishes: the wait runs out after its bound and every kernel still
ends normally.
"""
import numpy as np
import pytest

import oracle
from helpers import bits_of, gpu_available, to_gpu
from paper_1710_07358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1710_07358_amd as rd  # noqa: E402
from paper_1710_07358_amd import _native as N  # noqa: E402


def test_status_clear_after_normal_calls():
    x = to_gpu(W.plain(2 ** 20 + 7, "int32", "sum", salt=1), "int32")
    rd.reduce(x, "sum")
    rd.scan(x, "sum")
    rd.argreduce(x, "max")
    off = torch.tensor([0, 10, 5000, 2 ** 20 + 7], dtype=torch.int64, device="cuda")
    rd.segmented(x, off, "xor")
    assert rd.workspace_status() == 0


@pytest.mark.sets_wait_status
def test_forced_timeout_reduce_is_reported_then_cleared():
    x_np = W.plain(2 ** 20 + 7, "int32", "xor", salt=2)
    x = to_gpu(x_np, "int32")
    ws = rd.Workspace()
    assert rd.workspace_status(ws) == 0
    print("[wait] forced grid-stage timeout, rd_reduce int32 xor", flush=True)
    rd.debug_force_wait_timeout(True)
    try:
        rd.reduce(x, "xor", workspace=ws)
    finally:
        rd.debug_force_wait_timeout(False)
    flags = rd.workspace_status(ws)
    assert flags & N.RD_WAIT_GRID, flags
    assert rd.workspace_status(ws) == 0  # reading cleared it
    # the workspace keeps working: the next launch is correct and clean
    assert bits_of(rd.reduce(x, "xor", workspace=ws)) == oracle.reduce(x_np, "xor", "int32")
    assert rd.workspace_status(ws) == 0
    ws.close()


@pytest.mark.sets_wait_status
def test_forced_timeout_scan_is_reported_and_the_next_scan_is_whole():
    n = 3 * 2 ** 20 + 5  # many tiles: later tiles wait on earlier ones
    x_np = W.plain(n, "int32", "sum", config=1, salt=3)
    x = to_gpu(x_np, "int32")
    ws = rd.Workspace()
    print("[wait] forced scan look-back timeout, int32 sum", flush=True)
    rd.debug_force_wait_timeout(True)
    try:
        rd.scan(x, "sum", workspace=ws)
    finally:
        rd.debug_force_wait_timeout(False)
    flags = rd.workspace_status(ws)
    assert flags & N.RD_WAIT_SCAN, flags
    # The give-up of that launch is tagged with its epoch: the next scans wait
    # as long as they need and are exact.
    ref = oracle.scan(x_np, "sum", "int32")
    for _ in range(3):
        out = rd.scan(x, "sum", workspace=ws)
        got = out.cpu().numpy().view(np.uint32).astype(np.uint64)
        assert np.array_equal(got, ref)
    assert rd.workspace_status(ws) == 0
    ws.close()
