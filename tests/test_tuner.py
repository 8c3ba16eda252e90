"""The autotuner on the GPU: coordinate descent over a two-value space times
real launches, its best configuration goes through the table writer, and
rd_tune_load installs the written table so the library launches with it."""
import os

import numpy as np
import pytest

import oracle
from helpers import gpu_available

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1710_07358_amd import _native as N  # noqa: E402
from paper_1710_07358_amd import api as rd  # noqa: E402
from paper_1710_07358_amd import tune  # noqa: E402


def test_descend_writes_a_table_that_loads(tmp_path):
    n = 1 << 20
    x = torch.randint(-1000, 1000, (n,), dtype=torch.int32, device="cuda")
    out = torch.empty((), dtype=torch.int32, device="cuda")
    start = {"block": 256, "unroll": 2, "blocks_per_cu": 2, "nontemporal": 0, "layout": 0}
    installed = rd.config_get("plain", torch.int32, "sum", n)
    space = {"unroll": [2, 4], "blocks_per_cu": [1, 2]}
    seen = []

    def timer(fn):
        t = tune.time_call(fn, reps=5, batches=2, warm_s=0.0)
        seen.append(rd.config_get("plain", torch.int32, "sum", n))  # the forced shape
        # every timed candidate computes the right sum
        assert out.item() == int(x.sum().item())
        return t

    best, t = tune.descend("plain", start, lambda: rd.reduce(x, "sum", out=out), passes=1, space=space,
                           timer=timer)
    assert t > 0.0
    assert best["unroll"] in (2, 4) and best["blocks_per_cu"] in (1, 2)
    assert {(c["unroll"], c["blocks_per_cu"]) for c in seen} >= {(2, 2), (4, 2)}
    assert rd.config_get("plain", torch.int32, "sum", n) == installed  # descend leaves nothing forced
    line = tune.table_line("plain", 4, 0, 0, 62, best)
    path = tmp_path / "table.txt"
    path.write_text(tune.TABLE_HEADER + "\n" + line + "\n")
    try:
        rd.tune_load(str(path))
        got = rd.config_get("plain", torch.int32, "sum", n)
        assert got == best, (got, best)
        # a launch with the loaded table still reduces correctly
        xs = x.cpu().numpy()
        assert rd.reduce(x, "sum").item() % 2 ** 32 == oracle.reduce(xs, "sum", "int32")
    finally:
        table = os.environ.get("RD_TUNE_TABLE", N.TUNED_TABLE)
        rd.tune_load(table if table != "none" and os.path.exists(table) else None)
    assert rd.config_get("plain", torch.int32, "sum", n) == installed


def test_unroll_sweep_rows():
    rows = tune.unroll_sweep(1 << 20, lambda msg: None)
    assert [r["unroll"] for r in rows] == [1, 2, 4, 8, 16]
    assert all(r["ms"] > 0 and np.isfinite(r["GBps"]) for r in rows)
    assert rows[0]["speedup"] == 1.0
