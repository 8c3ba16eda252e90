import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workloads")
    config.addinivalue_line("markers", "sets_wait_status: forces a bounded wait to run out (checks the status itself)")


def read_golden(name):
    """Parse a golden fixture: '#' comments, whitespace-separated rows."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


@pytest.fixture(autouse=True)
def _bounded_waits_never_ran_out(request):
    """After every GPU test: no bounded wait inside a kernel ran out, in any
    workspace of the device (reading the status words also clears them)."""
    yield
    if request.node.get_closest_marker("gpu") is None or request.node.get_closest_marker("sets_wait_status"):
        return
    torch = sys.modules.get("torch")
    api = sys.modules.get("paper_1710_07358_amd.api")
    if torch is None or api is None or not torch.cuda.is_available():
        return
    flags = api.workspace_status()
    assert flags == 0, f"a bounded wait inside a kernel ran out during this test (status bits {flags:#x})"
