"""Host-side AddressSanitizer + UndefinedBehaviorSanitizer builds (CPU only).

* The CPU oracle (plain C) is built with gcc under both sanitizers and driven
  through every entry point on small and edge-case inputs.
* The C ABI's host code (validation, workspace bookkeeping, the launch-table
  parser and lookup, configuration forcing, error reporting) is built with
  hipcc, sanitizers on the host side only, and linked against stand-ins for
  the kernel translation units, so no GPU is needed or touched.

Any sanitizer report, or a wrong value the drivers check, fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
SAN_C = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, cwd):
    proc = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV)
    noise = "packed-fp32-ops"  # the host pass does not know the device feature
    msg = "\n".join(l for l in (proc.stdout + proc.stderr).splitlines() if noise not in l)
    return proc.returncode, msg


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, msg = _run(["gcc", "-O1", "-g", *SAN_C, "-pthread", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_driver.c"),
                    "-o", exe, "-lm"], tmp_path)
    assert rc == 0, msg
    rc, msg = _run([exe], tmp_path)
    assert rc == 0 and "oracle driver ok" in msg and "Sanitizer" not in msg, msg


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("gcc") is None, reason="needs hipcc and gcc")
def test_c_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1710_07358_amd", "csrc")]
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    hip = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", *inc, *host_san, "-x", "hip", "-c"]
    for src, obj in ((os.path.join(ROOT, "paper_1710_07358_amd", "csrc", "rd_api.cpp"), "rd_api.o"),
                     (os.path.join(SAN, "launch_stubs.cpp"), "stubs.o")):
        rc, msg = _run([*hip, src, "-o", obj], tmp_path)
        assert rc == 0, msg
    rc, msg = _run(["gcc", "-O1", "-g", *SAN_C, *inc, "-c", os.path.join(SAN, "abi_driver.c"), "-o", "driver.o"],
                   tmp_path)
    assert rc == 0, msg
    rc, msg = _run([HIPCC, *host_san, "--offload-arch=gfx950", "rd_api.o", "stubs.o", "driver.o", "-o",
                    "abi_driver"], tmp_path)
    assert rc == 0, msg
    table = os.path.join(ROOT, "paper_1710_07358_amd", "tuned_gfx950.txt")
    rc, msg = _run([str(tmp_path / "abi_driver"), table, str(tmp_path / "scratch_table.txt")], tmp_path)
    assert rc == 0 and "abi driver ok" in msg and "Sanitizer" not in msg and "runtime error" not in msg, msg
