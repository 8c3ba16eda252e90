"""Static check of our own gfx950 code objects: no kernel may write through
the scalar data cache (scalar stores or atomics, its write-back or discard).
Disassembles each compiled translation unit of librd with the ROCm LLVM tools."""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm/bin"
FORBIDDEN = re.compile(r"^\s+(s_store_\w+|s_atomic_\w+|s_buffer_store\w*|s_buffer_atomic\w*|"
                       r"s_scratch_store\w*|s_dcache_wb\w*|s_dcache_discard\w*)\b", re.M)


def _objects():
    return sorted(glob.glob(os.path.join(ROOT, "_build", "*.o")))


@pytest.mark.skipif(not os.path.exists(os.path.join(LLVM, "llvm-objdump")), reason="ROCm LLVM tools absent")
def test_no_scalar_cache_writes(tmp_path):
    objs = _objects()
    if not objs:
        pytest.skip("library not built yet (no _build objects)")
    checked = 0
    for obj in objs:
        fat = tmp_path / "fat.bin"
        scratch = tmp_path / "copy.o"
        r = subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", obj, str(scratch)],
                           capture_output=True)
        if r.returncode != 0 or not fat.exists():
            continue  # host-only object
        co = tmp_path / "dev.co"
        subprocess.check_call([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                               "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fat}", f"--output={co}"])
        asm = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", str(co)],
                             capture_output=True, text=True, check=True).stdout
        bad = FORBIDDEN.findall(asm)
        assert not bad, f"{os.path.basename(obj)}: {sorted(set(bad))}"
        checked += 1
        fat.unlink()
    assert checked >= 8
