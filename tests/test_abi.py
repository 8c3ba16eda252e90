"""The C-ABI library: loads, exports every function include/rd.h declares,
and rejects bad arguments on the host before touching a device.  No GPU
needed (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rd.h")


@pytest.fixture(scope="module")
def N():
    from paper_1710_07358_amd import _native

    if not os.path.exists(_native.LIB_PATH):
        from paper_1710_07358_amd.build import build

        build()
    _native.lib()
    return _native


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rd_[a-z_0-9]+)\s*\(", text)))


def _enum_values():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for body in re.findall(r"typedef enum \w+ \{(.*?)\}", text, flags=re.S):
        nxt = 0
        for item in body.split(","):
            item = item.strip()
            if not item:
                continue
            if "=" in item:
                name, v = (s.strip() for s in item.split("="))
                nxt = int(v)
            else:
                name = item
            vals[name] = nxt
            nxt += 1
    return vals


def test_every_declared_symbol_is_exported(N):
    decl = _declared_functions()
    assert len(decl) >= 15
    lib = N.lib()
    for name in decl:
        assert hasattr(lib, name), name
        assert name in N.SIGNATURES, f"binding lacks {name}"
    assert set(N.SIGNATURES) == set(decl)


# Entry points that compute (or describe) the method: each one's comment in
# the header names the passage of the paper that defines the operation.
METHOD_ENTRY_POINTS = ("rd_reduce", "rd_reduce_compensated", "rd_argreduce", "rd_reduce_paper_design",
                       "rd_segmented_reduce", "rd_scan", "rd_segmented_scan", "rd_saved_bytes",
                       "rd_rowreduce_fwd", "rd_rowreduce_bwd", "rd_workspace_status")


def _comment_before(name):
    text = open(HEADER).read()
    m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*(?:[\w\s*]+?)\b" + name + r"\s*\(", text, flags=re.S)
    return m.group(1) if m else ""


def test_every_method_entry_point_cites_the_paper():
    decl = _declared_functions()
    for name in METHOD_ENTRY_POINTS:
        assert name in decl, name
        comment = _comment_before(name)
        assert re.search(r"Section \d(\.\d)?|Algorithm 1", comment), f"{name}: no citation in its header comment"


def test_enum_values_match_header(N):
    vals = _enum_values()
    for name, v in vals.items():
        assert getattr(N, name) == v, name


def test_out_dtype_table(N):
    lib = N.lib()
    out = ctypes.c_int()
    expect = {
        (N.RD_I32, N.RD_SUM): N.RD_I32, (N.RD_U32, N.RD_PROD): N.RD_U32,
        (N.RD_F32, N.RD_SUM): N.RD_F32, (N.RD_F64, N.RD_MAX): N.RD_F64,
        (N.RD_F16, N.RD_SUM): N.RD_F32, (N.RD_BF16, N.RD_PROD): N.RD_F32,
        (N.RD_F16, N.RD_MIN): N.RD_F16, (N.RD_BF16, N.RD_XOR): N.RD_BF16,
    }
    for (dt, op), want in expect.items():
        assert lib.rd_out_dtype(dt, op, ctypes.byref(out)) == N.RD_OK
        assert out.value == want, (dt, op)
    assert lib.rd_dtype_size(N.RD_F64) == 8 and lib.rd_dtype_size(N.RD_BF16) == 2


def test_host_errors_before_any_device_call(N):
    lib = N.lib()
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: the call fails validation first
    assert lib.rd_reduce(fake, -1, N.RD_F32, N.RD_SUM, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert b"n = -1" in lib.rd_last_error()
    assert lib.rd_reduce(fake, 4, 17, N.RD_SUM, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce(fake, 4, N.RD_F32, 42, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce(None, 4, N.RD_F32, N.RD_SUM, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce(ctypes.c_void_p(0x10001), 4, N.RD_F32, N.RD_SUM, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert b"aligned" in lib.rd_last_error()
    assert lib.rd_reduce(fake, 4, N.RD_F32, N.RD_SUM, None, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_noalloc(fake, -1, N.RD_F32, N.RD_SUM, fake, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_noalloc(fake, 4, 17, N.RD_SUM, fake, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_noalloc(None, 4, N.RD_F32, N.RD_SUM, fake, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_noalloc(fake, 4, N.RD_F32, N.RD_SUM, ctypes.c_void_p(0x10002), None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_reduce_compensated(fake, 4, N.RD_I32, fake, None, None) == N.RD_ERR_UNSUPPORTED
    assert lib.rd_reduce_compensated(fake, 4, N.RD_F64, fake, None, None) == N.RD_ERR_UNSUPPORTED
    assert lib.rd_segmented_reduce(fake, fake, -1, N.RD_F32, N.RD_SUM, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_segmented_reduce(fake, fake, 0, N.RD_F32, N.RD_SUM, fake, None, None) == N.RD_OK
    assert lib.rd_segmented_reduce(fake, ctypes.c_void_p(0x10004), 3, N.RD_F32, N.RD_SUM, fake, None,
                                   None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_rowreduce_fwd(fake, 2, 2, N.RD_F64, N.RD_SUM, fake, fake, None) == N.RD_ERR_UNSUPPORTED
    assert lib.rd_rowreduce_fwd(fake, 2, 2, N.RD_F32, N.RD_XOR, fake, fake, None) == N.RD_ERR_UNSUPPORTED
    assert lib.rd_rowreduce_fwd(fake, -2, 2, N.RD_F32, N.RD_SUM, fake, fake, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_rowreduce_fwd(fake, 2, 2 ** 31, N.RD_F32, N.RD_MAX, fake, fake, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_rowreduce_fwd(fake, 2, 2, N.RD_F32, N.RD_MAX, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_rowreduce_bwd(fake, fake, None, 2, 2, N.RD_F32, N.RD_PROD, fake, None) == N.RD_ERR_INVALID_ARG
    # scans: validation happens on the host before any device call
    assert lib.rd_scan(fake, -1, N.RD_F32, N.RD_SUM, 0, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_scan(fake, 0, N.RD_F32, N.RD_SUM, 0, fake, None, None) == N.RD_OK  # nothing to do
    assert lib.rd_scan(fake, 4, N.RD_F32, 9, 0, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_scan(fake, 4, N.RD_F16, N.RD_SUM, 0, ctypes.c_void_p(0x10002), None, None) == N.RD_ERR_INVALID_ARG
    assert b"out" in lib.rd_last_error()  # float16 sums write float32: 2-byte alignment is not enough
    assert lib.rd_segmented_scan(fake, 8, fake, -1, N.RD_I32, N.RD_SUM, 0, fake, None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_segmented_scan(fake, 8, fake, 1 << 31, N.RD_I32, N.RD_SUM, 0, fake, None,
                                 None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_segmented_scan(fake, 8, ctypes.c_void_p(0x10004), 3, N.RD_I32, N.RD_SUM, 1, fake, None,
                                 None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_workspace_reset(None, None) == N.RD_ERR_INVALID_ARG
    assert lib.rd_workspace_destroy(None) == N.RD_OK


def test_saved_bytes(N):
    lib = N.lib()
    assert lib.rd_saved_bytes(N.RD_SUM, 4096, 262144) == 0
    assert lib.rd_saved_bytes(N.RD_MAX, 4096, 262144) == 4096 * 8
    # product: 16-byte row header + two doubles (products of the chunks before
    # and after) per 16384-column chunk
    assert lib.rd_saved_bytes(N.RD_PROD, 4096, 262144) == 4096 * 16 + 4096 * 16 * 16
    assert lib.rd_saved_bytes(N.RD_PROD, 3, 16385) == 3 * 16 + 3 * 2 * 16


def test_config_force_and_tune_table(N, tmp_path):
    lib = N.lib()
    cfg = N.RdConfig(256, 3, 8, 0, 0)  # unroll 3 has no kernel
    assert lib.rd_config_force(N.RD_KIND_PLAIN, ctypes.byref(cfg)) == N.RD_ERR_INVALID_ARG
    cfg = N.RdConfig(96, 4, 8, 0, 0)  # block not a multiple of 64
    assert lib.rd_config_force(N.RD_KIND_PLAIN, ctypes.byref(cfg)) == N.RD_ERR_INVALID_ARG
    good = N.RdConfig(512, 16, 2, 1, 2)
    assert lib.rd_config_force(N.RD_KIND_PLAIN, ctypes.byref(good)) == N.RD_OK
    got = N.RdConfig()
    assert lib.rd_config_get(N.RD_KIND_PLAIN, N.RD_F32, N.RD_SUM, 1 << 28, ctypes.byref(got)) == N.RD_OK
    assert (got.block, got.unroll, got.blocks_per_cu, got.nontemporal, got.layout) == (512, 16, 2, 1, 2)
    bad_layout = N.RdConfig(256, 4, 1, 0, 3)
    assert lib.rd_config_force(N.RD_KIND_PLAIN, ctypes.byref(bad_layout)) == N.RD_ERR_INVALID_ARG
    assert lib.rd_config_force(N.RD_KIND_PLAIN, None) == N.RD_OK
    assert lib.rd_config_get(N.RD_KIND_SCAN, N.RD_F32, N.RD_SUM, 1 << 28, ctypes.byref(got)) == N.RD_OK
    assert got.block % 64 == 0 and got.blocks_per_cu >= 1
    assert lib.rd_config_get(N.RD_KIND_SEGMENTED_SCAN, N.RD_BF16, N.RD_SUM, 1 << 28, ctypes.byref(got)) == N.RD_OK
    assert lib.rd_config_force(N.RD_KIND_SEGMENTED_SCAN + 1, None) == N.RD_ERR_INVALID_ARG
    table = tmp_path / "tune.txt"
    table.write_text("# kind esize opclass lo hi block unroll bpc nt layout\n0 4 0 20 30 1024 4 2 1 1\n")
    assert lib.rd_tune_load(str(table).encode()) == N.RD_OK
    assert lib.rd_config_get(N.RD_KIND_PLAIN, N.RD_F32, N.RD_SUM, 1 << 28, ctypes.byref(got)) == N.RD_OK
    assert (got.block, got.unroll, got.blocks_per_cu, got.nontemporal, got.layout) == (1024, 4, 2, 1, 1)
    assert lib.rd_config_get(N.RD_KIND_PLAIN, N.RD_F64, N.RD_SUM, 1 << 10, ctypes.byref(got)) == N.RD_OK
    assert got.block == 256  # uncovered entries keep the defaults
    bad = tmp_path / "bad.txt"
    bad.write_text("0 4 0 20 30 1024 5 2 1 0\n")
    assert lib.rd_tune_load(str(bad).encode()) == N.RD_ERR_INVALID_ARG
    assert lib.rd_tune_load(None) == N.RD_OK


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_1710_07358_amd as rd

    with pytest.raises(ValueError):
        rd.reduce(torch.ones(4), "sum")
    with pytest.raises(ValueError):
        rd.api._op("mean")


def test_bench_bandwidth_convention_matches_paper_table():
    # Section 4's table: input bytes / time, decimal GB/s
    import bench
    from conftest import read_golden

    rows = read_golden("execution_times_table.txt")
    n = int(rows[0][1])
    esize = int(rows[1][1])
    for f, ms, speedup, bw, usage in rows[2:]:
        assert abs(bench.gbps(n * esize, float(ms) / 1e3) - float(bw)) <= 1e-6 * float(bw), f
        base_ms = float(rows[2][1])
        assert abs(base_ms / float(ms) - float(speedup)) <= 1e-6 * float(speedup)


def test_missing_library_fails_loudly(N, monkeypatch, tmp_path):
    # No CPU fallback anywhere: without librd.so every entry point raises.
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "librd.so"))
    with pytest.raises(RuntimeError, match="missing"):
        N.lib()
