"""The C-ABI library loads and exports every symbol include/clbm.h declares,
and its host-only helpers behave (no GPU compute here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clbm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clbm_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1705_11092_amd import clbm
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(clbm.lib, n), n
    assert sorted(clbm.EXPORTED) == names


def test_host_helpers():
    from paper_1705_11092_amd import clbm, inputs
    assert clbm.nonslip_s3(0.5) == pytest.approx(1.6, abs=1e-15)  # Sec. IV A
    assert clbm.nonslip_s3(1.0) == pytest.approx(8.0 / 7.0)
    assert clbm.nonslip_s3(1.754) == pytest.approx(inputs.nonslip_s3(1.754))
    assert clbm.s_from_nu(0.01) == pytest.approx(1.0 / 0.53)
    # Buffer sizes: 9 direction runs per row, each padded to 8 elements,
    # or, for rows wider than 64 nodes, to a whole number of 128-byte lines
    # (32 FP32, 16 FP64, 64 16-bit elements).
    G = 64  # spare bytes after the last row
    assert clbm.buffer_bytes(4096, 4096, "f32") == 9 * 4096 * 4096 * 4 + G
    assert clbm.buffer_bytes(4096, 4096, "f16") == 9 * 4096 * 4096 * 2 + G
    assert clbm.buffer_bytes(4096, 4096, "bf16sr") == 9 * 4096 * 4096 * 2 + G
    assert clbm.buffer_bytes(64, 32, "f64") == 9 * 64 * 32 * 8 + G
    # Narrow lattices keep R = 2^k rows per block (runs of a direction in a
    # block reach 16 KB or R reaches the height), and ny rounds up to whole
    # blocks: 37 x 23 FP32 has 160-byte runs, R = 16, 32 rows allocated;
    # 1030 x 9 has 4224-byte runs (1056 elements), R = 4, 12 rows; 1030 x 3
    # stops at R = 2 (the height), 4 rows; 4100-wide FP32 rows (4128
    # elements) exceed 16 KB, R = 1.
    assert clbm.buffer_bytes(37, 23, "f32") == 9 * 40 * 32 * 4 + G
    assert clbm.buffer_bytes(37, 16, "f32") == 9 * 40 * 16 * 4 + G
    assert clbm.buffer_bytes(1030, 9, "f32") == 9 * 1056 * 12 * 4 + G
    assert clbm.buffer_bytes(1030, 3, "f32") == 9 * 1056 * 4 * 4 + G
    assert clbm.buffer_bytes(4100, 3, "f32") == 9 * 4128 * 3 * 4 + G
    # The line padding starts above 64 nodes: 64 x 1 keeps 64 elements,
    # 65 x 1 takes 96 (FP32), 80 (FP64) or 128 (16-bit) per run, and
    # R = 2^k grows the rows as before (65 x 64 FP32: 384-byte runs, R = 64).
    assert clbm.buffer_bytes(64, 1, "f32") == 9 * 64 * 1 * 4 + G
    assert clbm.buffer_bytes(65, 1, "f32") == 9 * 96 * 1 * 4 + G
    assert clbm.buffer_bytes(65, 1, "f64") == 9 * 80 * 1 * 8 + G
    assert clbm.buffer_bytes(65, 1, "bf16") == 9 * 128 * 1 * 2 + G
    assert clbm.buffer_bytes(65, 64, "f32") == 9 * 96 * 64 * 4 + G
    assert clbm.buffer_bytes(0, 5, "f32") == 0
    assert clbm.lib.clbm_buffer_bytes(5, 5, 9) == 0
    assert clbm.lib.clbm_buffer_bytes(5, 5, 6) == 0


def test_create_rejects_bad_arguments_before_touching_the_gpu():
    from paper_1705_11092_amd import clbm
    h = ctypes.c_void_p()
    base = dict(nx=8, ny=8, bc_y=0, storage=1, scheme=0, streaming=0, s0=1, s1=1, sb=1, s2=1,
                s3=1, s4=1, rho0=1.0, pop_a=None, pop_b=None, stream=None)
    bad = [dict(nx=0), dict(bc_y=3), dict(storage=7), dict(scheme=5), dict(streaming=2),
           dict(streaming=1, pop_b=0x1000),
           dict(s2=0.0), dict(s3=2.5), dict(s4=float("nan")), dict(rho0=-1.0)]
    for change in bad:
        cfg = clbm._Config(**{**base, **change})
        assert clbm.lib.clbm_create(ctypes.byref(cfg), ctypes.byref(h)) == clbm.CLBM_EINVAL, change
        assert clbm.lib.clbm_last_error()
    assert clbm.lib.clbm_create(None, ctypes.byref(h)) == clbm.CLBM_EINVAL
    assert clbm.lib.clbm_destroy(None) == clbm.CLBM_OK
    assert clbm.lib.clbm_batch_destroy(None) == clbm.CLBM_OK
    assert clbm.lib.clbm_step(None, 1) == clbm.CLBM_EINVAL
    assert clbm.lib.clbm_set_occupancy(None, 3) == clbm.CLBM_EINVAL
    assert clbm.lib.clbm_get_occupancy(None) == -1
    assert clbm.lib.clbm_set_resident_limit(None, 512) == clbm.CLBM_EINVAL
    assert clbm.lib.clbm_set_step_pairs(None, 1) == clbm.CLBM_EINVAL
    assert clbm.lib.clbm_get_step_pairs(None) == -1
    assert clbm.lib.clbm_batch_variant_count() >= 1
