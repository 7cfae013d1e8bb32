"""The library's node update, compiled for the host, against the oracle
(no GPU).

tests/host_collide.hip wraps collide() of the kernels' header with the rate
constants the library derives for a lattice; it is built here with
hipcc --offload-host-only.  The kernel expands M, N(u), N^-1(u) and M^-1 by
hand (factorised shifts, deviations from the rest state); the oracle applies
the printed matrices as dense products.  They must agree to FP64 rounding
for every forcing scheme (Eq. 12, Eq. 21 and Eqs. 17-19) over random states,
velocities up to 0.15 and random rates, and to FP32 rounding in FP32.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("host_collide") / "libhost_collide.so"
    subprocess.check_call([HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-fPIC", "-shared",
                           "-ffp-contract=on", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1705_11092_amd", "csrc"),
                           "-o", str(out), os.path.join(ROOT, "tests", "host_collide.hip")],
                          stderr=subprocess.DEVNULL)
    h = ctypes.CDLL(str(out))
    dp = ctypes.POINTER(ctypes.c_double)
    for fn in (h.host_collide_f64, h.host_collide_f32):
        fn.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double, ctypes.c_int, dp]
    return h


def _run(fn, f, Fx, Fy, s, rho0, scheme):
    dp = ctypes.POINTER(ctypes.c_double)
    f = np.ascontiguousarray(f, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.empty(9)
    fn(f.ctypes.data_as(dp), Fx, Fy, s.ctypes.data_as(dp), rho0, scheme, out.ctypes.data_as(dp))
    return out


@pytest.mark.parametrize("scheme", [oracle.SCHEME_CONSISTENT, oracle.SCHEME_GUO_LBL,
                                    oracle.SCHEME_PREMNATH])
def test_kernel_collision_matches_oracle(lib, scheme):
    rng = np.random.default_rng(400 + scheme)
    one = np.ones((1, 1))
    w64 = w32 = 0.0
    for _ in range(400):
        rho0 = rng.choice([1.0, 0.7, 2.5])
        rho = rho0 * (1 + rng.uniform(-0.05, 0.05))
        ux, uy = rng.uniform(-0.15, 0.15, 2)
        Fx, Fy = rng.uniform(-5e-3, 5e-3, 2)
        f = oracle.init(rho * one, ux * one, uy * one, Fx * one, Fy * one)[:, 0, 0]
        f = f + rng.normal(0.0, 3e-3 * rho0, 9)
        s = oracle.s6(*rng.uniform(0.3, 1.98, 6))
        ref = oracle.collide(f, Fx, Fy, s, scheme)
        w64 = max(w64, np.max(np.abs(_run(lib.host_collide_f64, f, Fx, Fy, s, rho0, scheme) - ref)) / rho0)
        w32 = max(w32, np.max(np.abs(_run(lib.host_collide_f32, f, Fx, Fy, s, rho0, scheme) - ref)) / rho0)
    assert w64 < 2e-15, w64
    assert w32 < 1e-7, w32


def test_premnath_is_the_consistent_collision_at_s3_2(lib):
    # Remark 6 on the kernel's arithmetic: with s3 = 2 the two schemes give
    # the same post-collision state.
    rng = np.random.default_rng(410)
    one = np.ones((1, 1))
    for _ in range(50):
        f = oracle.init(one, 0.05 * one, -0.03 * one, 1e-3 * one, 2e-3 * one)[:, 0, 0]
        f = f + rng.normal(0.0, 1e-3, 9)
        s = oracle.s6(*rng.uniform(0.5, 1.9, 6))
        s[4] = 2.0
        a = _run(lib.host_collide_f64, f, 1e-3, 2e-3, s, 1.0, oracle.SCHEME_CONSISTENT)
        b = _run(lib.host_collide_f64, f, 1e-3, 2e-3, s, 1.0, oracle.SCHEME_PREMNATH)
        assert np.array_equal(a, b)
