"""The oracle: TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of the D2Q9 cascaded lattice Boltzmann step
with the consistent forcing scheme (Fei & Luo, Sec. II), written in C
(``clbm_oracle.c``) and driven from here through ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It imports nothing from the GPU package and the GPU
package never imports it.

Arrays follow one layout: populations are ``[9, ny, nx]`` float64 (x
fastest), per-node fields are ``[ny, nx]`` float64.  The direction order is
the one of Eq. (1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "clbm_oracle.c")
_LIB = os.path.join(_HERE, "libclbm_oracle.so")

#: Forcing schemes: Eq. (12) (the paper's), Eq. (21) (Lycett-Brown & Luo
#: with Guo's term) and Eqs. (17)-(19) (Premnath et al., Sec. III A).
SCHEME_CONSISTENT = 0
SCHEME_GUO_LBL = 1
SCHEME_PREMNATH = 2

BC_PERIODIC = 0
BC_BOUNCEBACK = 1

_lib = None


def build() -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    cmd = [
        "gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
        "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.oracle_matrix_M.argtypes = [dp]
    lib.oracle_matrix_Minv.argtypes = [dp]
    lib.oracle_matrix_N.argtypes = [dbl, dbl, dp]
    lib.oracle_matrix_Ninv.argtypes = [dbl, dbl, dp]
    lib.oracle_collide.argtypes = [dp, dbl, dbl, dp, i32, i32, dp]
    lib.oracle_premnath_delta_f.argtypes = [dbl, dbl, dbl, dbl, dp]
    lib.oracle_step.argtypes = [i32, i32, i32, dp, i32, dp, dp, dp, dp, i32]
    lib.oracle_step.restype = i32
    lib.oracle_run.argtypes = [i32, i32, i32, dp, i32, dp, dp, dp, dp, i64, i32]
    lib.oracle_run.restype = i32
    lib.oracle_init.argtypes = [i32, i32, dp, dp, dp, dp, dp, dp]
    lib.oracle_init.restype = i32
    lib.oracle_moments.argtypes = [i32, i32, dp, dp, dp, dp, dp, dp]
    lib.oracle_moments.restype = i32
    lib.oracle_max_threads.restype = i32
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    """OpenMP threads the oracle uses when none are requested."""
    return int(_load().oracle_max_threads())


def matrix_M() -> np.ndarray:
    """M as printed in Eq. (5)."""
    out = np.empty((9, 9))
    _load().oracle_matrix_M(_p(out))
    return out


def matrix_Minv() -> np.ndarray:
    """M^-1 as printed in the Appendix."""
    out = np.empty((9, 9))
    _load().oracle_matrix_Minv(_p(out))
    return out


def matrix_N(ux: float, uy: float) -> np.ndarray:
    """N(u) as printed in Eq. (6)."""
    out = np.empty((9, 9))
    _load().oracle_matrix_N(float(ux), float(uy), _p(out))
    return out


def matrix_Ninv(ux: float, uy: float) -> np.ndarray:
    """N^-1(u) as printed in the Appendix."""
    out = np.empty((9, 9))
    _load().oracle_matrix_Ninv(float(ux), float(uy), _p(out))
    return out


def s6(s0=1.0, s1=1.0, sb=1.0, s2=1.0, s3=1.0, s4=1.0) -> np.ndarray:
    """The six distinct rates of S = diag(s0,s1,s1,sb,s2,s2,s3,s3,s4)."""
    return np.array([s0, s1, sb, s2, s3, s4], dtype=np.float64)


def collide(f, Fx: float, Fy: float, s, scheme: int = SCHEME_CONSISTENT,
            shift: bool = True) -> np.ndarray:
    """Post-collision populations at one node (Eqs. 11-15, 9).

    ``shift=False`` replaces N by the identity (Remark 2)."""
    f = _c(f).reshape(9)
    s = _c(s).reshape(6)
    out = np.empty(9)
    _load().oracle_collide(_p(f), float(Fx), float(Fy), _p(s), int(scheme),
                           1 if shift else 0, _p(out))
    return out


def premnath_delta_f(Fx: float, Fy: float, ux: float, uy: float) -> np.ndarray:
    """Delta f_i of Sec. III A (Eq. 18) at velocity u: the discrete
    distribution whose central moments are C_P of Eq. (19)."""
    out = np.empty(9)
    _load().oracle_premnath_delta_f(float(Fx), float(Fy), float(ux), float(uy), _p(out))
    return out


def force_field(kind: str, params, nx: int, ny: int):
    """Force density per node for the force kinds the lattices use.

    ``const``: (Fx, Fy) everywhere.  ``kolmogorov``: Fx = A sin(2 pi k y/ny),
    Fy = 0, with y the row index.  ``none``: zero.  ``field``: (fx, fy)
    arrays given in ``params``."""
    if kind == "none":
        return np.zeros((ny, nx)), np.zeros((ny, nx))
    if kind == "const":
        Fx, Fy = params
        return np.full((ny, nx), float(Fx)), np.full((ny, nx), float(Fy))
    if kind == "kolmogorov":
        A, k = params
        y = np.arange(ny, dtype=np.float64)
        col = float(A) * np.sin(2.0 * np.pi * float(k) * y / ny)
        return np.repeat(col[:, None], nx, axis=1), np.zeros((ny, nx))
    if kind == "field":
        fx, fy = params
        return _c(fx).reshape(ny, nx).copy(), _c(fy).reshape(ny, nx).copy()
    raise ValueError(f"unknown force kind {kind!r}")


def init(rho, ux, uy, fx, fy) -> np.ndarray:
    """Pre-collision f(x, 0) whose Eq. (15) moments are (rho, u)."""
    rho, ux, uy, fx, fy = (_c(a) for a in (rho, ux, uy, fx, fy))
    ny, nx = rho.shape
    f = np.empty((9, ny, nx))
    rc = _load().oracle_init(nx, ny, _p(rho), _p(ux), _p(uy), _p(fx), _p(fy), _p(f))
    if rc:
        raise ValueError("oracle_init rejected its arguments")
    return f


def moments(f, fx, fy):
    """(rho, ux, uy) of a pre-collision state (Eqs. 11 and 15)."""
    f, fx, fy = _c(f), _c(fx), _c(fy)
    _, ny, nx = f.shape
    rho, ux, uy = np.empty((ny, nx)), np.empty((ny, nx)), np.empty((ny, nx))
    rc = _load().oracle_moments(nx, ny, _p(f), _p(fx), _p(fy), _p(rho), _p(ux), _p(uy))
    if rc:
        raise ValueError("oracle_moments rejected its arguments")
    return rho, ux, uy


def step(f, fx, fy, s, bc_y: int = BC_PERIODIC, scheme: int = SCHEME_CONSISTENT,
         nthreads: int = 0) -> np.ndarray:
    """One collide-and-stream step; returns the new pre-collision state."""
    f, fx, fy, s = _c(f), _c(fx), _c(fy), _c(s)
    _, ny, nx = f.shape
    out = np.empty_like(f)
    rc = _load().oracle_step(nx, ny, int(bc_y), _p(s), int(scheme), _p(fx), _p(fy),
                             _p(f), _p(out), int(nthreads))
    if rc:
        raise ValueError("oracle_step rejected its arguments")
    return out


def run(f, fx, fy, s, nsteps: int, bc_y: int = BC_PERIODIC,
        scheme: int = SCHEME_CONSISTENT, nthreads: int = 0) -> np.ndarray:
    """``nsteps`` steps from pre-collision state ``f`` (not modified)."""
    f = _c(f).copy()
    fx, fy, s = _c(fx), _c(fy), _c(s)
    _, ny, nx = f.shape
    work = np.empty_like(f)
    rc = _load().oracle_run(nx, ny, int(bc_y), _p(s), int(scheme), _p(fx), _p(fy),
                            _p(f), _p(work), int(nsteps), int(nthreads))
    if rc:
        raise ValueError("oracle_run rejected its arguments")
    return f


def rel_l2(u, v, u_ref, v_ref) -> float:
    """E2 of Eq. (24): sqrt(sum |u - u_ref|^2 / sum |u_ref|^2) over both
    components and all nodes."""
    num = np.sum((np.asarray(u) - u_ref) ** 2) + np.sum((np.asarray(v) - v_ref) ** 2)
    den = np.sum(np.asarray(u_ref) ** 2) + np.sum(np.asarray(v_ref) ** 2)
    return float(np.sqrt(num / den))
