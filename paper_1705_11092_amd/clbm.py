"""ctypes binding of libclbm.so (include/clbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the
library is missing the import of this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclbm.so")

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f16sr": 4, "bf16sr": 5}
ELEM_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f16sr": 2, "bf16sr": 2}
BC = {"periodic": 0, "bounceback": 1}
STREAM_TWO_BUFFERS, STREAM_IN_PLACE = 0, 1
FORCE = {"none": 0, "const": 1, "kolmogorov": 2, "field": 3, "shan_chen": 4}
SCHEME = {"consistent": 0, "guo_lbl": 1, "premnath": 2}

CLBM_OK, CLBM_EINVAL, CLBM_EHIP, CLBM_ESTATE, CLBM_ENONFINITE = 0, -1, -2, -3, -4


class ClbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"clbm error {code}: {msg}")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_y", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("streaming", ctypes.c_int32),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("sb", ctypes.c_double),
        ("s2", ctypes.c_double), ("s3", ctypes.c_double), ("s4", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("pop_a", ctypes.c_void_p), ("pop_b", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1705_11092_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, dp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double))
    sig = {
        "clbm_buffer_bytes": (ctypes.c_size_t, [i32, i32, i32]),
        "clbm_create": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.POINTER(vp)]),
        "clbm_destroy": (ctypes.c_int, [vp]),
        "clbm_set_force": (ctypes.c_int, [vp, i32, dp, vp, vp]),
        "clbm_init": (ctypes.c_int, [vp, vp, vp, vp]),
        "clbm_step": (ctypes.c_int, [vp, i64]),
        "clbm_set_occupancy": (ctypes.c_int, [vp, i32]),
        "clbm_set_resident_limit": (ctypes.c_int, [vp, i64]),
        "clbm_set_step_pairs": (ctypes.c_int, [vp, i32]),
        "clbm_get_step_pairs": (i32, [vp]),
        "clbm_get_occupancy": (i32, [vp]),
        "clbm_step_count": (i64, [vp]),
        "clbm_moments": (ctypes.c_int, [vp, vp, vp, vp, dp]),
        "clbm_moments_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "clbm_error_norms": (ctypes.c_int, [vp, vp, vp, dp]),
        "clbm_get_populations": (ctypes.c_int, [vp, vp]),
        "clbm_set_populations": (ctypes.c_int, [vp, vp]),
        "clbm_set_graph_steps": (ctypes.c_int, [vp, i32]),
        "clbm_last_error": (ctypes.c_char_p, []),
        "clbm_nonslip_s3": (dbl, [dbl]),
        "clbm_s_from_nu": (dbl, [dbl]),
        "clbm_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, vp, ctypes.POINTER(vp)]),
        "clbm_batch_step": (ctypes.c_int, [vp, i64]),
        "clbm_batch_step_each": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
        "clbm_batch_autotune": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.POINTER(i32)]),
        "clbm_batch_variant_count": (i32, []),
        "clbm_batch_set_variant": (ctypes.c_int, [vp, i32]),
        "clbm_batch_get_variant": (i32, [vp]),
        "clbm_batch_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()

#: Every symbol include/clbm.h declares.
EXPORTED = (
    "clbm_buffer_bytes", "clbm_create", "clbm_destroy", "clbm_set_force", "clbm_init",
    "clbm_step", "clbm_step_count", "clbm_moments", "clbm_moments_noalloc", "clbm_error_norms",
    "clbm_get_populations", "clbm_set_populations", "clbm_set_graph_steps",
    "clbm_set_occupancy", "clbm_get_occupancy", "clbm_set_resident_limit",
    "clbm_set_step_pairs", "clbm_get_step_pairs",
    "clbm_last_error", "clbm_nonslip_s3", "clbm_s_from_nu", "clbm_batch_create",
    "clbm_batch_step", "clbm_batch_step_each", "clbm_batch_autotune",
    "clbm_batch_variant_count", "clbm_batch_set_variant", "clbm_batch_get_variant",
    "clbm_batch_destroy",
)


def _check(rc: int):
    if rc != CLBM_OK:
        raise ClbmError(rc, lib.clbm_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _field(a, shape, device) -> Optional[torch.Tensor]:
    """FP64 contiguous device tensor of `shape` from numpy / torch / None."""
    if a is None:
        return None
    if not isinstance(a, torch.Tensor):
        a = np.asarray(a, dtype=np.float64)
        if not a.flags.writeable:  # e.g. a broadcast view: torch wants its own copy
            a = a.copy()
    t = torch.as_tensor(a)
    t = t.to(device=device, dtype=torch.float64).contiguous()
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def buffer_bytes(nx: int, ny: int, storage: str) -> int:
    return int(lib.clbm_buffer_bytes(nx, ny, STORAGE[storage]))


def nonslip_s3(s2: float) -> float:
    return float(lib.clbm_nonslip_s3(s2))


def s_from_nu(nu: float) -> float:
    return float(lib.clbm_s_from_nu(nu))


class Lattice:
    """One D2Q9 lattice on the GPU (see include/clbm.h for the semantics)."""

    def __init__(self, nx: int, ny: int, s: Sequence[float], storage: str = "f32",
                 bc_y: str = "periodic", rho0: float = 1.0, scheme: str = "consistent",
                 device: str = "cuda", stream: Optional[torch.cuda.Stream] = None,
                 inplace: bool = False):
        self.nx, self.ny, self.storage = int(nx), int(ny), storage
        self.inplace = bool(inplace)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = buffer_bytes(self.nx, self.ny, storage)
        if nbytes == 0:
            raise ClbmError(CLBM_EINVAL, "invalid lattice size or storage")
        with torch.cuda.stream(self.stream):
            self.pop_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.pop_b = (None if self.inplace else
                          torch.empty(nbytes, dtype=torch.uint8, device=self.device))
        s = [float(v) for v in s]
        cfg = _Config(self.nx, self.ny, BC[bc_y], STORAGE[storage], SCHEME[scheme],
                      STREAM_IN_PLACE if self.inplace else STREAM_TWO_BUFFERS,
                      s[0], s[1], s[2], s[3], s[4], s[5], float(rho0),
                      self.pop_a.data_ptr(), None if self.inplace else self.pop_b.data_ptr(),
                      self.stream.cuda_stream)
        self._cfg = cfg
        h = ctypes.c_void_p()
        _check(lib.clbm_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._force_keep = None

    # -- state ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib.clbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def footprint_bytes(self) -> int:
        return (1 if self.inplace else 2) * self.pop_a.numel()

    def set_force(self, kind: str, params=None, fx=None, fy=None):
        p = None
        if params is not None:
            arr = (ctypes.c_double * len(params))(*[float(v) for v in params])
            p = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        with torch.cuda.stream(self.stream):
            tfx = _field(fx, (self.ny, self.nx), self.device)
            tfy = _field(fy, (self.ny, self.nx), self.device)
            _check(lib.clbm_set_force(self._h, FORCE[kind], p, _ptr(tfx), _ptr(tfy)))
        self._force_keep = (tfx, tfy)  # keep alive until the stream passes the copy
        return self

    def init(self, rho=None, ux=None, uy=None):
        shape = (self.ny, self.nx)
        with torch.cuda.stream(self.stream):
            tr, tu, tv = (_field(a, shape, self.device) for a in (rho, ux, uy))
            _check(lib.clbm_init(self._h, _ptr(tr), _ptr(tu), _ptr(tv)))
        # The input fields are freed into torch's allocator on this stream, so
        # later work on the stream cannot reuse them before the kernel reads.
        return self

    def step(self, n: int = 1):
        _check(lib.clbm_step(self._h, int(n)))
        return self

    @property
    def steps(self) -> int:
        return int(lib.clbm_step_count(self._h))

    def set_graph_steps(self, n: int):
        _check(lib.clbm_set_graph_steps(self._h, int(n)))

    def set_resident_limit(self, max_groups: int):
        """Largest lattice (in groups of nodes) stepped by the resident
        kernel; 0 turns it off."""
        _check(lib.clbm_set_resident_limit(self._h, int(max_groups)))
        return self

    @property
    def step_pairs(self) -> bool:
        """Whether this lattice advances two fused steps per launch."""
        return int(lib.clbm_get_step_pairs(self._h)) == 1

    @step_pairs.setter
    def step_pairs(self, enable: Optional[bool]):
        """True: pairs wherever supported; False: never; None: the default
        (pairs wherever supported)."""
        _check(lib.clbm_set_step_pairs(self._h, -1 if enable is None else (1 if enable else 0)))

    @property
    def occupancy(self) -> int:
        """Cap on the step kernel's blocks per compute unit (0 = none)."""
        return int(lib.clbm_get_occupancy(self._h))

    @occupancy.setter
    def occupancy(self, blocks_per_cu: int):
        _check(lib.clbm_set_occupancy(self._h, int(blocks_per_cu)))

    def moments(self, fields: bool = True, totals: bool = True):
        """(rho, ux, uy, totals): FP64 device fields (or None) and the host
        FP64 totals {mass, x-momentum, y-momentum} (or None)."""
        shape = (self.ny, self.nx)
        with torch.cuda.stream(self.stream):
            if fields:
                rho, ux, uy = (torch.empty(shape, dtype=torch.float64, device=self.device)
                               for _ in range(3))
            else:
                rho = ux = uy = None
            tot = (ctypes.c_double * 3)() if totals else None
            _check(lib.clbm_moments(self._h, _ptr(rho), _ptr(ux), _ptr(uy),
                                    ctypes.cast(tot, ctypes.POINTER(ctypes.c_double)) if totals else None))
        return rho, ux, uy, (list(tot) if totals else None)

    def moments_noalloc(self, rho=None, ux=None, uy=None, totals=None):
        """clbm_moments_noalloc into caller-owned FP64 device tensors (each
        may be None; totals holds 3 values).  Enqueues only: the library
        allocates nothing and does not wait for the device."""
        _check(lib.clbm_moments_noalloc(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(totals)))

    def error_norms(self, ux_ref, uy_ref):
        """(sum |u - u_ref|^2, sum |u_ref|^2) in FP64 on the GPU."""
        shape = (self.ny, self.nx)
        with torch.cuda.stream(self.stream):
            a, b = _field(ux_ref, shape, self.device), _field(uy_ref, shape, self.device)
            out = (ctypes.c_double * 2)()
            _check(lib.clbm_error_norms(self._h, _ptr(a), _ptr(b),
                                        ctypes.cast(out, ctypes.POINTER(ctypes.c_double))))
        return out[0], out[1]

    def get_populations(self) -> torch.Tensor:
        with torch.cuda.stream(self.stream):
            f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
            _check(lib.clbm_get_populations(self._h, _ptr(f)))
        return f

    def set_populations(self, f):
        with torch.cuda.stream(self.stream):
            t = _field(f, (9, self.ny, self.nx), self.device)
            _check(lib.clbm_set_populations(self._h, _ptr(t)))
        return self


class Batch:
    """Many lattices advanced by one persistent launch per step."""

    def __init__(self, lattices: Sequence[Lattice], stream: Optional[torch.cuda.Stream] = None):
        self.lattices = list(lattices)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (ctypes.c_void_p * len(self.lattices))(*[l.handle.value for l in self.lattices])
        b = ctypes.c_void_p()
        _check(lib.clbm_batch_create(arr, len(self.lattices), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(b)))
        self._b = b

    def close(self):
        if getattr(self, "_b", None):
            lib.clbm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(lib.clbm_batch_step(self._b, int(n)))
        return self

    def step_each(self, counts: Sequence[int]):
        arr = (ctypes.c_int64 * len(counts))(*[int(c) for c in counts])
        _check(lib.clbm_batch_step_each(self._b, arr))
        return self

    def autotune(self, cache_path: Optional[str] = None) -> int:
        v = ctypes.c_int32(-1)
        _check(lib.clbm_batch_autotune(self._b, cache_path.encode() if cache_path else None,
                                       ctypes.byref(v)))
        return int(v.value)

    @staticmethod
    def variant_count() -> int:
        return int(lib.clbm_batch_variant_count())

    @property
    def variant(self) -> int:
        return int(lib.clbm_batch_get_variant(self._b))

    @variant.setter
    def variant(self, v: int):
        _check(lib.clbm_batch_set_variant(self._b, int(v)))


def lattice_from_workload(wl, storage: str = "f32", device: str = "cuda",
                          stream: Optional[torch.cuda.Stream] = None, init: bool = True,
                          inplace: bool = False, scheme: str = "consistent") -> Lattice:
    """A Lattice set up from an inputs.Workload (force then start state)."""
    lat = Lattice(wl.nx, wl.ny, wl.s, storage=storage,
                  bc_y="bounceback" if wl.bc_y == 1 else "periodic", rho0=wl.rho0,
                  device=device, stream=stream, inplace=inplace, scheme=scheme)
    if wl.force_kind == "field":
        lat.set_force("field", fx=wl.force_params[0], fy=wl.force_params[1])
    elif wl.force_kind == "none":
        lat.set_force("none")
    else:
        lat.set_force(wl.force_kind, params=wl.force_params)
    if init:
        lat.init(wl.rho, wl.ux, wl.uy)
    return lat
