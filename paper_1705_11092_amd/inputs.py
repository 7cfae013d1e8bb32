"""Seeded synthetic inputs for the lattice workloads.

This module holds no arithmetic of the collide-and-stream step: it only
builds initial fields (density and velocity per node), force parameters and
relaxation rates for the flows the paper and the workload list use.  Both
the GPU path and the oracle receive what it produces; it imports neither.

Every workload is an analytic flow; nothing here stands in for a dataset.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

RHO0 = 1.0


def s_from_nu(nu: float) -> float:
    """s2 = 1/(3 nu + 0.5) (Sec. II A)."""
    return 1.0 / (3.0 * nu + 0.5)


def nonslip_s3(s2: float) -> float:
    """Remark 4: s3 = (16 - 8 s2)/(8 - s2) removes the numerical slip of
    half-way bounce-back in Poiseuille flow."""
    return (16.0 - 8.0 * s2) / (8.0 - s2)


@dataclasses.dataclass
class Workload:
    """One lattice problem: sizes, boundaries, rates, force and start state."""

    name: str
    nx: int
    ny: int
    bc_y: int  # 0 periodic, 1 half-way bounce-back walls
    s: Tuple[float, float, float, float, float, float]  # s0, s1, sb, s2, s3, s4
    force_kind: str  # "none" | "const" | "kolmogorov" | "field" | "shan_chen"
    force_params: tuple
    rho: np.ndarray  # [ny, nx]
    ux: np.ndarray
    uy: np.ndarray
    steps: int
    rho0: float = RHO0
    meta: dict = dataclasses.field(default_factory=dict)


def _rest(nx: int, ny: int):
    return np.full((ny, nx), RHO0), np.zeros((ny, nx)), np.zeros((ny, nx))


def poiseuille(nx: int = 64, ny: int = 32, Fx: float = 1e-6, tau: float = 1.0,
               s3: Optional[float] = None, steps: int = 10_000) -> Workload:
    """Body-force-driven channel (Sec. IV A): periodic in x, bounce-back walls
    in y, started from rest.  Rates follow the paper's Poiseuille recipe:
    every rate equals s2 except s3, which takes the no-slip value unless
    given."""
    s2 = 1.0 / tau
    s3v = nonslip_s3(s2) if s3 is None else float(s3)
    rho, ux, uy = _rest(nx, ny)
    return Workload("poiseuille", nx, ny, 1, (s2, s2, s2, s2, s3v, s2), "const",
                    (Fx, 0.0), rho, ux, uy, steps,
                    meta={"Fx": Fx, "nu": (tau - 0.5) / 3.0})


def taylor_green(n: int, u0: float = 0.01, nu: float = 0.01,
                 F: Tuple[float, float] = (1e-6, 5e-7), steps: int = 20_000,
                 ny: Optional[int] = None) -> Workload:
    """Decaying Taylor-Green vortex on a periodic n x n box plus a uniform body
    force.  Velocity u0 [sin(phi x) sin(phi y), cos(phi x) cos(phi y)] with
    phi = 2 pi/n (the spatial form of Sec. IV B) and density from the
    pressure p0 + u0^2/4 [cos(2 phi x) - cos(2 phi y)] through p = rho cs^2.
    Rates: s2 from nu, sb = s2, the rest 1 (the recipe of Sec. IV B)."""
    nx = n
    ny = n if ny is None else ny
    phi_x = 2.0 * math.pi / nx
    phi_y = 2.0 * math.pi / ny
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    ux = u0 * np.sin(phi_x * x) * np.sin(phi_y * y)
    uy = u0 * np.cos(phi_x * x) * np.cos(phi_y * y)
    p_dev = 0.25 * u0 * u0 * (np.cos(2 * phi_x * x) - np.cos(2 * phi_y * y))
    rho = RHO0 + 3.0 * p_dev
    s2 = s_from_nu(nu)
    kind = "none" if (F[0] == 0.0 and F[1] == 0.0) else "const"
    return Workload(f"taylor_green_{nx}x{ny}", nx, ny, 0, (1.0, 1.0, s2, s2, 1.0, 1.0),
                    kind, (float(F[0]), float(F[1])) if kind == "const" else (),
                    rho, ux, uy, steps, meta={"u0": u0, "nu": nu, "F": F})


def kolmogorov(n: int, A: float, k: int, tau: float, steps: int = 1000) -> Workload:
    """Kolmogorov flow from rest: Fx = A sin(2 pi k y / n), periodic box."""
    s2 = 1.0 / tau
    rho, ux, uy = _rest(n, n)
    return Workload(f"kolmogorov_{n}", n, n, 0, (1.0, 1.0, s2, s2, 1.0, 1.0), "kolmogorov",
                    (float(A), int(k)), rho, ux, uy, steps,
                    meta={"A": A, "k": k, "nu": (tau - 0.5) / 3.0})


def steady_taylor_green(N: int, Re: float, u0: float = 0.05, scheme: str = "consistent",
                        steps: int = 0) -> Workload:
    """Steady forced Taylor-Green flow of Sec. IV B on an N x N periodic box:
    u_a = u0 [sin(phi x) sin(phi y), cos(phi x) cos(phi y)], phi = 2 pi/N,
    held by the force F = 2 nu phi^2 u_a, with nu = u0 N / Re; started from
    u_a and the density of p_a.  Rates: sb = s2, s1 = s2 for the
    Lycett-Brown & Luo scheme and 1 otherwise, the rest 1."""
    nu = u0 * N / Re
    s2 = s_from_nu(nu)
    phi = 2.0 * math.pi / N
    x = np.arange(N, dtype=np.float64)[None, :]
    y = np.arange(N, dtype=np.float64)[:, None]
    ux = np.ascontiguousarray(np.broadcast_to(u0 * np.sin(phi * x) * np.sin(phi * y), (N, N)))
    uy = np.ascontiguousarray(np.broadcast_to(u0 * np.cos(phi * x) * np.cos(phi * y), (N, N)))
    rho = np.ascontiguousarray(np.broadcast_to(
        RHO0 + 3.0 * 0.25 * u0 * u0 * (np.cos(2 * phi * x) - np.cos(2 * phi * y)), (N, N)))
    fx = 2.0 * nu * phi * phi * ux
    fy = 2.0 * nu * phi * phi * uy
    s1 = s2 if scheme == "guo_lbl" else 1.0
    return Workload(f"steady_tg_{N}_Re{Re:g}_{scheme}", N, N, 0, (1.0, s1, s2, s2, 1.0, 1.0),
                    "field", (fx, fy), rho, ux, uy, steps,
                    meta={"Re": Re, "nu": nu, "u0": u0, "scheme": scheme})


def channel(width: int, Fx: float, s2: float, s3: float, s1: Optional[float] = None,
            scheme: str = "consistent", length: int = 1) -> Workload:
    """Poiseuille channel of Sec. IV A: `width` nodes between half-way
    bounce-back walls, periodic in x over `length` nodes, from rest, every
    rate s2 except s3 (and s1 = 1 unless given)."""
    rho, ux, uy = _rest(length, width)
    s1v = 1.0 if s1 is None else s1
    return Workload(f"channel_{width}_{scheme}", length, width, 1, (s2, s1v, s2, s2, s3, s2),
                    "const", (Fx, 0.0), rho, ux, uy, 0,
                    meta={"Fx": Fx, "nu": (1.0 / s2 - 0.5) / 3.0, "scheme": scheme})


def droplet(n: int = 200, R: float = 50.0, s3: float = 1.0, s2: float = 1.4,
            scheme: str = "consistent", G: float = -10.0 / 3.0, psi0: float = 1.0,
            rho_ref: float = 1.0, rho_l: float = 2.783, rho_v: float = 0.3675,
            steps: int = 0) -> Workload:
    """Static droplet of Sec. IV C on an n x n periodic box: density rho_l
    inside a circle of radius R about the box centre ((n - 1)/2, (n - 1)/2),
    rho_v outside, at rest, under the Shan-Chen force with parameters
    (G, psi0, rho_ref).  Rates: sb = s2 (= s_v), s3 as given, the rest 1;
    s1 = s2 for the Lycett-Brown & Luo scheme (momentum conservation)."""
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    rho = np.where((x - c) ** 2 + (y - c) ** 2 < R * R, rho_l, rho_v)
    z = np.zeros((n, n))
    s1 = s2 if scheme == "guo_lbl" else 1.0
    return Workload(f"droplet_{n}_R{R:g}_s3_{s3:g}_{scheme}", n, n, 0, (1.0, s1, s2, s2, s3, 1.0),
                    "shan_chen", (float(G), float(psi0), float(rho_ref)), rho, z, z.copy(), steps,
                    meta={"R": R, "scheme": scheme, "rho_l": rho_l, "rho_v": rho_v})


def slab(n: int = 128, width: int = 64, ny: int = 4, s2: float = 1.4, s3: float = 1.0,
         G: float = -10.0 / 3.0, rho_l: float = 2.783, rho_v: float = 0.3675,
         steps: int = 0) -> Workload:
    """Flat liquid slab (a planar interface pair): rho_l on the `width` middle
    columns of an n x ny periodic box, rho_v elsewhere, at rest, under the
    Shan-Chen force.  With no curvature both phases settle at the
    coexistence densities."""
    x = np.arange(n, dtype=np.float64)[None, :]
    lo = (n - width) // 2
    rho = np.ascontiguousarray(np.broadcast_to(np.where((x >= lo) & (x < lo + width), rho_l, rho_v),
                                               (ny, n)))
    z = np.zeros((ny, n))
    return Workload(f"slab_{n}x{ny}_w{width}", n, ny, 0, (1.0, 1.0, s2, s2, s3, 1.0), "shan_chen",
                    (float(G), 1.0, 1.0), rho, z, z.copy(), steps, meta={"width": width})


def random_state(nx: int, ny: int, seed: int, amp_rho: float = 0.02,
                 amp_u: float = 0.05, bc_y: int = 0, s=None,
                 force: str = "field", amp_f: float = 1e-3, steps: int = 10) -> Workload:
    """White-noise density and velocity per node and (by default) a white-noise
    force field: every node differs from its neighbours, so any streaming or
    indexing slip shows up node by node."""
    rng = np.random.default_rng(seed)
    rho = RHO0 + amp_rho * rng.uniform(-1, 1, (ny, nx))
    ux = amp_u * rng.uniform(-1, 1, (ny, nx))
    uy = amp_u * rng.uniform(-1, 1, (ny, nx))
    if s is None:
        s = tuple(rng.uniform(0.6, 1.9, 6))
    if force == "field":
        fp = (amp_f * rng.uniform(-1, 1, (ny, nx)), amp_f * rng.uniform(-1, 1, (ny, nx)))
    elif force == "const":
        fp = (float(amp_f * rng.uniform(-1, 1)), float(amp_f * rng.uniform(-1, 1)))
    elif force == "kolmogorov":
        fp = (float(amp_f), int(rng.integers(1, 4)))
    else:
        fp = ()
    return Workload(f"random_{nx}x{ny}_s{seed}", nx, ny, bc_y, tuple(float(v) for v in s),
                    force, fp, rho, ux, uy, steps)


def kolmogorov_batch(count: int = 256, seed: int = 0, n_lo: int = 32, n_hi: int = 512,
                     steps: int = 1000) -> List[Workload]:
    """The batch of uneven Kolmogorov lattices: for each lattice, in this
    order, side N = round(exp(U(ln n_lo, ln n_hi))), A ~ U(1e-6, 1e-5),
    k in {1, 2, 4}, tau ~ U(0.55, 1.5)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        A = float(rng.uniform(1e-6, 1e-5))
        k = int(rng.choice([1, 2, 4]))
        tau = float(rng.uniform(0.55, 1.5))
        out.append(kolmogorov(n, A, k, tau, steps))
    return out


@dataclasses.dataclass
class Request:
    """One solve submitted to the server."""

    rid: int
    arrival: float  # seconds from stream start
    workload: Workload
    storage: str  # "f32" | "f16" | "bf16" | "f64"


def served_stream(count: int = 400, seed: int = 1, rate: float = 4.8,
                  n_lo: int = 64, n_hi: int = 2048, steps_lo: float = 1e3,
                  steps_hi: float = 1e5, storage_16: str = "f16sr") -> List[Request]:
    """Poisson arrivals of solves with sides log-uniform in [n_lo, n_hi], step
    counts log-uniform in [steps_lo, steps_hi], forcing uniform over
    {constant, Kolmogorov, none} (none = decaying Taylor-Green), storage FP32
    or 16-bit with equal odds (FP16 with stochastic rounding unless told
    otherwise: the more accurate 16-bit form on long runs), tau ~ U(0.55, 1.5)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        steps = int(round(math.exp(rng.uniform(math.log(steps_lo), math.log(steps_hi)))))
        kind = ["const", "kolmogorov", "none"][int(rng.integers(0, 3))]
        storage = "f32" if rng.uniform() < 0.5 else storage_16
        tau = float(rng.uniform(0.55, 1.5))
        nu = (tau - 0.5) / 3.0
        if kind == "const":
            F0 = min(1e-6, 0.05 / steps)
            wl = taylor_green(n, u0=0.0, nu=nu, F=(F0, F0 / 2), steps=steps)
            wl.name = f"const_{n}"
        elif kind == "kolmogorov":
            A = float(rng.uniform(1e-6, 1e-5))
            A = min(A, 0.05 / steps)
            k = int(rng.choice([1, 2, 4]))
            wl = kolmogorov(n, A, k, tau, steps)
        else:
            wl = taylor_green(n, u0=0.01, nu=nu, F=(0.0, 0.0), steps=steps)
        out.append(Request(rid, t, wl, storage))
    return out
