"""Definitions the tests check the oracle against, written from the paper's
definitions and from textbook solutions of the Navier-Stokes equations,
independently of the oracle's typed-in matrices.

Nothing here imports the oracle or the GPU package.
"""
from __future__ import annotations

import math

import numpy as np

# Eq. (1)
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
CS2 = 1.0 / 3.0

# (m, n) exponents behind the recombined vector of Eq. (3).
_SLOTS = [
    [((0, 0), 1.0)],
    [((1, 0), 1.0)],
    [((0, 1), 1.0)],
    [((2, 0), 1.0), ((0, 2), 1.0)],
    [((2, 0), 1.0), ((0, 2), -1.0)],
    [((1, 1), 1.0)],
    [((2, 1), 1.0)],
    [((1, 2), 1.0)],
    [((2, 2), 1.0)],
]


def moment_matrix(ux: float = 0.0, uy: float = 0.0) -> np.ndarray:
    """A with A f = recombined central moments about u (Eqs. 2-3); at u = 0
    these are the raw moments."""
    cx, cy = EX - ux, EY - uy
    A = np.zeros((9, 9))
    for r, terms in enumerate(_SLOTS):
        for (m, n), c in terms:
            A[r] += c * cx**m * cy**n
    return A


def central_moments(f, ux: float, uy: float) -> np.ndarray:
    """Recombined central moments of f by direct summation (Eqs. 2-3)."""
    f = np.asarray(f, dtype=np.float64)
    cx, cy = EX - ux, EY - uy

    def k(m, n):
        return float(np.sum(f * cx**m * cy**n))

    return np.array([k(0, 0), k(1, 0), k(0, 1), k(2, 0) + k(0, 2), k(2, 0) - k(0, 2),
                     k(1, 1), k(2, 1), k(1, 2), k(2, 2)])


def velocity(f, Fx: float, Fy: float):
    """Eq. (11) and Eq. (15)."""
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum()
    return rho, (np.dot(f, EX) + 0.5 * Fx) / rho, (np.dot(f, EY) + 0.5 * Fy) / rho


def from_central_moments(T, ux: float, uy: float) -> np.ndarray:
    """The unique f whose recombined central moments about u are T (a linear
    solve on the definition, not the printed inverses)."""
    return np.linalg.solve(moment_matrix(ux, uy), np.asarray(T, dtype=np.float64))


def product_equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    """rho Psi(e_x) Psi(e_y) with the 1-D D1Q3 factors Psi(0) = 2/3 - u^2 and
    Psi(+-1) = (1/3 + u^2 +- u)/2: the D2Q9 population whose central moments
    are those of the continuous Maxwellian up to k22 (tensor product of two
    1-D three-velocity equilibria)."""

    def psi(e, u):
        return np.where(e == 0, 2.0 / 3.0 - u * u, (1.0 / 3.0 + u * u + e * u) / 2.0)

    return rho * psi(EX, ux) * psi(EY, uy)


W = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


def guo_term(Fx: float, Fy: float, ux: float, uy: float) -> np.ndarray:
    """Guo's R_Gi (Remark 3)."""
    eu = EX * ux + EY * uy
    ax = (EX - ux) / CS2 + eu * EX / CS2**2
    ay = (EY - uy) / CS2 + eu * EY / CS2**2
    return W * (ax * Fx + ay * Fy)


def he_term(f_eq, rho: float, Fx: float, Fy: float, ux: float, uy: float) -> np.ndarray:
    """He's R_i of Eq. (13)."""
    return (Fx * (EX - ux) + Fy * (EY - uy)) / (rho * CS2) * f_eq


def mirror_x(field: np.ndarray) -> np.ndarray:
    """Node field under x -> -x on a periodic row of length nx."""
    return np.roll(field[..., ::-1], 1, axis=-1)


# Direction index under x -> -x (Eq. 1 order).
MIRROR_X_DIR = [0, 3, 2, 1, 4, 6, 5, 8, 7]


# --------------------------------------------------------------------------
# Closed-form flows
# --------------------------------------------------------------------------

def poiseuille_steady(ny: int, Fx: float, nu: float, rho0: float = 1.0) -> np.ndarray:
    """Steady channel profile u = Fx (L^2 - eta^2)/(2 rho0 nu), walls half a
    link outside rows 0 and ny-1, so 2L = ny (Eq. 23 with its L^2 factor)."""
    L = ny / 2.0
    eta = np.arange(ny) - (ny - 1) / 2.0
    return Fx / (2.0 * rho0 * nu) * (L * L - eta * eta)


def poiseuille_startup(ny: int, Fx: float, nu: float, t: float, nterms: int = 400,
                       rho0: float = 1.0) -> np.ndarray:
    """Channel flow started from rest: the steady profile minus its cosine
    series, each mode decaying as exp(-nu lambda_n^2 t)."""
    L = ny / 2.0
    eta = np.arange(ny) - (ny - 1) / 2.0
    s = L * L - eta * eta
    for n in range(nterms):
        lam = (2 * n + 1) * math.pi / (2 * L)
        a = 32.0 * L * L * (-1) ** n / ((2 * n + 1) ** 3 * math.pi**3)
        s = s - a * np.cos(lam * eta) * math.exp(-nu * lam * lam * t)
    return Fx / (2.0 * rho0 * nu) * s


def taylor_green_decay(nx: int, ny: int, u0: float, nu: float, F, t: float):
    """Decaying Taylor-Green vortex carried by a uniform body force:
    u = F t + u0 [sin(phi X) sin(phi Y), cos(phi X) cos(phi Y)] e^{-2 nu phi^2 t}
    with X = x - Fx t^2/2, Y = y - Fy t^2/2 (Galilean shift of the classic
    solution by the uniformly accelerated frame; exact for incompressible
    Navier-Stokes on a square box, phi = 2 pi/n)."""
    assert nx == ny
    phi = 2.0 * math.pi / nx
    Fx, Fy = F
    x = np.arange(nx)[None, :] - 0.5 * Fx * t * t
    y = np.arange(ny)[:, None] - 0.5 * Fy * t * t
    d = math.exp(-2.0 * nu * phi * phi * t)
    ux = Fx * t + u0 * np.sin(phi * x) * np.sin(phi * y) * d
    uy = Fy * t + u0 * np.cos(phi * x) * np.cos(phi * y) * d
    return np.broadcast_to(ux, (ny, nx)), np.broadcast_to(uy, (ny, nx))


def kolmogorov_startup(n: int, A: float, k: int, nu: float, t: float):
    """Kolmogorov flow from rest under Fx = A sin(kappa y):
    ux = A/(nu kappa^2) (1 - e^{-nu kappa^2 t}) sin(kappa y), kappa = 2 pi k/n."""
    kap = 2.0 * math.pi * k / n
    y = np.arange(n)[:, None]
    ux = A / (nu * kap * kap) * (1.0 - math.exp(-nu * kap * kap * t)) * np.sin(kap * y)
    return np.broadcast_to(ux, (n, n)), np.zeros((n, n))


def steady_taylor_green(N: int, u0: float, nu: float):
    """Steady forced Taylor-Green flow (Sec. IV B): u_a and the force that
    holds it, F = 2 nu phi^2 u_a (the force printed in Sec. IV B has its
    components exchanged; this one makes u_a, p_a an exact steady solution)."""
    phi = 2.0 * math.pi / N
    x = np.arange(N)[None, :]
    y = np.arange(N)[:, None]
    ua = np.broadcast_to(u0 * np.sin(phi * x) * np.sin(phi * y), (N, N))
    va = np.broadcast_to(u0 * np.cos(phi * x) * np.cos(phi * y), (N, N))
    rho = np.broadcast_to(1.0 + 3.0 * 0.25 * u0 * u0 * (np.cos(2 * phi * x) - np.cos(2 * phi * y)),
                          (N, N))
    fx = 2.0 * nu * phi * phi * ua
    fy = 2.0 * nu * phi * phi * va
    return (np.ascontiguousarray(ua), np.ascontiguousarray(va), np.ascontiguousarray(rho),
            np.ascontiguousarray(fx), np.ascontiguousarray(fy))


def rel_l2(u, v, ur, vr) -> float:
    """E2 of Eq. (24) over both components."""
    num = np.sum((np.asarray(u) - ur) ** 2) + np.sum((np.asarray(v) - vr) ** 2)
    den = np.sum(np.asarray(ur) ** 2) + np.sum(np.asarray(vr) ** 2)
    return float(np.sqrt(num / den))
