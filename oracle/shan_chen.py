"""The Shan-Chen interaction force for the static-droplet workload
(Sec. IV C): TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Plain numpy, FP64, written from the definitions:

* pseudopotential psi(rho) = psi0 exp(-rho_ref / rho);
* force F(x) = -G psi(x) sum_i w_i psi(x + e_i) e_i over the eight moving
  directions, w = 1/3 where |e_i|^2 = 1 and 1/12 where |e_i|^2 = 2, on a
  lattice periodic in x and y;
* pressure p = rho cs^2 + G psi^2 / 2 (cs^2 = 1/3), used for the Laplace law.

The force depends on the state, so a step of this workload is: density of
the pre-collision state (Eq. 11), force from that density, then the ordinary
collide-and-stream step of the oracle with that force field.

Sign convention: with this form of F, G < 0 pulls each node toward denser
neighbours; the liquid-vapour coexistence densities the paper quotes
(0.3675 and 2.783 for psi0 = rho_ref = 1) belong to G = -10/3.
"""
from __future__ import annotations

import numpy as np

from . import BC_PERIODIC, SCHEME_CONSISTENT, init, moments, step

CS2 = 1.0 / 3.0
#: Lattice directions of Eq. (1) and the Shan-Chen weights of Sec. IV C.
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
W_SC = (0.0, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12)

#: The paper's droplet parameters: G (attractive sign), psi0, rho_ref.
PAPER_G, PAPER_PSI0, PAPER_RHO_REF = -10.0 / 3.0, 1.0, 1.0


def psi(rho, psi0: float = PAPER_PSI0, rho_ref: float = PAPER_RHO_REF) -> np.ndarray:
    """psi0 exp(-rho_ref / rho)."""
    return psi0 * np.exp(-rho_ref / np.asarray(rho, dtype=np.float64))


def neighbour(field: np.ndarray, i: int) -> np.ndarray:
    """field(x + e_i) on the periodic lattice ([ny, nx] arrays, x fastest)."""
    return np.roll(np.roll(field, -EX[i], axis=1), -EY[i], axis=0)


def force(rho, G: float = PAPER_G, psi0: float = PAPER_PSI0,
          rho_ref: float = PAPER_RHO_REF):
    """(Fx, Fy) = -G psi(x) sum_i w_i psi(x + e_i) e_i at every node."""
    p = psi(rho, psi0, rho_ref)
    sx = np.zeros_like(p)
    sy = np.zeros_like(p)
    for i in range(1, 9):
        nb = neighbour(p, i)
        sx += W_SC[i] * EX[i] * nb
        sy += W_SC[i] * EY[i] * nb
    return -G * p * sx, -G * p * sy


def pressure(rho, G: float = PAPER_G, psi0: float = PAPER_PSI0,
             rho_ref: float = PAPER_RHO_REF) -> np.ndarray:
    """p = rho cs^2 + G psi^2 / 2 (Sec. IV C)."""
    return CS2 * np.asarray(rho) + 0.5 * G * psi(rho, psi0, rho_ref) ** 2


def density(f) -> np.ndarray:
    """rho = sum_i f_i (Eq. 11)."""
    return np.sum(np.asarray(f), axis=0)


def start(rho, ux=None, uy=None, G: float = PAPER_G, psi0: float = PAPER_PSI0,
          rho_ref: float = PAPER_RHO_REF) -> np.ndarray:
    """Start state with density rho and velocity u (zero if not given) under
    the force of that density."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    fx, fy = force(rho, G, psi0, rho_ref)
    z = np.zeros_like(rho)
    return init(rho, z if ux is None else ux, z if uy is None else uy, fx, fy)


def run(f, s, nsteps: int, G: float = PAPER_G, psi0: float = PAPER_PSI0,
        rho_ref: float = PAPER_RHO_REF, scheme: int = SCHEME_CONSISTENT,
        nthreads: int = 0) -> np.ndarray:
    """``nsteps`` steps with the force recomputed from the density each step."""
    for _ in range(nsteps):
        fx, fy = force(density(f), G, psi0, rho_ref)
        f = step(f, fx, fy, s, bc_y=BC_PERIODIC, scheme=scheme, nthreads=nthreads)
    return f


def state(f, G: float = PAPER_G, psi0: float = PAPER_PSI0, rho_ref: float = PAPER_RHO_REF):
    """(rho, ux, uy) of a state, with Eq. (15)'s force taken from its density."""
    fx, fy = force(density(f), G, psi0, rho_ref)
    return moments(f, fx, fy)

