"""Helpers shared by the GPU tests: run a workload on the HIP path and on the
oracle from the same seeded inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_force(wl):
    return oracle.force_field(wl.force_kind, wl.force_params, wl.nx, wl.ny)


def oracle_run(wl, steps, scheme=oracle.SCHEME_CONSISTENT, nthreads=0):
    if wl.force_kind == "shan_chen":
        from oracle import shan_chen
        G, psi0, rho_ref = wl.force_params
        f = shan_chen.start(wl.rho, wl.ux, wl.uy, G, psi0, rho_ref)
        f = shan_chen.run(f, wl.s, steps, G, psi0, rho_ref, scheme=scheme, nthreads=nthreads)
        rho, ux, uy = shan_chen.state(f, G, psi0, rho_ref)
        return f, rho, ux, uy
    fx, fy = oracle_force(wl)
    f = oracle.init(wl.rho, wl.ux, wl.uy, fx, fy)
    if steps:
        f = oracle.run(f, fx, fy, wl.s, steps, bc_y=wl.bc_y, scheme=scheme, nthreads=nthreads)
    rho, ux, uy = oracle.moments(f, fx, fy)
    return f, rho, ux, uy


def gpu_lattice(wl, storage, scheme="consistent", inplace=False):
    from paper_1705_11092_amd import clbm
    lat = clbm.Lattice(wl.nx, wl.ny, wl.s, storage=storage,
                       bc_y="bounceback" if wl.bc_y == 1 else "periodic", rho0=wl.rho0,
                       scheme=scheme, inplace=inplace)
    if wl.force_kind == "field":
        lat.set_force("field", fx=wl.force_params[0], fy=wl.force_params[1])
    elif wl.force_kind == "none":
        lat.set_force("none")
    else:
        lat.set_force(wl.force_kind, params=wl.force_params)
    lat.init(wl.rho, wl.ux, wl.uy)
    return lat


def gpu_run(wl, storage, steps, scheme="consistent", graph_steps=None, inplace=False):
    lat = gpu_lattice(wl, storage, scheme, inplace=inplace)
    if graph_steps is not None:
        lat.set_graph_steps(graph_steps)
    lat.step(steps)
    rho, ux, uy, tot = lat.moments()
    f = lat.get_populations().cpu().numpy()
    out = (f, rho.cpu().numpy(), ux.cpu().numpy(), uy.cpu().numpy(), tot)
    lat.close()
    return out


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b**2)))


def e2_u(ux, uy, uxr, uyr):
    num = np.sum((ux - uxr) ** 2) + np.sum((uy - uyr) ** 2)
    den = np.sum(uxr**2) + np.sum(uyr**2)
    return float(np.sqrt(num / den))
