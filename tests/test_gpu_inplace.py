"""In-place streaming (the AA pattern, one buffer) on the GPU.

The in-place step does each node's arithmetic exactly as the two-buffer
step and only stores it elsewhere, so every result must be bitwise equal to
the two-buffer result: after odd and even step counts (the two phases),
for every storage type, force mode, forcing scheme and y boundary, on
ragged and degenerate sizes, through graphs, batches mixing both forms,
every batch launch shape, the autotuner and the solve server.

Hazard test: in place, a step reads and writes the same buffer.  The
streaming maps give every location exactly one reader and one writer, the
same node, so no ordering between threads is needed.  A wrong map or a
location shared between two nodes shows up as a bitwise difference from the
two-buffer result that depends on the launch shape; the batch test runs
every variant (nodes per thread x blocks per CU) and the single-lattice
tests use 1 to 8 nodes per thread.
"""
import numpy as np
import pytest

import oracle
from paper_1705_11092_amd import inputs
from tests.gpu_util import e2_u, gpu_lattice, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

STORAGES = ["f64", "f32", "f16", "bf16", "f16sr", "bf16sr"]
CASES = [
    (37, 23, 0, "field"),
    (300, 70, 1, "field"),
    (1030, 9, 0, "kolmogorov"),
    (64, 32, 1, "const"),
    (1, 17, 1, "const"),
    (19, 1, 0, "field"),
    (2, 2, 0, "field"),
    (257, 130, 0, "none"),
    (520, 3, 1, "kolmogorov"),
    (256, 12, 1, "field"),  # rows of exactly one wave of groups at 4 nodes per thread
]


def _case(ci, seed):
    nx, ny, bc, force = CASES[ci]
    return inputs.random_state(nx, ny, seed=seed, bc_y=bc, force=force, amp_f=1e-3)


def _state(lat):
    rho, ux, uy, tot = lat.moments()
    return (lat.get_populations().cpu().numpy(), rho.cpu().numpy(), ux.cpu().numpy(),
            uy.cpu().numpy(), np.array(tot))


def _assert_same(a, b, what):
    for x, y, name in zip(a, b, ("f", "rho", "ux", "uy", "totals")):
        assert np.array_equal(x, y), f"{what}: {name} differs"


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_in_place_equals_two_buffers(storage, ci):
    wl = _case(ci, 400 + ci)
    log(f"in place vs two buffers: case {ci} {wl.nx}x{wl.ny} bc={wl.bc_y} {storage}")
    a = gpu_lattice(wl, storage)
    b = gpu_lattice(wl, storage, inplace=True)
    a.set_graph_steps(0)
    b.set_graph_steps(0)
    done = 0
    for n in (1, 1, 5, 2):  # phases 1, 0, 1, 0 after the calls
        a.step(n)
        b.step(n)
        done += n
        _assert_same(_state(a), _state(b), f"after {done} steps")
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16sr"])
@pytest.mark.parametrize("scheme", ["consistent", "guo_lbl"])
def test_in_place_through_graphs(storage, scheme):
    wl = _case(1, 501)
    a = gpu_lattice(wl, storage, scheme=scheme)
    b = gpu_lattice(wl, storage, scheme=scheme, inplace=True)
    for n in (64, 3, 128, 1):
        a.step(n)
        b.step(n)
    _assert_same(_state(a), _state(b), f"{storage} {scheme}")
    a.close()
    b.close()


@pytest.mark.parametrize("ci", [0, 1, 3, 5])
def test_in_place_matches_oracle(ci):
    wl = _case(ci, 600 + ci)
    fo, ro, uo, vo = oracle_run(wl, 13)
    fg, rg, ug, vg, _ = gpu_run(wl, "f64", 13, inplace=True)
    assert np.max(np.abs(fg - fo)) <= 1e-13
    _, _, ug32, vg32, _ = gpu_run(wl, "f32", 13, inplace=True)
    assert e2_u(ug32, vg32, uo, vo) <= 1e-5
    fo2, _, _, _ = oracle_run(wl, 10, scheme=oracle.SCHEME_GUO_LBL)
    fg2, _, _, _, _ = gpu_run(wl, "f64", 10, scheme="guo_lbl", inplace=True)
    assert np.max(np.abs(fg2 - fo2)) <= 1e-13


def test_in_place_reads_only_what_it_wrote():
    # The whole buffer is NaN before the start state is written; the state
    # must stay finite (no step reads a slot that no step or the start state
    # wrote, e.g. the row padding).
    import torch
    wl = _case(1, 701)
    lat = gpu_lattice(wl, "f32", inplace=True)
    lat.pop_a.fill_(0xFF)
    lat.init(wl.rho, wl.ux, wl.uy)
    for k in range(4):
        lat.step(1)
        assert torch.isfinite(lat.get_populations()).all().item(), f"step {k}"
    lat.close()


def test_batch_mixing_both_forms_every_variant():
    from paper_1705_11092_amd import clbm
    wls = [
        (_case(0, 801), "f32", True),
        (_case(1, 802), "f32", False),
        (_case(2, 803), "f16", True),
        (_case(3, 804), "bf16", True),
        (_case(7, 805), "f64", True),
        (inputs.kolmogorov(211, 5e-6, 2, 0.7), "f32", True),
        (_case(4, 806), "f16sr", True),
        (_case(8, 807), "bf16sr", False),
        (_case(6, 808), "bf16sr", True),
    ]
    steps = [40, 37, 41, 5, 0, 71, 44, 39, 3]
    ref = []
    for (wl, st, _), n in zip(wls, steps):
        lat = gpu_lattice(wl, st)
        lat.step(n)
        ref.append(_state(lat))
        lat.close()
    for variant in range(clbm.Batch.variant_count()):
        lats = [gpu_lattice(wl, st, inplace=ip) for wl, st, ip in wls]
        b = clbm.Batch(lats)
        b.variant = variant
        b.step_each(steps)
        for j, lat in enumerate(lats):
            _assert_same(_state(lat), ref[j], f"variant {variant} lattice {j}")
        b.close()
        for lat in lats:
            lat.close()


def test_autotune_leaves_in_place_lattices_untouched(tmp_path):
    from paper_1705_11092_amd import clbm
    wls = [inputs.kolmogorov(n, 3e-6, 1, 0.9) for n in (32, 45, 100, 180)]
    ref = []
    for wl in wls:
        lat = gpu_lattice(wl, "f32")
        lat.step(51)
        ref.append(_state(lat))
        lat.close()
    lats = [gpu_lattice(wl, "f32", inplace=True) for wl in wls]
    b = clbm.Batch(lats)
    b.step(1)  # phase 1: the tuner's launches must not disturb either phase
    v = b.autotune(str(tmp_path / "tune.txt"))
    assert 0 <= v < clbm.Batch.variant_count()
    b.step(20)
    b.autotune(None)
    b.step(30)
    for lat, r in zip(lats, ref):
        _assert_same(_state(lat), r, "after autotune")
    b.close()


def test_in_place_shan_chen():
    wl = inputs.droplet(n=48, R=12.0, s3=1.4)
    a = gpu_lattice(wl, "f64")
    b = gpu_lattice(wl, "f64", inplace=True)
    for n in (1, 64, 7):
        a.step(n)
        b.step(n)
    _assert_same(_state(a), _state(b), "shan-chen")
    a.close()
    b.close()


def test_served_in_place_equals_two_buffers_and_halves_the_footprint():
    from paper_1705_11092_amd import clbm
    from paper_1705_11092_amd.serve import GpuBackend, Server
    reqs = inputs.served_stream(count=10, seed=7, rate=80.0, n_lo=24, n_hi=160, steps_lo=40,
                                steps_hi=700, storage_16="f16sr")
    one = max(2 * clbm.buffer_bytes(r.workload.nx, r.workload.ny, r.storage) for r in reqs)
    two = Server(GpuBackend(budget_bytes=2 * one), min_tick=32, max_tick=256,
                 tick_s=0.002).run(reqs)
    reqs = inputs.served_stream(count=10, seed=7, rate=80.0, n_lo=24, n_hi=160, steps_lo=40,
                                steps_hi=700, storage_16="f16sr")
    be = GpuBackend(budget_bytes=2 * one, inplace=True)
    assert all(be.footprint(r) == clbm.buffer_bytes(r.workload.nx, r.workload.ny, r.storage)
               for r in reqs)
    one_buf = Server(be, min_tick=32, max_tick=256, tick_s=0.002).run(reqs)
    log(f"two buffers: max active {two.max_active}; in place: {one_buf.max_active}")
    assert one_buf.max_active >= two.max_active
    for r in reqs:
        x, y = two.results[r.rid], one_buf.results[r.rid]
        assert x.status == y.status == "done"
        assert np.array_equal(x.ux, y.ux) and np.array_equal(x.rho, y.rho)
