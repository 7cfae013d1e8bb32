"""clbm_moments_noalloc (the entry point for callers that cannot allocate)
against clbm_moments, through the C-ABI: the same fields and totals, bit for
bit, on two calls in a row, the second on a smaller lattice, in several
storage types and force modes (the Shan-Chen psi pass included)."""
import numpy as np
import pytest
import torch

from paper_1705_11092_amd import inputs
from tests.gpu_util import gpu_lattice, log

pytestmark = pytest.mark.gpu

# (nx, ny, bc_y, force, storage): the first of each pair is the larger.
CALLS = [
    [(300, 70, 1, "field", "f32"), (37, 23, 0, "field", "f32")],
    [(1030, 9, 0, "kolmogorov", "f64"), (19, 1, 0, "const", "f64")],
    [(2048, 600, 0, "const", "f16sr"), (64, 32, 1, "const", "f16sr")],
]


def _compare(lat):
    rho, ux, uy, tot = lat.moments()
    shape = (lat.ny, lat.nx)
    # Outputs poisoned with NaN: everything the call owes must be written.
    outs = [torch.full(shape, float("nan"), dtype=torch.float64, device=lat.device) for _ in range(3)]
    tdev = torch.full((3,), float("nan"), dtype=torch.float64, device=lat.device)
    with torch.cuda.stream(lat.stream):
        lat.moments_noalloc(*outs, totals=tdev)
    lat.stream.synchronize()
    for a, b in zip((rho, ux, uy), outs):
        assert torch.equal(a, b)
    got = tdev.cpu().numpy()
    log(f"  totals {tot} vs noalloc {got.tolist()}")
    assert np.array_equal(np.array(tot), got)
    # Fields only, and totals only.
    t2 = torch.full((3,), float("nan"), dtype=torch.float64, device=lat.device)
    with torch.cuda.stream(lat.stream):
        lat.moments_noalloc(totals=t2)
        lat.moments_noalloc(outs[0], None, None, None)
    lat.stream.synchronize()
    assert np.array_equal(t2.cpu().numpy(), got)


@pytest.mark.parametrize("pair", range(len(CALLS)))
def test_noalloc_moments_equal_clbm_moments(pair):
    for nx, ny, bc, force, storage in CALLS[pair]:
        log(f"noalloc moments {nx}x{ny} bc={bc} force={force} storage={storage}")
        wl = inputs.random_state(nx, ny, seed=700 + nx, bc_y=bc, force=force, amp_f=1e-3)
        lat = gpu_lattice(wl, storage)
        lat.step(7)
        _compare(lat)
        lat.close()


def test_noalloc_moments_shan_chen():
    for n, R in ((96, 20.0), (48, 12.0)):
        log(f"noalloc moments Shan-Chen droplet {n}^2")
        wl = inputs.droplet(n, R)
        lat = gpu_lattice(wl, "f64")
        lat.step(5)
        _compare(lat)
        lat.close()


def test_noalloc_moments_errors():
    from paper_1705_11092_amd import clbm
    wl = inputs.random_state(16, 8, seed=3)
    lat = clbm.Lattice(16, 8, wl.s, storage="f32")
    with pytest.raises(clbm.ClbmError) as e:
        lat.moments_noalloc(totals=torch.empty(3, dtype=torch.float64, device="cuda"))
    assert e.value.code == clbm.CLBM_ESTATE
    lat.init(wl.rho, wl.ux, wl.uy)
    host = torch.empty(3, dtype=torch.float64)
    with pytest.raises(clbm.ClbmError) as e:
        lat.moments_noalloc(totals=host)  # host memory where device memory is due
    assert e.value.code == clbm.CLBM_EINVAL
    lat.close()
