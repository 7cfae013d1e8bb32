"""The largest lattice the library accepts: 46336 x 46336 nodes (2,147,024,896,
just below 2^31), FP16 storage, two buffers of 38.6 GB each.

Kolmogorov forcing from rest is independent of x, so at any size the
result is known from a one-column lattice of the same height: every column
of the GPU result must be bitwise the same (an index that overflowed 32 bits
would break that), and each column must match the FP64 oracle on the
1 x 46336 lattice within the FP16 storage tolerance of the parity tests.
Fields are read on the device and only a few columns come to the host.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import e2_u, log

pytestmark = pytest.mark.gpu

N = 46336
STEPS = 12
A, K, TAU = 1e-4, 3, 0.8


def test_largest_square_lattice_fp16():
    import torch
    from paper_1705_11092_amd import clbm
    s2 = 1.0 / TAU
    rates = (1.0, 1.0, s2, s2, 1.0, 1.0)
    assert N * N < 2**31 and clbm.buffer_bytes(N, N, "f16") == 9 * N * N * 2 + 64
    lat = clbm.Lattice(N, N, rates, storage="f16")
    lat.set_force("kolmogorov", params=(A, K))
    lat.init()  # rest state, rho0 everywhere
    lat.step(STEPS)
    rho, ux, uy, tot = lat.moments()
    xs = torch.tensor([0, 1, 7, 4095, N // 2, N - 2, N - 1], device=rho.device)
    cols_u = ux.index_select(1, xs).cpu().numpy()
    cols_v = uy.index_select(1, xs).cpu().numpy()
    cols_r = rho.index_select(1, xs).cpu().numpy()
    del rho, ux, uy
    lat.close()
    torch.cuda.empty_cache()
    log(f"{N}^2 f16 after {STEPS} steps: mass {tot[0]:.6e}, x-momentum {tot[1]:.6e}")
    for c in range(1, len(xs)):
        assert np.array_equal(cols_u[:, c], cols_u[:, 0]), f"column {int(xs[c])}"
        assert np.array_equal(cols_r[:, c], cols_r[:, 0]), f"column {int(xs[c])}"
    for c in range(1, len(xs)):
        assert np.array_equal(cols_v[:, c], cols_v[:, 0]), f"column {int(xs[c])}"

    fx, fy = oracle.force_field("kolmogorov", (A, K), 1, N)
    one, zero = np.ones((N, 1)), np.zeros((N, 1))
    f = oracle.run(oracle.init(one, zero, zero, fx, fy), fx, fy, np.array(rates), STEPS)
    ro, uo, vo = oracle.moments(f, fx, fy)
    e = e2_u(cols_u[:, :1], cols_v[:, :1], uo, vo)
    log(f"  E2(u) of a column against the oracle's 1 x {N} lattice: {e:.3e}")
    assert e <= 3e-3
    # Momentum grows by the summed force each step: zero for a whole number
    # of sine periods; mass stays.
    assert abs(tot[0] - float(N) * N) <= 1e-6 * N * N


@pytest.mark.parametrize("storage,n", [("f32", 11000), ("f64", 7800)])
def test_two_step_kernel_above_4gb(storage, n):
    # A lattice whose buffers exceed 4 GB (FP32 11000^2: 4.36 GB each, FP64
    # 7800^2: 4.38 GB) takes the two-step kernel's 64-bit addressing; its
    # result must equal single steps bitwise (fields compared on the device).
    import torch
    from paper_1705_11092_amd import clbm
    assert clbm.buffer_bytes(n, n, storage) > 2**32
    rates = (1.0, 1.0, 1.25, 1.25, 1.0, 1.0)
    out = []
    for pairs in (False, True):
        lat = clbm.Lattice(n, n, rates, storage=storage, bc_y="bounceback")
        lat.set_force("kolmogorov", params=(1e-4, 2))
        lat.init()
        lat.step_pairs = pairs
        assert lat.step_pairs == pairs
        lat.step(5)
        rho, ux, uy, tot = lat.moments()
        out.append((rho, ux, uy))
        lat.close()
        del lat
    log(f"{n}^2 {storage}, 5 steps: pairs vs single steps compared on the device")
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    del out
    torch.cuda.empty_cache()
