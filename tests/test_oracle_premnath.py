"""Pins of the oracle's scheme of Premnath et al. (M1, Sec. III A).

The paper writes M1 as relaxation toward T~eq - C_P/2 (Eq. 17) with the
force moments cut at first order, C_P = [0, Fx, Fy, 0, ..., 0] (Eq. 19),
followed by the addition of the discrete change Delta f (Eq. 18), which it
cites without printing.  The oracle reads Delta f as the distribution whose
central moments are C_P, Delta f = M^-1 N^-1(u) C_P.  What pins that
reading and the code:

- Table I (Sec. IV A): M1's E2 of the channel, 2.739e-4, for every force;
- Table II (Sec. IV B): M1's column of the steady forced Taylor-Green flow
  at N = 10 and 20 for Re = 50, 100, 150, to the printed digits;
- Remark 6: at s3 = 2 the paper's scheme and M1 coincide;
- Eq. (20): Delta f_0 = -2 F.u + O(u^3);
- Remark 5: M1 leaves s0 and s1 free (mass and momentum are conserved
  and the force adds exactly F to the momentum);
- a planted sign error in Eq. (17) fails the momentum pin.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1705_11092_amd import inputs
from tests import defs
from tests.test_oracle_flows import _steady_channel, _steady_tg, _table

M1 = oracle.SCHEME_PREMNATH


def _random_node(rng, u=0.05, F=2e-3):
    rho = 1.0 + rng.uniform(-0.02, 0.02)
    ux, uy = rng.uniform(-u, u, 2)
    Fx, Fy = rng.uniform(-F, F, 2)
    one = np.ones((1, 1))
    f = oracle.init(rho * one, ux * one, uy * one, Fx * one, Fy * one)[:, 0, 0]
    return f + rng.normal(0.0, 1e-3, 9), Fx, Fy


@pytest.mark.parametrize("Fx", [1e-6, 7e-6])
def test_table1_M1_column(Fx):
    # Channel 50 nodes wide, every rate 1.754 except s3 from Remark 4 and
    # s1 = 1: the printed 2.739e-4 for every force.
    tab = _table("paper_table1.txt")
    row = tab[np.argmin(np.abs(tab[:, 0] - Fx))]
    s3 = inputs.nonslip_s3(1.754)
    e = _steady_channel(50, oracle.s6(1.754, 1.0, 1.754, 1.754, s3, 1.754), Fx, scheme=M1)
    assert e * 1e4 == pytest.approx(row[1], abs=6e-4)


@pytest.mark.parametrize("Re,N", [(50, 10), (50, 20), (100, 10), (100, 20), (150, 10), (150, 20)])
def test_table2_M1_column(Re, N):
    tab = _table("paper_table2.txt")
    row = tab[(tab[:, 0] == Re) & (tab[:, 1] == N)][0]
    e = _steady_tg(N, Re, scheme=M1)
    assert e * 1e2 == pytest.approx(row[3], abs=1.0e-4)


def test_remark6_m1_is_the_present_scheme_at_s3_2():
    rng = np.random.default_rng(61)
    for _ in range(20):
        f, Fx, Fy = _random_node(rng)
        s = oracle.s6(*rng.uniform(0.6, 1.9, 6))
        s_two = s.copy()
        s_two[4] = 2.0
        a = oracle.collide(f, Fx, Fy, s_two, oracle.SCHEME_CONSISTENT)
        b = oracle.collide(f, Fx, Fy, s_two, M1)
        assert np.max(np.abs(a - b)) < 1e-15
        # Elsewhere they differ by the third-order force moments,
        # (1 - s3/2) F/3 in k~21 and k~12.
        c = oracle.collide(f, Fx, Fy, s, oracle.SCHEME_CONSISTENT)
        d = oracle.collide(f, Fx, Fy, s, M1)
        assert np.max(np.abs(c - d)) > 1e-2 * abs(1 - s[4] / 2) * max(abs(Fx), abs(Fy))


def test_remark6_on_a_lattice():
    wl = inputs.random_state(14, 11, seed=62, bc_y=1, force="field", amp_f=1e-3)
    fx, fy = wl.force_params
    s = np.array(wl.s, dtype=np.float64)
    s[4] = 2.0
    f = oracle.init(wl.rho, wl.ux, wl.uy, fx, fy)
    a = oracle.run(f, fx, fy, s, 30, bc_y=1)
    b = oracle.run(f, fx, fy, s, 30, bc_y=1, scheme=M1)
    assert np.max(np.abs(a - b)) < 1e-14


def test_eq20_delta_f0():
    # Delta f_0 + 2 F.u is O(u^3): halving u divides it by 8.
    F = np.array([1e-3, 2e-3])
    d = np.array([0.8, 0.6])
    rem = []
    for u in (0.04, 0.02, 0.01):
        ux, uy = u * d
        df = oracle.premnath_delta_f(F[0], F[1], ux, uy)
        lead = -2.0 * (F[0] * ux + F[1] * uy)
        assert df[0] == pytest.approx(lead, rel=0.05)
        rem.append(df[0] - lead)
    assert rem[0] / rem[1] == pytest.approx(8.0, rel=1e-9)
    assert rem[1] / rem[2] == pytest.approx(8.0, rel=1e-9)
    # Guo's R_G0 of Eq. (20) is -3 F.u: the two differ at first order in u.
    assert abs(df[0] - (-3.0 * (F[0] * ux + F[1] * uy))) > 0.3 * abs(lead)


def test_delta_f_carries_no_mass_and_momentum_F():
    rng = np.random.default_rng(63)
    for _ in range(10):
        Fx, Fy = rng.uniform(-1e-2, 1e-2, 2)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        df = oracle.premnath_delta_f(Fx, Fy, ux, uy)
        assert abs(df.sum()) < 1e-17
        assert abs(defs.EX @ df - Fx) < 1e-17
        assert abs(defs.EY @ df - Fy) < 1e-17


def test_m1_conserves_and_frees_s0_s1():
    # Remark 5: mass conserved, momentum + F, and the post-collision state
    # does not depend on s0 and s1.
    rng = np.random.default_rng(64)
    for _ in range(10):
        f, Fx, Fy = _random_node(rng)
        r = rng.uniform(0.6, 1.9, 6)
        a = oracle.collide(f, Fx, Fy, oracle.s6(*r), M1)
        assert abs(a.sum() - f.sum()) < 1e-15
        assert abs(defs.EX @ a - (defs.EX @ f + Fx)) < 1e-15
        assert abs(defs.EY @ a - (defs.EY @ f + Fy)) < 1e-15
        r2 = r.copy()
        r2[0], r2[1] = rng.uniform(0.3, 1.9, 2)
        b = oracle.collide(f, Fx, Fy, oracle.s6(*r2), M1)
        assert np.max(np.abs(a - b)) < 1e-15


def test_planted_sign_of_eq17_is_caught(tmp_path):
    # Plant T~eq + C_P/2 in place of T~eq - C_P/2: a uniform force from rest
    # no longer gives u(n) = n F.
    src = open(oracle._SRC).read()
    old = "S[k] * (Teq[k] - CP[k] / 2.0)"
    assert old in src
    path = tmp_path / "planted.c"
    path.write_text(src.replace(old, "S[k] * (Teq[k] + CP[k] / 2.0)"))
    so = tmp_path / "libplanted.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                           str(path), "-lm"])
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_run.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_int, dp, dp, dp, dp,
                                                   ctypes.c_int64, ctypes.c_int]
    n, F = 40, (1e-6, -4e-7)
    fx, fy = oracle.force_field("const", F, 4, 4)
    one = np.ones((4, 4))
    f0 = oracle.init(one, 0 * one, 0 * one, fx, fy)
    s = oracle.s6(1.0, 0.7, 1.2, 1.3, 1.1, 1.0)
    _, ux, uy = oracle.moments(oracle.run(f0, fx, fy, s, n, scheme=M1), fx, fy)
    np.testing.assert_allclose(ux, n * F[0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(uy, n * F[1], rtol=0, atol=1e-15)
    f, work = f0.copy(), np.empty_like(f0)
    p = lambda a: np.ascontiguousarray(a).ctypes.data_as(dp)  # noqa: E731
    assert lib.oracle_run(4, 4, 0, p(s), M1, p(fx), p(fy), p(f), p(work), n, 1) == 0
    _, ux_bad, _ = oracle.moments(f, fx, fy)
    assert not np.allclose(ux_bad, n * F[0], rtol=1e-3)
