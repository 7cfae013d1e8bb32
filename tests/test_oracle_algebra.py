"""Pins of the oracle's algebra against the paper's definitions.

Each test ties a piece of the oracle to something other than itself: the
moment definitions of Eqs. (2)-(3), linear solves on those definitions,
the textbook product-form equilibrium, Guo's and He's force terms, and the
invariants the paper states (conservation, Remarks 2, 3 and 5).
"""
import numpy as np
import pytest

import oracle
from tests import defs

RNG = np.random.default_rng(20170531)


def _random_node(rng, amp_u=0.08, amp_ne=0.01):
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    ux, uy = amp_u * rng.uniform(-1, 1, 2)
    f = defs.product_equilibrium(rho, ux, uy) * (1.0 + amp_ne * rng.uniform(-1, 1, 9))
    return f


def test_M_is_the_raw_moment_definition():
    # Eq. (5) against Eqs. (2)-(3) evaluated on the velocities of Eq. (1).
    np.testing.assert_array_equal(oracle.matrix_M(), defs.moment_matrix(0.0, 0.0))


def test_printed_Minv_inverts_M_exactly():
    # The Appendix inverse against the definition of M; dyadic entries, so exact.
    A = defs.moment_matrix(0.0, 0.0)
    np.testing.assert_array_equal(oracle.matrix_Minv() @ A, np.eye(9))
    np.testing.assert_array_equal(A @ oracle.matrix_Minv(), np.eye(9))


@pytest.mark.parametrize("seed", range(5))
def test_N_maps_raw_to_central_moments(seed):
    # Eq. (6): N(u) M f must be the central moments of Eq. (2) about u.
    rng = np.random.default_rng(seed)
    ux, uy = rng.uniform(-0.3, 0.3, 2)
    lhs = oracle.matrix_N(ux, uy) @ oracle.matrix_M()
    np.testing.assert_allclose(lhs, defs.moment_matrix(ux, uy), atol=1e-15)
    f = rng.uniform(0, 1, 9)
    np.testing.assert_allclose(oracle.matrix_N(ux, uy) @ oracle.matrix_M() @ f,
                               defs.central_moments(f, ux, uy), atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_printed_Ninv_inverts_N(seed):
    rng = np.random.default_rng(100 + seed)
    ux, uy = rng.uniform(-0.3, 0.3, 2)
    N, NI = oracle.matrix_N(ux, uy), oracle.matrix_Ninv(ux, uy)
    np.testing.assert_allclose(NI @ N, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(N @ NI, np.eye(9), atol=1e-15)
    # Shifting back by u is shifting by -u.
    np.testing.assert_allclose(NI, oracle.matrix_N(-ux, -uy), atol=0)
    # And against the definitions: N(u) = A(u) A(0)^-1, so N^-1 = A(0) A(u)^-1.
    np.testing.assert_allclose(NI, defs.moment_matrix(0, 0) @ np.linalg.inv(defs.moment_matrix(ux, uy)),
                               atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_is_the_generalized_local_equilibrium(seed):
    # Init with F = 0 gives M^-1 N^-1 T~eq (Eq. 8).  Its central moments must
    # be T~eq by direct summation, it must equal the textbook product form,
    # and at u = 0 it must give the rest weights.
    rng = np.random.default_rng(200 + seed)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1)
    ux, uy = rng.uniform(-0.2, 0.2, 2)
    one = np.ones((1, 1))
    f = oracle.init(rho * one, ux * one, uy * one, 0 * one, 0 * one)[:, 0, 0]
    teq = np.array([rho, 0, 0, 2 * rho / 3, 0, 0, 0, 0, rho / 9])
    np.testing.assert_allclose(defs.central_moments(f, ux, uy), teq, atol=1e-15)
    np.testing.assert_allclose(f, defs.product_equilibrium(rho, ux, uy), atol=1e-15)
    f0 = oracle.init(one, 0 * one, 0 * one, 0 * one, 0 * one)[:, 0, 0]
    np.testing.assert_allclose(f0, defs.W, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_init_reproduces_requested_moments_under_force(seed):
    rng = np.random.default_rng(300 + seed)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1)
    ux, uy = rng.uniform(-0.2, 0.2, 2)
    Fx, Fy = rng.uniform(-1e-2, 1e-2, 2)
    one = np.ones((1, 1))
    f = oracle.init(rho * one, ux * one, uy * one, Fx * one, Fy * one)
    r, u, v = oracle.moments(f, Fx * one, Fy * one)
    assert abs(r[0, 0] - rho) < 1e-15 and abs(u[0, 0] - ux) < 1e-16 and abs(v[0, 0] - uy) < 1e-16
    # Brute-force check on the same quantities, Eqs. (11) and (15).
    r2, u2, v2 = defs.velocity(f[:, 0, 0], Fx, Fy)
    assert abs(r2 - rho) < 1e-15 and abs(u2 - ux) < 1e-16 and abs(v2 - uy) < 1e-16


@pytest.mark.parametrize("seed", range(20))
def test_collision_conserves_mass_and_adds_F_to_momentum(seed):
    # Eq. (12): mass conserved, momentum sum_i f e_i grows by exactly F.
    rng = np.random.default_rng(400 + seed)
    f = _random_node(rng)
    Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
    s = rng.uniform(0.2, 1.95, 6)
    fs = oracle.collide(f, Fx, Fy, s)
    assert abs(fs.sum() - f.sum()) < 2e-15
    assert abs(np.dot(fs, defs.EX) - (np.dot(f, defs.EX) + Fx)) < 2e-15
    assert abs(np.dot(fs, defs.EY) - (np.dot(f, defs.EY) + Fy)) < 2e-15


@pytest.mark.parametrize("seed", range(10))
def test_collision_relaxes_each_central_moment_at_its_own_rate(seed):
    # Post-collision central moments (about the pre-collision Eq. 15 u, by
    # direct summation) against T~ relaxed slot by slot.  This checks the
    # use of the matrices (no transposed operand, no wrong slot) rather than
    # the formula of Eq. (12) itself, which the flow tests pin.
    rng = np.random.default_rng(500 + seed)
    f = _random_node(rng, amp_ne=0.05)
    Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
    s = rng.uniform(0.2, 1.95, 6)
    S = np.array([s[0], s[1], s[1], s[2], s[3], s[3], s[4], s[4], s[5]])
    rho, ux, uy = defs.velocity(f, Fx, Fy)
    Tt = defs.central_moments(f, ux, uy)
    Ts = defs.central_moments(oracle.collide(f, Fx, Fy, s), ux, uy)
    teq = np.array([rho, 0, 0, 2 * rho / 3, 0, 0, 0, 0, rho / 9])
    dev_before, dev_after = Tt - teq, Ts - teq
    # Second-order and fourth-order slots carry no force term.
    for k in (3, 4, 5, 8):
        assert abs(dev_after[k] - (1 - S[k]) * dev_before[k]) < 1e-15
    # First-order slots: -F/2 before, +F/2 after, whatever s1 is.
    np.testing.assert_allclose(Tt[1:3], [-Fx / 2, -Fy / 2], atol=1e-16)
    np.testing.assert_allclose(Ts[1:3], [Fx / 2, Fy / 2], atol=1e-16)
    assert abs(Ts[0] - rho) < 1e-15


@pytest.mark.parametrize("seed", range(10))
def test_force_moments_match_eq13_in_the_slots_it_fixes(seed):
    # The third-order force slots of Eq. (14) against the central moments of
    # He's term R_i (Eq. 13) with the generalized equilibrium: k~21 of R is
    # cs^2 Fy and k~12 is cs^2 Fx.  The printed order of Eq. (14) has them
    # exchanged; this test fails on it.
    rng = np.random.default_rng(600 + seed)
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    ux, uy = rng.uniform(-0.1, 0.1, 2)
    Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
    s = rng.uniform(0.2, 1.7, 6)
    S = np.array([s[0], s[1], s[1], s[2], s[3], s[3], s[4], s[4], s[5]])
    one = np.ones((1, 1))
    f = oracle.init(rho * one, ux * one, uy * one, Fx * one, Fy * one)[:, 0, 0]
    fs = oracle.collide(f, Fx, Fy, s)
    teq = np.array([rho, 0, 0, 2 * rho / 3, 0, 0, 0, 0, rho / 9])
    C = (defs.central_moments(fs, ux, uy) - teq) / (1 - S / 2)
    feq = defs.from_central_moments(teq, ux, uy)
    CR = defs.central_moments(defs.he_term(feq, rho, Fx, Fy, ux, uy), ux, uy)
    np.testing.assert_allclose(C[[3, 4, 5, 6, 7, 8]],
                               [0, 0, 0, Fy / 3, Fx / 3, 0], atol=1e-15)
    np.testing.assert_allclose(CR[[0, 1, 2, 5, 6, 7]], [0, Fx, Fy, 0, Fy / 3, Fx / 3], atol=1e-15)
    # The slots Eq. (14) sets to zero differ from Eq. (13) by O(F u^3).
    bound = 6 * max(abs(Fx), abs(Fy)) * max(abs(ux), abs(uy)) ** 3
    assert np.all(np.abs(CR[[3, 4, 8]]) <= bound + 1e-18)


@pytest.mark.parametrize("seed", range(10))
def test_s0_s1_do_not_matter(seed):
    # Remark 5.
    rng = np.random.default_rng(700 + seed)
    f = _random_node(rng, amp_ne=0.05)
    Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
    s = rng.uniform(0.2, 1.95, 6)
    a = oracle.collide(f, Fx, Fy, s)
    s2 = s.copy()
    s2[0], s2[1] = rng.uniform(0.1, 1.99, 2)
    np.testing.assert_allclose(oracle.collide(f, Fx, Fy, s2), a, atol=3e-16)


@pytest.mark.parametrize("seed", range(10))
def test_bgk_limit_with_guo_forcing(seed):
    # Remark 3: with every rate equal to s the scheme is BGK with a forcing
    # term whose central moments are C, relaxed at (1 - s/2).
    rng = np.random.default_rng(800 + seed)
    f = _random_node(rng, amp_ne=0.05)
    Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
    s = float(rng.uniform(0.3, 1.9))
    rho, ux, uy = defs.velocity(f, Fx, Fy)
    feq = defs.product_equilibrium(rho, ux, uy)
    Rc = defs.from_central_moments([0, Fx, Fy, 0, 0, 0, Fy / 3, Fx / 3, 0], ux, uy)
    bgk = f - s * (f - feq) + (1 - s / 2) * Rc
    np.testing.assert_allclose(oracle.collide(f, Fx, Fy, [s] * 6), bgk, atol=1e-16)


def test_bgk_limit_differs_from_guo_term_at_order_F_u2():
    # Remark 3: Eq. (13)'s term equals Guo's R_G plus higher-order terms.
    # With all rates s, the collision minus BGK with Guo's R_G is
    # (1 - s/2)(R_c - R_G) = O(F u^2): halving u quarters it.
    s = 1.3
    Fx, Fy = 1e-4, -7e-5
    diffs = []
    for scale in (1.0, 0.5, 0.25):
        ux, uy = 0.08 * scale, -0.05 * scale
        feq = defs.product_equilibrium(1.0, ux, uy)
        # Equilibrium apart from the first-order slots, which Eq. (15) fixes
        # at -F/2 so that the collision sees exactly this u.
        f = defs.from_central_moments([1.0, -Fx / 2, -Fy / 2, 2 / 3, 0, 0, 0, 0, 1 / 9], ux, uy)
        guo = f - s * (f - feq) + (1 - s / 2) * defs.guo_term(Fx, Fy, ux, uy)
        diffs.append(np.max(np.abs(oracle.collide(f, Fx, Fy, [s] * 6) - guo)))
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, diffs


@pytest.mark.parametrize("seed", range(10))
def test_mrt_limit_of_remark2(seed):
    # Remark 2: with N = I the collision is a raw-moment MRT whose
    # equilibrium and force vectors are the raw moments of the generalized
    # equilibrium and of the distribution with central moments C.  Built
    # here from the moment definitions alone.
    rng = np.random.default_rng(900 + seed)
    f = _random_node(rng, amp_ne=0.05)
    Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
    s = rng.uniform(0.3, 1.9, 6)
    S = np.diag([s[0], s[1], s[1], s[2], s[3], s[3], s[4], s[4], s[5]])
    rho, ux, uy = defs.velocity(f, Fx, Fy)
    A = defs.moment_matrix(0, 0)
    Teq = A @ defs.product_equilibrium(rho, ux, uy)
    Craw = A @ defs.from_central_moments([0, Fx, Fy, 0, 0, 0, Fy / 3, Fx / 3, 0], ux, uy)
    T = A @ f
    mrt = np.linalg.solve(A, T - S @ (T - Teq) + (np.eye(9) - S / 2) @ Craw)
    np.testing.assert_allclose(oracle.collide(f, Fx, Fy, s, shift=False), mrt, atol=2e-16)
    # With one rate for all moments the shift changes nothing.
    sb = [float(s[3])] * 6
    np.testing.assert_allclose(oracle.collide(f, Fx, Fy, sb, shift=False),
                               oracle.collide(f, Fx, Fy, sb, shift=True), atol=2e-16)


def test_mrt_limit_force_is_guo_up_to_order_F_u2():
    # Remark 2: the N = I force term (I - S/2) N^-1 C against the MRT with
    # Guo's forcing, (I - S/2) M R_G: they differ at O(F u^2).
    s = [1.0, 1.0, 1.2, 1.6, 0.9, 1.1]
    Fx, Fy = 2e-4, 1e-4
    diffs = []
    for scale in (1.0, 0.5, 0.25):
        ux, uy = 0.06 * scale, 0.04 * scale
        f = defs.from_central_moments([1.0, -Fx / 2, -Fy / 2, 2 / 3, 0, 0, 0, 0, 1 / 9], ux, uy)
        out = oracle.collide(f, Fx, Fy, s, shift=False)
        feq = defs.product_equilibrium(1.0, ux, uy)
        A = defs.moment_matrix(0, 0)
        S = np.diag([s[0], s[1], s[1], s[2], s[3], s[3], s[4], s[4], s[5]])
        T = A @ f
        mrt = np.linalg.solve(A, T - S @ (T - A @ feq) +
                              (np.eye(9) - S / 2) @ (A @ defs.guo_term(Fx, Fy, ux, uy)))
        diffs.append(np.max(np.abs(out - mrt)))
    assert 3.5 < diffs[0] / diffs[1] < 4.5 and 3.5 < diffs[1] / diffs[2] < 4.5, diffs


def test_guo_lbl_scheme_is_eq21():
    # Eq. (21): the Lycett-Brown & Luo scheme adds (1 - s2/2) N M R_G.
    rng = np.random.default_rng(1000)
    f = _random_node(rng, amp_ne=0.05)
    Fx, Fy = 3e-4, -2e-4
    s = rng.uniform(0.3, 1.9, 6)
    S = np.array([s[0], s[1], s[1], s[2], s[3], s[3], s[4], s[4], s[5]])
    rho, ux, uy = defs.velocity(f, Fx, Fy)
    Tt = defs.central_moments(f, ux, uy)
    teq = np.array([rho, 0, 0, 2 * rho / 3, 0, 0, 0, 0, rho / 9])
    CG = defs.central_moments(defs.guo_term(Fx, Fy, ux, uy), ux, uy)
    Ts = (1 - S) * Tt + S * teq + (1 - s[3] / 2) * CG
    expect = defs.from_central_moments(Ts, ux, uy)
    np.testing.assert_allclose(oracle.collide(f, Fx, Fy, s, scheme=oracle.SCHEME_GUO_LBL),
                               expect, atol=3e-16)
