"""Pins of the oracle's analytic Jacobian and VJP (CPU only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import Reaction, nasa_const, tiny_mechanism
from metrics import jac_scaled_error

R = 8314.46261815324
P0 = 101325.0


def _states(m, n, seed, with_anchors=False):
    st = synth.state_c0(m.n_species, n=n, seed=seed)
    T, p, Y = st["T"], st["p"] * np.where(np.arange(n) % 2, 10.0, 1.0), np.ascontiguousarray(st["Y"].T)
    if with_anchors:
        a = synth.load_anchors()
        T = np.concatenate([T, a["T"][:4]])
        p = np.concatenate([p, a["p"][:4]])
        Y = np.concatenate([Y, a["Y"][:4]])
    return T, p, Y


def _scaled(J1, J2, m, T, p, Y):
    _, G = oracle.jacobian(m, T, p, Y, return_gross=True)
    return jac_scaled_error(J1, J2, G, T, Y)


@pytest.mark.parametrize("which", ["c0", "c1"])
def test_analytic_jacobian_matches_complex_step(which, c0_path, c1_path):
    m = oracle.read_mechanism(c0_path if which == "c0" else c1_path)
    T, p, Y = _states(m, 8, 11, with_anchors=(which == "c1"))
    J = oracle.jacobian(m, T, p, Y)
    Jc = oracle.complex_step_jacobian(m, T, p, Y)
    assert _scaled(J, Jc, m, T, p, Y).max() <= 1e-12


def test_central_differences_agree(c0_path):
    m = oracle.read_mechanism(c0_path)
    T, p, Y = _states(m, 16, 12)
    J = oracle.jacobian(m, T, p, Y)
    Jf = oracle.central_fd_jacobian(m, T, p, Y)
    assert _scaled(Jf, J, m, T, p, Y).max() <= 1e-6


def test_gross_jacobian_bounds_the_jacobian(c1_path):
    m = oracle.read_mechanism(c1_path)
    T, p, Y = _states(m, 6, 14, with_anchors=True)
    J, G = oracle.jacobian(m, T, p, Y, return_gross=True)
    assert np.all(np.abs(J) <= G * (1 + 1e-12) + 1e-300)


def test_vjp_dot_product_identity(c1_path):
    m = oracle.read_mechanism(c1_path)
    T, p, Y = _states(m, 6, 13)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((6, m.n_species))
    uh = rng.standard_normal(6)
    v = rng.standard_normal((6, m.n_species + 1))
    J = oracle.jacobian(m, T, p, Y)
    gT, gY = oracle.vjp(m, T, p, Y, u, uh)
    lhs = (np.concatenate([uh[:, None], u], axis=1) * np.einsum("nrc,nc->nr", J, v)).sum(axis=1)
    rhs = gT * v[:, 0] + (gY * v[:, 1:]).sum(axis=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11)


def test_isomer_jacobian_by_hand(tmp_path):
    # A <=> B, k_f = 1, K_c = 2 at 1000 K, equal molar masses W:
    # q = C_A - C_B/2; dC_A/dY_A = rho/W (1 - Y_A), dC_B/dY_A = -rho Y_B / W
    # => d w_A / d Y_A = -(rho/W) (1 - Y_A + Y_B/2) = -0.75 rho/W at Y = (1/2, 1/2)
    sp = [("A", (1, 1), nasa_const(), None), ("B", (1, 1), nasa_const(a6=-1000.0 * math.log(2.0)), None)]
    rx = [Reaction("elementary", {0: 1}, {1: 1}, 0.0, 0.0, 0.0)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "iso.mech", sp, rx))
    W = 1.008 + 15.999
    rho = P0 * W / (R * 1000.0)
    J = oracle.jacobian(m, np.array([1000.0]), np.array([P0]), np.array([[0.5, 0.5]]))
    assert J[0, 1, 1] == pytest.approx(-0.75 * rho / W, rel=1e-14)
    assert J[0, 2, 1] == pytest.approx(0.75 * rho / W, rel=1e-14)
    # d w_A / d Y_B = -(dC_A/dY_B - dC_B/dY_B / 2) = -(-rho Y_A/W - rho (1 - Y_B)/(2W)) = 0.75 rho/W
    # (C is homogeneous of degree 0 in Y, so the Y columns dotted with Y vanish)
    assert J[0, 1, 2] == pytest.approx(0.75 * rho / W, rel=1e-14)
    assert abs(J[0, 1, 1:] @ np.array([0.5, 0.5])) <= 1e-15 * rho / W


@pytest.mark.parametrize("which", ["c0", "c1"])
def test_jvp_matches_complex_step_along_v(which, c0_path, c1_path):
    """J v of the oracle against one complex step of the forward oracle along v (exact
    to rounding, independent of the analytic chain rule); scale of row k:
    sum_c G_kc |v_c| with G the gross Jacobian."""
    m = oracle.read_mechanism(c0_path if which == "c0" else c1_path)
    T, p, Y = _states(m, 8, 21, with_anchors=(which == "c1"))
    rng = np.random.default_rng(5)
    n = T.shape[0]
    vT = rng.standard_normal(n) * T * 1e-2
    vY = rng.standard_normal((n, m.n_species)) * Y
    jh, jw = oracle.jvp(m, T, p, Y, vT, vY)
    ch, cw = oracle.complex_step_jvp(m, T, p, Y, vT, vY)
    _, G = oracle.jacobian(m, T, p, Y, return_gross=True)
    scale = np.einsum("nrc,nc->nr", G, np.abs(np.concatenate([vT[:, None], vY], axis=1)))
    err = np.abs(np.concatenate([(jh - ch)[:, None], jw - cw], axis=1)) / scale
    assert err.max() <= 1e-12


def test_jvp_of_a_single_column_is_that_column(c0_path):
    """v = e_c gives column c of the Jacobian (and the T column for v = e_T)."""
    m = oracle.read_mechanism(c0_path)
    T, p, Y = _states(m, 3, 22)
    J = oracle.jacobian(m, T, p, Y)
    for c in (0, 1, m.n_species):
        vT = np.full(3, 1.0 if c == 0 else 0.0)
        vY = np.zeros((3, m.n_species))
        if c > 0:
            vY[:, c - 1] = 1.0
        jh, jw = oracle.jvp(m, T, p, Y, vT, vY)
        np.testing.assert_array_equal(jh, J[:, 0, c])
        np.testing.assert_array_equal(jw, J[:, 1:, c])
