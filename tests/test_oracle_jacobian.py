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
