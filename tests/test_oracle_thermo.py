"""Pins of the oracle's mixture state and NASA-7 thermodynamics (CPU only).

Every expected number below is worked out by hand from the definitions for a
special case (single-coefficient polynomials, isomers, pure species) or is an
exact identity of the polynomials checked by complex-step differentiation.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import nasa_const, tiny_mechanism

R = 8314.46261815324


def _one_species(tmp_path, a_lo, a_hi=None):
    path = tiny_mechanism(tmp_path / "one.mech", [("X", (2, 0), a_lo, a_hi)], [])
    return oracle.read_mechanism(path)


@pytest.mark.parametrize("coef,T,cp,hrt,sr", [
    # a1 = 3.5, a6 = -1000, a7 = 5 at T = 500: cp/R = 3.5, h/RT = 3.5 - 2, s/R = 3.5 ln 500 + 5
    ([3.5, 0, 0, 0, 0, -1000.0, 5.0], 500.0, 3.5, 1.5, 3.5 * math.log(500.0) + 5.0),
    # a2 only: cp/R = a2 T, h/RT = a2 T / 2, s/R = a2 T
    ([0, 0.002, 0, 0, 0, 0, 0], 500.0, 1.0, 0.5, 1.0),
    # a3 only at T = 1000 (still the low range): cp/R = 1, h/RT = 1/3, s/R = 1/2
    ([0, 0, 1e-6, 0, 0, 0, 0], 1000.0, 1.0, 1.0 / 3.0, 0.5),
    ([0, 0, 0, 1e-9, 0, 0, 0], 1000.0, 1.0, 0.25, 1.0 / 3.0),
    ([0, 0, 0, 0, 1e-12, 0, 0], 1000.0, 1.0, 0.2, 0.25),
])
def test_nasa_single_coefficient_closed_forms(tmp_path, coef, T, cp, hrt, sr):
    m = _one_species(tmp_path, coef)
    cpR, hRT, sR, gRT = oracle.nasa7(m, np.array([T]))
    assert cpR[0, 0] == pytest.approx(cp, rel=1e-14)
    assert hRT[0, 0] == pytest.approx(hrt, rel=1e-14)
    assert sR[0, 0] == pytest.approx(sr, rel=1e-14)
    assert gRT[0, 0] == pytest.approx(hrt - sr, rel=1e-13, abs=1e-14)


def test_nasa_range_selection(tmp_path):
    # low range used at T <= T_mid, high range above
    m = _one_species(tmp_path, nasa_const(a1=2.0), nasa_const(a1=7.0))
    cpR, _, _, _ = oracle.nasa7(m, np.array([999.0, 1000.0, 1000.5, 2500.0]))
    assert list(cpR[:, 0]) == [2.0, 2.0, 7.0, 7.0]


def test_thermo_dimensional_units(tmp_path):
    m = _one_species(tmp_path, nasa_const(a1=3.5, a6=-1000.0, a7=5.0))
    T = np.array([500.0])
    props = oracle.thermo_properties(m, T, np.array([101325.0]), np.array([[1.0]]))
    W = 2 * 1.008
    assert props["cp_k"][0, 0] == pytest.approx(3.5 * R, rel=1e-14)
    assert props["h_k"][0, 0] == pytest.approx(R * (3.5 * 500 - 1000), rel=1e-14)
    assert props["s_k"][0, 0] == pytest.approx(R * (3.5 * math.log(500) + 5), rel=1e-14)
    assert props["g_k"][0, 0] == pytest.approx(props["h_k"][0, 0] - 500 * props["s_k"][0, 0], rel=1e-13)
    assert props["cp_mass"][0] == pytest.approx(3.5 * R / W, rel=1e-14)
    assert props["rho"][0] == pytest.approx(101325.0 * W / (R * 500.0), rel=1e-14)
    assert props["Wbar"][0] == pytest.approx(W, rel=1e-15)


def test_nasa_derivative_identities_by_complex_step(c1_path):
    """d(h/R)/dT = cp/R and d(s/R)/dT = cp/(R T): exact polynomial identities."""
    m = oracle.read_mechanism(c1_path)
    T = np.array([350.0, 800.0, 999.0, 1400.0, 2450.0])
    h = 1e-30
    cpR, _, _, _ = oracle.nasa7(m, T)
    _, hRTc, sRc, _ = oracle.nasa7(m, T.astype(complex) + 1j * h)
    dh = ((T + 1j * h)[:, None] * hRTc).imag / h
    ds = sRc.imag / h
    np.testing.assert_allclose(dh, cpR, rtol=1e-13)
    np.testing.assert_allclose(ds, cpR / T[:, None], rtol=1e-13)


def test_generated_nasa_continuity_at_tmid(c1_path):
    """The generator chooses the upper-range a6, a7 so that h and s are continuous."""
    m = oracle.read_mechanism(c1_path)
    t = m.t_mid

    def evaluate(a, T):
        cp = sum(a[:, j] * T ** j for j in range(5))
        h = a[:, 0] + sum(a[:, j] * T ** j / (j + 1) for j in range(1, 5)) + a[:, 5] / T
        s = a[:, 0] * np.log(T) + sum(a[:, j] * T ** j / j for j in range(1, 5)) + a[:, 6]
        return cp, h, s
    cl, hl, sl = evaluate(m.a_lo, t)
    ch, hh, sh = evaluate(m.a_hi, t)
    np.testing.assert_allclose(hh, hl, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sh, sl, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ch, cl, rtol=0.05)        # cp: continuous to fit accuracy only


def test_mixture_state_closed_forms(tmp_path):
    # isomers (same composition => same molar mass): X = Y; sum C = p/(RT)
    species = [("A", (1, 1), nasa_const(), None), ("B", (1, 1), nasa_const(), None),
               ("C", (1, 1), nasa_const(), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "iso.mech", species, []))
    Y = np.array([[0.2, 0.3, 0.5], [0.6, 0.1, 0.3]])
    T = np.array([700.0, 1900.0])
    p = np.array([101325.0, 1013250.0])
    Wbar, rho, X, C = oracle.mixture_state(m, T, p, Y)
    W = 1.008 + 15.999
    np.testing.assert_allclose(X, Y, rtol=1e-15)
    np.testing.assert_allclose(Wbar, W, rtol=1e-15)
    np.testing.assert_allclose(rho, p * W / (R * T), rtol=1e-15)
    np.testing.assert_allclose(C.sum(axis=1), p / (R * T), rtol=1e-15)


def test_mixture_state_unequal_weights(tmp_path):
    # H (1.008) and O (15.999): Wbar = 1/(Y_H/W_H + Y_O/W_O); X_H = Wbar Y_H / W_H
    species = [("H", (1, 0), nasa_const(), None), ("O", (0, 1), nasa_const(), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "ho.mech", species, []))
    Y = np.array([[0.5, 0.5]])
    Wbar, rho, X, C = oracle.mixture_state(m, np.array([1000.0]), np.array([101325.0]), Y)
    wbar = 1.0 / (0.5 / 1.008 + 0.5 / 15.999)
    assert Wbar[0] == pytest.approx(wbar, rel=1e-15)
    assert X[0, 0] == pytest.approx(15.999 / (1.008 + 15.999), rel=1e-15)
    assert C[0].sum() == pytest.approx(101325.0 / (R * 1000.0), rel=1e-15)
