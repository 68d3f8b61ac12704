"""Pins of the oracle's optional rate forms (CPU only): PLOG, Chebyshev, SRI and Lindemann
falloff, explicit reverse rates, irreversible reactions and non-integer forward orders,
each against a closed form worked by hand, and their derivatives against complex steps."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import Reaction, nasa_const, tiny_mechanism
from metrics import jac_scaled_error

R = 8314.46261815324
P0 = 101325.0


def _iso(tmp_path, rx, name="v.mech", three=False):
    """Species A, B (isomers, H:1 O:1) and C = A+B dimer (H:2 O:2) with a1-only thermo."""
    sp = [("A", (1, 1), nasa_const(a1=3.5), None), ("B", (1, 1), nasa_const(a1=3.5, a7=math.log(3.0)), None),
          ("C", (2, 2), nasa_const(a1=4.5, a6=-5000.0), None)]
    return oracle.read_mechanism(tiny_mechanism(tmp_path / name, sp, rx))


def _state(T, p, Y):
    return np.array([T], float), np.array([p], float), np.array([Y], float)


def _conc(m, T, p, Y):
    _, _, _, C = oracle.mixture_state(m, T, p, Y)
    return C[0]


def test_plog_tabulated_interpolated_and_clamped(tmp_path):
    e1, e2 = (1e4, math.log(2e3), 0.5, 1000.0), (1e6, math.log(7e4), -0.2, 3000.0)
    rx = [Reaction("plog", {0: 1}, {1: 1}, e1[1], e1[2], e1[3], extra={"plog": [e1, e2]})]
    m = _iso(tmp_path, rx)
    T = 1300.0
    k1 = math.exp(e1[1]) * T ** e1[2] * math.exp(-e1[3] / T)
    k2 = math.exp(e2[1]) * T ** e2[2] * math.exp(-e2[3] / T)
    for p, want in ((1e4, k1), (1e6, k2), (1e5, math.sqrt(k1 * k2)), (3e3, k1), (5e7, k2)):
        kf = oracle.rates_of_progress(m, *_state(T, p, [0.5, 0.3, 0.2]))["kf"][0, 0]
        assert kf == pytest.approx(want, rel=1e-13), p
    # a quarter of the way in ln p: k1^(3/4) k2^(1/4)
    kf = oracle.rates_of_progress(m, *_state(T, 1e4 * 10 ** 0.5, [0.5, 0.3, 0.2]))["kf"][0, 0]
    assert kf == pytest.approx(k1 ** 0.75 * k2 ** 0.25, rel=1e-13)


def test_chebyshev_closed_forms(tmp_path):
    Tmin, Tmax, Pmin, Pmax = 300.0, 2500.0, 1e3, 1e7
    D = 1.0 / Tmax - 1.0 / Tmin
    a = np.zeros((3, 2))
    a[0, 0], a[1, 0], a[0, 1], a[2, 0] = 3.0, -1.2, 0.4, 0.25
    rx = [Reaction("chebyshev", {0: 1}, {1: 1}, 0.0, 0.0, 0.0, extra={"cheb": (Tmin, Tmax, Pmin, Pmax, a)})]
    m = _iso(tmp_path, rx)
    for T, p in ((700.0, 1e5), (1900.0, 3e3), (350.0, 8e6)):
        Tr = (2.0 / T - 1.0 / Tmin - 1.0 / Tmax) / D
        Pr = (2.0 * math.log10(p) - math.log10(Pmin) - math.log10(Pmax)) / (math.log10(Pmax) - math.log10(Pmin))
        # T_0 = 1, T_1(x) = x, T_2(x) = 2 x^2 - 1
        want = 10 ** (3.0 - 1.2 * Tr + 0.4 * Pr + 0.25 * (2 * Tr ** 2 - 1))
        kf = oracle.rates_of_progress(m, *_state(T, p, [0.5, 0.3, 0.2]))["kf"][0, 0]
        assert kf == pytest.approx(want, rel=1e-12)
    # first degree in Tr only: an Arrhenius law with b = 0 and theta = -2 ln(10) alpha_10 / D
    a1 = np.zeros((2, 1))
    a1[0, 0], a1[1, 0] = 2.0, -0.7
    m1 = _iso(tmp_path, [Reaction("chebyshev", {0: 1}, {1: 1}, 0.0, 0.0, 0.0,
                                  extra={"cheb": (Tmin, Tmax, Pmin, Pmax, a1)})], "v1.mech")
    theta = -2.0 * math.log(10.0) * (-0.7) / D
    lnA = math.log(10.0) * (2.0 + 0.7 * (1.0 / Tmin + 1.0 / Tmax) / D)
    for T in (400.0, 1000.0, 2400.0):
        kf = oracle.rates_of_progress(m1, *_state(T, 2e4, [0.5, 0.3, 0.2]))["kf"][0, 0]
        assert kf == pytest.approx(math.exp(lnA - theta / T), rel=1e-12)


def test_sri_at_unit_reduced_pressure_and_scaling(tmp_path):
    """At P_r = 1, X = 1 and F = d (a e^(-b/T) + e^(-T/c)) T^e, so k_f = kinf F / 2; at
    P_r = 100, X = 1/5; F (and k_f) scale with d everywhere."""
    lnA, b, th = math.log(1e10), 0.3, 2000.0
    k0 = (math.log(1e14), -0.8, 500.0)
    sri = (0.8, 300.0, 900.0, 1.2, 0.15)
    rx = [Reaction("sri", {0: 1, 1: 1}, {2: 1}, lnA, b, th, extra={"k0": k0, "sri": sri})]
    m = _iso(tmp_path, rx)
    T = 1100.0
    kinf = math.exp(lnA) * T ** b * math.exp(-th / T)
    k0v = math.exp(k0[0]) * T ** k0[1] * math.exp(-k0[2] / T)
    M = kinf / k0v                                        # [M] with P_r = 1
    rho = M * R * T / R / T                               # total concentration M: p = M R T
    p = M * R * T
    T_, p_, Y_ = _state(T, p, [0.4, 0.35, 0.25])
    r = oracle.rates_of_progress(m, T_, p_, Y_)
    assert r["M"][0, 0] == pytest.approx(M, rel=1e-12) and rho == pytest.approx(M)
    a_, b_, c_, d_, e_ = sri
    F = d_ * (a_ * math.exp(-b_ / T) + math.exp(-T / c_)) * T ** e_
    assert r["kf"][0, 0] == pytest.approx(kinf * 0.5 * F, rel=1e-12)
    # at P_r = 100, log10 P_r = 2 and X = 1/5: F = d S^(1/5) T^e, k_f = kinf (100/101) F
    T_, p_, Y_ = _state(T, 100.0 * p, [0.4, 0.35, 0.25])
    r = oracle.rates_of_progress(m, T_, p_, Y_)
    F100 = d_ * (a_ * math.exp(-b_ / T) + math.exp(-T / c_)) ** 0.2 * T ** e_
    assert r["kf"][0, 0] == pytest.approx(kinf * 100.0 / 101.0 * F100, rel=1e-12)
    m2 = _iso(tmp_path, [Reaction("sri", {0: 1, 1: 1}, {2: 1}, lnA, b, th,
                                  extra={"k0": k0, "sri": sri[:3] + (2 * d_, e_)})], "v2.mech")
    T2, p2, Y2 = _state(1700.0, 3 * P0, [0.2, 0.3, 0.5])
    np.testing.assert_allclose(oracle.rates_of_progress(m2, T2, p2, Y2)["kf"],
                               2 * oracle.rates_of_progress(_iso(tmp_path, rx, "v3.mech"), T2, p2, Y2)["kf"],
                               rtol=1e-13)


def test_lindemann_limits(tmp_path):
    """F = 1: k_f = kinf P_r/(1 + P_r) -> k0 [M] at low pressure, kinf at high pressure."""
    lnA, b, th = math.log(1e9), 0.0, 1000.0
    k0 = (math.log(1e13), 0.0, 0.0)
    m = _iso(tmp_path, [Reaction("lindemann", {0: 1, 1: 1}, {2: 1}, lnA, b, th, extra={"k0": k0})])
    T = 1000.0
    kinf = 1e9 * math.exp(-1.0)
    for p in (10.0, 1e5, 1e9):
        T_, p_, Y_ = _state(T, p, [0.4, 0.35, 0.25])
        r = oracle.rates_of_progress(m, T_, p_, Y_)
        M = r["M"][0, 0]
        Pr = 1e13 * M / kinf
        assert r["kf"][0, 0] == pytest.approx(kinf * Pr / (1 + Pr), rel=1e-13)
    assert r["kf"][0, 0] == pytest.approx(kinf, rel=1e-3)


def test_explicit_reverse_irreversible_and_orders_by_hand(tmp_path):
    rev = (math.log(5e3), 0.4, 7000.0)
    rx = [Reaction("elementary", {0: 1}, {1: 1}, math.log(2e6), 0.0, 4000.0, extra={"reverse": rev}),
          Reaction("elementary", {0: 1, 1: 1}, {2: 1}, math.log(3e8), 0.2, 1500.0,
                   extra={"irreversible": True, "orders": {0: 0.5, 1: 1.7}})]
    m = _iso(tmp_path, rx)
    T, p, Y = _state(1400.0, 2 * P0, [0.45, 0.35, 0.2])
    C = _conc(m, T, p, Y)
    r = oracle.rates_of_progress(m, T, p, Y)
    kf0 = 2e6 * math.exp(-4000.0 / 1400.0)
    kr0 = 5e3 * 1400.0 ** 0.4 * math.exp(-7000.0 / 1400.0)
    assert r["q"][0, 0] == pytest.approx(kf0 * C[0] - kr0 * C[1], rel=1e-13)
    kf1 = 3e8 * 1400.0 ** 0.2 * math.exp(-1500.0 / 1400.0)
    assert r["q"][0, 1] == pytest.approx(kf1 * C[0] ** 0.5 * C[1] ** 1.7, rel=1e-13)
    assert r["qr"][0, 1] == 0.0
    # the stoichiometry keeps its integer coefficients: w_C = q_1
    w = oracle.production_rates(m, T, p, Y)["wdot"]
    assert w[0, 2] == pytest.approx(r["q"][0, 1], rel=1e-14)


@pytest.fixture(scope="module")
def variant_mech(tmp_path_factory):
    path = tmp_path_factory.mktemp("var") / "v.mech"
    path.write_text(synth.mechanism_text(synth.generate_variant_mechanism()))
    return oracle.read_mechanism(str(path))


def _vstates(m, n, seed):
    st = synth.state_c0(m.n_species, n=n, seed=seed)
    return st["T"], st["p"] * np.geomspace(0.05, 60.0, n), np.ascontiguousarray(st["Y"].T)


def test_variant_jacobian_matches_complex_step(variant_mech):
    """Every rate form's analytic derivatives (PLOG across and beyond its pressures,
    Chebyshev, SRI, Lindemann, explicit reverse, irreversible, fractional orders) against
    complex-step differentiation of the forward rates."""
    m = variant_mech
    kinds = set(m.kind)
    assert {"plog", "chebyshev", "sri", "lindemann", "troe", "threebody"} <= kinds
    T, p, Y = _vstates(m, 10, 51)
    J, G = oracle.jacobian(m, T, p, Y, return_gross=True)
    Jc = oracle.complex_step_jacobian(m, T, p, Y)
    assert jac_scaled_error(J, Jc, G, T, Y).max() <= 1e-12
    assert np.all(np.abs(J) <= G * (1 + 1e-12) + 1e-300)


def test_variant_conservation(variant_mech):
    m = variant_mech
    T, p, Y = _vstates(m, 10, 52)
    r = oracle.production_rates(m, T, p, Y)
    el = r["wdot"] @ m.comp
    assert np.max(np.abs(el) / (r["turnover"] @ m.comp + 1e-300)) <= 1e-13
    assert np.max(np.abs(r["r_mass"]) / (r["turnover"] @ m.W)) <= 1e-13
