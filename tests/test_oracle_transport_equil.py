"""Pins of the oracle's mixture-averaged transport and of its equilibrium solver (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from helpers import Reaction, nasa_const, tiny_mechanism

R = 8314.46261815324
P0 = 101325.0


def test_pure_species_limits(c0_path):
    m = oracle.read_mechanism(c0_path)
    ns = m.n_species
    T = np.full(ns, 1234.0)
    Y = np.eye(ns)
    with np.errstate(invalid="ignore", divide="ignore"):   # D_k of a pure species is 0/0
        tp = oracle.transport_properties(m, T, np.full(ns, P0), Y)
    L = math.log(1234.0)
    for k in range(ns):
        mu_k = math.exp(sum(m.mu_fit[k, j] * L ** j for j in range(4)))
        lam_k = math.exp(sum(m.lam_fit[k, j] * L ** j for j in range(4)))
        assert tp["mu"][k] == pytest.approx(mu_k, rel=1e-14)          # Phi_kk = 1 exactly
        assert tp["lambda"][k] == pytest.approx(lam_k, rel=1e-14)


def test_fit_evaluation_at_ln_T_equal_one(tmp_path):
    # at T = e, ln mu = c0 + c1 + c2 + c3
    mu = [[-10.0, 0.5, 0.25, -0.125], [-11.0, 0.7, 0.0, 0.0]]
    lam = [[-3.0, 0.8, 0.0, 0.0], [-2.5, 0.8, 0.01, 0.0]]
    dif = {(0, 1): np.array([-9.0, 1.75, 0.0, 0.0])}
    sp = [("A", (1, 0), nasa_const(), None), ("B", (0, 1), nasa_const(), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "t.mech", sp, [], transport=(mu, lam, dif)))
    mu_k, lam_k, D = oracle.transport.species_transport(m, np.array([math.e]), np.array([P0]))
    assert mu_k[0, 0] == pytest.approx(math.exp(-10.0 + 0.5 + 0.25 - 0.125), rel=1e-14)
    assert lam_k[0, 1] == pytest.approx(math.exp(-2.5 + 0.8 + 0.01), rel=1e-14)
    assert D[0, 0, 1] == pytest.approx(math.exp(-9.0 + 1.75), rel=1e-14)
    assert D[0, 1, 0] == D[0, 0, 1]


def test_identical_species_mixture(tmp_path):
    # two species with the same molar mass and fits behave as one: mu = mu_k, lambda = lambda_k
    fit = [-10.5, 0.7, 0.0, 0.0]
    lfit = [-3.0, 0.8, 0.0, 0.0]
    sp = [("A", (1, 1), nasa_const(), None), ("B", (1, 1), nasa_const(), None)]
    dif = {(0, 1): np.array([-9.0, 1.75, 0.0, 0.0])}
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "same.mech", sp, [], transport=([fit, fit], [lfit, lfit], dif)))
    tp = oracle.transport_properties(m, np.array([900.0]), np.array([P0]), np.array([[0.3, 0.7]]))
    L = math.log(900.0)
    assert tp["mu"][0] == pytest.approx(math.exp(-10.5 + 0.7 * L), rel=1e-14)
    assert tp["lambda"][0] == pytest.approx(math.exp(-3.0 + 0.8 * L), rel=1e-14)


def test_binary_wilke_and_mathur_saxena_unequal_masses(tmp_path):
    """Hand-worked binary mixture: W_B = 4 W_A, mu_A = 4 mu_B, lambda_A = 4 lambda_B, and
    Y = (0.2, 0.8), which gives X = (1/2, 1/2), so X differs from Y.

    Wilke, with (mu_A/mu_B)^(1/2) = 2 and (W_B/W_A)^(1/4) = 2^(1/2):
      Phi_AB = 8^(-1/2) (1 + 1/4)^(-1/2) (1 + 2 2^(1/2))^2 = (9 + 4 2^(1/2)) / 10^(1/2)
      Phi_BA = 8^(-1/2) (1 + 4)^(-1/2) (1 + 2^(-3/2))^2   = (9/8 + 2^(-1/2)) / 40^(1/2)
      mu = X_A mu_A / (X_A + X_B Phi_AB) + X_B mu_B / (X_B + X_A Phi_BA)
         = mu_A / (1 + Phi_AB) + mu_B / (1 + Phi_BA)          (X_A = X_B)
    Mathur-Saxena, lambda_A = 0.1, lambda_B = 0.025:
      sum X lambda = 0.0625, sum X / lambda = 25, lambda = (0.0625 + 1/25) / 2 = 0.05125.
    Swapping W_j/W_k inside Phi, or weighting by Y instead of X, changes both values.
    """
    mu_a, mu_b = 4e-5, 1e-5
    mu = [[math.log(mu_a), 0.0, 0.0, 0.0], [math.log(mu_b), 0.0, 0.0, 0.0]]
    lam = [[math.log(0.1), 0.0, 0.0, 0.0], [math.log(0.025), 0.0, 0.0, 0.0]]
    dif = {(0, 1): np.array([math.log(5e-5), 0.0, 0.0, 0.0])}
    sp = [("H", (1,), nasa_const(), None), ("H4", (4,), nasa_const(), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "wilke.mech", sp, [], elements=("H",),
                                             transport=(mu, lam, dif)))
    assert m.W[1] / m.W[0] == pytest.approx(4.0, rel=1e-15)
    T = np.array([700.0, 1800.0])            # constant fits: no temperature dependence
    Y = np.array([[0.2, 0.8], [0.2, 0.8]])
    tp = oracle.transport_properties(m, T, np.full(2, P0), Y)
    _, _, X, _ = oracle.mixture_state(m, T, np.full(2, P0), Y)
    np.testing.assert_allclose(X, 0.5, rtol=1e-15)
    s2 = math.sqrt(2.0)
    phi_ab = (9.0 + 4.0 * s2) / math.sqrt(10.0)
    phi_ba = (9.0 / 8.0 + 1.0 / s2) / math.sqrt(40.0)
    mu_ref = mu_a / (1.0 + phi_ab) + mu_b / (1.0 + phi_ba)
    np.testing.assert_allclose(tp["mu"], mu_ref, rtol=1e-14)
    np.testing.assert_allclose(tp["lambda"], 0.05125, rtol=1e-14)


def test_wilke_ternary_permutation_and_scaling(tmp_path):
    """Three species of unequal mass: relabelling the species leaves mu and lambda unchanged,
    and scaling every pure viscosity by s scales mu by s (Phi depends on ratios only)."""
    base = [math.log(3e-5), math.log(1.2e-5), math.log(2.5e-5)]
    lams = [math.log(0.08), math.log(0.03), math.log(0.15)]
    comps = [(1, 0), (0, 2), (2, 1)]

    def build(order, shift, name):
        mu = [[base[i] + shift, 0.0, 0.0, 0.0] for i in order]
        lam = [[lams[i], 0.0, 0.0, 0.0] for i in order]
        dif = {(j, k): np.array([math.log(5e-5), 0.0, 0.0, 0.0]) for j in range(3) for k in range(j + 1, 3)}
        sp = [(f"S{i}", comps[i], nasa_const(), None) for i in order]
        return oracle.read_mechanism(tiny_mechanism(tmp_path / name, sp, [], transport=(mu, lam, dif)))
    Y = np.array([[0.5, 0.3, 0.2]])
    a = oracle.transport_properties(build([0, 1, 2], 0.0, "a.mech"), np.array([1000.0]), np.array([P0]), Y)
    b = oracle.transport_properties(build([2, 0, 1], 0.0, "b.mech"), np.array([1000.0]), np.array([P0]),
                                    Y[:, [2, 0, 1]])
    c = oracle.transport_properties(build([0, 1, 2], math.log(3.0), "c.mech"), np.array([1000.0]),
                                    np.array([P0]), Y)
    assert b["mu"][0] == pytest.approx(a["mu"][0], rel=1e-14)
    assert b["lambda"][0] == pytest.approx(a["lambda"][0], rel=1e-14)
    assert c["mu"][0] == pytest.approx(3.0 * a["mu"][0], rel=1e-14)


def test_binary_and_trace_diffusion(tmp_path):
    sp = [("H", (1, 0), nasa_const(), None), ("O", (0, 1), nasa_const(), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "bin.mech", sp, []))
    T = np.array([800.0, 800.0])
    p = np.array([P0, P0])
    Y = np.array([[0.25, 0.75], [1e-12, 1.0 - 1e-12]])
    tp = oracle.transport_properties(m, T, p, Y)
    _, _, X, _ = oracle.mixture_state(m, T, p, Y)
    d12 = math.exp(math.log(5e-5))
    # binary: D_1 = D_12 Y_2 / X_2
    assert tp["Dmix"][0, 0] == pytest.approx(d12 * Y[0, 1] / X[0, 1], rel=1e-14)
    # trace H in pure O: D_H -> D_HO
    assert tp["Dmix"][1, 0] == pytest.approx(d12, rel=1e-10)


def test_pressure_dependence(c0_path):
    m = oracle.read_mechanism(c0_path)
    rng = np.random.default_rng(0)
    Y = rng.dirichlet(np.full(m.n_species, 0.5), size=4)
    T = np.array([400.0, 900.0, 1500.0, 2400.0])
    a = oracle.transport_properties(m, T, np.full(4, P0), Y)
    b = oracle.transport_properties(m, T, np.full(4, 4 * P0), Y)
    np.testing.assert_allclose(b["Dmix"], a["Dmix"] / 4.0, rtol=1e-14)
    np.testing.assert_allclose(b["mu"], a["mu"], rtol=1e-15)
    np.testing.assert_allclose(b["lambda"], a["lambda"], rtol=1e-15)


# ------------------------------------------------------------------ equilibrium
def test_equilibrium_isomers(tmp_path):
    # g_B - g_A = -RT ln 2 at 1000 K: x_B / x_A = 2
    sp = [("A", (1, 1), nasa_const(), None), ("B", (1, 1), nasa_const(a6=-1000.0 * math.log(2.0)), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "iso.mech", sp, []))
    Y, info = oracle.equilibrate(m, 1000.0, P0, np.array([0.9, 0.1]))
    assert Y[1] / Y[0] == pytest.approx(2.0, rel=1e-13)


@pytest.mark.parametrize("pfac,xh", [(1.0, (math.sqrt(5.0) - 1.0) / 2.0),
                                     (4.0, (math.sqrt(17.0) - 1.0) / 8.0)])
def test_equilibrium_dissociation(tmp_path, pfac, xh):
    # H2 = 2H with all g = 0: x_H^2 / x_H2 = p0/p, x_H + x_H2 = 1
    sp = [("H", (1, 0), nasa_const(), None), ("H2", (2, 0), nasa_const(), None)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "diss.mech", sp, []))
    Y, _ = oracle.equilibrate(m, 1500.0, pfac * P0, np.array([0.0, 1.0]))
    nh, nh2 = Y[0] / 1.008, Y[1] / 2.016
    assert nh / (nh + nh2) == pytest.approx(xh, rel=1e-13)


def test_equilibrium_conservation_and_stationarity(c1_path):
    m = oracle.read_mechanism(c1_path)
    rng = np.random.default_rng(2)
    Y0 = rng.dirichlet(np.full(m.n_species, 0.3))
    Y, info = oracle.equilibrate(m, 1900.0, 10 * P0, Y0)
    b0 = (Y0 / m.W) @ m.comp
    b1 = (Y / m.W) @ m.comp
    np.testing.assert_allclose(b1, b0, rtol=1e-12)
    # mu_k = sum_e a_ek pi_e for every species
    np.testing.assert_allclose(info["mu"], m.comp @ info["pi"], rtol=1e-12, atol=1e-10)


def test_stored_anchor_states_are_equilibria(c1_path):
    """The stored near-equilibrium anchors are Gibbs minima of the 53-species mechanism."""
    from synth.state import load_anchors
    m = oracle.read_mechanism(c1_path)
    a = load_anchors()
    idx = np.arange(0, a["T"].shape[0], 17)
    r = oracle.rates_of_progress(m, a["T"][idx], a["p"][idx], a["Y"][idx])
    assert np.all(np.abs(r["q"]) <= 1e-9 * np.abs(r["qf"]))
