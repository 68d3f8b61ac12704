"""Pins of the oracle's rates of progress and production rates (CPU only).

Hand-worked single-reaction cases (NASA data with a6 only, so g/RT = a6/T and the
equilibrium constants are closed forms), the Troe centre and Lindemann points,
third-body efficiency scaling, detailed balance at the Gibbs minimum, element and
mass conservation, additivity and permutation equivariance.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import Reaction, nasa_const, tiny_mechanism

R = 8314.46261815324
P0 = 101325.0
T1000 = np.array([1000.0])


def _isomer_mech(tmp_path):
    # A <=> B, k_f = 1, g_B/RT - g_A/RT = -ln 2 at 1000 K  =>  K_c = 2 (dimensionless)
    species = [("A", (1, 1), nasa_const(), None),
               ("B", (1, 1), nasa_const(a6=-1000.0 * math.log(2.0)), None)]
    rx = [Reaction("elementary", {0: 1}, {1: 1}, 0.0, 0.0, 0.0)]
    return oracle.read_mechanism(tiny_mechanism(tmp_path / "iso.mech", species, rx))


def test_isomerisation_hand_values(tmp_path):
    m = _isomer_mech(tmp_path)
    ctot = P0 / (R * 1000.0)
    p = np.array([P0] * 3)
    Y = np.array([[1.0, 0.0], [1.0 / 3.0, 2.0 / 3.0], [0.5, 0.5]])
    r = oracle.rates_of_progress(m, np.full(3, 1000.0), p, Y)
    assert r["lnKc"][0, 0] == pytest.approx(math.log(2.0), rel=1e-15)
    assert r["q"][0, 0] == pytest.approx(ctot, rel=1e-14)              # q = k_f C_A
    assert abs(r["q"][1, 0]) <= 1e-15 * r["qf"][1, 0]                   # C_B/C_A = K_c
    assert r["q"][2, 0] == pytest.approx(ctot / 4.0, rel=1e-14)         # C/2 - (C/2)/2
    w = oracle.production_rates(m, np.full(3, 1000.0), p, Y)["wdot"]
    np.testing.assert_allclose(w[:, 1], -w[:, 0], rtol=0, atol=0)
    assert w[2, 1] == pytest.approx(ctot / 4.0, rel=1e-14)


def _assoc_mech(tmp_path, kind="elementary", eff=None, troe=(), lnA=math.log(2.0), b=1.0, theta=0.0):
    # H + O <=> HO with g_HO/RT = -ln 4 at 1000 K  =>  K_c = 4 R T / p0  (dnu = -1)
    species = [("H", (1, 0), nasa_const(), None), ("O", (0, 1), nasa_const(), None),
               ("HO", (1, 1), nasa_const(a6=-1000.0 * math.log(4.0)), None)]
    rx = [Reaction(kind, {0: 1, 1: 1}, {2: 1}, lnA, b, theta, eff or {}, troe)]
    return oracle.read_mechanism(tiny_mechanism(tmp_path / f"assoc_{kind}.mech", species, rx))


def _conc_to_Y(m, C):
    """Mass fractions of a state with concentrations C (kmol/m^3)."""
    mass = C * m.W
    return mass / mass.sum()


def test_association_rate_constant_and_equilibrium(tmp_path):
    m = _assoc_mech(tmp_path)
    Kc = 4.0 * R * 1000.0 / P0
    # k_f = A T^b = 2 * 1000 at 1000 K
    ctot = P0 / (R * 1000.0)
    Y = np.array([[0.5, 0.5, 0.0]])
    r = oracle.rates_of_progress(m, T1000, np.array([P0]), Y)
    _, _, _, C = oracle.mixture_state(m, T1000, np.array([P0]), Y)
    assert r["kf"][0, 0] == pytest.approx(2000.0, rel=1e-14)
    assert math.exp(r["lnKc"][0, 0]) == pytest.approx(Kc, rel=1e-14)
    assert r["q"][0, 0] == pytest.approx(2000.0 * C[0, 0] * C[0, 1], rel=1e-14)
    # equilibrium state: C_H = C_O = c, C_HO = Kc c^2, with 2c + Kc c^2 = p/(RT)
    c = (-2.0 + math.sqrt(4.0 + 4.0 * Kc * ctot)) / (2.0 * Kc)
    Yeq = _conc_to_Y(m, np.array([c, c, Kc * c * c]))[None, :]
    r = oracle.rates_of_progress(m, T1000, np.array([P0]), Yeq)
    assert abs(r["q"][0, 0]) <= 1e-13 * r["qf"][0, 0]


def test_activation_temperature(tmp_path):
    # theta = 1000 ln 2 halves k at 1000 K
    m = _assoc_mech(tmp_path, lnA=0.0, b=0.0, theta=1000.0 * math.log(2.0))
    r = oracle.rates_of_progress(m, T1000, np.array([P0]), np.array([[0.5, 0.5, 0.0]]))
    assert r["kf"][0, 0] == pytest.approx(0.5, rel=1e-14)


def test_pressure_scaling_of_forward_and_reverse_rates(tmp_path):
    m = _assoc_mech(tmp_path)
    Y = np.array([[0.3, 0.3, 0.4]] * 2)
    T = np.array([1300.0, 1300.0])
    r = oracle.rates_of_progress(m, T, np.array([P0, 3.0 * P0]), Y)
    assert r["qf"][1, 0] / r["qf"][0, 0] == pytest.approx(9.0, rel=1e-13)   # sum nu' = 2
    assert r["qr"][1, 0] / r["qr"][0, 0] == pytest.approx(3.0, rel=1e-13)   # sum nu'' = 1


def test_second_order_in_one_species(tmp_path):
    # H + H <=> H2 with k_f = 1: q_f = C_H^2
    species = [("H", (1, 0), nasa_const(), None), ("H2", (2, 0), nasa_const(), None)]
    rx = [Reaction("elementary", {0: 2}, {1: 1}, 0.0, 0.0, 0.0)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "h2.mech", species, rx))
    r = oracle.rates_of_progress(m, T1000, np.array([P0]), np.array([[1.0, 0.0]]))
    assert r["qf"][0, 0] == pytest.approx((P0 / (R * 1000.0)) ** 2, rel=1e-14)
    w = oracle.production_rates(m, T1000, np.array([P0]), np.array([[1.0, 0.0]]))["wdot"]
    assert w[0, 0] == pytest.approx(-2.0 * r["q"][0, 0], rel=1e-15)
    assert w[0, 1] == pytest.approx(r["q"][0, 0], rel=1e-15)


def test_three_body_efficiencies(tmp_path):
    Y = np.array([[0.3, 0.3, 0.4]])
    p = np.array([P0])
    q_el = oracle.rates_of_progress(_assoc_mech(tmp_path), T1000, p, Y)["q"][0, 0]
    q_tb = oracle.rates_of_progress(_assoc_mech(tmp_path, "threebody"), T1000, p, Y)["q"][0, 0]
    assert q_tb == pytest.approx(q_el * P0 / (R * 1000.0), rel=1e-14)     # [M] = p/(RT)
    zero = _assoc_mech(tmp_path, "threebody", eff={0: 0.0, 1: 0.0, 2: 0.0})
    assert oracle.rates_of_progress(zero, T1000, p, Y)["q"][0, 0] == 0.0
    scaled = _assoc_mech(tmp_path, "threebody", eff={0: 2.5, 1: 2.5, 2: 2.5})
    assert oracle.rates_of_progress(scaled, T1000, p, Y)["q"][0, 0] == pytest.approx(2.5 * q_tb, rel=1e-14)
    # a single efficiency changes [M] by (eps - 1) C_k
    one = _assoc_mech(tmp_path, "threebody", eff={2: 3.0})
    _, _, _, C = oracle.mixture_state(one, T1000, p, Y)
    r = oracle.rates_of_progress(one, T1000, p, Y)
    assert r["M"][0, 0] == pytest.approx(C.sum() + 2.0 * C[0, 2], rel=1e-14)


def test_troe_lindemann_limit(tmp_path):
    # T3, T1, T2 -> 1e30: F_cent = 1 so F = 1 and k_f = kinf P_r / (1 + P_r); kinf = 1, k0 = 1000
    troe = (math.log(1000.0), 0.0, 0.0, 0.6, 1e30, 1e30, 1e30)
    m = _assoc_mech(tmp_path, "troe", troe=troe, lnA=0.0, b=0.0)
    r = oracle.rates_of_progress(m, T1000, np.array([P0]), np.array([[0.3, 0.3, 0.4]]))
    pr = 1000.0 * P0 / (R * 1000.0)
    assert r["kf"][0, 0] == pytest.approx(pr / (1.0 + pr), rel=1e-14)


def _troe_at(tmp_path, target_f1):
    """Troe reaction at 1000 K with F_cent = e^-1 and k0 chosen so that f1 = target."""
    ctot = P0 / (R * 1000.0)
    lfc = -1.0 / math.log(10.0)
    c = -0.4 - 0.67 * lfc
    n = 0.75 - 1.27 * lfc
    d = 0.14
    # u / (n - d u) = f1  =>  u = f1 n / (1 + d f1);   log10 Pr = u - c
    u = target_f1 * n / (1.0 + d * target_f1)
    pr = 10.0 ** (u - c)
    lnA0 = math.log(pr / ctot)                      # kinf = 1, [M] = ctot
    troe = (lnA0, 0.0, 0.0, 0.5, 1000.0, 1000.0, 1e30)   # F_cent = e^-1/2 + e^-1/2 + 0
    m = _assoc_mech(tmp_path, "troe", troe=troe, lnA=0.0, b=0.0)
    r = oracle.rates_of_progress(m, T1000, np.array([P0]), np.array([[0.3, 0.3, 0.4]]))
    return r["kf"][0, 0], pr


def test_troe_centre_point(tmp_path):
    # f1 = 0: F = F_cent = e^-1
    kf, pr = _troe_at(tmp_path, 0.0)
    assert kf == pytest.approx(pr / (1.0 + pr) * math.exp(-1.0), rel=1e-13)


def test_troe_unit_f1_point(tmp_path):
    # f1 = 1: log10 F = log10 F_cent / 2, F = sqrt(F_cent)
    kf, pr = _troe_at(tmp_path, 1.0)
    assert kf == pytest.approx(pr / (1.0 + pr) * math.exp(-0.5), rel=1e-13)


def test_troe_rate_does_not_multiply_by_M(tmp_path):
    # doubling every efficiency doubles P_r only (k_f changes through P_r/(1+P_r) and F, not x2)
    troe = (math.log(1000.0), 0.0, 0.0, 0.6, 1e30, 1e30, 1e30)
    Y = np.array([[0.3, 0.3, 0.4]])
    m2 = _assoc_mech(tmp_path, "troe", eff={0: 2.0, 1: 2.0, 2: 2.0}, troe=troe, lnA=0.0, b=0.0)
    r = oracle.rates_of_progress(m2, T1000, np.array([P0]), Y)
    pr = 2000.0 * P0 / (R * 1000.0)
    assert r["kf"][0, 0] == pytest.approx(pr / (1.0 + pr), rel=1e-14)


def test_heat_release_sign(tmp_path):
    # H + O -> HO with h_HO = R a6 < 0: exothermic; with no HO present q > 0 and hrr = -h_HO q > 0
    m = _assoc_mech(tmp_path)
    out = oracle.production_rates(m, T1000, np.array([P0]), np.array([[0.5, 0.5, 0.0]]))
    q = out["q"][0, 0]
    h_ho = R * (-1000.0 * math.log(4.0))
    assert q > 0
    assert out["hrr"][0] == pytest.approx(-h_ho * q, rel=1e-14)
    assert out["hrr"][0] > 0


def _random_states(ns, n, seed):
    st = synth.state_c0(ns, n=n, seed=seed)
    return st["T"], st["p"], np.ascontiguousarray(st["Y"].T)


@pytest.mark.parametrize("which", ["c0", "c1"])
def test_element_and_mass_conservation(which, c0_path, c1_path):
    m = oracle.read_mechanism(c0_path if which == "c0" else c1_path)
    T, p, Y = _random_states(m.n_species, 200, 3)
    out = oracle.production_rates(m, T, p, Y)
    el = out["wdot"] @ m.comp
    scale_el = out["turnover"] @ m.comp
    assert np.all(np.abs(el) <= 1e-13 * scale_el)
    assert np.all(np.abs(out["r_mass"]) <= 1e-13 * (out["turnover"] @ m.W))


def test_additivity_over_mechanism_halves(tmp_path):
    mech = synth.generate_mechanism(synth.MECH_C1)
    whole = oracle.read_mechanism(synth.write_mechanism(mech, tmp_path / "all.mech"))
    import copy
    h1 = copy.deepcopy(mech); h1.reactions = mech.reactions[::2]
    h2 = copy.deepcopy(mech); h2.reactions = mech.reactions[1::2]
    m1 = oracle.read_mechanism(synth.write_mechanism(h1, tmp_path / "h1.mech"))
    m2 = oracle.read_mechanism(synth.write_mechanism(h2, tmp_path / "h2.mech"))
    T, p, Y = _random_states(whole.n_species, 50, 4)
    w = oracle.production_rates(whole, T, p, Y)
    w1 = oracle.production_rates(m1, T, p, Y)
    w2 = oracle.production_rates(m2, T, p, Y)
    np.testing.assert_allclose(w1["wdot"] + w2["wdot"], w["wdot"], rtol=0,
                               atol=1e-14 * w["turnover"].max())


def test_permutation_equivariance(tmp_path):
    mech = synth.generate_mechanism(synth.MECH_C0)
    m = oracle.read_mechanism(synth.write_mechanism(mech, tmp_path / "a.mech"))
    rng = np.random.default_rng(7)
    perm = rng.permutation(len(mech.names))          # new index j holds old species perm[j]
    inv = np.argsort(perm)
    import copy
    pm = copy.deepcopy(mech)
    pm.names = [mech.names[k] for k in perm]
    pm.comp = mech.comp[perm]
    pm.nasa_lo = mech.nasa_lo[perm]
    pm.nasa_hi = mech.nasa_hi[perm]
    pm.mu = mech.mu[perm]
    pm.lam = mech.lam[perm]
    pm.dif = {}
    for (j, k), c in mech.dif.items():
        a, b = sorted((int(inv[j]), int(inv[k])))
        pm.dif[(a, b)] = c
    pm.reactions = []
    for r in mech.reactions[::-1]:
        rr = copy.deepcopy(r)
        rr.reactants = {int(inv[k]): v for k, v in r.reactants.items()}
        rr.products = {int(inv[k]): v for k, v in r.products.items()}
        rr.efficiencies = {int(inv[k]): v for k, v in r.efficiencies.items()}
        pm.reactions.append(rr)
    mp = oracle.read_mechanism(synth.write_mechanism(pm, tmp_path / "b.mech"))
    T, p, Y = _random_states(m.n_species, 40, 5)
    a = oracle.production_rates(m, T, p, Y)
    b = oracle.production_rates(mp, T, p, Y[:, perm])
    np.testing.assert_allclose(b["wdot"], a["wdot"][:, perm], rtol=1e-13,
                               atol=1e-14 * a["turnover"].max())
    np.testing.assert_allclose(b["hrr"], a["hrr"], rtol=1e-11, atol=1e-14 * np.abs(a["hrr"]).max())


@pytest.mark.parametrize("which,T,p", [("c0", 1200.0, P0), ("c0", 2400.0, 10 * P0),
                                       ("c1", 1600.0, P0), ("c1", 2300.0, 10 * P0)])
def test_detailed_balance_at_gibbs_minimum(which, T, p, c0_path, c1_path):
    """At the equilibrium of equil.py every rate of progress vanishes: pins K_c."""
    m = oracle.read_mechanism(c0_path if which == "c0" else c1_path)
    rng = np.random.default_rng(int(T))
    Y0 = rng.dirichlet(np.full(m.n_species, 0.3))
    Yeq, _ = oracle.equilibrate(m, T, p, Y0)
    r = oracle.rates_of_progress(m, np.array([T]), np.array([p]), Yeq[None, :])
    assert np.all(np.abs(r["q"][0]) <= 1e-10 * np.abs(r["qf"][0]))
