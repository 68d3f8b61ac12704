"""Pins of the oracle's point-wise chemistry source terms (CPU only): dY_k/dt, dT/dt
and the point-wise part of Q_T (Section 2, Eq. (1a), Eq. (1b), Eq. (3))."""
import numpy as np
import pytest

import oracle
import synth


def _states(m, n, seed, with_anchors=True):
    st = synth.state_c0(m.n_species, n=n, seed=seed)
    T, p, Y = st["T"], st["p"] * np.where(np.arange(n) % 2, 10.0, 1.0), np.ascontiguousarray(st["Y"].T)
    if with_anchors and m.n_species == 53:
        a = synth.load_anchors()
        T = np.concatenate([T, a["T"][:4]])
        p = np.concatenate([p, a["p"][:4]])
        Y = np.concatenate([Y, a["Y"][:4]])
    return T, p, Y


@pytest.fixture(scope="module", params=["c0", "c1"])
def mech(request, c0_path, c1_path):
    return oracle.read_mechanism(c0_path if request.param == "c0" else c1_path)


def test_mass_fraction_rates_conserve_mass(mech):
    """sum_k dY_k/dt = sum_k W_k w_k / rho = 0 for an element-balanced mechanism."""
    T, p, Y = _states(mech, 12, 1)
    s = oracle.chemistry_source(mech, T, p, Y)
    gross = (np.abs(s["wdot"]) * mech.W[None, :]).sum(axis=1) / s["rho"]
    assert np.max(np.abs(s["dYdt"].sum(axis=1)) / gross) <= 1e-13


@pytest.mark.parametrize("dp", [0.0, 2.5e5])
def test_enthalpy_balance(mech, dp):
    """Adiabatic low-Mach energy balance: rho d(h_mass)/dt = dp0/dt along the source,
    with h_mass = sum_k Y_k h_k(T) / W_k, i.e. rho (sum_k h_k/W_k dY_k/dt + c_p dT/dt) = dp0/dt.
    A wrong sign of the heat release, or a molar c_p, fails it."""
    T, p, Y = _states(mech, 12, 2)
    s = oracle.chemistry_source(mech, T, p, Y, dp0dt=dp)
    th = oracle.thermo_properties(mech, T, p, Y)
    dh = (th["h_k"] / mech.W[None, :] * s["dYdt"]).sum(axis=1) + th["cp_mass"] * s["dTdt"]
    gross = (np.abs(th["h_k"] / mech.W[None, :] * s["dYdt"])).sum(axis=1) + np.abs(th["cp_mass"] * s["dTdt"])
    assert np.max(np.abs(s["rho"] * dh - dp) / (s["rho"] * gross + abs(dp))) <= 1e-13


@pytest.mark.parametrize("dp", [0.0, -4.0e4])
def test_divergence_constraint_is_the_density_rate(mech, dp):
    """Q_T = -(1/rho) d rho/dt along the source (Eq. (3)): the rate of the ideal-gas density of
    Eq. (1d) along (dT/dt, dp0/dt, dY/dt), taken by one complex step of the oracle's mixture
    state (no use of the Q_T formula)."""
    T, p, Y = _states(mech, 12, 3)
    s = oracle.chemistry_source(mech, T, p, Y, dp0dt=dp)
    Wbar = 1.0 / (Y / mech.W[None, :]).sum(axis=1)
    scale = np.abs(s["dTdt"] / T) + (Wbar[:, None] / mech.W[None, :] * np.abs(s["dYdt"])).sum(axis=1) + abs(dp) / p
    h = 1e-30 / scale                       # a relative step of 1e-30 in every variable
    _, rho_c, _, _ = oracle.mixture_state(mech, T + 1j * h * s["dTdt"], p + 1j * h * dp,
                                          Y + 1j * h[:, None] * s["dYdt"])
    qt_ref = -(rho_c.imag / h) / s["rho"]
    assert np.max(np.abs(s["QT"] - qt_ref) / scale) <= 1e-13


def test_source_scales_with_the_production_rates(mech):
    """Doubling every pre-exponential factor (ln A + ln 2, Troe k0 too) doubles the
    production rates, so dY/dt, dT/dt and Q_T double (dp0/dt = 0)."""
    import copy
    T, p, Y = _states(mech, 6, 4, with_anchors=False)
    s1 = oracle.chemistry_source(mech, T, p, Y)
    m2 = copy.deepcopy(mech)
    m2.lnA = mech.lnA + np.log(2.0)
    tr = m2.troe.copy()
    tr[:, 0] = np.where(np.array(mech.kind) == "troe", tr[:, 0] + np.log(2.0), tr[:, 0])
    m2.troe = tr
    s2 = oracle.chemistry_source(m2, T, p, Y)
    for k in ("dYdt", "dTdt", "QT"):
        np.testing.assert_allclose(s2[k], 2.0 * s1[k], rtol=1e-12, atol=1e-300)
