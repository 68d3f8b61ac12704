"""Pins of the oracle's constant-pressure reactor step (CPU only): the Jacobian of the
source terms, and the two-stage Rosenbrock step built on it."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import Reaction, nasa_const, tiny_mechanism

R = 8314.46261815324
P0 = 101325.0
GAMMA = 1.0 + 1.0 / math.sqrt(2.0)


def _states(m, n, seed):
    st = synth.state_c0(m.n_species, n=n, seed=seed)
    return st["T"], st["p"] * np.where(np.arange(n) % 2, 10.0, 1.0), np.ascontiguousarray(st["Y"].T)


@pytest.mark.parametrize("which", ["c0", "c1"])
def test_source_jacobian_matches_complex_step(which, c0_path, c1_path):
    """A = df/dx against one complex step of f per column (exact to rounding, no use of
    the chain rule); entries of row r measured against max_c |A_rc| x_c of the complex-step
    Jacobian with x = (T, Y)."""
    m = oracle.read_mechanism(c0_path if which == "c0" else c1_path)
    T, p, Y = _states(m, 6, 31)
    A = oracle.source_jacobian(m, T, p, Y)
    n, ns = Y.shape
    h = 1e-30
    Acs = np.zeros_like(A)
    for c in range(ns + 1):
        Tc, Yc = T.astype(complex), Y.astype(complex)
        step = h * T if c == 0 else np.full(n, h)
        if c == 0:
            Tc = Tc + 1j * step
        else:
            Yc[:, c - 1] += 1j * step
        Acs[:, :, c] = oracle.rhs(m, Tc, p, Yc).imag / step[:, None]
    x = np.concatenate([T[:, None], Y], axis=1)
    scale = (np.abs(Acs) * x[:, None, :]).max(axis=2, keepdims=True)
    assert np.max(np.abs(A - Acs) * x[:, None, :] / scale) <= 1e-12


def _isomer_mech(tmp_path, lnA=math.log(10.0), K=3.0):
    """A <=> B, isomers (same W), identical c_p and h, entropies differing by ln K: the
    reaction is thermoneutral, so T and rho stay constant and
    dY_A/dt = -(k_f + k_r) Y_A + k_r (Y_A + Y_B), with k_r = k_f / K."""
    sp = [("A", (1, 1), nasa_const(a1=3.5), None), ("B", (1, 1), nasa_const(a1=3.5, a7=math.log(K)), None)]
    rx = [Reaction("elementary", {0: 1}, {1: 1}, lnA, 0.0, 0.0)]
    return oracle.read_mechanism(tiny_mechanism(tmp_path / "iso.mech", sp, rx))


def test_one_step_is_the_stability_function(tmp_path):
    """On the linear isomerisation one ROS2 step multiplies Y_A - Y_eq by
    R(z) = (1 + (1 - 2 gamma) z) / (1 - gamma z)^2 with z = -(k_f + k_r) h."""
    m = _isomer_mech(tmp_path)
    kf, kr = 10.0, 10.0 / 3.0
    lam, yeq = kf + kr, kr / (kf + kr)
    T, p, Y = np.array([1200.0, 800.0]), np.array([P0, 5 * P0]), np.array([[0.9, 0.1], [0.05, 0.95]])
    for h in (1e-3, 0.05, 2.0, 1e3):
        T1, Y1 = oracle.ros2_step(m, T, p, Y, h, 1)
        z = -lam * h
        Rz = (1 + (1 - 2 * GAMMA) * z) / (1 - GAMMA * z) ** 2
        np.testing.assert_allclose(Y1[:, 0] - yeq, Rz * (Y[:, 0] - yeq), rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(T1, T, rtol=1e-14)
        np.testing.assert_allclose(Y1.sum(axis=1), 1.0, rtol=0, atol=1e-13)


def test_second_order_convergence(tmp_path):
    """Against the exact relaxation Y_A(t) - Y_eq = (Y_A(0) - Y_eq) exp(-(k_f + k_r) t), the
    error at t = 0.3 s falls by four when the substeps double (order two)."""
    m = _isomer_mech(tmp_path)
    lam, yeq = 10.0 + 10.0 / 3.0, (10.0 / 3.0) / (10.0 + 10.0 / 3.0)
    T, p, Y = np.array([1000.0]), np.array([P0]), np.array([[0.8, 0.2]])
    exact = yeq + (0.8 - yeq) * math.exp(-lam * 0.3)
    errs = [abs(oracle.ros2_step(m, T, p, Y, 0.3, k)[1][0, 0] - exact) for k in (256, 512, 1024)]
    assert 3.8 < errs[0] / errs[1] < 4.1 and 3.9 < errs[1] / errs[2] < 4.1


def test_equilibrium_is_a_fixed_point(tmp_path):
    """At the Gibbs minimum (equil.py, an independent solver) every rate of progress vanishes,
    so f = 0 and a step of any size leaves the state where it is."""
    sp = [("H2", (2, 0), nasa_const(a1=3.5, a6=0.0, a7=-1.0), None),
          ("H", (1, 0), nasa_const(a1=2.5, a6=26000.0, a7=-0.5), None),
          ("O2", (0, 2), nasa_const(a1=3.5, a6=0.0, a7=2.0), None),
          ("O", (0, 1), nasa_const(a1=2.5, a6=29000.0, a7=1.5), None),
          ("OH", (1, 1), nasa_const(a1=3.5, a6=4000.0, a7=1.0), None)]
    rx = [Reaction("elementary", {0: 1}, {1: 2}, math.log(1e8), 0.0, 2000.0),
          Reaction("elementary", {2: 1}, {3: 2}, math.log(1e8), 0.0, 3000.0),
          Reaction("elementary", {1: 1, 3: 1}, {4: 1}, math.log(1e7), 0.0, 0.0)]
    m = oracle.read_mechanism(tiny_mechanism(tmp_path / "eq.mech", sp, rx))
    T, p = 3000.0, P0
    Yeq, _ = oracle.equilibrate(m, T, p, np.array([0.12, 0.0, 0.88, 0.0, 0.0]))
    assert Yeq.min() > 1e-12                       # every species present at this temperature
    T1, Y1 = oracle.ros2_step(m, np.array([T]), np.array([p]), Yeq[None, :], 1e-3, 2)
    assert abs(T1[0] - T) <= 1e-9 * T
    np.testing.assert_allclose(Y1[0], Yeq, rtol=1e-8, atol=1e-14)


def test_step_conserves_mass_and_elements(c0_path):
    """sum_k Y_k and the element totals sum_k a_ek Y_k / W_k are linear invariants of f, which
    a Rosenbrock step with the exact Jacobian keeps to rounding."""
    import copy
    m = copy.deepcopy(oracle.read_mechanism(c0_path))
    # pre-exponential factors scaled by e^-48, so that the step's stiffness h |A| stays near
    # 1e2 to 1e4 (the rounding of a dense solve is ~ eps h |A| of the change it makes)
    m.lnA = m.lnA - 48.0
    T, p, Y = _states(m, 8, 32)
    T = np.maximum(T, 1200.0)
    T1, Y1 = oracle.ros2_step(m, T, p, Y, 1e-3, 3)
    assert np.max(np.abs(Y1.sum(axis=1) - Y.sum(axis=1))) <= 1e-13
    el0 = (Y / m.W[None, :]) @ m.comp
    el1 = (Y1 / m.W[None, :]) @ m.comp
    assert np.max(np.abs(el1 - el0) / np.abs(el0).sum(axis=1, keepdims=True)) <= 1e-12
    assert np.all(np.abs(T1 - T) > 0)
