"""Mixture state and NASA-7 thermodynamics (oracle).

Definitions:

* ideal gas, Eq. (1d): rho = p Wbar / (R T), with the mean molar mass
  Wbar = 1 / sum_k (Y_k / W_k) (the W-bar of Eq. (3));
* mole fractions X_k = Wbar Y_k / W_k (the X_k of Eq. (2)); concentrations
  C_k = rho Y_k / W_k;
* NASA 7-coefficient polynomials, the thermodynamic data of a Cantera-format
  mechanism (Section 2): with the low range for T <= T_mid and the high range
  above,
      cp/R   = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4
      h/(RT) = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T
      s/R    = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7
      g/(RT) = h/(RT) - s/R      (standard-state Gibbs energy)
  (the c_{p,k} and h_k of Eq. (1b)).

Pinned by: the exact polynomial identities d(h/R)/dT = cp/R and d(s/R)/dT = cp/(R T)
(complex step), the a1-only closed forms, X = Y for equal molar masses, and
sum_k C_k = p/(R T) for normalised Y.
"""
from __future__ import annotations

import numpy as np


def mixture_state(m, T, p, Y):
    """(Wbar [n], rho [n], X [n,Ns], C [n,Ns]) for T [n], p [n], Y [n,Ns]."""
    T = np.asarray(T)
    p = np.asarray(p)
    Y = np.asarray(Y)
    inv_wbar = (Y / m.W[None, :]).sum(axis=1)
    Wbar = 1.0 / inv_wbar
    rho = p * Wbar / (m.R * T)
    X = Wbar[:, None] * Y / m.W[None, :]
    C = rho[:, None] * Y / m.W[None, :]
    return Wbar, rho, X, C


def nasa7(m, T):
    """(cp/R, h/RT, s/R, g/RT), each [n, Ns], from the NASA-7 fits."""
    T = np.asarray(T)[:, None]
    low = (T.real <= m.t_mid[None, :])
    a = np.where(low[:, :, None], m.a_lo[None, :, :], m.a_hi[None, :, :])   # [n, Ns, 7]
    a1, a2, a3, a4, a5, a6, a7 = (a[:, :, j] for j in range(7))
    cp = a1 + a2 * T + a3 * T ** 2 + a4 * T ** 3 + a5 * T ** 4
    h = a1 + a2 * T / 2 + a3 * T ** 2 / 3 + a4 * T ** 3 / 4 + a5 * T ** 4 / 5 + a6 / T
    s = a1 * np.log(T) + a2 * T + a3 * T ** 2 / 2 + a4 * T ** 3 / 3 + a5 * T ** 4 / 4 + a7
    return cp, h, s, h - s


def thermo_properties(m, T, p, Y):
    """Dimensional per-species and mixture thermodynamic properties.

    Returns a dict with cp_k [J/(kmol K)], h_k [J/kmol], s_k [J/(kmol K)] (standard
    state), g_k = h_k - T s_k [J/kmol] (each [n, Ns]), and the mixture values
    cp_mass = sum Y_k cp_k / W_k [J/(kg K)], h_mass = sum Y_k h_k / W_k [J/kg],
    rho [kg/m^3] and Wbar [kg/kmol].
    """
    T = np.asarray(T)
    Y = np.asarray(Y)
    cpR, hRT, sR, gRT = nasa7(m, T)
    cp_k = m.R * cpR
    h_k = m.R * T[:, None] * hRT
    s_k = m.R * sR
    g_k = h_k - T[:, None] * s_k
    Wbar, rho, _, _ = mixture_state(m, T, p, Y)
    cp_mass = (Y * cp_k / m.W[None, :]).sum(axis=1)
    h_mass = (Y * h_k / m.W[None, :]).sum(axis=1)
    return {"cp_k": cp_k, "h_k": h_k, "s_k": s_k, "g_k": g_k,
            "cp_mass": cp_mass, "h_mass": h_mass, "rho": rho, "Wbar": Wbar}
