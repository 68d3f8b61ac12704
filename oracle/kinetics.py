"""Rates of progress and net production rates (oracle).

The net production rate w_k of Eq. (1a) and the heat-release term of Eq. (1b),
with the reaction kinetics of a Cantera-format mechanism (Section 2), written out
as the standard mass-action definitions:

* modified Arrhenius:  k = A T^b exp(-theta / T)          (theta = E_a / R)
* third body:          [M]_i = sum_k eps_ik C_k; the rate of progress of a
                       three-body reaction is multiplied by [M]_i in both directions
* Troe falloff:        k0, kinf from their Arrhenius forms; P_r = k0 [M] / kinf;
                       F_cent = (1-alpha) exp(-T/T3) + alpha exp(-T/T1) + exp(-T2/T);
                       c = -0.4 - 0.67 log10 F_cent, n = 0.75 - 1.27 log10 F_cent, d = 0.14;
                       f1 = (log10 P_r + c) / (n - d (log10 P_r + c));
                       log10 F = log10 F_cent / (1 + f1^2);
                       k_f = kinf P_r / (1 + P_r) F   ([M] enters through P_r only)
* equilibrium:         ln K_c,i = -sum_k dnu_ki g_k/(RT) + dnu_i ln(p0 / (R T)),
                       dnu = nu'' - nu', dnu_i = sum_k dnu_ki;  k_r = k_f / K_c
* rates of progress:   q_i = k_f,i prod_k C_k^nu'_ki - k_r,i prod_k C_k^nu''_ki
* production:          w_k = sum_i dnu_ki q_i
* heat release:        hrr = -sum_k h_k w_k with h_k the full NASA molar enthalpy
                       (positive when exothermic)
* mass residual:       r_mass = sum_k W_k w_k (zero for element-balanced reactions)

Pinned by: hand-computed single-reaction values, the Lindemann and Troe-centre
limits, efficiency scaling, detailed balance at the Gibbs minimum (equil.py),
element and mass conservation, mechanism additivity and permutation equivariance.
"""
from __future__ import annotations

import numpy as np

from . import rates
from .thermo import mixture_state, nasa7


def rates_of_progress(m, T, p, Y):
    """Per-reaction quantities, each [n, Nr]:

    kf  forward rate constant (falloff-blended, PLOG- or Chebyshev-evaluated)
    kr  reverse rate constant: kf / Kc, the explicit reverse expression, or 0
    lnKc
    M   third-body concentration sum_k eps_ik C_k (all reactions; used by three-body/falloff)
    qf, qr   forward / reverse rates including the [M] factor of three-body reactions,
             with the forward orders of rates.forward_orders
    q   net rate qf - qr
    """
    T = np.asarray(T)
    Y = np.asarray(Y)
    n = T.shape[0]
    p = np.broadcast_to(np.asarray(p), T.shape)
    Wbar, rho, X, C = mixture_state(m, T, p, Y)
    _, _, _, gRT = nasa7(m, T)
    nr = m.n_reactions
    dtype = np.result_type(T, Y, np.asarray(p), float)
    out = {k: np.zeros((n, nr), dtype=dtype) for k in ("kf", "kr", "lnKc", "M", "qf", "qr", "q")}
    dnu = m.nu_r - m.nu_f
    lnp0RT = np.log(m.p0 / (m.R * T))
    M_all = C @ m.eff.T                                      # [n, Nr]
    for i in range(nr):
        M = M_all[:, i]
        kf, dkf, dkM = rates.forward(m, i, T, p, M)
        lnKc = -(gRT * dnu[i][None, :]).sum(axis=1) + dnu[i].sum() * lnp0RT
        kr, _, _ = rates.reverse(m, i, T, kf, dkf, dkM, lnKc, 0.0 * T)
        pf = np.ones(n, dtype=dtype)
        pr = np.ones(n, dtype=dtype)
        for k, o in rates.forward_orders(m, i).items():
            pf = pf * rates.power(C[:, k], o)
        for k in np.nonzero(m.nu_r[i])[0]:
            pr = pr * C[:, k] ** int(m.nu_r[i, k])
        fac = M if m.kind[i] == "threebody" else 1.0
        qf = fac * kf * pf
        qr = fac * kr * pr
        for key, val in (("kf", kf), ("kr", kr), ("lnKc", lnKc), ("M", M), ("qf", qf), ("qr", qr),
                         ("q", qf - qr)):
            out[key][:, i] = val
    return out


def production_rates(m, T, p, Y):
    """dict(wdot [n,Ns] kmol/(m^3 s), hrr [n] W/m^3, r_mass [n] kg/(m^3 s), turnover [n,Ns])."""
    T = np.asarray(T)
    r = rates_of_progress(m, T, p, Y)
    dnu = m.nu_r - m.nu_f                                   # [Nr, Ns]
    wdot = r["q"] @ dnu                                     # sum_i dnu_ki q_i
    _, hRT, _, _ = nasa7(m, T)
    h = m.R * T[:, None] * hRT
    hrr = -(h * wdot).sum(axis=1)
    r_mass = wdot @ m.W
    turnover = (np.abs(r["qf"]) + np.abs(r["qr"])) @ np.abs(dnu)
    return {"wdot": wdot, "hrr": hrr, "r_mass": r_mass, "turnover": turnover, "q": r["q"],
            "qf": r["qf"], "qr": r["qr"]}
