"""Point-wise chemistry source terms of the thermochemistry subsystem (oracle).

Section 2, Eq. (1a)-(1b), keeps only the terms that involve no spatial derivative
(a homogeneous mixture at the point): with the molar production rates w_k of
kinetics.py (kmol/(m^3 s)), the heat-release rate hrr = -sum_k h_k w_k and the
thermodynamic-pressure rate dp0/dt (an input; zero for an open domain),

    dY_k/dt = W_k w_k / rho                            (Eq. (1a); w_k in mass units is W_k w_k)
    dT/dt   = (hrr + dp0/dt) / (rho c_p)               (Eq. (1b); c_p per unit mass)

and the point-wise part of the divergence constraint, Eq. (3), evaluated with
these two rates in place of the material derivatives:

    Q_T = (1/T) dT/dt + sum_k (Wbar / W_k) dY_k/dt - (1/p0) dp0/dt.

Pinned by: mass conservation (sum_k dY_k/dt = 0 for an element-balanced
mechanism), enthalpy conservation at constant pressure (d h_mass/dt = 0 along the
source), and Q_T = -(1/rho) d rho/dt along the source, taken by a complex step of
the ideal-gas density of Eq. (1d) (independent of the Q_T formula).
"""
from __future__ import annotations

import numpy as np

from .kinetics import production_rates
from .thermo import thermo_properties


def chemistry_source(m, T, p, Y, dp0dt=None):
    """dict(dYdt [n, Ns] 1/s, dTdt [n] K/s, QT [n] 1/s, rho [n], cp_mass [n], wdot, hrr)."""
    T = np.asarray(T)
    p = np.broadcast_to(np.asarray(p, dtype=float), T.shape)
    Y = np.asarray(Y)
    r = production_rates(m, T, p, Y)
    th = thermo_properties(m, T, p, Y)
    rho, cp, Wbar = th["rho"], th["cp_mass"], th["Wbar"]
    dp = np.zeros_like(T, dtype=float) if dp0dt is None else np.broadcast_to(np.asarray(dp0dt, float), T.shape)
    dYdt = r["wdot"] * m.W[None, :] / rho[:, None]
    dTdt = (r["hrr"] + dp) / (rho * cp)
    QT = dTdt / T + (Wbar[:, None] / m.W[None, :] * dYdt).sum(axis=1) - dp / p
    return {"dYdt": dYdt, "dTdt": dTdt, "QT": QT, "rho": rho, "cp_mass": cp,
            "wdot": r["wdot"], "hrr": r["hrr"]}
