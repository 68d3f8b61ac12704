"""Analytic Jacobian and vector-Jacobian product of (hrr, w_1..w_Ns) w.r.t. (T, Y_1..Y_Ns) (oracle).

The paper's integrator needs derivatives of the chemistry source in every Newton
and Krylov iteration; it approximates J v by difference quotients (Section 2).
The oracle differentiates the production rates of kinetics.py exactly, by the
chain rule, with plain loops over reactions:

* rows:    0 = hrr, 1..Ns = w_k;  columns: 0 = T, 1..Ns = Y_j (p fixed, every Y_j
  independent, no renormalisation);
* dC_m/dY_j = delta_mj rho / W_m - C_m Wbar / W_j   and   dC_m/dT = -C_m / T;
* d ln k/dT = (b + theta/T) / T for an Arrhenius constant;
* d(g/RT)/dT = -(h/RT) / T, hence d ln K_c/dT = (sum_k dnu_k h_k/(RT) - dnu) / T;
* Troe: closed-form derivatives of F through P_r and F_cent;
* d hrr/dx = -sum_k h_k dw_k/dx, plus -sum_k cp_k w_k for x = T (dh_k/dT = cp_k).

Pinned by: complex-step differentiation of the forward oracle (exact to rounding),
central finite differences, and the dot-product identity of the VJP.
"""
from __future__ import annotations

import numpy as np

from . import rates
from .kinetics import production_rates
from .thermo import mixture_state, nasa7

def jacobian(m, T, p, Y, return_gross=False):
    """J [n, Ns+1, Ns+1]: rows (hrr, w_1..Ns), columns (T, Y_1..Ns).

    With return_gross, also the gross magnitude G of every entry: the same chain
    rule with every reaction's contribution taken in absolute value,
    G_kx = sum_i |dnu_ki| |dq_i/dx| (each chain-rule term separately), row 0 =
    sum_k |h_k| G_kx (+ sum_k |cp_k w_k| for x = T).  G bounds the rounding of any
    summation order of J the way the gross turnover bounds that of w.
    """
    T = np.asarray(T)
    p = np.asarray(p)
    Y = np.asarray(Y)
    n, ns = Y.shape
    Wbar, rho, X, C = mixture_state(m, T, p, Y)
    cpR, hRT, _, gRT = nasa7(m, T)
    dnu = m.nu_r - m.nu_f
    lnp0RT = np.log(m.p0 / (m.R * T))
    dtype = np.result_type(T, Y, p, float)
    JC = np.zeros((n, ns, ns), dtype=dtype)      # d w_k / d C_j
    JTC = np.zeros((n, ns), dtype=dtype)         # d w_k / d T at fixed C
    if return_gross:
        GY = np.zeros((n, ns, ns))
        GT = np.zeros((n, ns))
    for i in range(m.n_reactions):
        M = C @ m.eff[i]
        kf, dkf_dT, dkf_dM = rates.forward(m, i, T, p, M)
        lnKc = -(gRT * dnu[i][None, :]).sum(axis=1) + dnu[i].sum() * lnp0RT
        dlnKc_dT = ((hRT * dnu[i][None, :]).sum(axis=1) - dnu[i].sum()) / T
        kr, dkr_terms, dkr_dM = rates.reverse(m, i, T, kf, dkf_dT, dkf_dM, lnKc, dlnKc_dT)
        dkr_dT = sum(dkr_terms) if dkr_terms else 0.0 * kf
        orders = rates.forward_orders(m, i)
        prod = np.nonzero(m.nu_r[i])[0]
        pf = np.ones(n, dtype=dtype)
        pr = np.ones(n, dtype=dtype)
        for k, o in orders.items():
            pf = pf * rates.power(C[:, k], o)
        for k in prod:
            pr = pr * C[:, k] ** int(m.nu_r[i, k])
        # d(prod_k C_k^o_k)/dC_j for each j of the product (no division by C)
        dpf = {}
        for j, oj in orders.items():
            v = rates.dpower(C[:, j], oj)
            for k, o in orders.items():
                if k != j:
                    v = v * rates.power(C[:, k], o)
            dpf[j] = v
        dpr = {}
        for j in prod:
            v = m.nu_r[i, j] * C[:, j] ** int(m.nu_r[i, j] - 1)
            for k in prod:
                if k != j:
                    v = v * C[:, k] ** int(m.nu_r[i, k])
            dpr[j] = v
        falloff = m.kind[i] in rates.FALLOFF
        fac = M if m.kind[i] == "threebody" else np.ones_like(M)
        dq_dC = np.zeros((n, ns), dtype=dtype)
        for j, v in dpf.items():
            dq_dC[:, j] += fac * kf * v
        for j, v in dpr.items():
            dq_dC[:, j] -= fac * kr * v
        # [M] = sum_k eps_k C_k: the whole rate for three-body reactions, k_f (and k_r) for falloff
        dq_dM = (kf * pf - kr * pr) if m.kind[i] == "threebody" else \
            (dkf_dM * pf - dkr_dM * pr) if falloff else np.zeros_like(kf)
        dq_dC += dq_dM[:, None] * m.eff[i][None, :]
        dq_dT = fac * (dkf_dT * pf - dkr_dT * pr)
        JC += dnu[i][None, :, None] * dq_dC[:, None, :]
        JTC += dnu[i][None, :] * dq_dT[:, None]
        if return_gross:
            a = np.zeros((n, ns))
            for j, v in dpf.items():
                a[:, j] += np.abs(fac * kf * v)
            for j, v in dpr.items():
                a[:, j] += np.abs(fac * kr * v)
            if m.kind[i] == "threebody":
                a += (np.abs(kf * pf) + np.abs(kr * pr))[:, None] * m.eff[i][None, :]
            elif falloff:
                a += (np.abs(dkf_dM * pf) + np.abs(dkr_dM * pr))[:, None] * m.eff[i][None, :]
            sig = (a * C).sum(axis=1)
            tabs = np.abs(fac) * (np.abs(dkf_dT * pf) + sum(np.abs(t * pr) for t in dkr_terms))
            gy = rho[:, None] * a / m.W[None, :] + (Wbar[:, None] / m.W[None, :]) * sig[:, None]
            GY += np.abs(dnu[i])[None, :, None] * gy[:, None, :]
            GT += np.abs(dnu[i])[None, :] * (tabs + sig / T)[:, None]
    # chain rule to (T, Y)
    dC_dY = rho[:, None, None] * np.eye(ns)[None] / m.W[None, :, None] \
        - C[:, :, None] * (Wbar[:, None] / m.W[None, :])[:, None, :]          # [n, m, j]
    JY = np.einsum("nkm,nmj->nkj", JC, dC_dY)
    JT = JTC - np.einsum("nkm,nm->nk", JC, C) / T[:, None]
    w = production_rates(m, T, p, Y)["wdot"]
    h = m.R * T[:, None] * hRT
    cp = m.R * cpR
    J = np.zeros((n, ns + 1, ns + 1), dtype=dtype)
    J[:, 1:, 0] = JT
    J[:, 1:, 1:] = JY
    J[:, 0, 0] = -(h * JT).sum(axis=1) - (cp * w).sum(axis=1)
    J[:, 0, 1:] = -np.einsum("nk,nkj->nj", h, JY)
    if not return_gross:
        return J
    G = np.zeros((n, ns + 1, ns + 1))
    G[:, 1:, 0] = GT
    G[:, 1:, 1:] = GY
    G[:, 0, 0] = (np.abs(h) * GT).sum(axis=1) + np.abs(cp * w).sum(axis=1)
    G[:, 0, 1:] = np.einsum("nk,nkj->nj", np.abs(h), GY)
    return J, G


def vjp(m, T, p, Y, u, u_hrr=None):
    """(gT [n], gY [n, Ns]) = u^T J with u [n, Ns] the cotangent of w and u_hrr [n] of hrr."""
    J = jacobian(m, T, p, Y)
    n = J.shape[0]
    uu = np.concatenate([np.zeros((n, 1)) if u_hrr is None else np.asarray(u_hrr)[:, None],
                         np.asarray(u)], axis=1)
    g = np.einsum("nr,nrc->nc", uu, J)
    return g[:, 0], g[:, 1:]


def jvp(m, T, p, Y, vT, vY):
    """(jv_hrr [n], jv_w [n, Ns]) = J v for the tangent v = (vT [n], vY [n, Ns]) of (T, Y).

    The forward-mode derivative of (hrr, w) along v: the plain product of the
    analytic Jacobian with v.  Pinned by complex-step differentiation of the
    forward oracle along v (complex_step_jvp).
    """
    J = jacobian(m, T, p, Y)
    v = np.concatenate([np.asarray(vT)[:, None], np.asarray(vY)], axis=1)
    jv = np.einsum("nrc,nc->nr", J, v)
    return jv[:, 0], jv[:, 1:]


def complex_step_jvp(m, T, p, Y, vT, vY, h=1e-30):
    """J v by one complex step of the forward oracle along v: Im f(x + i h v) / h."""
    T = np.asarray(T, dtype=float)
    Y = np.asarray(Y, dtype=float)
    f = _forward_vector(m, T + 1j * h * np.asarray(vT), p, Y + 1j * h * np.asarray(vY)).imag / h
    return f[:, 0], f[:, 1:]


def _forward_vector(m, T, p, Y):
    r = production_rates(m, T, p, Y)
    return np.concatenate([r["hrr"][:, None], r["wdot"]], axis=1)


def complex_step_jacobian(m, T, p, Y, h=1e-30):
    """Jacobian by complex-step differentiation of the forward oracle (exact to rounding)."""
    T = np.asarray(T, dtype=float)
    Y = np.asarray(Y, dtype=float)
    n, ns = Y.shape
    J = np.zeros((n, ns + 1, ns + 1))
    for c in range(ns + 1):
        Tc = T.astype(complex)
        Yc = Y.astype(complex)
        if c == 0:
            step = h * T
            Tc = Tc + 1j * step
        else:
            step = np.full(n, h)
            Yc[:, c - 1] = Yc[:, c - 1] + 1j * step
        J[:, :, c] = _forward_vector(m, Tc, p, Yc).imag / step[:, None]
    return J


def central_fd_jacobian(m, T, p, Y, rel=1e-6, y_floor=1e-10):
    """Central finite differences, h_T = rel*T, h_j = rel*max(Y_j, y_floor)."""
    T = np.asarray(T, dtype=float)
    Y = np.asarray(Y, dtype=float)
    n, ns = Y.shape
    J = np.zeros((n, ns + 1, ns + 1))
    for c in range(ns + 1):
        if c == 0:
            hh = rel * T
            fp = _forward_vector(m, T + hh, p, Y)
            fm = _forward_vector(m, T - hh, p, Y)
        else:
            hh = rel * np.maximum(Y[:, c - 1], y_floor)
            Yp = Y.copy(); Yp[:, c - 1] += hh
            Ym = Y.copy(); Ym[:, c - 1] -= hh
            fp = _forward_vector(m, T, p, Yp)
            fm = _forward_vector(m, T, p, Ym)
        J[:, :, c] = (fp - fm) / (2.0 * hh[:, None])
    return J
