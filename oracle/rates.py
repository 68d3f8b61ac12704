"""Rate constants of one reaction in every form the mechanism format allows (oracle).

The paper takes its kinetics from a Cantera-format mechanism (Section 2); these are the
standard definitions of the rate forms such a mechanism uses, in SI-kmol units:

* Arrhenius:   k = A T^b exp(-theta/T);  d ln k/dT = (b + theta/T)/T.
* falloff:     k0 (low-pressure Arrhenius), kinf (the reaction's Arrhenius), P_r = k0 [M]/kinf,
               k_f = kinf P_r/(1 + P_r) F with the broadening factor F of
               - troe: the Gilbert-Luther-Troe form with F_cent = (1-alpha) e^(-T/T3)
                 + alpha e^(-T/T1) + e^(-T2/T), c = -0.4 - 0.67 log10 F_cent,
                 n = 0.75 - 1.27 log10 F_cent, d = 0.14, f1 = (log10 P_r + c)/(n - d (log10 P_r + c)),
                 log10 F = log10 F_cent / (1 + f1^2);
               - lindemann: F = 1;
               - sri: F = d (a exp(-b/T) + exp(-T/c))^X T^e,  X = 1/(1 + (log10 P_r)^2).
* plog:        Arrhenius expressions k_j at pressures p_j (ascending); at p_j <= p <= p_{j+1}
               ln k is linear in ln p between ln k_j and ln k_{j+1}; below p_1 and above the
               last pressure the end expression applies.
* chebyshev:   log10 k = sum_t sum_q alpha_tq T_t(Tr) T_q(Pr), T_n the Chebyshev polynomials,
               Tr = (2/T - 1/Tmin - 1/Tmax)/(1/Tmax - 1/Tmin),
               Pr = (2 log10 p - log10 Pmin - log10 Pmax)/(log10 Pmax - log10 Pmin).
* reverse:     k_r = k_f / K_c, or an explicit reverse Arrhenius expression, or 0 for an
               irreversible reaction.
* orders:      forward rate k_f prod_k C_k^(o_k) with the given (possibly non-integer) orders
               of the reactants; the stoichiometry of the production rates is unchanged.

Each function returns the value and its temperature derivative at fixed p and [M] (and
the [M] derivative for falloff); p is never differentiated.  All work on complex T and
concentrations (complex-step differentiation), comparing real parts only.

Pinned by (tests/test_oracle_variants.py): PLOG at a tabulated pressure and midway in
ln p (geometric mean), clamping beyond the table; Chebyshev single-coefficient cases and
the closed form of a first-degree expansion in 1/T (an Arrhenius law); SRI at P_r = 1
(X = 1) and its d, e scaling; Lindemann's k0 [M] and kinf limits; explicit-reverse and
irreversible single-reaction rates by hand; fractional orders by hand; complex-step
derivatives of every form.
"""
from __future__ import annotations

import numpy as np

LN10 = np.log(10.0)
FALLOFF = ("troe", "lindemann", "sri")


def arrhenius(lnA, b, theta, T):
    return np.exp(lnA) * T ** b * np.exp(-theta / T)


def dlnk_dT(b, theta, T):
    return (b + theta / T) / T


def _log10_guard(x):
    return np.log10(np.where(np.real(x) < 1e-300, 1e-300, x))


def broadening(kind, T, Pr, troe=None, sri=None):
    """(F, d log10 F / d log10 P_r at fixed T, d log10 F / dT at fixed P_r)."""
    if kind == "lindemann":
        one = np.ones_like(T * Pr)
        return one, 0.0 * one, 0.0 * one
    ell = _log10_guard(Pr)
    if kind == "sri":
        a, b, c, d, e = sri
        S = a * np.exp(-b / T) + np.exp(-T / c)
        dS = a * b / T ** 2 * np.exp(-b / T) - np.exp(-T / c) / c
        X = 1.0 / (1.0 + ell ** 2)
        F = d * S ** X * T ** e
        dlogF_dell = -2.0 * ell * X ** 2 * np.log10(S)
        dlogF_dT = (X * dS / S + e / T) / LN10
        return F, dlogF_dell, dlogF_dT
    # troe
    _, _, _, alpha, T3, T1, T2 = troe
    Fcent = (1.0 - alpha) * np.exp(-T / T3) + alpha * np.exp(-T / T1) + np.exp(-T2 / T)
    dFcent = -(1.0 - alpha) / T3 * np.exp(-T / T3) - alpha / T1 * np.exp(-T / T1) + T2 / T ** 2 * np.exp(-T2 / T)
    lFc = _log10_guard(Fcent)
    c = -0.4 - 0.67 * lFc
    n = 0.75 - 1.27 * lFc
    d = 0.14
    u = ell + c
    den = n - d * u
    f1 = u / den
    g = 1.0 / (1.0 + f1 ** 2)
    F = 10.0 ** (lFc * g)
    df1_dell = n / den ** 2
    df1_dlFc = (-0.67 * den - u * (-1.27 + 0.67 * d)) / den ** 2
    dlogF_dell = -lFc * 2.0 * f1 * df1_dell * g ** 2
    dlogF_dlFc = g - lFc * 2.0 * f1 * df1_dlFc * g ** 2
    return F, dlogF_dell, dlogF_dlFc * dFcent / (Fcent * LN10)


def plog(entries, T, p):
    """(k, d ln k/dT) of a PLOG expression at (T, p); p real."""
    lnp = np.log(np.real(p))
    P = np.array([e[0] for e in entries])
    lk = [e[1] + e[2] * np.log(T) - e[3] / T for e in entries]
    dk = [dlnk_dT(e[2], e[3], T) for e in entries]
    lnk = np.zeros_like(lk[0])
    dln = np.zeros_like(dk[0])
    lnP = np.log(P)
    j = np.clip(np.searchsorted(lnP, lnp, side="right") - 1, 0, max(len(P) - 2, 0))
    for jj in range(len(P)):
        if len(P) == 1:
            sel = np.ones_like(lnp, dtype=bool)
            w = np.zeros_like(lnp)
        else:
            sel = j == jj
            if jj == len(P) - 1:
                continue
            w = np.clip((lnp - lnP[jj]) / (lnP[jj + 1] - lnP[jj]), 0.0, 1.0)
        nxt = min(jj + 1, len(P) - 1)
        lnk = np.where(sel, (1 - w) * lk[jj] + w * lk[nxt], lnk)
        dln = np.where(sel, (1 - w) * dk[jj] + w * dk[nxt], dln)
    return np.exp(lnk), dln


def _cheb_polys(x, n):
    """T_0..T_{n-1}(x) and their derivatives (T_t' = t U_{t-1})."""
    Tn = [np.ones_like(x), x]
    U = [np.ones_like(x), 2 * x]
    for t in range(2, n):
        Tn.append(2 * x * Tn[-1] - Tn[-2])
        U.append(2 * x * U[-1] - U[-2])
    dT = [np.zeros_like(x)] + [t * U[t - 1] for t in range(1, n)]
    return Tn[:n], dT[:n]


def chebyshev(cheb, T, p):
    """(k, d ln k/dT) of a Chebyshev expression at (T, p); p real."""
    Tmin, Tmax, Pmin, Pmax, alpha = cheb
    nT, nP = alpha.shape
    Tr = (2.0 / T - 1.0 / Tmin - 1.0 / Tmax) / (1.0 / Tmax - 1.0 / Tmin)
    dTr = -2.0 / T ** 2 / (1.0 / Tmax - 1.0 / Tmin)
    Pr = (2.0 * np.log10(np.real(p)) - np.log10(Pmin) - np.log10(Pmax)) / (np.log10(Pmax) - np.log10(Pmin))
    phT, dphT = _cheb_polys(Tr, nT)
    phP, _ = _cheb_polys(Pr + 0.0 * Tr.real, nP)
    lg = 0.0 * Tr
    dlg = 0.0 * Tr
    for t in range(nT):
        for q in range(nP):
            lg = lg + alpha[t, q] * phT[t] * phP[q]
            dlg = dlg + alpha[t, q] * dphT[t] * phP[q]
    return 10.0 ** lg, LN10 * dlg * dTr


def forward(m, i, T, p, M):
    """(k_f, dk_f/dT at fixed p and [M], dk_f/d[M] at fixed T) of reaction i ([M] enters falloff only)."""
    kind = m.kind[i]
    ex = m.extra[i] if m.extra else {}
    if kind == "plog":
        k, d = plog(ex["plog"], T, p)
        return k, k * d, 0.0 * k
    if kind == "chebyshev":
        k, d = chebyshev(ex["cheb"], T, p)
        return k, k * d, 0.0 * k
    kinf = arrhenius(m.lnA[i], m.b[i], m.theta[i], T)
    dinf = dlnk_dT(m.b[i], m.theta[i], T)
    if kind not in FALLOFF:
        return kinf, kinf * dinf, 0.0 * kinf
    lnA0, b0, th0 = (m.troe[i][:3] if kind == "troe" else ex["k0"])
    k0 = arrhenius(lnA0, b0, th0, T)
    Pr = k0 * M / kinf
    F, dF_dell, dF_dT = broadening(kind, T, Pr, troe=m.troe[i], sri=ex.get("sri"))
    kf = kinf * Pr / (1.0 + Pr) * F
    dlnPr = dlnk_dT(b0, th0, T) - dinf
    # d ln F/dT = LN10 (dlog10F/dell dell/dT + dlog10F/dT), dell/dT = dlnPr / LN10
    dlnF = dF_dell * dlnPr + LN10 * dF_dT
    dkf_dT = kf * (dinf + dlnPr / (1.0 + Pr) + dlnF)
    # d ln k_f / d ln P_r = 1/(1 + P_r) + dlog10F/dell,  k_f / [M] = k0 F / (1 + P_r)
    dkf_dM = k0 * F / (1.0 + Pr) * (1.0 / (1.0 + Pr) + dF_dell)
    return kf, dkf_dT, dkf_dM


def reverse(m, i, T, kf, dkf_dT, dkf_dM, lnKc, dlnKc_dT):
    """(k_r, [terms of dk_r/dT], dk_r/d[M]); the terms sum to dk_r/dT (kept apart for the
    gross Jacobian)."""
    ex = m.extra[i] if m.extra else {}
    if ex.get("irreversible"):
        z = 0.0 * kf
        return z, [], z
    if "reverse" in ex:
        lnA, b, th = ex["reverse"]
        kr = arrhenius(lnA, b, th, T)
        return kr, [kr * dlnk_dT(b, th, T)], 0.0 * kr
    invKc = np.exp(-lnKc)
    kr = kf * invKc
    return kr, [dkf_dT * invKc, -kr * dlnKc_dT], dkf_dM * invKc


def forward_orders(m, i):
    """{species: order} of the forward rate law (stoichiometric coefficients unless given)."""
    ex = m.extra[i] if m.extra else {}
    o = {int(k): float(m.nu_f[i, k]) for k in np.nonzero(m.nu_f[i])[0]}
    o.update({int(k): float(v) for k, v in ex.get("orders", {}).items()})
    return o


def power(C, o):
    """C^o, with integer orders as plain integer powers."""
    return C ** int(o) if float(o).is_integer() else C ** o


def dpower(C, o):
    """d(C^o)/dC = o C^(o-1)."""
    return o * (C ** int(o - 1) if float(o).is_integer() else C ** (o - 1.0))
