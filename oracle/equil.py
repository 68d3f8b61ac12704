"""Chemical equilibrium by Gibbs minimisation at fixed T, p and element totals (oracle).

Used to build near-equilibrium test states and to pin the equilibrium constants
of kinetics.py (detailed balance: every rate of progress vanishes at the minimum).

Minimises  G/(RT) = sum_k n_k [g_k/(RT) + ln(p/p0) + ln(n_k/N)]  subject to
sum_k a_ek n_k = b_e, N = sum_k n_k, with the element-potential Newton iteration of
the classical free-energy-minimisation method (White, Johnson and Dantzig; the
"RAND" form used by Gordon and McBride): each step solves for the element
potentials pi_e and d ln N,

    sum_e' (sum_k a_ek a_e'k n_k) pi_e' + (sum_k a_ek n_k) dlnN = b_e - sum_k a_ek n_k + sum_k a_ek n_k mu_k
    sum_e  (sum_k a_ek n_k) pi_e + (sum_k n_k - N) dlnN        = N - sum_k n_k + sum_k n_k mu_k

with mu_k = g_k/(RT) + ln(p/p0) + ln(n_k/N), then d ln n_k = -mu_k + sum_e a_ek pi_e + dlnN,
damped so that no ln n_k moves by more than 2 per step.  The iteration works on
ln n_k throughout, so trace species down to exp(-700) stay representable.

Pinned by: the isomer closed form x_B/x_A = exp(-(g_B - g_A)/RT), the dissociation
closed form for A2 = 2A, element conservation, and the stationarity conditions
mu_k = sum_e a_ek pi_e for every species.
"""
from __future__ import annotations

import numpy as np

from .thermo import nasa7


def equilibrate(m, T, p, Y0, tol=1e-14, max_iter=2000):
    """Equilibrium mass fractions Y [Ns] at (T, p) with the element totals of Y0 [Ns].

    Returns (Y, info) where info has the element potentials 'pi' [Ne], 'iterations',
    and 'mu' (the final mu_k = g_k/RT + ln(p/p0) + ln x_k).
    """
    T = float(T)
    p = float(p)
    Y0 = np.asarray(Y0, dtype=float)
    A = m.comp.T.astype(float)                          # [Ne, Ns]
    b = A @ (Y0 / m.W)                                  # kmol of element per kg
    present_el = b > 0
    # species made only of present elements
    sp = np.all((m.comp[:, ~present_el] == 0), axis=1)
    A = A[present_el][:, sp]
    b = b[present_el]
    _, _, _, gRT = nasa7(m, np.array([T]))
    mu0 = gRT[0, sp] + np.log(p / m.p0)
    ns = A.shape[1]
    ne = A.shape[0]
    N = float((Y0 / m.W).sum())
    lnn = np.full(ns, np.log(N / ns))
    lnN = np.log(N)
    pi = np.zeros(ne)
    it = 0
    for it in range(1, max_iter + 1):
        n = np.exp(lnn)
        Nn = np.exp(lnN)
        mu = mu0 + lnn - lnN
        G = (A * n[None, :]) @ A.T
        An = A @ n
        M = np.zeros((ne + 1, ne + 1))
        M[:ne, :ne] = G
        M[:ne, ne] = An
        M[ne, :ne] = An
        M[ne, ne] = n.sum() - Nn
        rhs = np.concatenate([b - An + A @ (n * mu), [Nn - n.sum() + (n * mu).sum()]])
        # least squares: the element rows may be linearly dependent (e.g. only isomers present)
        sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
        pi, dlnN = sol[:ne], sol[ne]
        dlnn = -mu + A.T @ pi + dlnN
        big = max(np.max(np.abs(dlnn)), abs(dlnN))
        lam = 1.0 if big <= 2.0 else 2.0 / big
        lnn = lnn + lam * dlnn
        lnN = lnN + lam * dlnN
        xw = np.exp(lnn - lnN)
        if lam == 1.0 and np.max(xw * np.abs(dlnn)) < tol and abs(dlnN) < tol:
            break
    else:
        raise RuntimeError("equilibrium iteration did not converge")
    # final state in exact element-potential form: ln x_k = a_k . pi - mu0_k, normalised
    lnx = A.T @ pi - mu0
    lnx = lnx - np.log(np.exp(lnx - lnx.max()).sum()) - lnx.max()
    x = np.exp(lnx)
    Wsp = m.W[sp]
    Ysp = x * Wsp / (x * Wsp).sum()
    Y = np.zeros(m.n_species)
    Y[sp] = Ysp
    mu_final = np.full(m.n_species, np.nan)
    mu_final[sp] = mu0 + lnx
    return Y, {"pi": pi, "iterations": it, "mu": mu_final}
