"""Mixture-averaged transport properties (oracle).

The paper's transport model is mixture-averaged, without Soret or Dufour effects,
with the diffusion velocity V_k = -(D_k / X_k) grad X_k + V_c (Eq. (2)); the
mixture viscosity mu enters Eq. (4) and the conductivity lambda Eq. (1b).  The
standard mixture-averaged definitions (Chemkin/Cantera):

* pure-species fits (cubic in ln T):  ln mu_k = sum_m a_km (ln T)^m,
  ln lambda_k likewise, ln D_jk = sum_m d_jkm (ln T)^m + ln(p0 / p) (binary, symmetric)
* Wilke:   mu = sum_k X_k mu_k / sum_j X_j Phi_kj,
           Phi_kj = (1/sqrt 8) (1 + W_k/W_j)^(-1/2) [1 + (mu_k/mu_j)^(1/2) (W_j/W_k)^(1/4)]^2
* Mathur-Saxena:   lambda = (sum_k X_k lambda_k + 1 / sum_k (X_k / lambda_k)) / 2
* Hirschfelder-Curtiss, in the mole-fraction-gradient form of Eq. (2):
           D_k = (1 - Y_k) / sum_{j != k} (X_j / D_jk)

Pinned by: pure-species limits (Phi_kk = 1 exactly), identical species, trace
species in a pure bath (D_k -> D_kj), the binary closed form D_1 = D_12 Y_2 / X_2,
D proportional to 1/p, mu and lambda independent of p.
"""
from __future__ import annotations

import numpy as np

from .thermo import mixture_state


def _poly3(c, L):
    return c[..., 0] + c[..., 1] * L + c[..., 2] * L ** 2 + c[..., 3] * L ** 3


def species_transport(m, T, p):
    """mu_k, lambda_k [n, Ns] and D_jk [n, Ns, Ns] (diagonal left at zero)."""
    T = np.asarray(T)
    p = np.asarray(p)
    L = np.log(T)[:, None]
    mu_k = np.exp(_poly3(m.mu_fit[None, :, :], L))
    lam_k = np.exp(_poly3(m.lam_fit[None, :, :], L))
    ns = m.n_species
    D = np.zeros((T.shape[0], ns, ns), dtype=np.result_type(T, p, float))
    lnp = np.log(m.p0 / p)
    for j in range(ns):
        for k in range(j + 1, ns):
            d = np.exp(_poly3(m.dif_fit[j, k], np.log(T)) + lnp)
            D[:, j, k] = d
            D[:, k, j] = d
    return mu_k, lam_k, D


def transport_properties(m, T, p, Y):
    """dict(mu [n] Pa s, lambda [n] W/(m K), Dmix [n, Ns] m^2/s)."""
    Y = np.asarray(Y)
    _, _, X, _ = mixture_state(m, T, p, Y)
    mu_k, lam_k, D = species_transport(m, T, p)
    W = m.W
    ns = m.n_species
    phi = np.zeros((X.shape[0], ns, ns), dtype=mu_k.dtype)
    for k in range(ns):
        for j in range(ns):
            phi[:, k, j] = (1.0 / np.sqrt(8.0)) * (1.0 + W[k] / W[j]) ** -0.5 * \
                (1.0 + np.sqrt(mu_k[:, k] / mu_k[:, j]) * (W[j] / W[k]) ** 0.25) ** 2
    mu = (X * mu_k / np.einsum("nkj,nj->nk", phi, X)).sum(axis=1)
    lam = 0.5 * ((X * lam_k).sum(axis=1) + 1.0 / (X / lam_k).sum(axis=1))
    Dmix = np.zeros_like(X)
    for k in range(ns):
        s = 0.0
        for j in range(ns):
            if j != k:
                s = s + X[:, j] / D[:, j, k]
        Dmix[:, k] = (1.0 - Y[:, k]) / s
    return {"mu": mu, "lambda": lam, "Dmix": Dmix}
