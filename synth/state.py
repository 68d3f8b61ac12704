"""Seeded synthetic thermochemical states (T, p, Y) and cotangents.

Layouts returned here are the library's: ``T[n]``, ``p[n]`` and ``Y[Ns, n]``
(species-major, point-fastest).  All draws use ``numpy.random.default_rng``.

Workload shapes follow the paper's use: the production runs evaluate the
chemistry on 7th-order spectral elements (8^3 points per element, Section 3.3),
at 40 bar for the flame-kernel case, with 0.6-7 M points per GPU (Section 4.2).
"""
from __future__ import annotations

import os

import numpy as np

P_ATM = 101325.0
ANCHOR_FILE = os.path.join(os.path.dirname(__file__), "data", "c1_equil_anchors.npz")


def dirichlet_rows(rng, n, ns, alpha):
    """[n, ns] rows drawn from a symmetric Dirichlet(alpha) (rows sum to 1)."""
    return rng.dirichlet(np.full(ns, alpha), size=n)


def state_c0(ns, n=4096, seed=0):
    """T ~ U[300, 2500] K, p = 1 atm, Y ~ Dirichlet(0.5)."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(300.0, 2500.0, size=n)
    Y = dirichlet_rows(rng, n, ns, 0.5)
    p = np.full(n, P_ATM)
    return {"T": T, "p": p, "Y": np.ascontiguousarray(Y.T)}


def c1_anchor_requests(ns, n_anchor=256, seed=11):
    """Temperatures, pressures and element-total sources for the near-equilibrium anchors.

    Each anchor is equilibrated (fixed T, p, element totals of ``Y0``) outside this
    package; the result is stored in ``ANCHOR_FILE``.
    """
    rng = np.random.default_rng(seed)
    T = rng.uniform(1500.0, 2500.0, size=n_anchor)
    p = np.where(rng.uniform(size=n_anchor) < 0.5, P_ATM, 10.0 * P_ATM)
    Y0 = dirichlet_rows(rng, n_anchor, ns, 0.3)
    return T, p, Y0


def load_anchors(path=ANCHOR_FILE):
    with np.load(path, allow_pickle=False) as z:
        return {k: np.array(z[k]) for k in ("T", "p", "Y")}


def state_c1(ns, n=1 << 20, seed=1, anchors=None, near_eq_fraction=0.10):
    """The 53-species workload state.

    90 % of the points: T ~ U[300, 2500] K, Y ~ Dirichlet(0.3).  10 %: near-equilibrium
    states obtained by cycling the stored equilibrium anchors, perturbing every
    Y_k by a factor (1 + 1e-3 N(0,1)), renormalising and jittering T by up to 0.1 K.
    p is 1 atm or 10 atm with probability 1/2 each.  Rows are shuffled; "near_eq" marks the
    near-equilibrium rows.
    """
    rng = np.random.default_rng(seed)
    if anchors is None:
        anchors = load_anchors()
    n_eq = int(round(near_eq_fraction * n))
    n_rand = n - n_eq
    T = np.empty(n)
    p = np.empty(n)
    Y = np.empty((n, ns))
    T[:n_rand] = rng.uniform(300.0, 2500.0, size=n_rand)
    p[:n_rand] = np.where(rng.uniform(size=n_rand) < 0.5, P_ATM, 10.0 * P_ATM)
    Y[:n_rand] = dirichlet_rows(rng, n_rand, ns, 0.3)
    if n_eq:
        a = np.arange(n_eq) % anchors["T"].shape[0]
        Ye = anchors["Y"][a] * (1.0 + 1e-3 * rng.standard_normal((n_eq, ns)))
        Ye = np.abs(Ye)
        Y[n_rand:] = Ye / Ye.sum(axis=1, keepdims=True)
        T[n_rand:] = anchors["T"][a] + rng.uniform(-0.1, 0.1, size=n_eq)
        p[n_rand:] = anchors["p"][a]
    perm = rng.permutation(n)
    near_eq = np.arange(n) >= n_rand
    return {"T": T[perm], "p": p[perm], "Y": np.ascontiguousarray(Y[perm].T), "near_eq": near_eq[perm]}


def state_c3_cotangent(ns, n=1 << 20, seed=3):
    """Cotangent u ~ N(0, 1) of shape [Ns, n] for the VJP."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((n, ns)).T)


def gll_nodes(n_nodes=8):
    """Gauss-Lobatto-Legendre nodes on [-1, 1] (endpoints and roots of P'_{n-1})."""
    inner = np.polynomial.legendre.Legendre.basis(n_nodes - 1).deriv().roots()
    return np.sort(np.concatenate([[-1.0], np.real(inner), [1.0]]))


def c4_element_counts(seed=4, n_launch=8):
    """Uneven element counts per launch, U{1000..8000}, always containing 1000 and 8000."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(1000, 8001, size=n_launch)
    counts[0], counts[-1] = 1000, 8000
    return [int(c) for c in counts]


def state_c4_launch(ns, n_elements, seed=4, launch=0, p_pa=40.0 * P_ATM):
    """Points of ``n_elements`` spectral elements of 8^3 GLL nodes, lexicographic (i fastest).

    Per element: T = 300 + 2100 * (1 + tanh((n.x - d)/delta))/2 with a random unit
    normal n, d ~ U[-1.2, 1.2], delta ~ logU[0.05, 1]; Y = (1 - c) Y_u + c Y_b with
    c = (T - 300)/2100 and Y_u, Y_b ~ Dirichlet(0.3) per element; p = 40 atm.
    """
    rng = np.random.default_rng([seed, launch])
    x1 = gll_nodes(8)
    zz, yy, xx = np.meshgrid(x1, x1, x1, indexing="ij")
    X = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)          # [512, 3], i fastest
    nrm = rng.standard_normal((n_elements, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    d = rng.uniform(-1.2, 1.2, size=n_elements)
    delta = np.exp(rng.uniform(np.log(0.05), np.log(1.0), size=n_elements))
    s = (nrm @ X.T - d[:, None]) / delta[:, None]                      # [E, 512]
    T = 300.0 + 2100.0 * 0.5 * (1.0 + np.tanh(s))
    c = (T - 300.0) / 2100.0
    Yu = dirichlet_rows(rng, n_elements, ns, 0.3)
    Yb = dirichlet_rows(rng, n_elements, ns, 0.3)
    Y = (1.0 - c)[:, :, None] * Yu[:, None, :] + c[:, :, None] * Yb[:, None, :]
    n = n_elements * 512
    return {"T": T.reshape(n), "p": np.full(n, p_pa),
            "Y": np.ascontiguousarray(Y.reshape(n, ns).T)}


def state_c4_launch_device(ns, n_elements, seed=4, launch=0, p_pa=40.0 * P_ATM, device="cuda"):
    """state_c4_launch's recipe with its per-element draws taken from the same generator in
    the same order, and the [E x 512 x Ns] fields formed on the device with torch (for
    launches of thousands of elements; the per-point values agree with state_c4_launch to
    the rounding of tanh).  Returns torch tensors T [n], p [n], Y [Ns, n] (FP64)."""
    import torch
    rng = np.random.default_rng([seed, launch])
    x1 = gll_nodes(8)
    zz, yy, xx = np.meshgrid(x1, x1, x1, indexing="ij")
    X = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    nrm = rng.standard_normal((n_elements, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    d = rng.uniform(-1.2, 1.2, size=n_elements)
    delta = np.exp(rng.uniform(np.log(0.05), np.log(1.0), size=n_elements))
    Yu = dirichlet_rows(rng, n_elements, ns, 0.3)
    Yb = dirichlet_rows(rng, n_elements, ns, 0.3)
    dev = torch.device(device)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    s_ = (t(nrm) @ t(X).T - t(d)[:, None]) / t(delta)[:, None]        # [E, 512]
    T = 300.0 + 2100.0 * 0.5 * (1.0 + torch.tanh(s_))
    c = ((T - 300.0) / 2100.0).reshape(-1)                             # [n]
    n = n_elements * 512
    Yu_d, Yb_d = t(Yu.T.copy()), t(Yb.T.copy())                        # [Ns, E]
    Y = torch.empty((ns, n), dtype=torch.float64, device=dev)
    for k in range(ns):                                                # [Ns, n] species-major
        Y[k] = (1.0 - c) * Yu_d[k].repeat_interleave(512) + c * Yb_d[k].repeat_interleave(512)
    return T.reshape(n), torch.full((n,), p_pa, dtype=torch.float64, device=dev), Y
