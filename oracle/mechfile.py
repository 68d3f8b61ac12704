"""The oracle's own reader of the ``crf-mech 1`` mechanism text.

Independent of the library's C++ loader: both read the same file, so a reading
disagreement shows up as a parity failure.  Arrays are dense and plain
(stoichiometric matrices [Nr, Ns], efficiency matrix [Nr, Ns] with default 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class OracleMech:
    R: float
    p0: float
    elements: list
    aw: np.ndarray           # [Ne] atomic weights
    names: list
    comp: np.ndarray         # [Ns, Ne] element counts
    W: np.ndarray            # [Ns] molar masses, sum_e comp * aw
    t_lo: np.ndarray
    t_mid: np.ndarray
    t_hi: np.ndarray
    a_lo: np.ndarray         # [Ns, 7]
    a_hi: np.ndarray         # [Ns, 7]
    kind: list               # per reaction: "elementary" | "threebody" | "troe"
    nu_f: np.ndarray         # [Nr, Ns] reactant coefficients nu'
    nu_r: np.ndarray         # [Nr, Ns] product coefficients nu''
    lnA: np.ndarray
    b: np.ndarray
    theta: np.ndarray
    eff: np.ndarray          # [Nr, Ns] third-body efficiencies (1 by default)
    troe: np.ndarray         # [Nr, 7] (lnA0, b0, theta0, alpha, T3, T1, T2); zeros if not falloff
    mu_fit: np.ndarray       # [Ns, 4]
    lam_fit: np.ndarray      # [Ns, 4]
    dif_fit: np.ndarray      # [Ns, Ns, 4] symmetric, diagonal unused
    # per reaction, the optional rate forms and modifiers (empty dict for a plain reaction):
    #   "k0": (lnA0, b0, theta0)           low-pressure limit of a lindemann / sri falloff
    #   "sri": (a, b, c, d, e)
    #   "plog": [(p, lnA, b, theta), ...]  ascending p (Pa)
    #   "cheb": (Tmin, Tmax, Pmin, Pmax, alpha [nT, nP])
    #   "reverse": (lnA, b, theta)         explicit reverse Arrhenius
    #   "irreversible": True
    #   "orders": {species: order}         forward reaction orders (reactants)
    extra: list = None

    @property
    def n_species(self):
        return len(self.names)

    @property
    def n_reactions(self):
        return len(self.kind)


def _pairs(tokens, n, conv):
    out = {}
    for t in tokens[:n]:
        k, v = t.split(":")
        out[int(k)] = conv(v)
    return out


def read_mechanism(path) -> OracleMech:
    with open(path) as fh:
        lines = [ln.strip() for ln in fh if ln.strip() and not ln.lstrip().startswith("#")]
    it = iter(lines)
    head = next(it).split()
    if head != ["crf-mech", "1"]:
        raise ValueError(f"not a crf-mech 1 file: {head}")
    R = p0 = None
    tok = next(it).split()
    while tok[0] in ("gas-constant", "standard-pressure"):
        if tok[0] == "gas-constant":
            R = float(tok[1])
        else:
            p0 = float(tok[1])
        tok = next(it).split()
    assert tok[0] == "elements"
    ne = int(tok[1])
    elements, aw = [], []
    for _ in range(ne):
        e, w = next(it).split()
        elements.append(e)
        aw.append(float(w))
    aw = np.array(aw)
    tok = next(it).split()
    assert tok[0] == "species"
    ns = int(tok[1])
    names, comp, tl, tm, th, alo, ahi = [], [], [], [], [], [], []
    for _ in range(ns):
        t = next(it).split()
        names.append(t[0])
        comp.append([int(x) for x in t[1:1 + ne]])
        f = [float(x) for x in t[1 + ne:]]
        tl.append(f[0]); tm.append(f[1]); th.append(f[2])
        alo.append(f[3:10]); ahi.append(f[10:17])
    comp = np.array(comp, dtype=np.int64)
    tok = next(it).split()
    assert tok[0] == "reactions"
    nr = int(tok[1])
    kind = []
    nu_f = np.zeros((nr, ns)); nu_r = np.zeros((nr, ns))
    lnA = np.zeros(nr); b = np.zeros(nr); theta = np.zeros(nr)
    eff = np.ones((nr, ns)); troe = np.zeros((nr, 7))
    extra = []
    for i in range(nr):
        t = next(it).split()
        assert t[0] == "reaction"
        kind.append(t[1])
        p = 2
        assert t[p] == "reactants"; n = int(t[p + 1])
        for k, v in _pairs(t[p + 2:], n, int).items():
            nu_f[i, k] += v
        p += 2 + n
        assert t[p] == "products"; n = int(t[p + 1])
        for k, v in _pairs(t[p + 2:], n, int).items():
            nu_r[i, k] += v
        p += 2 + n
        assert t[p] == "arrhenius"
        lnA[i], b[i], theta[i] = (float(x) for x in t[p + 1:p + 4])
        p += 4
        assert t[p] == "efficiencies"; n = int(t[p + 1])
        for k, v in _pairs(t[p + 2:], n, float).items():
            eff[i, k] = v
        p += 2 + n
        ex = {}
        if t[1] == "troe":
            assert t[p] == "troe"
            troe[i] = [float(x) for x in t[p + 1:p + 8]]
            p += 8
        elif t[1] == "lindemann":
            assert t[p] == "falloff"
            ex["k0"] = tuple(float(x) for x in t[p + 1:p + 4])
            p += 4
        elif t[1] == "sri":
            assert t[p] == "sri"
            f = [float(x) for x in t[p + 1:p + 9]]
            ex["k0"], ex["sri"] = tuple(f[:3]), tuple(f[3:])
            p += 9
        elif t[1] == "plog":
            assert t[p] == "plog"
            n = int(t[p + 1])
            f = [float(x) for x in t[p + 2:p + 2 + 4 * n]]
            ex["plog"] = [tuple(f[4 * j:4 * j + 4]) for j in range(n)]
            p += 2 + 4 * n
        elif t[1] == "chebyshev":
            assert t[p] == "chebyshev"
            Tmin, Tmax, Pmin, Pmax = (float(x) for x in t[p + 1:p + 5])
            nT, nP = int(t[p + 5]), int(t[p + 6])
            a = np.array([float(x) for x in t[p + 7:p + 7 + nT * nP]]).reshape(nT, nP)
            ex["cheb"] = (Tmin, Tmax, Pmin, Pmax, a)
            p += 7 + nT * nP
        while p < len(t):
            if t[p] == "reverse":
                ex["reverse"] = tuple(float(x) for x in t[p + 1:p + 4])
                p += 4
            elif t[p] == "irreversible":
                ex["irreversible"] = True
                p += 1
            elif t[p] == "orders":
                n = int(t[p + 1])
                ex["orders"] = _pairs(t[p + 2:], n, float)
                p += 2 + n
            else:
                raise ValueError(f"reaction {i}: unknown token {t[p]}")
        extra.append(ex)
    assert next(it) == "transport"
    mu = np.zeros((ns, 4)); lam = np.zeros((ns, 4)); dif = np.zeros((ns, ns, 4))
    for line in it:
        t = line.split()
        if t[0] == "end":
            break
        if t[0] == "viscosity":
            mu[int(t[1])] = [float(x) for x in t[2:6]]
        elif t[0] == "conductivity":
            lam[int(t[1])] = [float(x) for x in t[2:6]]
        elif t[0] == "diffusion":
            j, k = int(t[1]), int(t[2])
            dif[j, k] = dif[k, j] = [float(x) for x in t[3:7]]
    W = comp @ aw
    return OracleMech(R, p0, elements, aw, names, comp, W, np.array(tl), np.array(tm), np.array(th),
                      np.array(alo), np.array(ahi), kind, nu_f, nu_r, lnA, b, theta, eff, troe,
                      mu, lam, dif, extra)
