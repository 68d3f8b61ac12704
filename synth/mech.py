"""Seeded synthetic reaction mechanisms, written in the ``crf-mech 1`` text format.

The paper's solver reads its chemistry "in Cantera format" (Section 2) and its
production runs use a 9-species / 21-reaction hydrogen mechanism (Section 4.2).
That mechanism is not available here, so mechanisms of the same shape are drawn
at random:

* species are distinct element-count vectors over the given elements;
* reactions are element-balanced by construction (rejection sampling over
  product multisets with the same element vector as the reactants);
* every reaction is reversible, written in its exothermic direction at 1000 K
  (judged on the generator's own smooth heat-capacity model, not on the
  fitted polynomials);
* NASA-7 coefficients are least-squares fits of a smooth sigmoidal c_p(T),
  with a6/a7 of the upper range chosen for continuity of h and s at T_mid;
* transport fits are cubics in ln T of power laws with small curvature.

File format (all indices 0-based, floats printed with ``repr`` so that every
reader recovers the same doubles)::

    crf-mech 1
    gas-constant <R J/(kmol K)>
    standard-pressure <p0 Pa>
    elements <Ne>
    <symbol> <atomic weight kg/kmol>                       (Ne lines)
    species <Ns>
    <name> <Ne counts> <Tlo> <Tmid> <Thi> <7 low coeffs> <7 high coeffs>
    reactions <Nr>
    reaction <elementary|threebody|troe> reactants <n> <k:nu>... products <n> <k:nu>...
        arrhenius <lnA> <b> <theta> efficiencies <n> <k:eps>... [troe <lnA0> <b0> <theta0> <alpha> <T3> <T1> <T2>]
    transport
    viscosity <k> <c0> <c1> <c2> <c3>                      (Ns lines, ln mu = sum c_m (ln T)^m)
    conductivity <k> <c0> <c1> <c2> <c3>                   (Ns lines)
    diffusion <j> <k> <c0> <c1> <c2> <c3>                  (j<k, at the standard pressure)
    end

(each ``reaction`` record is one line in the file).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ATOMIC_WEIGHT = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999}
GAS_CONSTANT = 8314.46261815324      # J/(kmol K)
STANDARD_PRESSURE = 101325.0         # Pa
T_LO, T_MID, T_HI = 300.0, 1000.0, 3000.0
T_REF = 298.15


@dataclass(frozen=True)
class MechSpec:
    name: str
    elements: tuple
    n_species: int
    max_atoms: int
    n_elementary: int
    n_threebody: int
    n_troe: int
    seed: int


MECH_C0 = MechSpec("c0", ("H", "O", "N"), 9, 4, 21, 0, 0, 0)
MECH_C1 = MechSpec("c1", ("C", "H", "O", "N"), 53, 6, 260, 40, 25, 1)
MECH_C4 = MechSpec("c4", ("C", "H", "O", "N"), 200, 8, 1050, 300, 150, 2)


@dataclass
class Reaction:
    kind: str                      # "elementary" | "threebody" | "troe"
    reactants: dict                # species -> stoichiometric coefficient
    products: dict
    lnA: float
    b: float
    theta: float
    efficiencies: dict = field(default_factory=dict)
    troe: tuple = ()               # (lnA0, b0, theta0, alpha, T3, T1, T2)
    # optional rate forms and modifiers: "k0" (lindemann/sri low-pressure Arrhenius),
    # "sri" (a, b, c, d, e), "plog" [(p, lnA, b, theta)], "cheb" (Tmin, Tmax, Pmin, Pmax,
    # alpha [nT, nP]), "reverse" (lnA, b, theta), "irreversible" True, "orders" {k: o}
    extra: dict = field(default_factory=dict)


@dataclass
class Mechanism:
    elements: tuple
    weights: tuple
    names: list
    comp: np.ndarray               # [Ns, Ne] int
    nasa_lo: np.ndarray            # [Ns, 7]
    nasa_hi: np.ndarray            # [Ns, 7]
    reactions: list
    mu: np.ndarray                 # [Ns, 4]
    lam: np.ndarray                # [Ns, 4]
    dif: dict                      # (j, k) j<k -> [4]


# ---------------------------------------------------------------- species
def _draw_species(rng, elements, n_species, max_atoms):
    """Monatomic species of every element first, then distinct random compositions.

    Starting from the atoms makes every element appear and gives every molecule
    balanced dissociation/recombination partners, so that small mechanisms
    (9 species) still admit enough distinct balanced reactions.
    """
    ne = len(elements)
    comps = [tuple(int(e == i) for e in range(ne)) for i in range(ne)]
    seen = set(comps)
    for _ in range(100000):
        if len(comps) >= n_species:
            break
        total = int(rng.integers(2, max_atoms + 1))
        c = rng.multinomial(total, np.full(ne, 1.0 / ne))
        key = tuple(int(x) for x in c)
        if key in seen:
            continue
        seen.add(key)
        comps.append(key)
    else:
        raise RuntimeError("could not draw enough distinct species compositions")
    comps = np.array(comps, dtype=np.int64)
    names = []
    for c in comps:
        s = "".join(f"{el}{n if n > 1 else ''}" for el, n in zip(elements, c) if n)
        names.append(s)
    return comps, names


# ---------------------------------------------------------------- heat capacity model
def _cp_params(rng, n_atoms):
    c_lo = 2.5 + rng.uniform(0.0, 1.5 * (n_atoms - 1))
    c_hi = c_lo + rng.uniform(0.5, 2.0 * n_atoms)
    t_c = rng.uniform(500.0, 1500.0)
    w = rng.uniform(200.0, 600.0)
    hf = rng.uniform(-3.0e4, 6.0e4)       # h_f(298.15)/R  [K]
    s0 = rng.uniform(15.0, 35.0)          # s(298.15)/R
    return c_lo, c_hi, t_c, w, hf, s0


def _cp_model(T, p):
    c_lo, c_hi, t_c, w = p[:4]
    return c_lo + (c_hi - c_lo) / (1.0 + np.exp(-(T - t_c) / w))


def _h_model(T, p):
    """h/R of the smooth model: h_f/R + integral of cp/R from T_REF (closed form)."""
    c_lo, c_hi, t_c, w, hf = p[:5]
    def prim(x):
        return c_lo * x + (c_hi - c_lo) * w * np.logaddexp(0.0, (x - t_c) / w)
    return hf + prim(T) - prim(T_REF)


def _fit_nasa(p):
    """Least-squares quartic fits of cp/R on both ranges; a6/a7 from h_f, s0 and continuity."""
    coeffs = []
    for lo, hi in ((T_LO, T_MID), (T_MID, T_HI)):
        t = np.linspace(lo, hi, 200)
        x = t / 1000.0
        bfit = np.polynomial.polynomial.polyfit(x, _cp_model(t, p), 4)
        coeffs.append(np.array([bfit[m] / 1000.0 ** m for m in range(5)]))
    lo, hi = coeffs

    def h_poly(a, T):   # integral of the quartic (without the constant)
        return sum(a[m] * T ** (m + 1) / (m + 1) for m in range(5))

    def s_poly(a, T):   # integral of quartic/T (without the constant)
        return a[0] * math.log(T) + sum(a[m] * T ** m / m for m in range(1, 5))

    hf, s0 = p[4], p[5]
    a6_lo = hf - h_poly(lo, T_REF)
    a7_lo = s0 - s_poly(lo, T_REF)
    a6_hi = h_poly(lo, T_MID) + a6_lo - h_poly(hi, T_MID)
    a7_hi = s_poly(lo, T_MID) + a7_lo - s_poly(hi, T_MID)
    return np.concatenate([lo, [a6_lo, a7_lo]]), np.concatenate([hi, [a6_hi, a7_hi]])


# ---------------------------------------------------------------- reactions
class _CompIndex:
    def __init__(self, comp):
        self.comp = comp
        self.base = int(comp.max()) * 3 + 1
        self.mult = self.base ** np.arange(comp.shape[1], dtype=np.int64)
        codes = comp @ self.mult
        self.order = np.argsort(codes)
        self.codes = codes[self.order]

    def lookup(self, vecs):
        """Species index per row of `vecs` ([m, Ne]) or -1."""
        vecs = np.atleast_2d(vecs)
        ok = np.all(vecs >= 0, axis=1) & np.all(vecs < self.base, axis=1)
        codes = np.where(ok, vecs @ self.mult, -1)
        pos = np.clip(np.searchsorted(self.codes, codes), 0, len(self.codes) - 1)
        hit = ok & (self.codes[pos] == codes)
        return np.where(hit, self.order[pos], -1)


def _product_candidates(ix, target, n_prod):
    comp = ix.comp
    ns = comp.shape[0]
    if n_prod == 1:
        k = ix.lookup(target[None, :])[0]
        return [(int(k),)] if k >= 0 else []
    if n_prod == 2:
        b = ix.lookup(target[None, :] - comp)
        return [(a, int(b[a])) for a in range(ns) if b[a] >= a]
    out = []
    for a in range(ns):
        rest = target - comp[a]
        if np.any(rest < 0):
            continue
        c = ix.lookup(rest[None, :] - comp[a:])
        for off in np.nonzero(c >= 0)[0]:
            bb = a + int(off)
            if c[off] >= bb:
                out.append((a, bb, int(c[off])))
    return out


def _multiset(idx):
    d = {}
    for k in idx:
        d[int(k)] = d.get(int(k), 0) + 1
    return d


def _draw_reaction_sides(rng, ix, shape, force=None):
    """One attempt at (reactants, products) multisets of the given sizes, element balanced.

    Returns None when the drawn reactants admit no distinct product multiset.
    """
    ns = ix.comp.shape[0]
    n_reac, n_prod = shape
    reac = list(rng.integers(0, ns, size=n_reac))
    if force is not None:
        reac[0] = force
    target = ix.comp[reac].sum(axis=0)
    cands = _product_candidates(ix, target, n_prod)
    cands = [c for c in cands if not (set(c) & set(int(r) for r in reac))]
    if not cands:
        return None
    prod = cands[int(rng.integers(0, len(cands)))]
    return _multiset(reac), _multiset(prod)


def _key(reac, prod):
    a = tuple(sorted(reac.items()))
    b = tuple(sorted(prod.items()))
    return (a, b) if a <= b else (b, a)


def _orient(reac, prod, cp_params):
    """Write the reaction in its exothermic direction at 1000 K (smooth model enthalpies)."""
    dh = sum(n * _h_model(1000.0, cp_params[k]) for k, n in prod.items()) \
        - sum(n * _h_model(1000.0, cp_params[k]) for k, n in reac.items())
    return (reac, prod) if dh < 0 else (prod, reac)


def generate_mechanism(spec: MechSpec) -> Mechanism:
    rng = np.random.default_rng(spec.seed)
    comp, names = _draw_species(rng, spec.elements, spec.n_species, spec.max_atoms)
    ns = comp.shape[0]
    n_atoms = comp.sum(axis=1)
    cp_params = [_cp_params(rng, int(n_atoms[k])) for k in range(ns)]
    nasa = [_fit_nasa(p) for p in cp_params]
    nasa_lo = np.array([a for a, _ in nasa])
    nasa_hi = np.array([b for _, b in nasa])
    ix = _CompIndex(comp)

    kinds = ["elementary"] * spec.n_elementary + ["threebody"] * spec.n_threebody + ["troe"] * spec.n_troe
    elem_shapes = [(2, 2), (2, 1), (1, 2), (2, 3)]

    def draw_shape(kind):
        if kind == "elementary":
            if rng.uniform() < 0.7:
                return (2, 2)
            return elem_shapes[1 + int(rng.integers(0, 3))]
        return (2, 1) if rng.uniform() < 0.5 else (1, 2)

    reactions, keys = [], set()
    for kind in kinds:
        for _ in range(200000):
            sides = _draw_reaction_sides(rng, ix, draw_shape(kind))
            if sides is None:
                continue
            reac, prod = _orient(*sides, cp_params)
            key = _key(reac, prod)
            if reac == prod or key in keys:
                continue
            keys.add(key)
            reactions.append(_draw_rate(rng, kind, reac, prod, ns))
            break
        else:
            raise RuntimeError(f"could not draw a new balanced {kind} reaction")

    # every species must take part in some reaction: replace elementary reactions
    # by reactions that use the uncovered species until none is left
    for _ in range(10 * ns):
        used = set()
        for r in reactions:
            used |= set(r.reactants) | set(r.products)
        missing = [k for k in range(ns) if k not in used]
        if not missing:
            break
        k = missing[0]
        for _try in range(200):
            shape = elem_shapes[int(rng.integers(0, 4))]
            sides = _draw_reaction_sides(rng, ix, shape, force=k)
            if sides is None:
                continue
            reac, prod = _orient(*sides, cp_params)
            key = _key(reac, prod)
            if key in keys:
                continue
            # replace an elementary reaction whose species all stay covered elsewhere
            for j in rng.permutation(len(reactions)):
                old = reactions[j]
                if old.kind != "elementary":
                    continue
                others = set()
                for i2, r2 in enumerate(reactions):
                    if i2 != j:
                        others |= set(r2.reactants) | set(r2.products)
                if (set(old.reactants) | set(old.products)) <= (others | set(reac) | set(prod)):
                    keys.discard(_key(old.reactants, old.products))
                    keys.add(key)
                    reactions[j] = _draw_rate(rng, "elementary", reac, prod, ns)
                    break
            break
    else:
        raise RuntimeError("could not cover every species with a reaction")

    mu, lam, dif = _draw_transport(rng, ns)
    weights = tuple(ATOMIC_WEIGHT[e] for e in spec.elements)
    return Mechanism(spec.elements, weights, names, comp, nasa_lo, nasa_hi, reactions, mu, lam, dif)


def _draw_rate(rng, kind, reac, prod, ns):
    lnA = rng.uniform(20.0, 35.0)
    b = rng.uniform(-1.5, 2.0)
    theta = rng.uniform(0.0, 30000.0)
    eff, troe = {}, ()
    if kind in ("threebody", "troe"):
        n_eff = int(rng.integers(0, 5))
        for k in rng.choice(ns, size=n_eff, replace=False):
            eff[int(k)] = float(rng.uniform(0.3, 6.0))
    if kind == "troe":
        lnA0 = lnA + rng.uniform(2.0, 10.0)
        b0 = b - rng.uniform(0.0, 2.0)
        theta0 = rng.uniform(0.0, 1.0) * theta
        alpha = rng.uniform(0.3, 0.8)
        t3, t1, t2 = np.exp(rng.uniform(math.log(1e2), math.log(1e4), size=3))
        troe = (lnA0, b0, theta0, alpha, float(t3), float(t1), float(t2))
    return Reaction(kind, reac, prod, float(lnA), float(b), float(theta), eff, troe)


def _cubic_in_lnT(ln_v300, slope, k1, k2):
    """Coefficients c0..c3 of ln v = ln v300 + slope*L + k1*L^2 + k2*L^3, L = ln T - ln 300."""
    l0 = math.log(300.0)
    p_L = np.array([ln_v300, slope, k1, k2])
    # substitute L = x - l0 and expand in powers of x = ln T
    shift = np.polynomial.polynomial.Polynomial([-l0, 1.0])
    poly = np.polynomial.polynomial.Polynomial([0.0])
    for m, c in enumerate(p_L):
        poly = poly + c * shift ** m
    out = np.zeros(4)
    out[: len(poly.coef)] = poly.coef
    return out


def _draw_transport(rng, ns):
    def logu(lo, hi):
        return rng.uniform(math.log(lo), math.log(hi))
    mu = np.array([_cubic_in_lnT(logu(1e-5, 3e-5), 0.7, rng.uniform(-0.02, 0.02), rng.uniform(-0.02, 0.02))
                   for _ in range(ns)])
    lam = np.array([_cubic_in_lnT(logu(0.01, 0.2), 0.8, rng.uniform(-0.02, 0.02), rng.uniform(-0.02, 0.02))
                    for _ in range(ns)])
    dif = {}
    for j in range(ns):
        for k in range(j + 1, ns):
            dif[(j, k)] = _cubic_in_lnT(logu(1e-5, 1e-4), 1.75, rng.uniform(-0.02, 0.02),
                                        rng.uniform(-0.02, 0.02))
    return mu, lam, dif


# ---------------------------------------------------------------- writer
def mechanism_text(m: Mechanism) -> str:
    f = repr
    lines = ["crf-mech 1", f"# synthetic mechanism: {len(m.names)} species, {len(m.reactions)} reactions",
             f"gas-constant {f(GAS_CONSTANT)}", f"standard-pressure {f(STANDARD_PRESSURE)}",
             f"elements {len(m.elements)}"]
    for e, w in zip(m.elements, m.weights):
        lines.append(f"{e} {f(float(w))}")
    lines.append(f"species {len(m.names)}")
    for k, name in enumerate(m.names):
        toks = [name] + [str(int(c)) for c in m.comp[k]] + [f(T_LO), f(T_MID), f(T_HI)]
        toks += [f(float(a)) for a in m.nasa_lo[k]] + [f(float(a)) for a in m.nasa_hi[k]]
        lines.append(" ".join(toks))
    lines.append(f"reactions {len(m.reactions)}")
    for r in m.reactions:
        toks = ["reaction", r.kind, "reactants", str(len(r.reactants))]
        toks += [f"{k}:{n}" for k, n in sorted(r.reactants.items())]
        toks += ["products", str(len(r.products))]
        toks += [f"{k}:{n}" for k, n in sorted(r.products.items())]
        toks += ["arrhenius", f(r.lnA), f(r.b), f(r.theta)]
        toks += ["efficiencies", str(len(r.efficiencies))]
        toks += [f"{k}:{f(e)}" for k, e in sorted(r.efficiencies.items())]
        if r.kind == "troe":
            toks += ["troe"] + [f(float(x)) for x in r.troe]
        ex = r.extra
        if r.kind == "lindemann":
            toks += ["falloff"] + [f(float(x)) for x in ex["k0"]]
        elif r.kind == "sri":
            toks += ["sri"] + [f(float(x)) for x in tuple(ex["k0"]) + tuple(ex["sri"])]
        elif r.kind == "plog":
            toks += ["plog", str(len(ex["plog"]))] + [f(float(x)) for e in ex["plog"] for x in e]
        elif r.kind == "chebyshev":
            Tmin, Tmax, Pmin, Pmax, a = ex["cheb"]
            a = np.asarray(a, dtype=float)
            toks += ["chebyshev"] + [f(float(x)) for x in (Tmin, Tmax, Pmin, Pmax)]
            toks += [str(a.shape[0]), str(a.shape[1])] + [f(float(x)) for x in a.ravel()]
        if "reverse" in ex:
            toks += ["reverse"] + [f(float(x)) for x in ex["reverse"]]
        if ex.get("irreversible"):
            toks += ["irreversible"]
        if ex.get("orders"):
            toks += ["orders", str(len(ex["orders"]))] + [f"{k}:{f(float(o))}" for k, o in sorted(ex["orders"].items())]
        lines.append(" ".join(toks))
    lines.append("transport")
    for k in range(len(m.names)):
        lines.append(" ".join(["viscosity", str(k)] + [f(float(c)) for c in m.mu[k]]))
    for k in range(len(m.names)):
        lines.append(" ".join(["conductivity", str(k)] + [f(float(c)) for c in m.lam[k]]))
    for (j, k), c in sorted(m.dif.items()):
        lines.append(" ".join(["diffusion", str(j), str(k)] + [f(float(x)) for x in c]))
    lines.append("end")
    return "\n".join(lines) + "\n"


# A mechanism that uses every optional rate form: the 53-species reaction set of MECH_C1's
# generator at a smaller size, with reactions converted by their own seeded draws.
MECH_V = MechSpec("v", ("C", "H", "O", "N"), 32, 6, 50, 6, 12, 11)


def generate_variant_mechanism(spec: MechSpec = MECH_V, orders: bool = True) -> Mechanism:
    """generate_mechanism(spec) with reactions converted to the optional forms:
    of the 12 falloff reactions, 4 Lindemann and 5 SRI (the rest Troe); of the elementary
    ones, 6 PLOG (3-4 pressures, 1e4-1e7 Pa, each Arrhenius perturbed from the reaction's),
    5 Chebyshev (4 x 3 coefficients around the reaction's Arrhenius at 1 atm), 6 with an
    explicit reverse expression, 6 irreversible of which 4 have non-integer orders (none
    with orders=False; the draws are the same either way)."""
    m = generate_mechanism(spec)
    rng = np.random.default_rng(spec.seed + 1000)
    fall = [i for i, r in enumerate(m.reactions) if r.kind == "troe"]
    elem = [i for i, r in enumerate(m.reactions) if r.kind == "elementary"]
    rng.shuffle(fall)
    rng.shuffle(elem)
    for i in fall[:4]:
        r = m.reactions[i]
        r.kind, r.extra = "lindemann", {"k0": tuple(r.troe[:3])}
        r.troe = ()
    for i in fall[4:9]:
        r = m.reactions[i]
        sri = (rng.uniform(0.5, 2.0), rng.uniform(0.0, 1500.0), rng.uniform(300.0, 3000.0),
               rng.uniform(0.6, 1.4), rng.uniform(-0.3, 0.3))
        r.kind, r.extra = "sri", {"k0": tuple(r.troe[:3]), "sri": sri}
        r.troe = ()
    k = 0
    for i in elem[k:k + 6]:
        r = m.reactions[i]
        npres = int(rng.integers(3, 5))
        ps = np.sort(np.exp(rng.uniform(np.log(1e4), np.log(1e7), npres)))
        r.kind = "plog"
        r.extra = {"plog": [(float(pp), r.lnA + rng.uniform(-1.5, 1.5), r.b + rng.uniform(-0.3, 0.3),
                             max(0.0, r.theta + rng.uniform(-2000.0, 2000.0))) for pp in ps]}
    k += 6
    for i in elem[k:k + 5]:
        r = m.reactions[i]
        Tmin, Tmax, Pmin, Pmax = 290.0, 3000.0, 1e3, 1e8
        # log10 k of the reaction's Arrhenius at four temperatures, as a cubic in Tr, plus
        # pressure terms
        Tr = np.cos(np.pi * (np.arange(4) + 0.5) / 4)
        Ts = 2.0 / (Tr * (1.0 / Tmax - 1.0 / Tmin) + 1.0 / Tmin + 1.0 / Tmax)
        lg = (r.lnA + r.b * np.log(Ts) - r.theta / Ts) / np.log(10.0)
        a = np.zeros((4, 3))
        a[:, 0] = np.polynomial.chebyshev.chebfit(Tr, lg, 3)
        a[:, 1] = rng.uniform(-0.3, 0.3, 4) * np.array([1.0, 0.5, 0.2, 0.1])
        a[:, 2] = rng.uniform(-0.1, 0.1, 4) * np.array([1.0, 0.5, 0.2, 0.1])
        r.kind = "chebyshev"
        r.extra = {"cheb": (Tmin, Tmax, Pmin, Pmax, a)}
    k += 5
    for i in elem[k:k + 6]:
        r = m.reactions[i]
        r.extra = {"reverse": (r.lnA - rng.uniform(0.0, 4.0), r.b + rng.uniform(-0.5, 0.5),
                               r.theta + rng.uniform(5000.0, 20000.0))}
    k += 6
    for j, i in enumerate(elem[k:k + 6]):
        r = m.reactions[i]
        r.extra = {"irreversible": True}
        if j < 4:
            o = {s_: round(float(n_) * rng.uniform(0.5, 1.5), 2) for s_, n_ in r.reactants.items()}
            if orders:
                r.extra["orders"] = o
    return m


def with_rate_shift(m: Mechanism, dlnA: float) -> Mechanism:
    """A copy of m with every pre-exponential factor (and every falloff k0's) multiplied by
    e^dlnA: the same chemistry on a slower clock, for integrator tests at a moderate
    stiffness."""
    import copy
    out = copy.deepcopy(m)
    for r in out.reactions:
        r.lnA = r.lnA + dlnA
        if r.kind == "troe":
            r.troe = (r.troe[0] + dlnA,) + tuple(r.troe[1:])
    return out


def write_mechanism(spec_or_mech, path) -> str:
    m = generate_mechanism(spec_or_mech) if isinstance(spec_or_mech, MechSpec) else spec_or_mech
    text = mechanism_text(m)
    with open(path, "w") as fh:
        fh.write(text)
    return str(path)
