"""Reader of Cantera's YAML mechanism format, writing the library's ``crf-mech 1`` text.

The paper's solver takes its combustion model "in Cantera format" and generates code
from it (Section 2).  This module reads that format's thermodynamics and kinetics and
writes the plain text mechanism that ``crf_load_mech`` (and the oracle's reader) load:

* units: the file's ``units`` map (length, quantity, time, activation-energy, pressure;
  Cantera's defaults m, kmol, s, J/kmol, Pa), and values written as "<number> <unit>";
  everything is converted to SI with kmol: A to (m^3/kmol)^(n-1)/s for a rate of order n
  (three-body rates and falloff low-pressure limits one order higher), activation energies
  to theta = Ea/R in K, pressures to Pa, Chebyshev coefficients shifted by the same factor;
* species: composition and NASA7 thermo with two temperature ranges;
* reactions: "A + 2 B <=> C" (or "=" reversible, "=>" irreversible), integer
  coefficients 1..3 and at most 3 distinct species per side; types elementary
  (Arrhenius), three-body ("+ M", efficiencies, default-efficiency), falloff ("(+M)";
  Lindemann, Troe with or without T2, SRI), pressure-dependent-Arrhenius (PLOG, one
  expression per pressure), Chebyshev; reaction orders (reactant species only).
  Anything else (surface or chemically-activated reactions, specific third-body
  colliders, non-integer stoichiometry, duplicate PLOG pressures) raises ValueError.
* transport: Cantera files give molecular parameters (Lennard-Jones diameter and
  well depth) while the library takes cubic fits in ln T of ln mu_k, ln lambda_k and
  ln D_jk; this reader derives them from the kinetic theory of dilute gases:
      mu_k  = (5/16) sqrt(pi m_k k_B T) / (pi sigma_k^2 Omega22*(T/eps_k)),
      D_jk  = (3/16) sqrt(2 pi k_B^3 T^3 / m_jk) / (p sigma_jk^2 pi Omega11*(T/eps_jk)),
      lambda_k = (mu_k / W_k) (c_p,k + 5/4 R)   (Eucken),
  with sigma_jk and eps_jk the arithmetic and geometric means, the collision integrals
  from the correlation of Neufeld, Janzen and Aziz (1972), and the fits taken by least
  squares over 300-3000 K at 1 atm.  This is the plain Lennard-Jones model (no polar or
  rotational-relaxation corrections), so these transport properties differ from
  Cantera's own; with transport=False constant placeholder fits are written instead.

Usage: ``text = cantera_yaml.to_crf_mech(open(path).read())`` or
``Mechanism.from_cantera_yaml(path)``.  Only ``yaml.safe_load`` is used.
"""
from __future__ import annotations

import math
import re

import numpy as np
import yaml

GAS_CONSTANT = 8314.46261815324          # J/(kmol K)
STANDARD_PRESSURE = 101325.0             # Pa
AVOGADRO = 6.02214076e26                 # 1/kmol
BOLTZMANN = 1.380649e-23                 # J/K
ATOMIC_WEIGHT = {"H": 1.008, "D": 2.014, "C": 12.011, "N": 14.007, "O": 15.999, "AR": 39.95, "AR_": 39.95,
                 "HE": 4.0026, "NE": 20.180, "S": 32.06, "CL": 35.45, "F": 18.998, "SI": 28.085, "E": 5.48579909e-4}

_LENGTH = {"m": 1.0, "cm": 1e-2, "mm": 1e-3}
_QUANTITY = {"kmol": 1.0, "mol": 1e-3, "molec": 1.0 / AVOGADRO, "molecule": 1.0 / AVOGADRO}
_TIME = {"s": 1.0, "ms": 1e-3, "min": 60.0, "h": 3600.0}
_ENERGY_PER_QTY = {"J/kmol": 1.0, "J/mol": 1e3, "kJ/mol": 1e6, "cal/mol": 4184.0, "kcal/mol": 4.184e6,
                   "eV": 1.602176634e-19 * AVOGADRO}
_PRESSURE = {"Pa": 1.0, "kPa": 1e3, "MPa": 1e6, "bar": 1e5, "atm": 101325.0, "torr": 101325.0 / 760.0}


class _Units:
    def __init__(self, u):
        u = u or {}
        for key, table in (("length", _LENGTH), ("quantity", _QUANTITY), ("time", _TIME)):
            if u.get(key, None) is not None and u[key] not in table:
                raise ValueError(f"unsupported {key} unit {u[key]!r}")
        self.L = _LENGTH[u.get("length", "m")]
        self.Q = _QUANTITY[u.get("quantity", "kmol")]
        self.t = _TIME[u.get("time", "s")]
        ea = u.get("activation-energy", "J/kmol")
        if ea != "K" and ea not in _ENERGY_PER_QTY:
            raise ValueError(f"unsupported activation-energy unit {ea!r}")
        self.ea = ea
        pu = u.get("pressure", "Pa")
        if pu not in _PRESSURE:
            raise ValueError(f"unsupported pressure unit {pu!r}")
        self.P = _PRESSURE[pu]

    def a_factor(self, order):
        """A in the file's units -> (m^3/kmol)^(order-1)/s."""
        return (self.L ** 3 / self.Q) ** (order - 1) / self.t

    def theta(self, ea):
        """Activation energy (number in the file's unit, or "<number> <unit>") -> Ea/R in K."""
        v, unit = _split_unit(ea, self.ea)
        if unit == "K":
            return v
        if unit not in _ENERGY_PER_QTY:
            raise ValueError(f"unsupported activation-energy unit {unit!r}")
        return v * _ENERGY_PER_QTY[unit] / GAS_CONSTANT

    def pressure(self, pv):
        v, unit = _split_unit(pv, None)
        if unit is None:
            return v * self.P
        if unit not in _PRESSURE:
            raise ValueError(f"unsupported pressure unit {unit!r}")
        return v * _PRESSURE[unit]


def _split_unit(x, default):
    if isinstance(x, (int, float)):
        return float(x), default
    parts = str(x).split()
    if len(parts) == 1:
        return float(parts[0]), default
    return float(parts[0]), " ".join(parts[1:])


def _plain_number(x, what):
    if isinstance(x, (int, float)):
        return float(x)
    raise ValueError(f"{what}: values with explicit units are supported for Ea and P only ({x!r})")


_TOKEN = re.compile(r"^(\d+)?\s*([A-Za-z][A-Za-z0-9_()\-,*#+\[\]]*?)$")


def _side(text, index):
    """{species index: coefficient}; '+ M' and '(+M)' removed by the caller."""
    out = {}
    for tok in [t.strip() for t in re.split(r"\s\+\s", " " + text.strip() + " ")]:
        if not tok:
            continue
        parts = tok.split()
        if len(parts) == 2:
            c, name = parts
            if not re.fullmatch(r"\d+", c):
                raise ValueError(f"non-integer stoichiometric coefficient in {tok!r}")
            nu = int(c)
        elif len(parts) == 1:
            m = re.fullmatch(r"(\d+)([A-Za-z].*)", parts[0])
            nu, name = (int(m.group(1)), m.group(2)) if m and m.group(2) not in index else (1, parts[0])
        else:
            raise ValueError(f"cannot read species term {tok!r}")
        if name not in index:
            raise ValueError(f"unknown species {name!r}")
        k = index[name]
        out[k] = out.get(k, 0) + nu
    return out


def _equation(eq, index):
    """(reactants, products, reversible, third_body: None | '+M' | '(+M)')."""
    if "<=>" in eq:
        lhs, rhs = eq.split("<=>")
        rev = True
    elif "=>" in eq:
        lhs, rhs = eq.split("=>")
        rev = False
    elif "=" in eq:
        lhs, rhs = eq.split("=")
        rev = True
    else:
        raise ValueError(f"no reaction arrow in {eq!r}")
    tb = None
    sides = []
    for s in (lhs, rhs):
        m = re.search(r"\(\s*\+\s*([A-Za-z0-9_]+)\s*\)", s)
        if m:
            if m.group(1) != "M":
                raise ValueError(f"specific falloff collider (+{m.group(1)}) is not supported")
            tb = "(+M)"
            s = s[:m.start()] + s[m.end():]
        elif re.search(r"(^|\s)\+\s*M\s*$", s) or re.fullmatch(r"\s*M\s*", s):
            tb = "+M"
            s = re.sub(r"\+\s*M\s*$", "", s.rstrip())
        sides.append(_side(s, index))
    return sides[0], sides[1], rev, tb


def _neufeld_omega22(Ts):
    return 1.16145 * Ts ** -0.14874 + 0.52487 * np.exp(-0.77320 * Ts) + 2.16178 * np.exp(-2.43787 * Ts)


def _neufeld_omega11(Ts):
    return (1.06036 * Ts ** -0.15610 + 0.19300 * np.exp(-0.47635 * Ts) + 1.03587 * np.exp(-1.52996 * Ts)
            + 1.76474 * np.exp(-3.89411 * Ts))


def _cubic_fit(T, v):
    """Coefficients c0..c3 of ln v = sum_m c_m (ln T)^m (least squares)."""
    L = np.log(T)
    return np.polynomial.polynomial.polyfit(L, np.log(v), 3)


def _cp_R(a_lo, a_hi, tmid, T):
    a = np.where((T <= tmid)[:, None], np.asarray(a_lo)[None, :], np.asarray(a_hi)[None, :])
    return a[:, 0] + a[:, 1] * T + a[:, 2] * T ** 2 + a[:, 3] * T ** 3 + a[:, 4] * T ** 4


def to_crf_mech(text, transport=True):
    """The ``crf-mech 1`` text of a Cantera YAML mechanism (a string)."""
    doc = yaml.safe_load(text)
    units = _Units(doc.get("units"))
    phase = doc["phases"][0] if doc.get("phases") else {}
    species = doc["species"]
    if phase.get("species") and isinstance(phase["species"], list) and all(isinstance(s, str) for s in phase["species"]):
        by = {s["name"]: s for s in species}
        species = [by[n] for n in phase["species"]]
    names = [s["name"] for s in species]
    index = {n: k for k, n in enumerate(names)}
    elements = phase.get("elements") or sorted({e for s in species for e in s["composition"]})
    for e in elements:
        if e.upper() not in ATOMIC_WEIGHT:
            raise ValueError(f"no atomic weight for element {e!r}")
    f = repr
    lines = ["crf-mech 1", "# converted from a Cantera YAML mechanism",
             f"gas-constant {f(GAS_CONSTANT)}", f"standard-pressure {f(STANDARD_PRESSURE)}",
             f"elements {len(elements)}"]
    lines += [f"{e} {f(ATOMIC_WEIGHT[e.upper()])}" for e in elements]
    lines.append(f"species {len(names)}")
    W = np.zeros(len(names))
    nasa = []
    for k, s in enumerate(species):
        th = s["thermo"]
        if th.get("model") != "NASA7" or len(th["data"]) != 2 or len(th["temperature-ranges"]) != 3:
            raise ValueError(f"species {s['name']}: only NASA7 thermo with two ranges is supported")
        comp = [int(s["composition"].get(e, 0)) for e in elements]
        if sum(s["composition"].values()) != sum(comp):
            raise ValueError(f"species {s['name']}: element not listed in the phase")
        W[k] = sum(c * ATOMIC_WEIGHT[e.upper()] for c, e in zip(comp, elements))
        tl, tm, thi = (float(x) for x in th["temperature-ranges"])
        lo, hi = [float(x) for x in th["data"][0]], [float(x) for x in th["data"][1]]
        nasa.append((lo, hi, tm))
        lines.append(" ".join([s["name"]] + [str(c) for c in comp] + [f(tl), f(tm), f(thi)]
                              + [f(x) for x in lo] + [f(x) for x in hi]))
    rxns = doc.get("reactions", [])
    lines.append(f"reactions {len(rxns)}")
    for i, r in enumerate(rxns):
        reac, prod, rev, tb = _equation(r["equation"], index)
        rtype = r.get("type", "elementary")
        for side in (reac, prod):
            if len(side) > 3 or any(v > 3 for v in side.values()) or sum(side.values()) > 3:
                raise ValueError(f"reaction {i}: at most 3 species and total order 3 per side")
        orders = {index[k]: float(v) for k, v in (r.get("orders") or {}).items()}
        for k in orders:
            if k not in reac:
                raise ValueError(f"reaction {i}: orders of non-reactant species are not supported")
        order = sum(orders.get(k, float(v)) for k, v in reac.items())

        def arr(rc, n):
            A = _plain_number(rc["A"], f"reaction {i} A") * units.a_factor(n)
            if A <= 0:
                raise ValueError(f"reaction {i}: A must be positive")
            return math.log(A), float(rc.get("b", 0.0)), units.theta(rc.get("Ea", 0.0))

        toks = []
        extra = []
        if rtype in ("elementary", "reaction") and tb is None:
            kind = "elementary"
            lnA, b, th = arr(r["rate-constant"], order)
        elif rtype == "three-body" or (rtype == "elementary" and tb == "+M"):
            kind = "threebody"
            lnA, b, th = arr(r["rate-constant"], order + 1)
        elif rtype == "falloff":
            lnA, b, th = arr(r["high-P-rate-constant"], order)
            lo = arr(r["low-P-rate-constant"], order + 1)
            if "Troe" in r:
                t = r["Troe"]
                kind = "troe"
                extra = ["troe"] + [f(x) for x in lo] + [f(float(t["A"])), f(float(t["T3"])), f(float(t["T1"])),
                                                       f(float(t.get("T2", 1e30)))]
            elif "SRI" in r:
                t = r["SRI"]
                kind = "sri"
                extra = ["sri"] + [f(x) for x in lo] + [f(float(t["A"])), f(float(t["B"])), f(float(t["C"])),
                                                      f(float(t.get("D", 1.0))), f(float(t.get("E", 0.0)))]
            else:
                kind = "lindemann"
                extra = ["falloff"] + [f(x) for x in lo]
        elif rtype == "pressure-dependent-Arrhenius":
            kind = "plog"
            ents = sorted(((units.pressure(e["P"]),) + arr(e, order) for e in r["rate-constants"]),
                          key=lambda e: e[0])
            if len({e[0] for e in ents}) != len(ents):
                raise ValueError(f"reaction {i}: several PLOG expressions at one pressure are not supported")
            lnA, b, th = ents[0][1:]
            extra = ["plog", str(len(ents))] + [f(x) for e in ents for x in e]
        elif rtype == "Chebyshev":
            kind = "chebyshev"
            Tmin, Tmax = (float(x) for x in r["temperature-range"])
            Pmin, Pmax = (units.pressure(x) for x in r["pressure-range"])
            a = np.array(r["data"], dtype=float)
            a[0, 0] += math.log10(units.a_factor(order))      # T_0 = 1: the constant term
            lnA, b, th = 0.0, 0.0, 0.0
            extra = ["chebyshev"] + [f(x) for x in (Tmin, Tmax, Pmin, Pmax)] + [str(a.shape[0]), str(a.shape[1])]
            extra += [f(float(x)) for x in a.ravel()]
        else:
            raise ValueError(f"reaction {i}: unsupported type {rtype!r}")
        effs = {}
        if kind in ("threebody", "troe", "sri", "lindemann"):
            dflt = float(r.get("default-efficiency", 1.0))
            given = {index[k]: float(v) for k, v in (r.get("efficiencies") or {}).items() if k in index}
            for k in range(len(names)):
                e = given.get(k, dflt)
                if e != 1.0:
                    effs[k] = e
        elif r.get("efficiencies"):
            raise ValueError(f"reaction {i}: efficiencies on a reaction without third body")
        toks = ["reaction", kind, "reactants", str(len(reac))] + [f"{k}:{v}" for k, v in sorted(reac.items())]
        toks += ["products", str(len(prod))] + [f"{k}:{v}" for k, v in sorted(prod.items())]
        toks += ["arrhenius", f(lnA), f(b), f(th), "efficiencies", str(len(effs))]
        toks += [f"{k}:{f(e)}" for k, e in sorted(effs.items())]
        toks += extra
        if not rev:
            toks.append("irreversible")
        if orders:
            toks += ["orders", str(len(orders))] + [f"{k}:{f(o)}" for k, o in sorted(orders.items())]
        lines.append(" ".join(toks))
    lines.append("transport")
    ns = len(names)
    Tg = np.linspace(300.0, 3000.0, 60)
    if transport:
        sig, eps = np.zeros(ns), np.zeros(ns)
        for k, s in enumerate(species):
            tr = s.get("transport")
            if not tr or "diameter" not in tr or "well-depth" not in tr:
                raise ValueError(f"species {s['name']}: no Lennard-Jones transport data (use transport=False)")
            sig[k] = float(tr["diameter"]) * 1e-10
            eps[k] = float(tr["well-depth"])
        m = W / AVOGADRO
        mu_fit, lam_fit = [], []
        for k in range(ns):
            mu = 5.0 / 16.0 * np.sqrt(np.pi * m[k] * BOLTZMANN * Tg) / (np.pi * sig[k] ** 2 * _neufeld_omega22(Tg / eps[k]))
            lo, hi, tm = nasa[k]
            lam = mu / W[k] * GAS_CONSTANT * (_cp_R(lo, hi, tm, Tg) + 1.25)
            mu_fit.append(_cubic_fit(Tg, mu))
            lam_fit.append(_cubic_fit(Tg, lam))
        for k in range(ns):
            lines.append(" ".join(["viscosity", str(k)] + [f(float(c)) for c in mu_fit[k]]))
        for k in range(ns):
            lines.append(" ".join(["conductivity", str(k)] + [f(float(c)) for c in lam_fit[k]]))
        for j in range(ns):
            for k in range(j + 1, ns):
                mjk = m[j] * m[k] / (m[j] + m[k])
                sjk, ejk = 0.5 * (sig[j] + sig[k]), math.sqrt(eps[j] * eps[k])
                D = 3.0 / 16.0 * np.sqrt(2.0 * np.pi * BOLTZMANN ** 3 * Tg ** 3 / mjk) / (
                    STANDARD_PRESSURE * np.pi * sjk ** 2 * _neufeld_omega11(Tg / ejk))
                lines.append(" ".join(["diffusion", str(j), str(k)] + [f(float(c)) for c in _cubic_fit(Tg, D)]))
    else:
        for k in range(ns):
            lines.append(f"viscosity {k} {f(math.log(2e-5))} 0.0 0.0 0.0")
        for k in range(ns):
            lines.append(f"conductivity {k} {f(math.log(0.05))} 0.0 0.0 0.0")
        for j in range(ns):
            for k in range(j + 1, ns):
                lines.append(f"diffusion {j} {k} {f(math.log(5e-5))} 0.0 0.0 0.0")
    lines.append("end")
    return "\n".join(lines) + "\n"
