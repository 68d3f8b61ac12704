"""Hand-made mechanisms for the oracle pin tests."""
import numpy as np

import synth
from synth.mech import Mechanism, Reaction, mechanism_text  # noqa: F401


def tiny_mechanism(path, species, reactions, elements=("H", "O"), transport=None):
    """Write a hand-made mechanism.

    species: list of (name, counts tuple, a_lo[7], a_hi[7] or None)
    reactions: list of Reaction
    transport: optional (mu [Ns,4], lam [Ns,4], dif {(j,k): [4]})
    """
    ns = len(species)
    comp = np.array([s[1] for s in species], dtype=np.int64)
    a_lo = np.array([s[2] for s in species], dtype=float)
    a_hi = np.array([s[3] if s[3] is not None else s[2] for s in species], dtype=float)
    if transport is None:
        mu = np.tile([np.log(2e-5), 0.0, 0.0, 0.0], (ns, 1))
        lam = np.tile([np.log(0.05), 0.0, 0.0, 0.0], (ns, 1))
        dif = {(j, k): np.array([np.log(5e-5), 0.0, 0.0, 0.0]) for j in range(ns) for k in range(j + 1, ns)}
    else:
        mu, lam, dif = transport
    weights = tuple(synth.mech.ATOMIC_WEIGHT[e] for e in elements)
    m = Mechanism(tuple(elements), weights, [s[0] for s in species], comp, a_lo, a_hi, reactions,
                  np.asarray(mu, float), np.asarray(lam, float), dif)
    with open(path, "w") as fh:
        fh.write(mechanism_text(m))
    return str(path)


def nasa_const(a1=0.0, a6=0.0, a7=0.0):
    return [a1, 0.0, 0.0, 0.0, 0.0, a6, a7]

