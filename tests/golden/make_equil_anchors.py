"""Write the near-equilibrium anchor states of the 53-species workload.

Calls only the oracle: each anchor request (T, p, element totals of a
Dirichlet(0.3) composition) is equilibrated by Gibbs minimisation and stored in
synth/data/c1_equil_anchors.npz.  The state generator cycles and perturbs these
anchors to make the 10 % near-equilibrium share of the workload.

    python tests/golden/make_equil_anchors.py
"""
import os
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth.state import ANCHOR_FILE, c1_anchor_requests  # noqa: E402


def compute_anchors():
    with tempfile.TemporaryDirectory() as d:
        path = synth.write_mechanism(synth.MECH_C1, os.path.join(d, "c1.mech"))
        m = oracle.read_mechanism(path)
    T, p, Y0 = c1_anchor_requests(m.n_species)
    Y = np.zeros_like(Y0)
    for a in range(T.shape[0]):
        Y[a], _ = oracle.equilibrate(m, T[a], p[a], Y0[a])
    return {"T": T, "p": p, "Y": Y}


if __name__ == "__main__":
    out = compute_anchors()
    os.makedirs(os.path.dirname(ANCHOR_FILE), exist_ok=True)
    np.savez(ANCHOR_FILE, **out)
    print("wrote", ANCHOR_FILE, {k: v.shape for k, v in out.items()})
