"""Per-species and per-row errors of the HIP path against the FP64 oracle (GPU; run as a
script, not collected by pytest):

    python tests/error_report.py > report.txt

* production rates w_k, 53 species (sampled points of the 2^20-point state; FP64 and the
  mixed mode) and 200 species (one launch of 2 spectral elements, 1024 points): E_norm,k =
  ||w_hat_k - w_k|| / ||w_k|| over the points and E_turn,k = max |w_hat - w| / (|w| + S_k);
* transport, 53 species: max relative error of D_k per species and of mu, lambda;
* Jacobian, 53 species (2^18-point state sample) and 200 species: per row, the scaled error
  of the T column and of the Y columns (tests/metrics.jac_scaled_errors).
"""
import os
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import torch  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2409_06404_amd as crf  # noqa: E402
from metrics import e_norm, e_turn, fp32_range_split, jac_scaled_errors, significant_species  # noqa: E402


def dev(st):
    d = torch.device("cuda", 0)
    return (torch.from_numpy(np.ascontiguousarray(st["T"])).to(d), torch.from_numpy(np.ascontiguousarray(st["p"])).to(d),
            torch.from_numpy(np.ascontiguousarray(st["Y"])).to(d).t())


def sub(st, idx):
    return {"T": st["T"][idx], "p": st["p"][idx], "Y": np.ascontiguousarray(st["Y"][:, idx])}


def wdot_table(g, om, st, label):
    T, p, Y = dev(st)
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    sig = significant_species(ref["wdot"], om.W)
    cols = {}
    for prec in ("fp64", "mixed"):
        w = crf.wdot(g, T, p, Y, prec)[0].cpu().numpy()
        cols[prec] = (e_norm(w, ref["wdot"]), e_turn(w, ref["wdot"], ref["turnover"]))
    print(f"\n## production rates, {label}: E_norm and E_turn per species (* = significant)")
    print(f"{'k':>4} {'name':>10}  {'E_norm fp64':>12} {'E_turn fp64':>12}  {'E_norm mixed':>12} {'E_turn mixed':>12}")
    for k in range(om.n_species):
        print(f"{k:4d} {om.names[k]:>10}{'*' if sig[k] else ' '} {cols['fp64'][0][k]:12.2e} {cols['fp64'][1][k]:12.2e}  "
              f"{cols['mixed'][0][k]:12.2e} {cols['mixed'][1][k]:12.2e}")
    for prec in ("fp64", "mixed"):
        print(f"   max over significant species, {prec}: E_norm {cols[prec][0][sig].max():.2e}, "
              f"E_turn {cols[prec][1].max():.2e}")


def transport_table(g, om, st, label):
    T, p, Y = dev(st)
    ref = oracle.transport_properties(om, st["T"], st["p"], st["Y"].T)
    print(f"\n## transport, {label}: max relative error")
    res = {}
    for prec in ("fp64", "mixed"):
        mu, lam, D = (x.cpu().numpy() for x in crf.transport(g, T, p, Y, prec))
        res[prec] = (np.max(np.abs(mu / ref["mu"] - 1)), np.max(np.abs(lam / ref["lambda"] - 1)),
                     np.max(np.abs(D / ref["Dmix"] - 1), axis=0))
        print(f"   {prec}: mu {res[prec][0]:.2e}, lambda {res[prec][1]:.2e}, D_k max {res[prec][2].max():.2e}")
    print(f"{'k':>4} {'name':>10}  {'D_k fp64':>10} {'D_k mixed':>10}")
    for k in range(om.n_species):
        print(f"{k:4d} {om.names[k]:>10}  {res['fp64'][2][k]:10.2e} {res['mixed'][2][k]:10.2e}")


def jac_table(g, om, st, label):
    T, p, Y = dev(st)
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    res = {}
    for prec in ("fp64", "mixed"):
        J = crf.wdot_jac(g, T, p, Y, prec)[0].double().cpu().numpy()
        Jref = Jr
        if prec == "mixed":
            J, Jref = fp32_range_split(J, Jr)
        res[prec] = jac_scaled_errors(J, Jref, G, st["T"], st["Y"].T, floor=1e-10 if prec == "mixed" else 0.0)
    print(f"\n## Jacobian, {label}: per row (0 = heat release, 1 + k = species k) scaled error of the T column "
          "and of the Y columns")
    print(f"{'row':>4} {'name':>10}  {'T fp64':>10} {'Y fp64':>10}  {'T mixed':>10} {'Y mixed':>10}")
    for r in range(om.n_species + 1):
        nm = "hrr" if r == 0 else om.names[r - 1]
        print(f"{r:4d} {nm:>10}  {res['fp64'][0][r]:10.2e} {res['fp64'][1][r]:10.2e}  "
              f"{res['mixed'][0][r]:10.2e} {res['mixed'][1][r]:10.2e}")
    for prec in ("fp64", "mixed"):
        print(f"   max over rows, {prec}: T column {res[prec][0].max():.2e}, Y columns {res[prec][1].max():.2e}")


def main():
    torch.cuda.init()
    with tempfile.TemporaryDirectory() as d:
        p1 = synth.write_mechanism(synth.MECH_C1, os.path.join(d, "c1.mech"))
        p4 = synth.write_mechanism(synth.MECH_C4, os.path.join(d, "c4.mech"))
        g1, o1 = crf.Mechanism(p1, device=0), oracle.read_mechanism(p1)
        g4, o4 = crf.Mechanism(p4, device=0), oracle.read_mechanism(p4)
        full = synth.state_c1(53, n=1 << 20, seed=1)
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(1 << 20, size=2000, replace=False))
        print("# errors of the HIP path against the FP64 oracle (tests/error_report.py)")
        print("# 53 species / 325 reactions: 2000 points sampled from the 2^20-point state (10 % near equilibrium)")
        wdot_table(g1, o1, sub(full, idx), "53 species, 2000 sampled points")
        transport_table(g1, o1, sub(full, idx), "53 species, 2000 sampled points")
        jac_table(g1, o1, sub(full, np.sort(rng.choice(1 << 18, size=64, replace=False))),
                  "53 species, 64 points sampled from the first 2^18")
        st4 = synth.state_c4_launch(200, 2, seed=4, launch=0)
        print("\n# 200 species / 1500 reactions: 2 spectral elements (1024 points) at 40 atm")
        wdot_table(g4, o4, st4, "200 species, 1024 points")
        jac_table(g4, o4, sub(st4, np.linspace(0, 1023, 16).astype(int)), "200 species, 16 points")
        g1.close()
        g4.close()


if __name__ == "__main__":
    main()
