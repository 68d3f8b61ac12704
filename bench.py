"""Benchmark: production rates + dense Jacobian, 53 species, FP64 and mixed precision, on one MI355X.

Workload: the 53-species / 325-reaction mechanism (40 three-body, 25 Troe falloff),
2^18 points (the first 2^18 rows of the 2^20-point state: T ~ U[300, 2500] K with
10 % near-equilibrium points, p in {1, 10} atm, Y ~ Dirichlet(0.3)), synthetic.
One step = one fused crf_wdot_jac call (state, thermo, rate constants, falloff,
equilibrium constants, rates of progress, production rates and the dense Jacobian)
over the whole batch.  The rest of the per-point path (thermo, transport, VJP) is
timed in the same run and reported under "path_mpoints_per_s"; "supporting" holds the
200-species figures (one launch of 1000 spectral elements of 8^3 points at 40 atm; the
mixed Jacobian on a chunk of 2^15 points).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-path] [--no-c4]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def jac_bytes_per_point(ns, prec):
    """Algorithmic HBM bytes per point of crf_wdot_jac: read T, p, Y; write J and w."""
    n1 = ns + 1
    return 8 * (2 + ns) + (8 if prec == "fp64" else 4) * n1 * n1 + 8 * ns


def kernel_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_2409_06404_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def jac_kernel_name(plan, prec):
    """Name (as rocprofv3 shows it, shortened) of the kernel crf_wdot_jac launches."""
    base = ("k_jac_seg" if plan.startswith("segmented") else
            "k_jac_rt" if plan.startswith("reaction-table") else "k_jac")
    return "%s<%s>" % (base, "false" if prec == "fp64" else "true")


def recorded_traffic(kernel, prec):
    """HBM bytes per launch of the Jacobian kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{prec}_53sp_2p18_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("RESULT "):
            for tok in line.split()[1:]:
                k, v = tok.split("=")
                rec[k] = v
    if rec.get("kernel_sha") != kernel_source_hash():
        return None
    return float(rec["bytes_per_launch"])


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps      # ms per call


def supporting_c4(crf, steps):
    """Supporting figures on the 200-species / 1500-reaction mechanism (300 third-body,
    150 Troe) at 40 atm: one launch of 1000 spectral elements of 8^3 points with flame
    fronts (512 000 points): production rates, transport and VJP in both modes, and the
    mixed-mode Jacobian (FP32, 201 x 201 per point) on a chunk of 2^15 points."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    with tempfile.TemporaryDirectory() as d:
        path = synth.write_mechanism(synth.MECH_C4, os.path.join(d, "c4.mech"))
        m = crf.Mechanism(path, device=0)
        ns = m.n_species
        st = synth.state_c4_launch(ns, 1000, seed=4, launch=0)
        n = st["T"].shape[0]
        T = torch.from_numpy(st["T"]).to(dev)
        p = torch.from_numpy(st["p"]).to(dev)
        Y = torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t()
        u = torch.randn((ns, n), dtype=torch.float64, device=dev).t()
        out = {"workload": "200 species / 1500 reactions (300 third-body, 150 Troe), 40 atm, "
                           "1000 elements x 8^3 points", "n_points": n, "unit": "Mpoints/s"}
        for prec in ("fp64", "mixed"):
            out[prec] = {
                "wdot": n / (timed(lambda: crf.wdot(m, T, p, Y, prec, hrr=True), steps, 1, stream) * 1e-3) / 1e6,
                "transport": n / (timed(lambda: crf.transport(m, T, p, Y, prec), steps, 1, stream) * 1e-3) / 1e6,
                "vjp": n / (timed(lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec), steps, 1, stream) * 1e-3) / 1e6,
            }
        nj = 1 << 15
        J = torch.empty((nj, ns + 1, ns + 1), dtype=torch.float32, device=dev)
        Tj, pj, Yj = T[:nj], p[:nj], Y[:nj]
        ms = timed(lambda: crf.wdot_jac(m, Tj, pj, Yj, "mixed", out=J), steps, 1, stream)
        out["mixed"]["jac_chunk"] = nj / (ms * 1e-3) / 1e6
        out["jac_chunk_points"] = nj
        out["jac_plan"] = m.jac_plan
        del J
        m.close()
        torch.cuda.empty_cache()
    return out


def cpu_baseline(mech_path, st, n_sample):
    """The FP64 numpy oracle (production rates + analytic Jacobian) on a bounded sample."""
    import numpy as np

    import oracle
    om = oracle.read_mechanism(mech_path)
    T, p, Y = st["T"][:n_sample], st["p"][:n_sample], np.ascontiguousarray(st["Y"][:, :n_sample].T)
    c0, w0 = time.process_time(), time.perf_counter()
    oracle.production_rates(om, T, p, Y)
    oracle.jacobian(om, T, p, Y)
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    return {"value": n_sample / wall / 1e6, "unit": "Mpoints/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"{n_sample} points of the same state (production rates + analytic Jacobian, FP64 numpy), "
                      f"{wall:.1f} s wall on {os.cpu_count()} host CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=1 << 18)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10240,
                    help="points of the oracle CPU baseline (about 10-30 s of host time)")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None, help="time one precision only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (the reference for HBM byte counters)")
    ap.add_argument("--no-path", action="store_true", help="time the fused wdot+Jacobian call only")
    ap.add_argument("--no-c4", action="store_true", help="skip the 200-species supporting figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the per-point chemistry shards trivially by points; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2409_06404_amd as crf

    dev = torch.device("cuda", 0)
    n = args.points
    with tempfile.TemporaryDirectory() as d:
        mech_path = synth.write_mechanism(synth.MECH_C1, os.path.join(d, "c1.mech"))
        m = crf.Mechanism(mech_path, device=0)
        ns = m.n_species
        full = synth.state_c1(ns, n=1 << 20, seed=1)
        st = {"T": full["T"][:n], "p": full["p"][:n], "Y": np.ascontiguousarray(full["Y"][:, :n])}
        T = torch.from_numpy(st["T"]).to(dev)
        p = torch.from_numpy(st["p"]).to(dev)
        Y = torch.from_numpy(st["Y"]).to(dev).t()
        u = torch.randn((ns, n), dtype=torch.float64, device=dev).t()
        stream = torch.cuda.current_stream(dev)
        if args.calib_copy:
            a = torch.ones(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            del a, b
            torch.cuda.empty_cache()
        res = {}
        precs = [args.only] if args.only else ["fp64", "mixed"]
        for prec in precs:
            J = torch.empty((n, ns + 1, ns + 1), dtype=torch.float64 if prec == "fp64" else torch.float32,
                            device=dev)
            ms = timed(lambda: crf.wdot_jac(m, T, p, Y, prec, out=J), args.steps, args.warmup, stream)
            kname = jac_kernel_name(m.jac_plan, prec)
            bpp = jac_bytes_per_point(ns, prec)
            achieved = bpp * n / (ms * 1e-3) / 1e9
            res[prec] = {"value": n / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                         "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": achieved / HBM_PEAK_GBS,
                                      "traffic": recorded_traffic(kname.split("<")[0], prec),
                                      "bytes_per_point": bpp, "kernel": kname}}
            del J
            torch.cuda.empty_cache()
        path = {}
        for prec in ([] if args.no_path else precs):
            path[prec] = {
                "wdot": n / (timed(lambda: crf.wdot(m, T, p, Y, prec, hrr=True), args.steps, 1, stream) * 1e-3) / 1e6,
                "transport": n / (timed(lambda: crf.transport(m, T, p, Y, prec), max(2, args.steps // 4), 1, stream) * 1e-3) / 1e6,
                "vjp": n / (timed(lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec), args.steps, 1, stream) * 1e-3) / 1e6,
                "jvp": n / (timed(lambda: crf.wdot_jvp(m, T, p, Y, u, T, prec), args.steps, 1, stream) * 1e-3) / 1e6,
                "source": n / (timed(lambda: crf.source(m, T, p, Y, prec), args.steps, 1, stream) * 1e-3) / 1e6,
            }
            work = crf.new_workspace(m, n, prec)
            path[prec]["wdot_fwd_store"] = n / (timed(lambda: crf.wdot_fwd(m, T, p, Y, work, prec), args.steps, 1,
                                                      stream) * 1e-3) / 1e6
            path[prec]["vjp_stored"] = n / (timed(lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec, work=work),
                                                  args.steps, 1, stream) * 1e-3) / 1e6
            del work
        if "fp64" in path:
            path["fp64"]["thermo"] = n / (timed(lambda: crf.thermo(m, T, p, Y), args.steps, 1, stream) * 1e-3) / 1e6
        m.close()
        head = "fp64" if "fp64" in res else precs[0]
        out = {
            "metric": "Mpoints/s wdot+Jacobian (53 sp), FP64 vs mixed precision, % of roofline",
            "value": res[head]["value"], "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res[head]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64" if head == "fp64" else "f32+f64",
            "data": "synthetic",
            "config": {"workload": "wdot + dense Jacobian (fused), 53 species / 325 reactions (40 three-body, "
                                   "25 Troe), 2^18 points, inputs resident in HBM",
                       "n_points": n, "species": ns, "reactions": 325, "precision": head},
            "roofline": res[head]["roofline"],
        }
        if "mixed" in res and head != "mixed":
            out["mixed"] = dict(res["mixed"], dtype="f32+f64")
        out["path_mpoints_per_s"] = path
        if not (args.no_path or args.no_c4):
            out["supporting"] = {"c4_200sp": supporting_c4(crf, max(3, args.steps // 4))}
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(mech_path, st, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
