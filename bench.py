"""Benchmark: production rates + dense Jacobian, 53 species, FP64 and mixed precision, on one MI355X.

Workload: the 53-species / 325-reaction mechanism (40 three-body, 25 Troe falloff),
2^18 points (the first 2^18 rows of the 2^20-point state: T ~ U[300, 2500] K with
10 % near-equilibrium points, p in {1, 10} atm, Y ~ Dirichlet(0.3)), synthetic.
One step = one fused crf_wdot_jac call (state, thermo, rate constants, falloff,
equilibrium constants, rates of progress, production rates and the dense Jacobian)
over the whole batch.  The rest of the per-point path is timed in the same run on the
2^20-point state ("path": production rates, transport, VJP, J v, source terms, the
stored-intermediate VJP and thermo, each with its HBM fraction and its fraction of the
bound set by its exponentials at the measured exponential rates in "peaks_measured"),
"c0" is the 9-species mechanism in microseconds per call, and "c4" the 200-species
figures aggregated over 8 launches of 1000-8000 spectral elements of 8^3 points at
40 atm (the mixed Jacobian in chunks of whole elements under a 12 GB budget).

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


def transcendentals(om, prec, kind):
    """FP64 and FP32 exponentials/logarithms per point of one call on this mechanism (the
    minimum the kernels evaluate): rate constants (one per reaction, FP32 in the mixed
    mode), 1/K_c (one FP64 per reaction in both modes), Troe P_r, F_cent (3), log F_cent,
    ln [M], F (6 per falloff reaction, plus k0 for derivatives); transport: mu_k, lambda_k
    and the pair diffusivities (FP32 in the mixed mode)."""
    nr = om.n_reactions
    nt = sum(1 for k in om.kind if k == "troe")
    ns = om.n_species
    if kind == "transport":
        n = 2 * ns + ns * (ns - 1) // 2
        return (0, n) if prec == "mixed" else (n, 0)
    deriv = kind in ("vjp", "jvp", "jac")
    rate = nr + 6 * nt + (nt if deriv else 0)
    return (nr, rate) if prec == "mixed" else (nr + rate, 0)


def measure_peaks(crf, stream):
    """Measured rates of the probe kinds (operations/s) and a plain HBM copy (GB/s)."""
    import ctypes

    import torch
    from paper_2409_06404_amd import _lib
    L = _lib.lib()
    threads = 256 * 256 * 8
    out = torch.empty(threads, dtype=torch.float64, device="cuda")
    res = {}
    for kind, name, iters in ((0, "exp_f64_library", 64), (1, "exp_f64_devicelib", 64), (2, "exp_f32_v_exp", 256),
                              (3, "fma_f64", 1024), (4, "fma_f32", 1024)):
        fn = lambda: _lib.check(L.crf_peak_rate(kind, threads, iters, ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(stream.cuda_stream)))
        ms = timed(fn, 3, 1, stream)
        res[name] = threads * iters * 8 / (ms * 1e-3)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    b = torch.empty_like(a)
    ms = timed(lambda: b.copy_(a), 5, 1, stream)
    res["hbm_copy_GBps"] = 2 * a.numel() * 8 / (ms * 1e-3) / 1e9
    del a, b, out
    torch.cuda.empty_cache()
    return res


def roof(n, ms, bytes_per_point, t64, t32, peaks):
    """Rate, HBM fraction and transcendental-bound fraction of one call."""
    rate = n / (ms * 1e-3)
    t_exp = t64 / peaks["exp_f64_library"] + t32 / peaks["exp_f32_v_exp"]      # s per point
    return {"mpoints_per_s": rate / 1e6, "bytes_per_point": bytes_per_point,
            "hbm_frac": rate * bytes_per_point / (HBM_PEAK_GBS * 1e9),
            "exp_per_point": [t64, t32], "exp_bound_mpoints_per_s": 1.0 / t_exp / 1e6 if t_exp > 0 else None,
            "exp_frac": rate * t_exp if t_exp > 0 else None}


def path_figures(crf, m, om, T, p, Y, u, prec, steps, stream, peaks):
    """Every per-point call on the 2^20-point state (C1: FP64; C2: mixed; C3: VJP)."""
    import torch
    n, ns = T.shape[0], om.n_species
    dev = T.device
    out = {}
    io = 8 * (2 + ns)
    calls = {
        "wdot": (lambda: crf.wdot(m, T, p, Y, prec, hrr=True), io + 8 * ns + 8, "wdot"),
        "transport": (lambda: crf.transport(m, T, p, Y, prec), io + 8 * ns + 16, "transport"),
        "vjp": (lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec), io + 8 * ns + 8 + 8 * ns, "vjp"),
        "jvp": (lambda: crf.wdot_jvp(m, T, p, Y, u, T, prec), io + 8 * ns + 8 + 8 * ns + 8, "jvp"),
        "source": (lambda: crf.source(m, T, p, Y, prec), io + 8 * ns + 24, "wdot"),
    }
    for name, (fn, bpp, kind) in calls.items():
        ms = timed(fn, steps, 1, stream)
        out[name] = roof(n, ms, bpp, *transcendentals(om, prec, kind), peaks)
    work = crf.new_workspace(m, n, prec)
    ms = timed(lambda: crf.wdot_fwd(m, T, p, Y, work, prec), steps, 1, stream)
    out["wdot_fwd_store"] = roof(n, ms, io + 8 * ns + 8 + 32 * om.n_reactions, *transcendentals(om, prec, "jac"),
                                 peaks)
    ms = timed(lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec, work=work), steps, 1, stream)
    out["vjp_stored"] = roof(n, ms, io + 16 * ns + 8 + 32 * om.n_reactions, 0, 0, peaks)
    del work
    torch.cuda.empty_cache()
    if prec == "fp64":
        ms = timed(lambda: crf.thermo(m, T, p, Y), steps, 1, stream)
        out["thermo"] = roof(n, ms, io + 4 * 8 * ns + 32, 0, 0, peaks)
    return out


def c0_latency(crf, steps, stream):
    """The 9-species / 21-reaction mechanism on 4096 points: microseconds per crf_wdot call
    (launch-bound by construction: fewer points than one wave per compute unit)."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda", 0)
    with tempfile.TemporaryDirectory() as d:
        path = synth.write_mechanism(synth.MECH_C0, os.path.join(d, "c0.mech"))
        m = crf.Mechanism(path, device=0)
        st = synth.state_c0(m.n_species, n=4096, seed=0)
        T = torch.from_numpy(st["T"]).to(dev)
        p = torch.from_numpy(st["p"]).to(dev)
        Y = torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t()
        us = timed(lambda: crf.wdot(m, T, p, Y, "fp64", hrr=True), max(steps, 200), 10, stream) * 1e3
        m.close()
    return {"workload": "9 species / 21 reactions, 4096 points, 1 atm", "us_per_call": us, "calls": max(steps, 200)}


def supporting_c4(crf, stream, budget_gb=12.0):
    """The 200-species / 1500-reaction mechanism (300 third-body, 150 Troe) at 40 atm over
    its 8 launches of U{1000..8000} spectral elements of 8^3 points (the same element-count
    draw as the parity state): production rates, transport and VJP over whole launches in both modes,
    and the mixed-mode Jacobian (201 x 201 FP32 per point) in chunks of whole elements
    that fit `budget_gb` GB, every chunk of every launch computed; aggregate rates."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda", 0)
    counts = synth.c4_element_counts(seed=4)
    with tempfile.TemporaryDirectory() as d:
        path = synth.write_mechanism(synth.MECH_C4, os.path.join(d, "c4.mech"))
        m = crf.Mechanism(path, device=0)
        ns = m.n_species
        n1 = ns + 1
        chunk = int(budget_gb * 1e9 / (n1 * n1 * 4)) // 512 * 512
        J = torch.empty((chunk, n1, n1), dtype=torch.float32, device=dev)
        tot = {"points": 0, "fp64": {"wdot": 0.0, "vjp": 0.0, "transport": 0.0},
               "mixed": {"wdot": 0.0, "vjp": 0.0, "transport": 0.0, "jac": 0.0}}
        per_launch = []
        for li, E in enumerate(counts):
            T, p, Ysm = synth.state_c4_launch_device(ns, E, seed=4, launch=li, device="cuda")
            Y = Ysm.t()
            n = T.shape[0]
            u = torch.randn((ns, n), dtype=torch.float64, device=dev).t()
            rec = {"elements": E, "points": n}
            for prec in ("fp64", "mixed"):
                for name, fn in (("wdot", lambda: crf.wdot(m, T, p, Y, prec, hrr=True)),
                                 ("vjp", lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec)),
                                 ("transport", lambda: crf.transport(m, T, p, Y, prec))):
                    ms = timed(fn, 1, 1 if li == 0 else 0, stream)
                    tot[prec][name] += ms
                    rec[f"{prec}_{name}_ms"] = ms
            def jac_all():
                for c0 in range(0, n, chunk):
                    c1 = min(n, c0 + chunk)
                    crf.wdot_jac(m, T[c0:c1], p[c0:c1], Y[c0:c1], "mixed", out=J[:c1 - c0], with_wdot=False)
            ms = timed(jac_all, 1, 1 if li == 0 else 0, stream)
            tot["mixed"]["jac"] += ms
            rec["mixed_jac_ms"] = ms
            tot["points"] += n
            per_launch.append(rec)
            del T, p, Ysm, Y, u
            torch.cuda.empty_cache()
        del J
        plan = m.jac_plan
        m.close()
        torch.cuda.empty_cache()
    agg = {prec: {k: tot["points"] / (v * 1e-3) / 1e6 for k, v in tot[prec].items()} for prec in ("fp64", "mixed")}
    jb = n1 * n1 * 4 + 8 * (2 + 2 * ns)
    return {"workload": "200 species / 1500 reactions (300 third-body, 150 Troe), 40 atm, 8 launches of "
                        f"{counts} elements x 8^3 points", "points": tot["points"], "unit": "Mpoints/s",
            "aggregate": agg, "jac_chunk_points": chunk, "jac_plan": plan,
            "jac_roofline": {"bound": "hbm", "bytes_per_point": jb,
                             "frac": agg["mixed"]["jac"] * 1e6 * jb / (HBM_PEAK_GBS * 1e9)},
            "per_launch": per_launch}


def reactor_figures(crf, m, full, stream, n=1 << 14, nsub=4, dt=1e-6):
    """crf_reactor_step on the first n points of the 2^20-point state (53 species): nsub ROS2
    substeps of dt/nsub per call, each a fused w + Jacobian evaluation, the Newton matrix and
    its LU factorisation per point, and the stage source terms; the state advances in place."""
    import numpy as np
    import torch
    dev = torch.device("cuda", 0)
    out = {"workload": f"53 species, {n} points, {nsub} ROS2 substeps of {dt / nsub:g} s per call", "points": n,
           "substeps": nsub}
    for prec in ("fp64", "mixed"):
        T = torch.from_numpy(full["T"][:n].copy()).to(dev)
        p = torch.from_numpy(full["p"][:n].copy()).to(dev)
        Y = torch.from_numpy(np.ascontiguousarray(full["Y"][:, :n])).to(dev).t()
        work = crf.reactor_workspace(m, n, prec)
        ms = timed(lambda: crf.reactor_step(m, T, p, Y, dt, nsub, prec, work=work), 5, 1, stream)
        out[prec] = {"ms_per_call": ms, "mpoint_substeps_per_s": n * nsub / (ms * 1e-3) / 1e6,
                     "workspace_bytes": int(work.numel())}
        del T, p, Y, work
        torch.cuda.empty_cache()
    return out


def variant_figures(crf, stream, n=1 << 18, steps=5):
    """The mechanism with every optional rate form (32 species; PLOG, Chebyshev, Lindemann,
    SRI, explicit reverse, irreversible and forward-order reactions) on n points of the
    9-species state's distributions with pressures over 0.05-60 atm: every per-point call
    (its Jacobian in the reaction-table kernel), and the Jacobian of the same mechanism
    without the non-integer orders (the segmented kernel)."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda", 0)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "v.mech")
        with open(path, "w") as fh:
            fh.write(synth.mechanism_text(synth.generate_variant_mechanism()))
        m = crf.Mechanism(path, device=0)
        ns = m.n_species
        st = synth.state_c0(ns, n=n, seed=7)
        st["p"] = st["p"] * np.geomspace(0.05, 60.0, n)[np.random.default_rng(7).permutation(n)]
        T = torch.from_numpy(st["T"]).to(dev)
        p = torch.from_numpy(st["p"]).to(dev)
        Y = torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t()
        u = torch.randn((ns, n), dtype=torch.float64, device=dev).t()
        out = {"workload": f"{ns} species / {m.n_reactions} reactions with every optional rate form, {n} points",
               "jac_plan": m.jac_plan}
        for prec in ("fp64", "mixed"):
            J = torch.empty((n, ns + 1, ns + 1), dtype=torch.float64 if prec == "fp64" else torch.float32, device=dev)
            calls = {"wdot": lambda: crf.wdot(m, T, p, Y, prec, hrr=True),
                     "transport": lambda: crf.transport(m, T, p, Y, prec),
                     "vjp": lambda: crf.wdot_vjp(m, T, p, Y, u, None, prec),
                     "jvp": lambda: crf.wdot_jvp(m, T, p, Y, u, T, prec),
                     "jac": lambda: crf.wdot_jac(m, T, p, Y, prec, out=J)}
            out[prec] = {k: n / (timed(fn, steps, 1, stream) * 1e-3) / 1e6 for k, fn in calls.items()}
            del J
            torch.cuda.empty_cache()
        m.close()
        # the same mechanism without its non-integer forward orders: the segmented Jacobian kernel
        path2 = os.path.join(d, "v_no_orders.mech")
        with open(path2, "w") as fh:
            fh.write(synth.mechanism_text(synth.generate_variant_mechanism(orders=False)))
        m2 = crf.Mechanism(path2, device=0)
        out["no_orders_jac_plan"] = m2.jac_plan
        for prec in ("fp64", "mixed"):
            J = torch.empty((n, ns + 1, ns + 1), dtype=torch.float64 if prec == "fp64" else torch.float32, device=dev)
            out[prec]["jac_no_orders"] = n / (timed(lambda: crf.wdot_jac(m2, T, p, Y, prec, out=J), steps, 1, stream)
                                              * 1e-3) / 1e6
            del J
            torch.cuda.empty_cache()
        m2.close()
    out["unit"] = "Mpoints/s"
    return out


def cpu_baseline(mech_path, st, n_sample):
    """The FP64 numpy oracle (production rates + analytic Jacobian) on a bounded sample;
    cores = the host threads it kept busy on average (process CPU time / wall time)."""
    import numpy as np

    import oracle
    om = oracle.read_mechanism(mech_path)
    T, p, Y = st["T"][:n_sample], st["p"][:n_sample], np.ascontiguousarray(st["Y"][:, :n_sample].T)
    try:
        from threadpoolctl import threadpool_info
        blas = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        blas = None
    c0, w0 = time.process_time(), time.perf_counter()
    oracle.production_rates(om, T, p, Y)
    w1 = time.perf_counter()
    oracle.jacobian(om, T, p, Y)
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    return {"value": n_sample / wall / 1e6, "unit": "Mpoints/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"{n_sample} points of the same state: production rates ({w1 - w0:.1f} s) + analytic "
                      f"Jacobian ({wall - (w1 - w0):.1f} s), FP64 numpy; {cpu / wall:.1f} threads busy on average "
                      f"(BLAS pool {blas}, host CPUs {os.cpu_count()})"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=1 << 18)
    ap.add_argument("--path-points", type=int, default=1 << 20,
                    help="points of the supporting per-point calls (the 2^20-point state)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10240,
                    help="points of the oracle CPU baseline (about 10-30 s of host time)")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None, help="time one precision only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (the reference for HBM byte counters)")
    ap.add_argument("--no-path", action="store_true", help="time the fused wdot+Jacobian call only")
    ap.add_argument("--no-c4", action="store_true", help="skip the 200-species supporting figures")
    ap.add_argument("--no-jac", action="store_true",
                    help="skip the headline Jacobian (profiling runs of the supporting calls)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the per-point chemistry shards trivially by points; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    import synth
    import paper_2409_06404_amd as crf

    dev = torch.device("cuda", 0)
    n = args.points
    with tempfile.TemporaryDirectory() as d:
        mech_path = synth.write_mechanism(synth.MECH_C1, os.path.join(d, "c1.mech"))
        om = oracle.read_mechanism(mech_path)
        m = crf.Mechanism(mech_path, device=0)
        ns = m.n_species
        full = synth.state_c1(ns, n=1 << 20, seed=1)
        st = {"T": full["T"][:n], "p": full["p"][:n], "Y": np.ascontiguousarray(full["Y"][:, :n])}
        T = torch.from_numpy(st["T"]).to(dev)
        p = torch.from_numpy(st["p"]).to(dev)
        Y = torch.from_numpy(st["Y"]).to(dev).t()
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
        for prec in ([] if args.no_jac else precs):
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
        path, peaks, c0, reactor, variants = {}, None, None, None, None
        if not args.no_path:
            peaks = measure_peaks(crf, stream)
            npath = args.path_points
            Tf = torch.from_numpy(full["T"][:npath]).to(dev)
            pf = torch.from_numpy(full["p"][:npath]).to(dev)
            Yf = torch.from_numpy(np.ascontiguousarray(full["Y"][:, :npath])).to(dev).t()
            uf = torch.randn((ns, npath), dtype=torch.float64, device=dev).t()
            for prec in precs:
                path[prec] = path_figures(crf, m, om, Tf, pf, Yf, uf, prec, max(3, args.steps // 4), stream, peaks)
            path["points"] = npath
            del Tf, pf, Yf, uf
            torch.cuda.empty_cache()
            c0 = c0_latency(crf, args.steps, stream)
            reactor = reactor_figures(crf, m, full, stream)
            variants = variant_figures(crf, stream)
        m.close()
        if args.no_jac:
            print(json.dumps({"path": path, "peaks_measured": peaks, "c0": c0, "reactor": reactor,
                              "variants": variants}), flush=True)
            return
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
        if not args.no_path:
            out["peaks_measured"] = peaks
            out["path"] = path
            out["c0"] = c0
            out["reactor"] = reactor
            out["variants"] = variants
        if not (args.no_path or args.no_c4):
            out["c4"] = supporting_c4(crf, stream)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(mech_path, st, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
