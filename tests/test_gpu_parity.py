"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Bounds: FP64 mode 1e-12 relative (E_norm on significant species, E_turn, scaled
Jacobian error); mixed mode 1e-5 on E_norm of significant species and on the
scaled Jacobian error.  Sizes span several tiles of 64 lanes with ragged tails;
full-size cases compare sampled points.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from metrics import (e_norm, e_turn, fp32_range_split, jac_scaled_error, significant_species,  # noqa: E402
                     vjp_scaled_error)

pytestmark = pytest.mark.gpu

R = 8314.46261815324


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.fixture(scope="module")
def crf():
    _need_gpu()
    import paper_2409_06404_amd as crf
    return crf


@pytest.fixture(scope="module")
def mechs(crf, c0_path, c1_path):
    out = {}
    for name, path in (("c0", c0_path), ("c1", c1_path)):
        out[name] = (crf.Mechanism(path, device=0), oracle.read_mechanism(path))
    yield out
    for g, _ in out.values():
        g.close()


def to_dev(st, ld=None):
    dev = torch.device("cuda", 0)
    Ysm = st["Y"]
    ns, n = Ysm.shape
    ld = ld or n
    buf = torch.full((ns, ld), float("nan"), dtype=torch.float64, device=dev)
    buf[:, :n] = torch.from_numpy(Ysm).to(dev)
    return (torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["p"]).to(dev), buf[:, :n].t())


def state(which, n, seed=0):
    ns = 9 if which == "c0" else 53
    if which == "c0":
        return synth.state_c0(ns, n=n, seed=seed)
    return synth.state_c1(ns, n=n, seed=seed + 1)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------ production rates
@pytest.mark.parametrize("which,n", [("c0", 3000), ("c1", 3001)])
def test_wdot_fp64(crf, mechs, which, n):
    g, om = mechs[which]
    st = state(which, n)
    T, p, Y = to_dev(st)
    log(f"wdot fp64 {which} n={n}")
    w, h, r = crf.wdot(g, T, p, Y, "fp64", hrr=True, mass_resid=True)
    torch.cuda.synchronize()
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    w = w.cpu().numpy()
    sig = significant_species(ref["wdot"], om.W)
    en = e_norm(w, ref["wdot"])
    et = e_turn(w, ref["wdot"], ref["turnover"])
    log(f"  E_norm max {en[sig].max():.2e}  E_turn max {et.max():.2e}")
    assert en[sig].max() <= 1e-12
    assert et.max() <= 1e-12
    _, hRT, _, _ = oracle.nasa7(om, st["T"])
    hscale = (np.abs(R * st["T"][:, None] * hRT) * (ref["turnover"] + np.abs(ref["wdot"]))).sum(axis=1)
    assert np.max(np.abs(h.cpu().numpy() - ref["hrr"]) / hscale) <= 1e-12
    assert np.max(np.abs(r.cpu().numpy()) / (ref["turnover"] @ om.W)) <= 1e-13


def test_wdot_mixed_c1(crf, mechs):
    g, om = mechs["c1"]
    st = state("c1", 4097)
    T, p, Y = to_dev(st)
    w, h, r = crf.wdot(g, T, p, Y, "mixed", hrr=True, mass_resid=True)
    torch.cuda.synchronize()
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    w = w.cpu().numpy()
    sig = significant_species(ref["wdot"], om.W)
    en = e_norm(w, ref["wdot"])
    et = e_turn(w, ref["wdot"], ref["turnover"])
    log(f"wdot mixed c1: E_norm max {en[sig].max():.2e} median {np.median(en[sig]):.2e}  E_turn max {et.max():.2e}")
    assert en[sig].max() <= 1e-5
    # the mass residual is formed in FP64 from the FP64-accumulated rates
    assert np.max(np.abs(r.cpu().numpy()) / (ref["turnover"] @ om.W)) <= 1e-13


@pytest.mark.parametrize("call", ["wdot", "jac"])
def test_mixed_near_equilibrium(crf, mechs, call):
    """Mixed mode on the near-equilibrium share of the 53-species state alone: there
    q_f and q_r cancel to about three digits, so the equilibrium constant (FP64 in both
    modes) decides q.  Bound: E_norm <= 1e-5 on significant species."""
    g, om = mechs["c1"]
    st = synth.state_c1(53, n=4000, seed=2)
    ne = st["near_eq"]
    sub = {"T": st["T"][ne], "p": st["p"][ne], "Y": np.ascontiguousarray(st["Y"][:, ne])}
    T, p, Y = to_dev(sub)
    if call == "wdot":
        w = crf.wdot(g, T, p, Y, "mixed", hrr=False)[0]
    else:
        w = crf.wdot_jac(g, T, p, Y, "mixed")[1]
    torch.cuda.synchronize()
    ref = oracle.production_rates(om, sub["T"], sub["p"], sub["Y"].T)
    q = oracle.rates_of_progress(om, sub["T"], sub["p"], sub["Y"].T)
    assert np.median(np.abs(q["q"]) / np.abs(q["qf"])) < 1e-2      # the share is near equilibrium
    w = w.cpu().numpy()
    sig = significant_species(ref["wdot"], om.W)
    en = e_norm(w, ref["wdot"])
    et = e_turn(w, ref["wdot"], ref["turnover"])
    log(f"mixed near-eq {call} ({int(ne.sum())} points): E_norm max {en[sig].max():.2e}  E_turn max {et.max():.2e}")
    assert en[sig].max() <= 1e-5


# ------------------------------------------------------------------ thermo / transport
def test_thermo_fp64(crf, mechs):
    g, om = mechs["c1"]
    st = state("c1", 1500)
    T, p, Y = to_dev(st)
    out = crf.thermo(g, T, p, Y)
    torch.cuda.synchronize()
    ref = oracle.thermo_properties(om, st["T"], st["p"], st["Y"].T)
    for k in ("cp_k", "h_k", "s_k", "g_k"):
        a = out[k].cpu().numpy()
        scale = np.abs(ref[k]).max(axis=0, keepdims=True)
        assert np.max(np.abs(a - ref[k]) / scale) <= 1e-13, k
    for k in ("cp_mass", "h_mass", "rho", "Wbar"):
        a = out[k].cpu().numpy()
        scale = np.abs(ref[k]).max()
        assert np.max(np.abs(a - ref[k]) / scale) <= 1e-13, k


@pytest.mark.parametrize("which,prec,tol", [("c0", "fp64", 1e-12), ("c1", "fp64", 1e-12), ("c1", "mixed", 1e-5)])
def test_transport(crf, mechs, which, prec, tol):
    g, om = mechs[which]
    st = state(which, 331)
    T, p, Y = to_dev(st)
    mu, lam, D = crf.transport(g, T, p, Y, prec)
    torch.cuda.synchronize()
    ref = oracle.transport_properties(om, st["T"], st["p"], st["Y"].T)
    e_mu = np.max(np.abs(mu.cpu().numpy() / ref["mu"] - 1))
    e_lam = np.max(np.abs(lam.cpu().numpy() / ref["lambda"] - 1))
    e_d = np.max(np.abs(D.cpu().numpy() / ref["Dmix"] - 1))
    log(f"transport {which} {prec}: mu {e_mu:.2e} lambda {e_lam:.2e} Dmix {e_d:.2e}")
    assert max(e_mu, e_lam, e_d) <= tol


# ------------------------------------------------------------------ derivatives
def _jac_err(Jg, Jr, om, st, floor=0.0):
    """Scaled Jacobian error; floor > 0 marks an FP32 result (range split + floor)."""
    T, p, Yn = st["T"], st["p"], st["Y"].T
    _, G = oracle.jacobian(om, T, p, Yn, return_gross=True)
    if floor > 0:
        Jg, Jr = fp32_range_split(Jg, Jr)
    return jac_scaled_error(Jg, Jr, G, T, Yn, floor=floor)


# The mixed-mode Jacobian is stored in FP32: rows below 1e-10 of a point's dominant row
# are measured against that floor (see metrics.jac_scaled_error).
MIXED_FLOOR = 1e-10


@pytest.mark.parametrize("which,prec,tol", [("c0", "fp64", 1e-12), ("c1", "fp64", 1e-12),
                                            ("c0", "mixed", 1e-5), ("c1", "mixed", 1e-5)])
def test_jacobian(crf, mechs, which, prec, tol):
    g, om = mechs[which]
    st = state(which, 130)
    T, p, Y = to_dev(st)
    log(f"jac {which} {prec}")
    J, w = crf.wdot_jac(g, T, p, Y, prec)
    torch.cuda.synchronize()
    Jr = oracle.jacobian(om, st["T"], st["p"], st["Y"].T)
    err = _jac_err(J.double().cpu().numpy(), Jr, om, st, floor=MIXED_FLOOR if prec == "mixed" else 0.0)
    log(f"  scaled J error per row: max {err.max():.2e} (row {int(err.argmax())})")
    assert err.max() <= tol
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    w = w.cpu().numpy()
    if prec == "fp64":
        assert e_turn(w, ref["wdot"], ref["turnover"]).max() <= 1e-12
    else:   # mixed: E_norm on significant species is the bound; E_turn is reported only
        sig = significant_species(ref["wdot"], om.W)
        assert e_norm(w, ref["wdot"])[sig].max() <= 1e-5
        log(f"  mixed fused w: E_turn max {e_turn(w, ref['wdot'], ref['turnover']).max():.2e}")


@pytest.mark.parametrize("which,prec,tol", [("c0", "fp64", 1e-12), ("c1", "fp64", 1e-12), ("c1", "mixed", 1e-5)])
def test_vjp(crf, mechs, which, prec, tol):
    g, om = mechs[which]
    st = state(which, 97)
    T, p, Y = to_dev(st)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(st["Y"].shape)             # species-major like Y
    uh = rng.standard_normal(st["T"].shape) * 1e-6
    ut = torch.from_numpy(u).cuda().t()
    gT, gY = crf.wdot_vjp(g, T, p, Y, ut, torch.from_numpy(uh).cuda(), prec)
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    uu = np.concatenate([uh[:, None], u.T], axis=1)
    gref = np.einsum("nr,nrc->nc", uu, Jr)
    got = np.concatenate([gT.cpu().numpy()[:, None], gY.cpu().numpy()], axis=1)
    err = vjp_scaled_error(got, gref, uu, G)
    log(f"vjp {which} {prec}: {err:.2e}")
    assert err <= tol


def test_jacobian_central_differences_1024(crf, mechs):
    """GPU Jacobian against central differences of the GPU production rates (h = 1e-6 relative)."""
    g, om = mechs["c1"]
    st = synth.state_c1(53, n=1024, seed=1)
    T, p, Y = to_dev(st)
    J, _ = crf.wdot_jac(g, T, p, Y, "fp64", with_wdot=False)
    n, ns = 1024, 53
    Jfd = torch.empty_like(J)
    Ysm = Y.t().contiguous()
    for c in range(ns + 1):
        if c == 0:
            h = 1e-6 * T
            wp, hp, _ = crf.wdot(g, T + h, p, Y)
            wm, hm, _ = crf.wdot(g, T - h, p, Y)
        else:
            h = 1e-6 * torch.clamp(Ysm[c - 1], min=1e-10)
            Yp = Ysm.clone(); Yp[c - 1] += h
            Ym = Ysm.clone(); Ym[c - 1] -= h
            wp, hp, _ = crf.wdot(g, T, p, Yp.t())
            wm, hm, _ = crf.wdot(g, T, p, Ym.t())
        Jfd[:, 0, c] = (hp - hm) / (2 * h)
        Jfd[:, 1:, c] = (wp - wm) / (2 * h[:, None])
    torch.cuda.synchronize()
    err = _jac_err(Jfd.cpu().numpy(), J.cpu().numpy(), om, st)
    log(f"central FD vs GPU J: {err.max():.2e}")
    assert err.max() <= 1e-6


def test_autograd_function(crf, mechs):
    g, om = mechs["c0"]
    rng = np.random.default_rng(5)
    n = 6
    Ysm = rng.dirichlet(np.full(9, 20.0), size=n).T.copy()
    st = {"T": rng.uniform(900, 2000, n), "p": np.full(n, 101325.0), "Y": Ysm}
    T, p, Y = to_dev(st)
    T = T.clone().requires_grad_(True)
    Yl = Y.detach().clone()        # keep the species-major layout for the leaf
    Ysm_leaf = Yl.t().contiguous().requires_grad_(True)
    w, h = crf.WdotFn.apply(T, Ysm_leaf.t(), p, g, "fp64")
    (w.sum() + 1e-3 * h.sum()).backward()
    torch.cuda.synchronize()
    gT_ref, gY_ref = oracle.vjp(om, st["T"], st["p"], st["Y"].T, np.ones((n, 9)), np.full(n, 1e-3))
    np.testing.assert_allclose(T.grad.cpu().numpy(), gT_ref, rtol=1e-10, atol=1e-10 * np.abs(gT_ref).max())
    np.testing.assert_allclose(Ysm_leaf.grad.t().cpu().numpy(), gY_ref, rtol=1e-10,
                               atol=1e-10 * np.abs(gY_ref).max())

    def f(Tv, Yv):
        return crf.WdotFn.apply(Tv, Yv.t(), p, g, "fp64")[0]
    T2 = torch.from_numpy(st["T"]).cuda().requires_grad_(True)
    Y2 = torch.from_numpy(Ysm).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(f, (T2, Y2), eps=1e-6, atol=1e-6, rtol=1e-4)


# ------------------------------------------------------------------ edge cases
def test_edge_cases(crf, mechs):
    g, om = mechs["c1"]
    dev = torch.device("cuda", 0)
    # n = 0: no-op
    e = torch.empty(0, dtype=torch.float64, device=dev)
    w, h, _ = crf.wdot(g, e, e, torch.empty((53, 0), dtype=torch.float64, device=dev).t())
    assert w.shape == (0, 53)
    # n = 1, scalar pressure, padded leading dimension, exact zeros in Y
    st = state("c1", 67)
    st["Y"][5, :] = 0.0
    st["Y"][17, 3] = 0.0
    st["p"][:] = 101325.0 * 10
    T, _, Y = to_dev(st, ld=80)
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    w, h, _ = crf.wdot(g, T, 101325.0 * 10, Y)
    torch.cuda.synchronize()
    assert w.stride() == (1, 80)
    w = w.cpu().numpy()
    assert np.all(np.isfinite(w))
    assert e_turn(w, ref["wdot"], ref["turnover"]).max() <= 1e-12
    J, _ = crf.wdot_jac(g, T[:1], torch.tensor(101325.0 * 10, dtype=torch.float64, device=dev), Y[:1])
    Jr = oracle.jacobian(om, st["T"][:1], st["p"][:1], st["Y"].T[:1])
    sub = {"T": st["T"][:1], "p": st["p"][:1], "Y": st["Y"][:, :1]}
    assert _jac_err(J.cpu().numpy(), Jr, om, sub).max() <= 1e-12
    assert np.all(np.isfinite(J.cpu().numpy()))


def test_bitwise_reproducible(crf, mechs):
    g, _ = mechs["c1"]
    st = state("c1", 2000)
    T, p, Y = to_dev(st)
    a = crf.wdot(g, T, p, Y)[0].clone()
    b = crf.wdot(g, T, p, Y)[0].clone()
    Ja = crf.wdot_jac(g, T[:200], p[:200], Y[:200])[0].clone()
    Jb = crf.wdot_jac(g, T[:200], p[:200], Y[:200])[0].clone()
    ta = [x.clone() for x in crf.transport(g, T, p, Y)]
    tb = [x.clone() for x in crf.transport(g, T, p, Y)]
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(Ja, Jb)
    assert all(torch.equal(x, y) for x, y in zip(ta, tb))


def test_invalid_arguments_raise(crf, mechs):
    g, _ = mechs["c0"]
    st = state("c0", 10)
    T, p, Y = to_dev(st)
    with pytest.raises(ValueError):
        crf.wdot(g, T, p, Y.contiguous())                 # point-major layout is rejected
    with pytest.raises(ValueError):
        crf.wdot(g, T, p, Y, precision="bf16")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_transport_ragged_tiles_and_partial_outputs(crf, mechs, prec, tol):
    """Transport works on tiles of 16 points: point counts around the tile size, a padded
    leading dimension, one pressure for all points, and each output requested alone."""
    g, om = mechs["c1"]
    dev = torch.device("cuda", 0)
    st = state("c1", 77)
    st["Y"][11, :] = 0.0
    ref = oracle.transport_properties(om, st["T"], np.full(77, 3e5), st["Y"].T)
    for n in (1, 15, 16, 17, 33, 77):
        sub = {"T": st["T"][:n], "p": np.full(n, 3e5), "Y": np.ascontiguousarray(st["Y"][:, :n])}
        T, _, Y = to_dev(sub, ld=n + 3)
        log(f"transport ragged {prec} n={n}")
        mu, lam, D = crf.transport(g, T, 3e5, Y, prec)
        torch.cuda.synchronize()
        assert np.max(np.abs(mu.cpu().numpy() / ref["mu"][:n] - 1)) <= tol
        assert np.max(np.abs(lam.cpu().numpy() / ref["lambda"][:n] - 1)) <= tol
        assert np.max(np.abs(D.cpu().numpy() / ref["Dmix"][:n] - 1)) <= tol
    T, _, Y = to_dev({"T": st["T"], "p": st["p"], "Y": st["Y"]})
    from paper_2409_06404_amd import _lib
    import ctypes
    L = _lib.lib()
    out = torch.full((77,), -1.0, dtype=torch.float64, device=dev)
    Dm = torch.full((53, 77), -1.0, dtype=torch.float64, device=dev)
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    pr = torch.full((77,), 3e5, dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    prec_id = 0 if prec == "fp64" else 1
    for which in ("mu", "lambda", "Dmix"):
        out.fill_(-1.0)
        Dm.fill_(-1.0)
        args = {"mu": None, "lambda": None, "Dmix": None}
        args[which] = Dm if which == "Dmix" else out
        _lib.check(L.crf_transport(g.handle, prec_id, 77, P(T), P(pr), 1, P(Y), Y.stride(1), P(args["mu"]),
                                   P(args["lambda"]), P(args["Dmix"]), stream))
        torch.cuda.synchronize()
        got = (Dm.t() if which == "Dmix" else out).cpu().numpy()
        assert np.max(np.abs(got / ref[which] - 1)) <= tol, which


# ------------------------------------------------------------------ full sizes (sampled)
@pytest.fixture(scope="module")
def c1_full():
    return synth.state_c1(53, n=1 << 20, seed=1)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_full_size_wdot_sampled(crf, mechs, c1_full, prec, tol):
    g, om = mechs["c1"]
    T, p, Y = to_dev(c1_full)
    log(f"full-size wdot {prec} n=2^20")
    w, h, r = crf.wdot(g, T, p, Y, prec, hrr=True, mass_resid=True)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(1 << 20, size=1500, replace=False)
    idx = np.concatenate([idx, [0, (1 << 20) - 1]])
    ref = oracle.production_rates(om, c1_full["T"][idx], c1_full["p"][idx], c1_full["Y"][:, idx].T)
    got = w[torch.from_numpy(idx).cuda()].cpu().numpy()
    sig = significant_species(ref["wdot"], om.W)
    en = e_norm(got, ref["wdot"])
    log(f"  E_norm max {en[sig].max():.2e}")
    assert en[sig].max() <= tol
    assert torch.isfinite(w).all() and torch.isfinite(h).all()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_full_size_transport_sampled(crf, mechs, c1_full, prec, tol):
    g, om = mechs["c1"]
    T, p, Y = to_dev(c1_full)
    log(f"full-size transport {prec} n=2^20")
    mu, lam, D = crf.transport(g, T, p, Y, prec)
    torch.cuda.synchronize()
    idx = np.concatenate([np.random.default_rng(2).choice(1 << 20, size=400, replace=False), [0, (1 << 20) - 1]])
    ref = oracle.transport_properties(om, c1_full["T"][idx], c1_full["p"][idx], c1_full["Y"][:, idx].T)
    ii = torch.from_numpy(idx).cuda()
    e = [np.max(np.abs(mu[ii].cpu().numpy() / ref["mu"] - 1)), np.max(np.abs(lam[ii].cpu().numpy() / ref["lambda"] - 1)),
         np.max(np.abs(D[ii].cpu().numpy() / ref["Dmix"] - 1))]
    log(f"  mu {e[0]:.2e} lambda {e[1]:.2e} Dmix {e[2]:.2e}")
    assert max(e) <= tol
    del mu, lam, D
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_full_size_jacobian_sampled(crf, mechs, c1_full, prec, tol):
    """The benchmarked configuration: 2^18 points, 53 species, fused w output."""
    g, om = mechs["c1"]
    n = 1 << 18
    sub = {"T": c1_full["T"][:n], "p": c1_full["p"][:n], "Y": np.ascontiguousarray(c1_full["Y"][:, :n])}
    T, p, Y = to_dev(sub)
    log(f"full-size jac {prec} n=2^18")
    J, w = crf.wdot_jac(g, T, p, Y, prec)
    torch.cuda.synchronize()
    idx = np.concatenate([np.random.default_rng(1).choice(n, size=48, replace=False), [0, n - 1]])
    Jr = oracle.jacobian(om, sub["T"][idx], sub["p"][idx], sub["Y"][:, idx].T)
    s = {"T": sub["T"][idx], "p": sub["p"][idx], "Y": sub["Y"][:, idx]}
    err = _jac_err(J[torch.from_numpy(idx).cuda()].double().cpu().numpy(), Jr, om, s,
                   floor=MIXED_FLOOR if prec == "mixed" else 0.0)
    log(f"  scaled J error max {err.max():.2e}")
    assert err.max() <= tol
    if prec == "fp64":
        assert torch.isfinite(J).all()
    del J
    torch.cuda.empty_cache()
