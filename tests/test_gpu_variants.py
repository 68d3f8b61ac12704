"""Parity on the mechanism with every optional rate form (PLOG, Chebyshev, SRI and
Lindemann falloff, explicit reverse, irreversible, non-integer orders; 32 species, 76
reactions), on the GPU through the C ABI, FP64 1e-12 and mixed 1e-5, with pressures from
0.05 to 60 atm (PLOG below, inside and above its tables)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from metrics import (e_norm, e_turn, jac_scaled_error, significant_species,  # noqa: E402
                     vjp_scaled_error)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def var(mech_dir):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2409_06404_amd as crf
    path = str(mech_dir / "variants.mech")
    open(path, "w").write(synth.mechanism_text(synth.generate_variant_mechanism()))
    g = crf.Mechanism(path, device=0)
    yield crf, g, oracle.read_mechanism(path)
    g.close()


def _state(ns, n, seed):
    st = synth.state_c0(ns, n=n, seed=seed)
    st["p"] = st["p"] * np.geomspace(0.05, 60.0, n)[np.random.default_rng(seed).permutation(n)]
    return st


def _dev(st):
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["p"]).to(dev),
            torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t())


def test_variant_plan_is_reaction_table(var):
    """Non-integer forward orders keep a mechanism out of the segmented plan."""
    crf, g, om = var
    assert g.jac_plan.startswith("reaction-table") and "orders" in g.jac_plan


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_variant_wdot(var, prec, tol):
    crf, g, om = var
    st = _state(om.n_species, 1500, 61)
    T, p, Y = _dev(st)
    w, h, r = crf.wdot(g, T, p, Y, prec, hrr=True, mass_resid=True)
    torch.cuda.synchronize()
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    got = w.cpu().numpy()
    sig = significant_species(ref["wdot"], om.W)
    en = e_norm(got, ref["wdot"])
    print(f"variant wdot {prec}: E_norm {en[sig].max():.2e}", flush=True)
    assert en[sig].max() <= tol
    if prec == "fp64":
        assert e_turn(got, ref["wdot"], ref["turnover"]).max() <= 1e-12
    assert np.max(np.abs(r.cpu().numpy()) / (ref["turnover"] @ om.W)) <= 1e-13


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_variant_jacobian_vjp_jvp(var, prec, tol):
    crf, g, om = var
    n = 70
    st = _state(om.n_species, n, 62)
    T, p, Y = _dev(st)
    J, w = crf.wdot_jac(g, T, p, Y, prec)
    rng = np.random.default_rng(63)
    u = rng.standard_normal(st["Y"].shape)
    uh = rng.standard_normal(n) * 1e-6
    gT, gY = crf.wdot_vjp(g, T, p, Y, torch.from_numpy(u).cuda().t(), torch.from_numpy(uh).cuda(), prec)
    vT = rng.standard_normal(n) * 10.0
    vY = rng.standard_normal(st["Y"].shape) * st["Y"]
    jh, jw, _ = crf.wdot_jvp(g, T, p, Y, torch.from_numpy(vY).cuda().t(), torch.from_numpy(vT).cuda(), prec)
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    floor = 1e-10 if prec == "mixed" else 0.0
    ej = jac_scaled_error(J.double().cpu().numpy(), Jr, G, st["T"], st["Y"].T, floor=floor).max()
    uu = np.concatenate([uh[:, None], u.T], axis=1)
    ev = vjp_scaled_error(np.concatenate([gT.cpu().numpy()[:, None], gY.cpu().numpy()], axis=1),
                          np.einsum("nr,nrc->nc", uu, Jr), uu, G)
    v = np.concatenate([vT[:, None], vY.T], axis=1)
    ejv = np.max(np.abs(np.concatenate([jh.cpu().numpy()[:, None], jw.cpu().numpy()], axis=1)
                        - np.einsum("nrc,nc->nr", Jr, v)) / (np.einsum("nrc,nc->nr", G, np.abs(v)) + 1e-300))
    print(f"variant {prec}: J {ej:.2e} VJP {ev:.2e} JVP {ejv:.2e}", flush=True)
    assert max(ej, ev, ejv) <= tol


def test_variant_stored_vjp_and_source(var):
    crf, g, om = var
    n = 90
    st = _state(om.n_species, n, 64)
    T, p, Y = _dev(st)
    u = torch.from_numpy(np.random.default_rng(65).standard_normal(st["Y"].shape)).cuda().t()
    work = crf.new_workspace(g, n)
    crf.wdot_fwd(g, T, p, Y, work)
    gT, gY = crf.wdot_vjp(g, T, p, Y, u, work=work)
    gT0, gY0 = crf.wdot_vjp(g, T, p, Y, u)
    out = crf.source(g, T, p, Y, dp0dt=1e4)
    torch.cuda.synchronize()
    assert torch.equal(gT, gT0) and torch.equal(gY, gY0)
    ref = oracle.chemistry_source(om, st["T"], st["p"], st["Y"].T, dp0dt=1e4)
    pr = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    S = pr["turnover"] + np.abs(pr["wdot"])
    assert np.max(np.abs(out["dYdt"].cpu().numpy() - ref["dYdt"]) / (S * om.W[None, :] / ref["rho"][:, None])) <= 1e-12


@pytest.fixture(scope="module")
def var_seg(mech_dir):
    """The same mechanism without the non-integer orders: the segmented Jacobian kernel with
    its optional-form rate phase."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2409_06404_amd as crf
    path = str(mech_dir / "variants_no_orders.mech")
    open(path, "w").write(synth.mechanism_text(synth.generate_variant_mechanism(orders=False)))
    g = crf.Mechanism(path, device=0)
    yield crf, g, oracle.read_mechanism(path)
    g.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_variant_segmented_jacobian(var_seg, prec, tol):
    """PLOG, Chebyshev, Lindemann, SRI, explicit-reverse and irreversible reactions in the
    segmented kernel: J and the fused w against the oracle (ragged point count, pressures
    over 0.05-60 atm), and two runs bitwise equal."""
    crf, g, om = var_seg
    assert g.jac_plan == "segmented", g.jac_plan
    n = 83
    st = _state(om.n_species, n, 67)
    T, p, Y = _dev(st)
    print(f"variant segmented {prec}", flush=True)
    J, w = crf.wdot_jac(g, T, p, Y, prec)
    J2, w2 = crf.wdot_jac(g, T, p, Y, prec)
    torch.cuda.synchronize()
    assert torch.equal(J, J2) and torch.equal(w, w2)
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    floor = 1e-10 if prec == "mixed" else 0.0
    ej = jac_scaled_error(J.double().cpu().numpy(), Jr, G, st["T"], st["Y"].T, floor=floor).max()
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    got = w.cpu().numpy()
    if prec == "fp64":
        ew = e_turn(got, ref["wdot"], ref["turnover"]).max()
    else:
        sig = significant_species(ref["wdot"], om.W)
        ew = e_norm(got, ref["wdot"])[sig].max()
    print(f"  J {ej:.2e} w {ew:.2e}", flush=True)
    assert ej <= tol and ew <= tol


def test_variant_reactor_step(var, mech_dir):
    """ROS2 substeps on the variant mechanism (rates scaled by e^-40 for a moderate stiffness)."""
    crf, _, _ = var
    m = synth.with_rate_shift(synth.generate_variant_mechanism(), -40.0)
    for r in m.reactions:            # tabulated forms: shift their own expressions too
        if r.kind == "plog":
            r.extra["plog"] = [(pp, a - 40.0, b, t) for pp, a, b, t in r.extra["plog"]]
        elif r.kind == "chebyshev":
            a = r.extra["cheb"][4].copy()
            a[0, 0] -= 40.0 / np.log(10.0)
            r.extra["cheb"] = r.extra["cheb"][:4] + (a,)
        if "reverse" in r.extra:
            lnA, b, t = r.extra["reverse"]
            r.extra["reverse"] = (lnA - 40.0, b, t)
    path = str(mech_dir / "variants_slow.mech")
    open(path, "w").write(synth.mechanism_text(m))
    g = crf.Mechanism(path, device=0)
    om = oracle.read_mechanism(path)
    st = _state(om.n_species, 40, 66)
    st["T"] = np.maximum(st["T"], 1100.0)
    A = oracle.source_jacobian(om, st["T"], st["p"], st["Y"].T)
    dt = 2e3 / np.abs(A).max()
    T, p, Y = _dev(st)
    crf.reactor_step(g, T, p, Y, dt, 2)
    torch.cuda.synchronize()
    Tr, Yr = oracle.ros2_step(om, st["T"], st["p"], st["Y"].T, dt, 2)
    d = np.maximum(np.abs(T.cpu().numpy() - Tr) / st["T"], np.abs(Y.cpu().numpy() - Yr).max(axis=1))
    ch = np.maximum(np.abs(Tr - st["T"]) / st["T"], np.abs(Yr - st["Y"].T).max(axis=1))
    err = np.max(np.maximum(d - 4 * 2.2e-16, 0.0) / ch)
    print(f"variant reactor: dt {dt:.2e}, error / change {err:.2e}", flush=True)
    assert err <= 1e-10
    g.close()
