"""Parity of crf_wdot_jvp (forward-mode J v) and crf_source (point-wise chemistry source
terms, Eq. (1a)-(1b), Eq. (3)) with the FP64 oracle, on the GPU, through the C ABI.

Bounds: FP64 1e-12, mixed 1e-5.  J v: row k measured against sum_c G_kc |v_c| (G the
oracle's gross Jacobian), the same scale the VJP uses.  Source terms: FP64 point-wise
against the gross turnover of the rates they are built from; mixed as E_norm over points.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from metrics import e_norm, significant_species  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2409_06404_amd as crf
    return crf


@pytest.fixture(scope="module")
def mechs(crf, c0_path, c1_path, mech_dir):
    c4_path = synth.write_mechanism(synth.MECH_C4, str(mech_dir / "c4.mech"))
    out = {}
    for name, path in (("c0", c0_path), ("c1", c1_path), ("c4", c4_path)):
        out[name] = (crf.Mechanism(path, device=0), oracle.read_mechanism(path))
    yield out
    for g, _ in out.values():
        g.close()


def _state(which, n, seed):
    if which == "c0":
        return synth.state_c0(9, n=n, seed=seed)
    if which == "c1":
        return synth.state_c1(53, n=n, seed=seed)
    st = synth.state_c4_launch(200, 1, seed=4, launch=0)           # one element, 512 points
    return {"T": st["T"][:n], "p": st["p"][:n], "Y": np.ascontiguousarray(st["Y"][:, :n])}


def _dev(st):
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["p"]).to(dev),
            torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t())


def _tangent(st, seed):
    rng = np.random.default_rng(seed)
    vT = rng.standard_normal(st["T"].shape) * 10.0
    vY = rng.standard_normal(st["Y"].shape) * st["Y"]               # species-major like Y
    return vT, vY


@pytest.mark.parametrize("which,n,prec,tol", [("c0", 1000, "fp64", 1e-12), ("c1", 301, "fp64", 1e-12),
                                              ("c1", 301, "mixed", 1e-5), ("c4", 37, "fp64", 1e-12),
                                              ("c4", 37, "mixed", 1e-5)])
def test_jvp(crf, mechs, which, n, prec, tol):
    g, om = mechs[which]
    st = _state(which, n, 7)
    vT, vY = _tangent(st, 8)
    T, p, Y = _dev(st)
    print(f"jvp {which} {prec} n={n}", flush=True)
    jh, jw, w = crf.wdot_jvp(g, T, p, Y, torch.from_numpy(vY).cuda().t(), torch.from_numpy(vT).cuda(), prec,
                             with_wdot=True)
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    v = np.concatenate([vT[:, None], vY.T], axis=1)
    ref = np.einsum("nrc,nc->nr", Jr, v)
    scale = np.einsum("nrc,nc->nr", G, np.abs(v)) + 1e-300
    got = np.concatenate([jh.cpu().numpy()[:, None], jw.cpu().numpy()], axis=1)
    err = np.abs(got - ref) / scale
    print(f"  scaled J v error max {err.max():.2e} (hrr row {err[:, 0].max():.2e})", flush=True)
    assert err.max() <= tol
    # the fused production rates of the same evaluation
    wr = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    sig = significant_species(wr["wdot"], om.W)
    assert e_norm(w.cpu().numpy(), wr["wdot"])[sig].max() <= tol


def test_jvp_vjp_dot_product(crf, mechs):
    """<u, J v> from crf_wdot_jvp equals <J^T u, v> from crf_wdot_vjp (two independent kernels)."""
    g, om = mechs["c1"]
    st = _state("c1", 2049, 9)
    vT, vY = _tangent(st, 10)
    rng = np.random.default_rng(11)
    u = rng.standard_normal(st["Y"].shape)
    uh = rng.standard_normal(st["T"].shape) * 1e-6
    T, p, Y = _dev(st)
    jh, jw, _ = crf.wdot_jvp(g, T, p, Y, torch.from_numpy(vY).cuda().t(), torch.from_numpy(vT).cuda())
    gT, gY = crf.wdot_vjp(g, T, p, Y, torch.from_numpy(u).cuda().t(), torch.from_numpy(uh).cuda())
    torch.cuda.synchronize()
    lhs = uh * jh.cpu().numpy() + (u.T * jw.cpu().numpy()).sum(axis=1)
    rhs = gT.cpu().numpy() * vT + (gY.cpu().numpy() * vY.T).sum(axis=1)
    idx = np.arange(0, 2049, 41)
    _, G = oracle.jacobian(om, st["T"][idx], st["p"][idx], st["Y"][:, idx].T, return_gross=True)
    uu = np.abs(np.concatenate([uh[idx, None], u.T[idx]], axis=1))
    vv = np.abs(np.concatenate([vT[idx, None], vY.T[idx]], axis=1))
    scale = np.einsum("nr,nrc,nc->n", uu, G, vv)
    assert np.max(np.abs(lhs[idx] - rhs[idx]) / scale) <= 1e-12


def test_jvp_edge_cases(crf, mechs):
    g, om = mechs["c1"]
    dev = torch.device("cuda", 0)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    jh, jw, _ = crf.wdot_jvp(g, e, e, torch.empty((53, 0), dtype=torch.float64, device=dev).t(),
                             torch.empty((53, 0), dtype=torch.float64, device=dev).t())
    assert jw.shape == (0, 53)
    # vT omitted (zero), one point, exact zeros in Y
    st = _state("c1", 65, 12)
    st["Y"][4, :] = 0.0
    _, vY = _tangent(st, 13)
    T, p, Y = _dev(st)
    jh, jw, _ = crf.wdot_jvp(g, T, p, Y, torch.from_numpy(vY).cuda().t())
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    v = np.concatenate([np.zeros((65, 1)), vY.T], axis=1)
    ref = np.einsum("nrc,nc->nr", Jr, v)
    got = np.concatenate([jh.cpu().numpy()[:, None], jw.cpu().numpy()], axis=1)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref) / (np.einsum("nrc,nc->nr", G, np.abs(v)) + 1e-300)) <= 1e-12


@pytest.mark.parametrize("which,prec,dp", [("c0", "fp64", 0.0), ("c1", "fp64", 0.0), ("c1", "fp64", 3.0e4),
                                           ("c1", "mixed", 0.0), ("c4", "fp64", 0.0), ("c4", "mixed", 1.0e5)])
def test_source(crf, mechs, which, prec, dp):
    g, om = mechs[which]
    st = _state(which, 2001 if which != "c4" else 512, 14)
    T, p, Y = _dev(st)
    print(f"source {which} {prec} dp0dt={dp}", flush=True)
    out = crf.source(g, T, p, Y, prec, dp0dt=dp)
    torch.cuda.synchronize()
    ref = oracle.chemistry_source(om, st["T"], st["p"], st["Y"].T, dp0dt=dp)
    pr = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    th = oracle.thermo_properties(om, st["T"], st["p"], st["Y"].T)
    rho, cp = ref["rho"], ref["cp_mass"]
    S = pr["turnover"] + np.abs(pr["wdot"])                               # gross rate per species
    sc_y = S * om.W[None, :] / rho[:, None]
    sc_t = ((np.abs(th["h_k"]) * S).sum(axis=1) + abs(dp)) / (rho * cp)
    Wbar = th["Wbar"]
    sc_q = sc_t / st["T"] + Wbar / rho * S.sum(axis=1) + abs(dp) / st["p"]
    got = {k: v.cpu().numpy() for k, v in out.items()}
    if prec == "fp64":
        ey = np.max(np.abs(got["dYdt"] - ref["dYdt"]) / sc_y)
        et = np.max(np.abs(got["dTdt"] - ref["dTdt"]) / sc_t)
        eq = np.max(np.abs(got["QT"] - ref["QT"]) / sc_q)
        print(f"  dYdt {ey:.2e} dTdt {et:.2e} QT {eq:.2e}", flush=True)
        assert max(ey, et, eq) <= 1e-12
    else:
        sig = significant_species(pr["wdot"], om.W)
        ey = e_norm(got["dYdt"], ref["dYdt"])[sig].max()
        et = e_norm(got["dTdt"][:, None], ref["dTdt"][:, None])[0]
        eq = e_norm(got["QT"][:, None], ref["QT"][:, None])[0]
        print(f"  E_norm dYdt {ey:.2e} dTdt {et:.2e} QT {eq:.2e}", flush=True)
        assert max(ey, et, eq) <= 1e-5
    sc_h = (np.abs(th["h_k"]) * S).sum(axis=1)
    if prec == "fp64":
        assert np.max(np.abs(got["hrr"] - ref["hrr"]) / sc_h) <= 1e-12
    else:
        assert e_norm(got["hrr"][:, None], ref["hrr"][:, None])[0] <= 1e-5


def test_source_invalid_arguments(crf, mechs):
    g, _ = mechs["c0"]
    st = _state("c0", 8, 15)
    T, p, Y = _dev(st)
    with pytest.raises(crf.CrfError):
        crf.source(g, T, p, Y, dp0dt=float("nan"))
