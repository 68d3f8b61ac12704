"""The stored-intermediate VJP: crf_wdot_fwd keeps every reaction's rate constants and
their derivatives in a caller workspace, crf_wdot_vjp reuses them (GPU, through the C ABI).

Checked against the FP64 oracle (1e-12 FP64, 1e-5 mixed, the VJP scale of the recompute
tests), against the recompute path, and through the autograd function under both
branches of its HBM-budget policy.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from metrics import e_norm, significant_species, vjp_scaled_error  # noqa: E402

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
    st = synth.state_c4_launch(200, 1, seed=4, launch=0)
    return {"T": st["T"][:n], "p": st["p"][:n], "Y": np.ascontiguousarray(st["Y"][:, :n])}


def _dev(st):
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["p"]).to(dev),
            torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t())


@pytest.mark.parametrize("which,n,prec,tol", [("c0", 300, "fp64", 1e-12), ("c1", 201, "fp64", 1e-12),
                                              ("c1", 201, "mixed", 1e-5), ("c4", 33, "fp64", 1e-12),
                                              ("c4", 33, "mixed", 1e-5)])
def test_stored_vjp(crf, mechs, which, n, prec, tol):
    g, om = mechs[which]
    st = _state(which, n, 21)
    T, p, Y = _dev(st)
    rng = np.random.default_rng(22)
    u = rng.standard_normal(st["Y"].shape)
    uh = rng.standard_normal(n) * 1e-6
    ut, uht = torch.from_numpy(u).cuda().t(), torch.from_numpy(uh).cuda()
    print(f"stored vjp {which} {prec} n={n}", flush=True)
    work = crf.new_workspace(g, n, prec)
    assert work.numel() == n * g.n_reactions * 32
    w, h = crf.wdot_fwd(g, T, p, Y, work, prec)
    gT, gY = crf.wdot_vjp(g, T, p, Y, ut, uht, prec, work=work)
    gT0, gY0 = crf.wdot_vjp(g, T, p, Y, ut, uht, prec)                     # recompute path
    w0, h0, _ = crf.wdot(g, T, p, Y, prec)
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    uu = np.concatenate([uh[:, None], u.T], axis=1)
    gref = np.einsum("nr,nrc->nc", uu, Jr)
    got = np.concatenate([gT.cpu().numpy()[:, None], gY.cpu().numpy()], axis=1)
    err = vjp_scaled_error(got, gref, uu, G)
    got0 = np.concatenate([gT0.cpu().numpy()[:, None], gY0.cpu().numpy()], axis=1)
    diff = vjp_scaled_error(got, got0, uu, G)
    print(f"  vs oracle {err:.2e}, vs recompute {diff:.2e}", flush=True)
    assert err <= tol
    assert diff <= 1e-14
    # the forward's production rates are those of crf_wdot
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    sig = significant_species(ref["wdot"], om.W)
    assert e_norm(w.cpu().numpy(), ref["wdot"])[sig].max() <= tol
    assert torch.equal(w, w0) and torch.equal(h, h0)


def test_workspace_too_small_raises(crf, mechs):
    g, _ = mechs["c0"]
    st = _state("c0", 64, 23)
    T, p, Y = _dev(st)
    small = torch.empty(64 * g.n_reactions * 32 - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(crf.CrfError) as e:
        crf.wdot_fwd(g, T, p, Y, small)
    assert e.value.status == 7
    with pytest.raises(crf.CrfError) as e:
        crf.wdot_vjp(g, T, p, Y, torch.zeros_like(Y), work=small)
    assert e.value.status == 7


@pytest.mark.parametrize("budget", ["0", "1e12"])
def test_autograd_budget_policy(crf, mechs, monkeypatch, budget):
    """WdotFn keeps the intermediates when they fit CRF_HBM_BUDGET and recomputes otherwise;
    both give the oracle's gradients."""
    monkeypatch.setenv("CRF_HBM_BUDGET", budget)
    g, om = mechs["c1"]
    st = _state("c1", 130, 24)
    T, p, Y = _dev(st)
    T = T.clone().requires_grad_(True)
    Ysm = Y.t().contiguous().requires_grad_(True)
    w, h = crf.WdotFn.apply(T, Ysm.t(), p, g, "fp64")
    rng = np.random.default_rng(25)
    u = torch.from_numpy(rng.standard_normal((130, 53))).cuda()
    (w * u).sum().backward()
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    uu = np.concatenate([np.zeros((130, 1)), u.cpu().numpy()], axis=1)
    gref = np.einsum("nr,nrc->nc", uu, Jr)
    got = np.concatenate([T.grad.cpu().numpy()[:, None], Ysm.grad.t().cpu().numpy()], axis=1)
    assert vjp_scaled_error(got, gref, uu, G) <= 1e-12
