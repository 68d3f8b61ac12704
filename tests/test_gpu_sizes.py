"""Mechanism sizes that select the other code paths, on the GPU, through the C ABI.

* 60 species: the reactor's Newton matrix (61 unknowns) is beyond the register-resident
  factorisation (up to 56), so the workgroup-per-point LU runs;
* 100 species: transport on point tiles with 8 wavefronts per workgroup (two or three
  workgroups fit a compute unit's LDS), the Jacobian's reaction-table kernel;
* 240 species: transport on point tiles with 16 wavefronts per workgroup (one workgroup per
  compute unit) in both modes;
* 400 species: in FP64 a point tile's species rows exceed one compute unit's LDS and the
  two-points-per-wavefront transport kernel runs; the mixed mode still uses tiles;
* 120 species with about 2 500 and 5 000 reactions: the reaction table exceeds the LDS, and
  the Jacobian's row-block kernel runs (in FP64 only for the first, whose FP32 table still
  fits in the mixed mode).
Point counts are not multiples of the tile size (16)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from metrics import jac_scaled_error, fp32_range_split  # noqa: E402

pytestmark = pytest.mark.gpu

SPECS = {
    60: synth.MechSpec("s60", ("C", "H", "O", "N"), 60, 6, 180, 20, 10, 21),
    100: synth.MechSpec("s100", ("C", "H", "O", "N"), 100, 7, 300, 30, 20, 22),
    240: synth.MechSpec("s240", ("C", "H", "O", "N"), 240, 9, 400, 40, 20, 23),
    400: synth.MechSpec("s400", ("C", "H", "O", "N"), 400, 10, 600, 40, 20, 24),
}


@pytest.fixture(scope="module")
def crf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2409_06404_amd as crf
    return crf


@pytest.fixture(scope="module")
def mechs(crf, mech_dir):
    out = {}
    for ns, spec in SPECS.items():
        path = synth.write_mechanism(spec, str(mech_dir / f"{spec.name}.mech"))
        out[ns] = (crf.Mechanism(path, device=0), oracle.read_mechanism(path), path)
    yield out
    for g, _, _ in out.values():
        g.close()


def _dev(st):
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(st["T"].copy()).to(dev), torch.from_numpy(st["p"].copy()).to(dev),
            torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev).t())


@pytest.mark.parametrize("ns", [60, 100, 240, 400])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_transport_sizes(crf, mechs, ns, prec, tol):
    g, om, _ = mechs[ns]
    st = synth.state_c0(ns, n=37, seed=ns)
    T, p, Y = _dev(st)
    print(f"transport {ns} species {prec}", flush=True)
    mu, lam, D = crf.transport(g, T, p, Y, prec)
    torch.cuda.synchronize()
    ref = oracle.transport_properties(om, st["T"], st["p"], st["Y"].T)
    e = [np.max(np.abs(mu.cpu().numpy() / ref["mu"] - 1)), np.max(np.abs(lam.cpu().numpy() / ref["lambda"] - 1)),
         np.max(np.abs(D.cpu().numpy() / ref["Dmix"] - 1))]
    print(f"  mu {e[0]:.2e} lambda {e[1]:.2e} Dmix {e[2]:.2e}", flush=True)
    assert max(e) <= tol


@pytest.mark.parametrize("ns", [60, 100])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_jacobian_sizes(crf, mechs, ns, prec, tol):
    g, om, _ = mechs[ns]
    st = synth.state_c0(ns, n=21, seed=ns + 1)
    T, p, Y = _dev(st)
    print(f"jacobian {ns} species {prec}: plan {g.jac_plan}", flush=True)
    J, _ = crf.wdot_jac(g, T, p, Y, prec)
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    Jg = J.double().cpu().numpy()
    if prec == "mixed":
        Jg, Jr = fp32_range_split(Jg, Jr)
    err = jac_scaled_error(Jg, Jr, G, st["T"], st["Y"].T, floor=1e-10 if prec == "mixed" else 0.0)
    print(f"  scaled error {err.max():.2e}", flush=True)
    assert err.max() <= tol


ROW_BLOCK = {
    "rb2500": synth.MechSpec("rb2500", ("C", "H", "O", "N"), 120, 8, 2400, 60, 30, 31),
    "rb5000": synth.MechSpec("rb5000", ("C", "H", "O", "N"), 120, 8, 5000, 60, 30, 31),
}


@pytest.mark.parametrize("name", ["rb2500", "rb5000"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_jacobian_row_blocks(crf, mech_dir, name, prec, tol):
    """Mechanisms whose reaction table does not fit: J and the fused w against the oracle on a
    ragged point count."""
    path = synth.write_mechanism(ROW_BLOCK[name], str(mech_dir / f"{name}.mech"))
    g = crf.Mechanism(path, device=0)
    om = oracle.read_mechanism(path)
    plan = g.jac_plan
    row_block = plan.startswith("row-block") or (prec == "fp64" and "row-block in FP64" in plan)
    assert row_block or (name == "rb2500" and prec == "mixed"), plan
    st = synth.state_c0(om.n_species, n=13, seed=33)
    T, p, Y = _dev(st)
    print(f"jacobian {name} ({om.n_reactions} reactions) {prec}: plan {plan}", flush=True)
    J, w = crf.wdot_jac(g, T, p, Y, prec)
    torch.cuda.synchronize()
    Jr, G = oracle.jacobian(om, st["T"], st["p"], st["Y"].T, return_gross=True)
    Jg = J.double().cpu().numpy()
    if prec == "mixed":
        Jg, Jr = fp32_range_split(Jg, Jr)
    err = jac_scaled_error(Jg, Jr, G, st["T"], st["Y"].T, floor=1e-10 if prec == "mixed" else 0.0)
    ref = oracle.production_rates(om, st["T"], st["p"], st["Y"].T)
    ew = np.max(np.abs(w.cpu().numpy() - ref["wdot"]) / (ref["turnover"] + np.abs(ref["wdot"])))
    print(f"  scaled error {err.max():.2e}, w {ew:.2e}", flush=True)
    g.close()
    assert err.max() <= tol and ew <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_reactor_workgroup_lu(crf, mechs, mech_dir, prec, tol):
    """61 unknowns: the workgroup-per-point factorisation.  Rates scaled by e^-64 and h = 1e-5 s
    keep h |A| below ~1.5e3, as in the other reactor tests: with e^-56 and h = 5e-5 s (h |A| up
    to 2e7) an FP32 Jacobian alone moves the step by up to 3e-3 of its size, in the oracle's own
    ROS2 step too, which is the mixed mode's arithmetic, not the kernel's."""
    _, _, path = mechs[60]
    slow = synth.with_rate_shift(synth.generate_mechanism(SPECS[60]), -64.0)
    spath = str(mech_dir / "s60_slow.mech")
    open(spath, "w").write(synth.mechanism_text(slow))
    g = crf.Mechanism(spath, device=0)
    om = oracle.read_mechanism(spath)
    st = synth.state_c0(60, n=19, seed=5)
    st["T"] = np.maximum(st["T"], 1200.0)
    T, p, Y = _dev(st)
    print(f"reactor 60 species {prec}", flush=True)
    crf.reactor_step(g, T, p, Y, 2e-5, 2, prec)
    torch.cuda.synchronize()
    Tr, Yr = oracle.ros2_step(om, st["T"], st["p"], st["Y"].T, 2e-5, 2)
    T1, Y1 = T.cpu().numpy(), Y.cpu().numpy()
    dT = np.abs(T1 - Tr) / st["T"]
    dY = np.abs(Y1 - Yr).max(axis=1)
    ch = np.maximum(np.abs(Tr - st["T"]) / st["T"], np.abs(Yr - st["Y"].T).max(axis=1))
    err = np.max(np.maximum(np.maximum(dT, dY) - 4 * 2.2e-16, 0.0) / ch)
    print(f"  error / change {err:.2e}", flush=True)
    assert err <= tol
    g.close()
