"""The seeded input generator: deterministic, element-balanced, complete (CPU only)."""
import hashlib

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("spec", [synth.MECH_C0, synth.MECH_C1])
def test_mechanism_deterministic_and_valid(spec, tmp_path):
    t1 = synth.mechanism_text(synth.generate_mechanism(spec))
    t2 = synth.mechanism_text(synth.generate_mechanism(spec))
    assert hashlib.sha256(t1.encode()).hexdigest() == hashlib.sha256(t2.encode()).hexdigest()
    path = tmp_path / "m.mech"
    path.write_text(t1)
    m = oracle.read_mechanism(str(path))
    assert m.n_species == spec.n_species
    assert m.n_reactions == spec.n_elementary + spec.n_threebody + spec.n_troe
    assert m.kind.count("threebody") == spec.n_threebody
    assert m.kind.count("troe") == spec.n_troe
    dnu = m.nu_r - m.nu_f
    assert np.all(dnu @ m.comp == 0)                           # element balance
    assert np.all((np.abs(m.nu_f) + np.abs(m.nu_r)).sum(axis=0) > 0)   # every species used
    assert np.all(m.nu_f.sum(axis=1) <= 3) and np.all(m.nu_r.sum(axis=1) <= 3)
    assert not np.any((m.nu_f > 0) & (m.nu_r > 0))             # no species on both sides
    assert np.all((m.lnA >= 20) & (m.lnA <= 35))
    assert np.all((m.b >= -1.5) & (m.b <= 2.0))
    assert np.all((m.theta >= 0) & (m.theta <= 30000))


def test_states_shapes_and_ranges():
    st = synth.state_c0(9, n=4096, seed=0)
    assert st["Y"].shape == (9, 4096)
    np.testing.assert_allclose(st["Y"].sum(axis=0), 1.0, rtol=1e-14)
    assert np.all(st["Y"] > 0)
    assert st["T"].min() >= 300 and st["T"].max() <= 2500
    s1 = synth.state_c1(53, n=20000, seed=1)
    np.testing.assert_allclose(s1["Y"].sum(axis=0), 1.0, rtol=1e-13)
    assert set(np.unique(s1["p"])) == {101325.0, 1013250.0}
    assert np.sum(s1["T"] >= 1499.9) >= 2000
    s1b = synth.state_c1(53, n=20000, seed=1)
    assert np.array_equal(s1["Y"], s1b["Y"]) and np.array_equal(s1["T"], s1b["T"])


def test_c4_launch_layout():
    counts = synth.c4_element_counts()
    assert len(counts) == 8 and min(counts) == 1000 and max(counts) == 8000
    st = synth.state_c4_launch(200, 3, seed=4, launch=1)
    assert st["Y"].shape == (200, 3 * 512)
    assert np.all(st["p"] == 40 * 101325.0)
    assert st["T"].min() >= 300.0 and st["T"].max() <= 2400.0
    np.testing.assert_allclose(st["Y"].sum(axis=0), 1.0, rtol=1e-13)
    x = synth.gll_nodes(8)
    assert x[0] == -1.0 and x[-1] == 1.0 and np.allclose(x, -x[::-1])


def test_anchor_file_reproduces():
    """The stored anchors are what the committed script computes with the oracle."""
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("mk", os.path.join(here, "golden", "make_equil_anchors.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    fresh = mk.compute_anchors()
    stored = synth.load_anchors()
    for k in ("T", "p", "Y"):
        np.testing.assert_allclose(stored[k], fresh[k], rtol=1e-10, atol=1e-300)
