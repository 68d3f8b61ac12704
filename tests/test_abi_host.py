"""The C-ABI library loads, exports every declared symbol, and validates on the host (CPU only).

No compute call reaches a device here: mechanisms are loaded host-only (device -1)
and every call is rejected by argument validation before any launch.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crf.h")


@pytest.fixture(scope="module")
def L():
    from paper_2409_06404_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2409_06404_amd.build import build_library
        build_library()
    return _lib.lib()


def declared_functions():
    text = "".join(open(os.path.join(ROOT, "include", h)).read() for h in sorted(os.listdir(os.path.join(ROOT, "include"))))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(crf_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    from paper_2409_06404_amd import _lib
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def _load(L, path, device=-1):
    h = ctypes.c_void_p()
    s = L.crf_load_mech(str(path).encode(), device, ctypes.byref(h))
    return s, h


def test_host_only_load_and_counts(L, c1_path):
    s, h = _load(L, c1_path)
    assert s == 0, L.crf_last_error()
    assert L.crf_n_species(h) == 53 and L.crf_n_reactions(h) == 325 and L.crf_device(h) == -1
    L.crf_free_mech(h)
    assert L.crf_n_species(None) == -1
    L.crf_free_mech(None)


def test_status_strings(L):
    assert L.crf_status_str(0) == b"CRF_OK"
    assert L.crf_status_str(6) == b"CRF_E_UNSUPPORTED"


def _edit(src, dst, fn):
    text = open(src).read()
    open(dst, "w").write(fn(text))
    return dst


@pytest.mark.parametrize("edit,status,msg", [
    (lambda t: t.replace("crf-mech 1", "crf-mech 2"), 2, "version"),
    (lambda t: "\n".join(t.splitlines()[:40]), 2, ""),                                   # truncated
    (lambda t: t.replace("reaction elementary reactants 2", "reaction surface reactants 2", 1), 6, "unsupported"),
    (lambda t: t.replace("reaction elementary reactants 2", "reaction plog reactants 2", 1), 2, "plog"),
    (lambda t: t.replace("gas-constant 8314.46261815324", "gas-constant -1"), 3, "positive"),
], ids=["version", "truncated", "kind", "plog-block", "gasconst"])
def test_malformed_files(L, c0_path, tmp_path, edit, status, msg):
    bad = _edit(c0_path, tmp_path / "bad.mech", edit)
    s, h = _load(L, bad)
    assert s == status, (s, L.crf_last_error())
    assert msg in L.crf_last_error().decode()
    assert not h.value


def test_species_limit(L, c0_path, tmp_path):
    """Mechanisms above 2048 species are refused at load (CRF_E_UNSUPPORTED), before the
    rest of the file is read: the per-point species arrays of the kernels live in LDS."""
    text = open(c0_path).read()
    bad = tmp_path / "big.mech"
    bad.write_text(text.replace("\nspecies 9\n", "\nspecies 2049\n"))
    assert "species 2049" in bad.read_text()
    s, h = _load(L, bad)
    assert s == 6, (s, L.crf_last_error())
    assert b"at most 2048" in L.crf_last_error()
    assert not h.value


def test_unbalanced_reaction_rejected(L, c0_path, tmp_path):
    lines = open(c0_path).read().splitlines()
    i = next(k for k, ln in enumerate(lines) if ln.startswith("reaction "))
    toks = lines[i].split()
    j = toks.index("products") + 2                  # first product token "k:nu"
    k, nu = toks[j].split(":")
    toks[j] = f"{k}:{int(nu) + 1}" if int(nu) < 3 else f"{k}:1"
    lines[i] = " ".join(toks)
    bad = tmp_path / "unbal.mech"
    bad.write_text("\n".join(lines) + "\n")
    s, _ = _load(L, bad)
    assert s in (3, 6), L.crf_last_error()
    assert "balanced" in L.crf_last_error().decode() or "order" in L.crf_last_error().decode()


def test_missing_file(L):
    s, h = _load(L, "/nonexistent/x.mech")
    assert s == 2 and b"cannot read" in L.crf_last_error()


def test_compute_calls_validate_before_launch(L, c0_path):
    s, h = _load(L, c0_path)
    assert s == 0
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: validation fails first
    # n < 0
    assert L.crf_wdot(h, 0, -1, fake, fake, 1, fake, 10, fake, null, null, null) == 1
    # ld < n
    assert L.crf_wdot(h, 0, 10, fake, fake, 1, fake, 5, fake, null, null, null) == 1
    # bad p_stride
    assert L.crf_transport(h, 0, 10, fake, fake, 2, fake, 10, fake, null, null, null) == 1
    # NULL state with n > 0
    assert L.crf_wdot_jac(h, 0, 10, null, fake, 1, fake, 10, fake, null, null) == 1
    # NULL mechanism
    assert L.crf_thermo(None, 10, fake, fake, 1, fake, 10, *([null] * 8), null) == 1
    # valid arguments on a host-only mechanism: device error, nothing launched
    assert L.crf_wdot(h, 0, 10, fake, fake, 1, fake, 10, fake, null, null, null) == 5
    assert b"without a device" in L.crf_last_error()
    # J v: vY and jv_w are required; a host-only mechanism is a device error
    assert L.crf_wdot_jvp(h, 0, 10, fake, fake, 1, fake, 10, null, null, null, fake, null, null) == 1
    assert L.crf_wdot_jvp(h, 0, 10, fake, fake, 1, fake, 10, null, fake, null, null, null, null) == 1
    assert L.crf_wdot_jvp(h, 0, 10, fake, fake, 1, fake, 10, null, fake, null, fake, null, null) == 5
    # source terms: at least one output; dp0dt finite
    assert L.crf_source(h, 0, 10, fake, fake, 1, fake, 10, ctypes.c_double(0.0), null, null, null, null, null) == 1
    assert L.crf_source(h, 0, 10, fake, fake, 1, fake, 10, ctypes.c_double(float("inf")), fake, null, null, null,
                        null) == 1
    assert b"finite" in L.crf_last_error()
    assert L.crf_source(h, 0, 10, fake, fake, 1, fake, 10, ctypes.c_double(0.0), fake, null, null, null, null) == 5
    # workspace: size query, then CRF_E_WORKSPACE for a missing, short or misaligned buffer
    nr = L.crf_n_reactions(h)
    assert L.crf_workspace_bytes(h, 0, 1, 10) == 10 * nr * 32
    assert L.crf_workspace_bytes(h, 1, 1, 0) == 0
    assert L.crf_workspace_bytes(h, 0, 3, 10) == 0 and b"unknown operation" in L.crf_last_error()
    r64, r32 = L.crf_workspace_bytes(h, 0, 2, 10), L.crf_workspace_bytes(h, 1, 2, 10)
    assert 10 * 8 * 10 * 10 < r64 < r32          # the mixed mode adds an FP64 copy of the matrices
    assert L.crf_workspace_bytes(h, 0, 2, 0) == 0
    # reactor step: dt and nsub validated, then the workspace, then the device
    step = lambda dt, nsub, work, nb: L.crf_reactor_step(h, 0, 10, fake, fake, 1, fake, 10, ctypes.c_double(dt),
                                                         nsub, work, ctypes.c_size_t(nb), null)
    assert step(0.0, 1, fake, r64) == 1 and b"dt" in L.crf_last_error()
    assert step(float("nan"), 1, fake, r64) == 1
    assert step(1e-3, 0, fake, r64) == 1 and b"nsub" in L.crf_last_error()
    assert step(1e-3, 1, null, r64) == 7
    assert step(1e-3, 1, ctypes.c_void_p(0x1180), r64) == 7 and b"aligned" in L.crf_last_error()
    assert step(1e-3, 1, fake, r64 - 1) == 7
    assert step(1e-3, 1, fake, r64) == 5
    assert L.crf_workspace_bytes(h, 5, 1, 10) == 0 and b"precision" in L.crf_last_error()
    big = ctypes.c_size_t(10 * nr * 32)
    assert L.crf_wdot_fwd(h, 0, 10, fake, fake, 1, fake, 10, fake, null, null, null, big, null) == 7
    assert L.crf_wdot_fwd(h, 0, 10, fake, fake, 1, fake, 10, fake, null, null, fake, ctypes.c_size_t(10 * nr * 32 - 1),
                          null) == 7
    assert b"needed" in L.crf_last_error()
    assert L.crf_wdot_fwd(h, 0, 10, fake, fake, 1, fake, 10, fake, null, null, ctypes.c_void_p(0x1008), big,
                          null) == 7
    assert b"aligned" in L.crf_last_error()
    assert L.crf_wdot_fwd(h, 0, 10, fake, fake, 1, fake, 10, fake, null, null, fake, big, null) == 5
    assert L.crf_wdot_vjp(h, 0, 10, fake, fake, 1, fake, 10, fake, null, fake, fake, ctypes.c_void_p(0x1004), big,
                          null) == 7
    assert L.crf_wdot_vjp(h, 0, 10, fake, fake, 1, fake, 10, fake, null, fake, fake, fake, ctypes.c_size_t(5),
                          null) == 7
    assert L.crf_wdot_vjp(h, 0, 10, fake, fake, 1, fake, 10, fake, null, fake, fake, null, ctypes.c_size_t(0),
                          null) == 5          # no workspace: the recompute path
    assert L.crf_status_str(7) == b"CRF_E_WORKSPACE"
    # bad precision is checked after the state
    assert L.crf_wdot_jvp(None, 0, 10, fake, fake, 1, fake, 10, null, fake, null, fake, null, null) == 1
    s2, h2 = _load(L, c0_path)
    L.crf_free_mech(h2)
    L.crf_free_mech(h)


def test_jacobian_plan_selection(mech_dir):
    """The segmented Jacobian kernel takes the 9- and 53-species mechanisms (its plan
    passes the builder's replay check) and the variant mechanism without non-integer orders;
    the 200-species one and the variant mechanism with orders go to the reaction-table kernel."""
    import synth
    import paper_2409_06404_amd as crf
    for spec, want in ((synth.MECH_C0, "segmented"), (synth.MECH_C1, "segmented"), (synth.MECH_C4, "reaction-table")):
        path = synth.write_mechanism(spec, str(mech_dir / f"plan_{spec.n_species}.mech"))
        m = crf.Mechanism(path, device=-1)
        try:
            assert m.jac_plan.startswith(want), m.jac_plan
        finally:
            m.close()
    # optional rate forms take the segmented plan, non-integer forward orders do not
    for orders, want in ((False, "segmented"), (True, "reaction-table")):
        path = str(mech_dir / f"plan_var_{orders}.mech")
        open(path, "w").write(synth.mechanism_text(synth.generate_variant_mechanism(orders=orders)))
        m = crf.Mechanism(path, device=-1)
        try:
            assert m.jac_plan.startswith(want), m.jac_plan
        finally:
            m.close()


_GARBAGE = ("", "nan", "inf", "-inf", "-1", "0", "1e400", "-1e-400", "2147483648", "-2147483649",
            "9223372036854775808", "x", "1:2:3", ":", "0:", ":1", "99999:1", "1:nan", "3.5", "-0")


@pytest.fixture(scope="module")
def variant_path(mech_dir):
    import synth
    return synth.write_mechanism(synth.MECH_V, str(mech_dir / "fuzz_v.mech"))


@pytest.mark.parametrize("which", ["c0", "v"])
def test_truncated_files_are_rejected(L, c0_path, variant_path, tmp_path, which):
    """A file cut after any of its lines (before the last one) is refused with a status, never
    read past its end; the variant mechanism holds the PLOG and Chebyshev blocks."""
    lines = open(c0_path if which == "c0" else variant_path).read().splitlines()
    last = max(i for i, ln in enumerate(lines) if ln.strip())
    bad = tmp_path / "cut.mech"
    for k in range(last):
        bad.write_text("\n".join(lines[:k + 1]) + "\n")
        s, h = _load(L, bad)
        assert s in (2, 3, 6), (k, s, lines[k])
        assert not h.value


@pytest.mark.parametrize("which", ["c0", "v"])
def test_corrupted_tokens_never_crash(L, c0_path, variant_path, tmp_path, which):
    """Single tokens replaced by garbage (empty, non-finite, out-of-range integers, malformed
    species:coefficient pairs): every load returns a status, and a file that still loads
    describes a usable mechanism."""
    import numpy as np
    lines = open(c0_path if which == "c0" else variant_path).read().splitlines()
    rng = np.random.default_rng(17 if which == "c0" else 18)
    spots = [(i, j) for i, ln in enumerate(lines) for j in range(len(ln.split()))]
    bad = tmp_path / "tok.mech"
    for n in rng.choice(len(spots), size=min(300, len(spots)), replace=False):
        i, j = spots[n]
        toks = lines[i].split()
        toks[j] = _GARBAGE[rng.integers(len(_GARBAGE))]
        bad.write_text("\n".join(lines[:i] + [" ".join(toks)] + lines[i + 1:]) + "\n")
        s, h = _load(L, bad)
        assert 0 <= s <= 7
        if s == 0:
            assert L.crf_n_species(h) > 0 and L.crf_n_reactions(h) > 0 and L.crf_jac_plan(h)
            L.crf_free_mech(h)
        else:
            assert not h.value and L.crf_last_error()
