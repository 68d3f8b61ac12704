"""crf_reactor_step_static (the allocation-free reactor entry point, static device scratch)
against crf_reactor_step (caller workspace), through the C ABI: two calls in a row on one
device, the second with fewer points, each bitwise equal to the workspace entry point;
the size limit of the static scratch is refused with CRF_E_WORKSPACE."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(mech_dir):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2409_06404_amd as crf
    from paper_2409_06404_amd import _lib
    m = synth.with_rate_shift(synth.generate_mechanism(synth.MECH_C1), -64.0)
    path = str(mech_dir / "c1_slow_static.mech")
    open(path, "w").write(synth.mechanism_text(m))
    g = crf.Mechanism(path, device=0)
    yield crf, _lib.lib(), g
    g.close()


def _state(n, seed):
    st = synth.state_c1(53, n=n, seed=seed)
    st["T"] = np.maximum(st["T"], 1000.0)
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(st["T"]).to(dev), torch.from_numpy(st["p"]).to(dev),
            torch.from_numpy(np.ascontiguousarray(st["Y"])).to(dev))


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", [0, 1])
def test_static_matches_workspace_entry_point(env, prec):
    crf, L, g = env
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, seed in ((3001, 5), (777, 6)):                 # the second call is smaller
        T0, p, Y0 = _state(n, seed)
        Ta, Ya = T0.clone(), Y0.clone()
        Tb, Yb = T0.clone(), Y0.clone()
        nb = L.crf_workspace_bytes(g.handle, prec, 2, n)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        print(f"static vs workspace reactor: prec {prec} n={n}", flush=True)
        s1 = L.crf_reactor_step(g.handle, prec, n, _p(Ta), _p(p), 1, _p(Ya), n, ctypes.c_double(2e-4), 2,
                                _p(work), ctypes.c_size_t(nb), stream)
        s2 = L.crf_reactor_step_static(g.handle, prec, n, _p(Tb), _p(p), 1, _p(Yb), n, ctypes.c_double(2e-4), 2,
                                       stream)
        torch.cuda.synchronize()
        assert s1 == 0 and s2 == 0, L.crf_last_error()
        assert torch.isfinite(Ta).all() and not torch.equal(Ta, T0)
        assert torch.equal(Ta, Tb) and torch.equal(Ya, Yb)


def test_static_limit_is_refused(env):
    crf, L, g = env
    n = 6000                                           # 53 species: above 128 MiB of scratch
    assert L.crf_workspace_bytes(g.handle, 0, 2, n) > 128 << 20
    T0, p, Y0 = _state(n, 7)
    s = L.crf_reactor_step_static(g.handle, 0, n, _p(T0), _p(p), 1, _p(Y0), n, ctypes.c_double(1e-4), 1,
                                  ctypes.c_void_p(0))
    assert s == 7 and b"static" in L.crf_last_error()
