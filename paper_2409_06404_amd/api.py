"""PyTorch-facing API.  torch supplies device memory and the current stream only:
every computation runs in the HIP kernels behind the C ABI (include/crf.h).

Layouts: ``T [n]``, ``p [n]`` (or a 0-d tensor / float for one pressure), and
``Y`` a logical ``[n, Ns]`` float64 tensor stored species-major, i.e. with
strides ``(1, ld)`` (``Y = Ysm.T`` for a contiguous ``Ysm [Ns, ld]``).  Other
layouts raise: there are no hidden copies.  Per-species outputs come back in the
same layout.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import _lib
from ._lib import CRF_FP64, CRF_MIXED, CRF_OP_REACTOR, CRF_OP_VJP, CrfError, check

_PREC = {"fp64": CRF_FP64, "mixed": CRF_MIXED}


def _prec(precision):
    try:
        return _PREC[precision]
    except KeyError:
        raise ValueError(f"precision must be 'fp64' or 'mixed', got {precision!r}") from None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Mechanism:
    """A mechanism loaded from a ``crf-mech 1`` file onto one HIP device (device=-1: host-only)."""

    def __init__(self, path, device=None):
        if device is None:
            device = torch.cuda.current_device()
        elif isinstance(device, torch.device):
            device = device.index if device.index is not None else torch.cuda.current_device()
        h = ctypes.c_void_p()
        check(_lib.lib().crf_load_mech(str(path).encode(), int(device), ctypes.byref(h)))
        self._h = h
        self.path = str(path)

    @classmethod
    def from_cantera_yaml(cls, path, device=None, transport=True):
        """Load a Cantera YAML mechanism (converted by cantera_yaml.to_crf_mech)."""
        import tempfile

        from . import cantera_yaml
        text = cantera_yaml.to_crf_mech(open(path).read(), transport=transport)
        with tempfile.NamedTemporaryFile("w", suffix=".mech", delete=False) as fh:
            fh.write(text)
            tmp = fh.name
        try:
            return cls(tmp, device=device)
        finally:
            os.unlink(tmp)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("mechanism has been freed")
        return self._h

    @property
    def n_species(self):
        return _lib.lib().crf_n_species(self.handle)

    @property
    def n_reactions(self):
        return _lib.lib().crf_n_reactions(self.handle)

    @property
    def jac_plan(self):
        """Which Jacobian kernel crf_wdot_jac runs: 'segmented' or 'row-block (<reason>)'."""
        return _lib.lib().crf_jac_plan(self.handle).decode()

    @property
    def device(self):
        return _lib.lib().crf_device(self.handle)

    def close(self):
        if getattr(self, "_h", None) is not None:
            if self.device >= 0:
                torch.cuda.synchronize(self.device)
            _lib.lib().crf_free_mech(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def species_major(Y_nk):
    """Copy a [n, Ns] tensor into the species-major layout the library reads."""
    return Y_nk.t().contiguous().t()


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _state(m, T, p, Y):
    ns = m.n_species
    dev = torch.device("cuda", m.device)
    if T.dtype != torch.float64 or T.dim() != 1 or T.device != dev or not T.is_contiguous():
        raise ValueError("T must be a contiguous float64 [n] tensor on the mechanism's device")
    n = T.shape[0]
    if not torch.is_tensor(p):
        p = torch.tensor(float(p), dtype=torch.float64, device=dev)
    if p.dtype != torch.float64 or p.device != dev:
        raise ValueError("p must be float64 on the mechanism's device")
    if p.dim() == 0 or (p.dim() == 1 and p.shape[0] == 1 and n != 1):
        ps = 0
    elif p.dim() == 1 and p.shape[0] == n and p.is_contiguous():
        ps = 1
    else:
        raise ValueError("p must be a scalar or a contiguous [n] tensor")
    if Y.dtype != torch.float64 or Y.device != dev or Y.dim() != 2 or Y.shape != (n, ns):
        raise ValueError(f"Y must be a float64 [n, {ns}] tensor on the mechanism's device")
    if n > 0 and (Y.stride(0) != 1 or (ns > 1 and Y.stride(1) < n)):
        raise ValueError("Y must be species-major: strides (1, ld) with ld >= n (use species_major())")
    ld = Y.stride(1) if ns > 1 else max(n, 1)
    return n, p, ps, ld, dev


def _species_out(ns, n, ld, dev, dtype=torch.float64):
    return torch.empty((ns, ld), dtype=dtype, device=dev)[:, :n].t()


def thermo(m, T, p, Y):
    """dict(cp_k, h_k, s_k, g_k [n, Ns], cp_mass, h_mass, rho, Wbar [n]) in SI-kmol units."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    ns = m.n_species
    out = {k: _species_out(ns, n, ld, dev) for k in ("cp_k", "h_k", "s_k", "g_k")}
    out.update({k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("cp_mass", "h_mass", "rho", "Wbar")})
    check(_lib.lib().crf_thermo(m.handle, n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                *[_ptr(out[k]) for k in ("cp_k", "h_k", "s_k", "g_k", "cp_mass", "h_mass", "rho", "Wbar")],
                                _stream(dev)))
    return out


def wdot(m, T, p, Y, precision="fp64", hrr=True, mass_resid=False):
    """(wdot [n, Ns], hrr [n] or None, mass_resid [n] or None)."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    w = _species_out(m.n_species, n, ld, dev)
    h = torch.empty(n, dtype=torch.float64, device=dev) if hrr else None
    r = torch.empty(n, dtype=torch.float64, device=dev) if mass_resid else None
    check(_lib.lib().crf_wdot(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                              _ptr(w), _ptr(h), _ptr(r), _stream(dev)))
    return w, h, r


def transport(m, T, p, Y, precision="fp64"):
    """(mu [n], lambda [n], Dmix [n, Ns])."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    mu = torch.empty(n, dtype=torch.float64, device=dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    D = _species_out(m.n_species, n, ld, dev)
    check(_lib.lib().crf_transport(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                   _ptr(mu), _ptr(lam), _ptr(D), _stream(dev)))
    return mu, lam, D


def workspace_bytes(m, n, precision="fp64"):
    """Bytes of the rate intermediates that wdot_fwd stores for a later wdot_vjp (n points)."""
    b = _lib.lib().crf_workspace_bytes(m.handle, _prec(precision), CRF_OP_VJP, int(n))
    if b == 0 and n > 0 and m.n_reactions > 0:
        raise CrfError(1, _lib.lib().crf_last_error().decode())
    return b


def new_workspace(m, n, precision="fp64"):
    """A device buffer of workspace_bytes(m, n) bytes (torch allocations are 512-byte aligned)."""
    return torch.empty(max(workspace_bytes(m, n, precision), 1), dtype=torch.uint8,
                       device=torch.device("cuda", m.device))


def wdot_fwd(m, T, p, Y, work, precision="fp64", hrr=True):
    """(wdot [n, Ns], hrr [n] or None), storing the rate intermediates in `work` for wdot_vjp."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    if work.dtype != torch.uint8 or work.device != dev or not work.is_contiguous():
        raise ValueError("work must be a contiguous uint8 tensor on the mechanism's device")
    w = _species_out(m.n_species, n, ld, dev)
    h = torch.empty(n, dtype=torch.float64, device=dev) if hrr else None
    check(_lib.lib().crf_wdot_fwd(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                  _ptr(w), _ptr(h), _ptr(None), _ptr(work), work.numel(), _stream(dev)))
    return w, h


def wdot_vjp(m, T, p, Y, u, u_hrr=None, precision="fp64", work=None):
    """(gT [n], gY [n, Ns]) = u^T d(hrr, w)/d(T, Y); u in the same layout as Y.

    work: the buffer a wdot_fwd call at the same state filled (the rate constants are
    then reused), or None (recomputed)."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    ns = m.n_species
    if u.dtype != torch.float64 or u.shape != (n, ns) or u.device != dev or (n > 0 and ns > 1 and
                                                                             (u.stride(0) != 1 or u.stride(1) != ld)):
        raise ValueError("u must be a float64 [n, Ns] tensor with the same species-major layout as Y")
    if u_hrr is not None and (u_hrr.dtype != torch.float64 or u_hrr.shape != (n,) or not u_hrr.is_contiguous()):
        raise ValueError("u_hrr must be a contiguous float64 [n] tensor")
    if work is not None and (work.dtype != torch.uint8 or work.device != dev or not work.is_contiguous()):
        raise ValueError("work must be a contiguous uint8 tensor on the mechanism's device")
    gT = torch.empty(n, dtype=torch.float64, device=dev)
    gY = _species_out(ns, n, ld, dev)
    check(_lib.lib().crf_wdot_vjp(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                  _ptr(u), _ptr(u_hrr), _ptr(gT), _ptr(gY), _ptr(work),
                                  0 if work is None else work.numel(), _stream(dev)))
    return gT, gY


def hbm_budget(dev):
    """Bytes the autograd forward may keep for the backward: CRF_HBM_BUDGET if set (then
    capped at the device memory free now), else 0.  The default recomputes: on MI355X the
    VJP kernel is not limited by the rate constants' exponentials, and reading them back
    (32 bytes per reaction and point) made it slower, not faster (53 species: 103.5
    against 113 M points/s in FP64)."""
    env = os.environ.get("CRF_HBM_BUDGET")
    if not env:
        return 0
    free, _ = torch.cuda.mem_get_info(dev)
    return min(int(float(env)), free)


def wdot_jvp(m, T, p, Y, vY, vT=None, precision="fp64", with_hrr=True, with_wdot=False):
    """(jv_hrr [n] or None, jv_w [n, Ns], wdot [n, Ns] or None) = d(hrr, w)/d(T, Y) . (vT, vY).

    vY in the same species-major layout as Y; vT [n] or None (zero)."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    ns = m.n_species
    if vY.dtype != torch.float64 or vY.shape != (n, ns) or vY.device != dev or (n > 0 and ns > 1 and
                                                                              (vY.stride(0) != 1 or vY.stride(1) != ld)):
        raise ValueError("vY must be a float64 [n, Ns] tensor with the same species-major layout as Y")
    if vT is not None and (vT.dtype != torch.float64 or vT.shape != (n,) or not vT.is_contiguous() or vT.device != dev):
        raise ValueError("vT must be a contiguous float64 [n] tensor on the mechanism's device")
    jh = torch.empty(n, dtype=torch.float64, device=dev) if with_hrr else None
    jw = _species_out(ns, n, ld, dev)
    w = _species_out(ns, n, ld, dev) if with_wdot else None
    check(_lib.lib().crf_wdot_jvp(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                  _ptr(vT), _ptr(vY), _ptr(jh), _ptr(jw), _ptr(w), _stream(dev)))
    return jh, jw, w


def source(m, T, p, Y, precision="fp64", dp0dt=0.0):
    """Point-wise chemistry source terms: dict(dYdt [n, Ns] 1/s, dTdt [n] K/s, QT [n] 1/s, hrr [n] W/m^3)."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    out = {"dYdt": _species_out(m.n_species, n, ld, dev)}
    out.update({k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("dTdt", "QT", "hrr")})
    check(_lib.lib().crf_source(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld, float(dp0dt),
                                *[_ptr(out[k]) for k in ("dYdt", "dTdt", "QT", "hrr")], _stream(dev)))
    return out


def wdot_jac(m, T, p, Y, precision="fp64", with_wdot=True, out=None):
    """(J [n, Ns+1, Ns+1] float64/float32, wdot [n, Ns] or None).

    Rows: (hrr, w_1..w_Ns); columns: (T, Y_1..Y_Ns); point-major, row-major per point.
    """
    n, p, ps, ld, dev = _state(m, T, p, Y)
    ns = m.n_species
    dt = torch.float64 if precision == "fp64" else torch.float32
    if out is None:
        out = torch.empty((n, ns + 1, ns + 1), dtype=dt, device=dev)
    elif out.dtype != dt or out.shape != (n, ns + 1, ns + 1) or not out.is_contiguous() or out.device != dev:
        raise ValueError("out has the wrong dtype, shape, layout or device")
    w = _species_out(ns, n, ld, dev) if with_wdot else None
    check(_lib.lib().crf_wdot_jac(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                  _ptr(out), _ptr(w), _stream(dev)))
    return out, w


def reactor_workspace(m, n, precision="fp64"):
    """A device buffer of the size crf_reactor_step needs for n points."""
    b = _lib.lib().crf_workspace_bytes(m.handle, _prec(precision), CRF_OP_REACTOR, int(n))
    return torch.empty(max(b, 1), dtype=torch.uint8, device=torch.device("cuda", m.device))


def reactor_step(m, T, p, Y, dt, nsub=1, precision="fp64", work=None):
    """Advance (T [n], Y [n, Ns] species-major) in place by dt seconds of an adiabatic
    constant-pressure reactor: nsub ROS2 substeps.  Returns (T, Y)."""
    n, p, ps, ld, dev = _state(m, T, p, Y)
    if work is None:
        work = reactor_workspace(m, n, precision)
    if work.dtype != torch.uint8 or work.device != dev or not work.is_contiguous():
        raise ValueError("work must be a contiguous uint8 tensor on the mechanism's device")
    check(_lib.lib().crf_reactor_step(m.handle, _prec(precision), n, _ptr(T), _ptr(p), ps, _ptr(Y), ld,
                                      float(dt), int(nsub), _ptr(work), work.numel(), _stream(dev)))
    return T, Y


class WdotFn(torch.autograd.Function):
    """(wdot, hrr) = WdotFn.apply(T, Y, p, mech, precision); backward = crf_wdot_vjp.

    The forward keeps the rate intermediates (crf_wdot_fwd) when they fit the HBM budget
    (hbm_budget: CRF_HBM_BUDGET bytes, 0 when unset); otherwise the backward recomputes
    them."""

    @staticmethod
    def forward(ctx, T, Y, p, mech, precision="fp64"):
        n = T.shape[0]
        need = workspace_bytes(mech, n, precision)
        work = None
        if 0 < need <= hbm_budget(T.device):
            work = new_workspace(mech, n, precision)
            w, h = wdot_fwd(mech, T, p, Y, work, precision=precision, hrr=True)
        else:
            w, h, _ = wdot(mech, T, p, Y, precision=precision, hrr=True)
        ctx.save_for_backward(T, Y)
        ctx.mech, ctx.p, ctx.precision, ctx.work = mech, p, precision, work
        return w, h

    @staticmethod
    def backward(ctx, g_w, g_h):
        T, Y = ctx.saved_tensors
        n, ns = Y.shape
        u = torch.zeros_like(Y) if g_w is None else g_w
        if u.stride(0) != 1 or (ns > 1 and u.stride(1) != Y.stride(1)):
            u2 = _species_out(ns, n, Y.stride(1) if ns > 1 else n, Y.device)
            u2.copy_(u)
            u = u2
        uh = None if g_h is None else g_h.contiguous()
        gT, gY = wdot_vjp(ctx.mech, T, ctx.p, Y, u, uh, precision=ctx.precision, work=ctx.work)
        ctx.work = None
        return gT, gY, None, None, None


__all__ = ["Mechanism", "species_major", "thermo", "wdot", "transport", "wdot_vjp", "wdot_jvp", "wdot_jac",
           "wdot_fwd", "workspace_bytes", "new_workspace", "hbm_budget", "source", "reactor_step", "reactor_workspace",
           "WdotFn", "CrfError"]
