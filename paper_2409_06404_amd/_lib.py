"""ctypes declarations of the C ABI in include/crf.h (argument marshalling only)."""
import ctypes
import os

# CRF_LIB names another build of the same ABI (the sanitized host-only build of the host tests)
LIB_PATH = os.environ.get("CRF_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcrf.so")

EXPORTED = (
    "crf_load_mech", "crf_free_mech", "crf_n_species", "crf_n_reactions", "crf_device", "crf_jac_plan",
    "crf_last_error", "crf_status_str", "crf_thermo", "crf_wdot", "crf_transport",
    "crf_wdot_vjp", "crf_wdot_jac", "crf_wdot_jvp", "crf_source", "crf_workspace_bytes", "crf_wdot_fwd",
    "crf_reactor_step", "crf_reactor_step_static", "crf_peak_rate",
)

CRF_OK, CRF_E_ARG, CRF_E_PARSE, CRF_E_MECH, CRF_E_NOMEM, CRF_E_DEVICE, CRF_E_UNSUPPORTED, CRF_E_WORKSPACE = range(8)
CRF_FP64, CRF_MIXED = 0, 1
CRF_OP_VJP, CRF_OP_REACTOR = 1, 2

_lib = None


class CrfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def status_name(s):
    return ["CRF_OK", "CRF_E_ARG", "CRF_E_PARSE", "CRF_E_MECH", "CRF_E_NOMEM", "CRF_E_DEVICE",
            "CRF_E_UNSUPPORTED", "CRF_E_WORKSPACE"][s] if 0 <= s < 8 else f"status {s}"


def lib():
    """The loaded library; raises if libcrf.so has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    L.crf_load_mech.argtypes = [ctypes.c_char_p, I, ctypes.POINTER(ctypes.c_void_p)]
    L.crf_load_mech.restype = I
    L.crf_free_mech.argtypes = [P]
    L.crf_free_mech.restype = None
    for f in ("crf_n_species", "crf_n_reactions", "crf_device"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = I
    L.crf_jac_plan.argtypes = [P]
    L.crf_jac_plan.restype = ctypes.c_char_p
    L.crf_last_error.argtypes = []
    L.crf_last_error.restype = ctypes.c_char_p
    L.crf_status_str.argtypes = [I]
    L.crf_status_str.restype = ctypes.c_char_p
    state = [P, I64, D, D, I64, D, I64]
    L.crf_thermo.argtypes = state + [D] * 8 + [P]
    L.crf_thermo.restype = I
    L.crf_wdot.argtypes = [P, I, I64, D, D, I64, D, I64, D, D, D, P]
    L.crf_wdot.restype = I
    L.crf_transport.argtypes = [P, I, I64, D, D, I64, D, I64, D, D, D, P]
    L.crf_transport.restype = I
    SZ = ctypes.c_size_t
    L.crf_wdot_vjp.argtypes = [P, I, I64, D, D, I64, D, I64, D, D, D, D, D, SZ, P]
    L.crf_wdot_vjp.restype = I
    L.crf_wdot_jac.argtypes = [P, I, I64, D, D, I64, D, I64, D, D, P]
    L.crf_wdot_jac.restype = I
    L.crf_wdot_jvp.argtypes = [P, I, I64, D, D, I64, D, I64, D, D, D, D, D, P]
    L.crf_wdot_jvp.restype = I
    L.crf_source.argtypes = [P, I, I64, D, D, I64, D, I64, ctypes.c_double, D, D, D, D, P]
    L.crf_source.restype = I
    L.crf_workspace_bytes.argtypes = [P, I, I, I64]
    L.crf_workspace_bytes.restype = SZ
    L.crf_wdot_fwd.argtypes = [P, I, I64, D, D, I64, D, I64, D, D, D, D, SZ, P]
    L.crf_wdot_fwd.restype = I
    L.crf_reactor_step.argtypes = [P, I, I64, D, D, I64, D, I64, ctypes.c_double, I, D, SZ, P]
    L.crf_reactor_step.restype = I
    L.crf_reactor_step_static.argtypes = [P, I, I64, D, D, I64, D, I64, ctypes.c_double, I, P]
    L.crf_reactor_step_static.restype = I
    L.crf_peak_rate.argtypes = [I, I64, I, D, P]
    L.crf_peak_rate.restype = I
    _lib = L
    return L


def check(status):
    if status != CRF_OK:
        raise CrfError(status, lib().crf_last_error().decode())
