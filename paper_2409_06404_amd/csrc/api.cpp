// C ABI entry points: host-side argument validation, then kernel launch.

#include <cmath>
#include <string>

#include "crf_bench.h"
#include "crf_internal.h"

namespace crf {

namespace {
thread_local std::string g_last_error;
}

crf_status fail(crf_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

void clear_error() { g_last_error.clear(); }

namespace {

// Validation of the state arguments common to every compute call.
crf_status check_state(const crf_mech *m, int64_t n, const double *T, const double *p, int64_t ps,
                       const double *Y, int64_t ld, const char *fn) {
    std::string f(fn);
    if (!m) return fail(CRF_E_ARG, f + ": mechanism is NULL");
    if (n < 0) return fail(CRF_E_ARG, f + ": n must be >= 0");
    if (n > ((int64_t)1 << 40)) return fail(CRF_E_ARG, f + ": n too large");
    if (ps != 0 && ps != 1) return fail(CRF_E_ARG, f + ": p_stride must be 0 or 1");
    if (ld < n) return fail(CRF_E_ARG, f + ": ld must be >= n");
    if (n > 0 && (!T || !p || !Y)) return fail(CRF_E_ARG, f + ": T, p and Y must not be NULL");
    return CRF_OK;
}

// The mechanism's tables are on a device (checked after every argument).
crf_status check_device(const crf_mech *m, const char *fn) {
    if (m->device < 0 || !m->dev_buf)
        return fail(CRF_E_DEVICE, std::string(fn) + ": mechanism was loaded without a device");
    return CRF_OK;
}

crf_status check_prec(crf_precision prec, const char *fn) {
    if (prec != CRF_FP64 && prec != CRF_MIXED) return fail(CRF_E_ARG, std::string(fn) + ": invalid precision");
    return CRF_OK;
}

// Runs `launch` with the mechanism's device current; restores the caller's device.
template <class F>
crf_status on_device(const crf_mech *m, const char *fn, F &&launch) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(CRF_E_DEVICE, std::string(fn) + ": hipGetDevice failed");
    if (prev != m->device && hipSetDevice(m->device) != hipSuccess)
        return fail(CRF_E_DEVICE, std::string(fn) + ": hipSetDevice failed");
    hipError_t e = launch();
    if (prev != m->device) hipSetDevice(prev);
    if (e != hipSuccess) return fail(CRF_E_DEVICE, std::string(fn) + ": launch failed: " + hipGetErrorString(e));
    return CRF_OK;
}

}  // namespace
}  // namespace crf

using namespace crf;

extern "C" {

crf_status crf_load_mech(const char *path, int device, crf_mech **out) {
    if (!out) return fail(CRF_E_ARG, "crf_load_mech: out is NULL");
    *out = nullptr;
    if (device < -1) return fail(CRF_E_ARG, "crf_load_mech: device must be >= -1");
    crf_mech *m = new (std::nothrow) crf_mech();
    if (!m) return fail(CRF_E_NOMEM, "crf_load_mech: out of host memory");
    crf_status s = parse_mechanism(path, m->host);
    if (s == CRF_OK) {
        build_jac_plan(m->host);
        const HostMech &h = m->host;
        if (h.jp_ok) m->plan_text = "segmented";
        else if (jac_rt_fits(h.ns(), h.nr(), false)) m->plan_text = "reaction-table (" + h.jp_why + ")";
        else if (jac_rt_fits(h.ns(), h.nr(), true))
            m->plan_text = "reaction-table in the mixed mode, row-block in FP64 (" + h.jp_why + ")";
        else m->plan_text = "row-block (" + h.jp_why + ")";
    }
    if (s == CRF_OK && device >= 0) s = upload_mechanism(m, device);
    if (s != CRF_OK) { delete m; return s; }
    *out = m;
    return CRF_OK;
}

void crf_free_mech(crf_mech *m) {
    if (!m) return;
    if (m->dev_buf) {
        int prev = -1;
        hipGetDevice(&prev);
        hipSetDevice(m->device);
        hipFree(m->dev_buf);
        if (prev >= 0) hipSetDevice(prev);
    }
    delete m;
}

int crf_n_species(const crf_mech *m) { return m ? m->host.ns() : -1; }
int crf_n_reactions(const crf_mech *m) { return m ? m->host.nr() : -1; }
int crf_device(const crf_mech *m) { return m ? m->device : -1; }

const char *crf_jac_plan(const crf_mech *m) { return m ? m->plan_text.c_str() : ""; }

const char *crf_last_error(void) { return crf::g_last_error.c_str(); }

const char *crf_status_str(crf_status s) {
    switch (s) {
        case CRF_OK: return "CRF_OK";
        case CRF_E_ARG: return "CRF_E_ARG";
        case CRF_E_PARSE: return "CRF_E_PARSE";
        case CRF_E_MECH: return "CRF_E_MECH";
        case CRF_E_NOMEM: return "CRF_E_NOMEM";
        case CRF_E_DEVICE: return "CRF_E_DEVICE";
        case CRF_E_UNSUPPORTED: return "CRF_E_UNSUPPORTED";
        case CRF_E_WORKSPACE: return "CRF_E_WORKSPACE";
    }
    return "CRF_UNKNOWN_STATUS";
}

crf_status crf_thermo(const crf_mech *m, int64_t n, const double *T, const double *p, int64_t ps,
                      const double *Y, int64_t ld, double *cp_k, double *h_k, double *s_k, double *g_k,
                      double *cp_mass, double *h_mass, double *rho, double *Wbar, crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_thermo");
    if (s != CRF_OK) return s;
    if (check_device(m, "crf_thermo") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_thermo", [&] {
        return launch_thermo(m->dev, n, T, p, ps, Y, ld, cp_k, h_k, s_k, g_k, cp_mass, h_mass, rho, Wbar,
                             (hipStream_t)stream);
    });
}

crf_status crf_wdot(const crf_mech *m, crf_precision prec, int64_t n, const double *T, const double *p,
                    int64_t ps, const double *Y, int64_t ld, double *wdot, double *hrr, double *mass_resid,
                    crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_wdot");
    if (s == CRF_OK) s = check_prec(prec, "crf_wdot");
    if (s != CRF_OK) return s;
    if (n > 0 && !wdot) return fail(CRF_E_ARG, "crf_wdot: wdot must not be NULL");
    if (check_device(m, "crf_wdot") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_wdot", [&] {
        return launch_wdot(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, wdot, hrr, mass_resid, nullptr,
                           (hipStream_t)stream);
    });
}

crf_status crf_transport(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                         const double *p, int64_t ps, const double *Y, int64_t ld, double *mu,
                         double *lambda, double *Dmix, crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_transport");
    if (s == CRF_OK) s = check_prec(prec, "crf_transport");
    if (s != CRF_OK) return s;
    if (check_device(m, "crf_transport") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0 || (!mu && !lambda && !Dmix)) return CRF_OK;
    return on_device(m, "crf_transport", [&] {
        return launch_transport(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, mu, lambda, Dmix,
                                (hipStream_t)stream);
    });
}

size_t crf_workspace_bytes(const crf_mech *m, crf_precision prec, int op, int64_t n) {
    if (!m) { fail(CRF_E_ARG, "crf_workspace_bytes: mechanism is NULL"); return 0; }
    if (check_prec(prec, "crf_workspace_bytes") != CRF_OK) return 0;
    if (n < 0 || n > ((int64_t)1 << 40)) { fail(CRF_E_ARG, "crf_workspace_bytes: n out of range"); return 0; }
    if (op == CRF_OP_VJP) return (size_t)n * (size_t)m->host.nr() * VJP_WORK_PER_RXN;
    if (op == CRF_OP_REACTOR) return reactor_work_bytes(m->host.ns(), prec == CRF_MIXED, n);
    fail(CRF_E_ARG, "crf_workspace_bytes: unknown operation");
    return 0;
}

namespace {
crf_status check_work(const crf_mech *m, int64_t n, const void *work, size_t work_bytes, const char *fn) {
    const size_t need = (size_t)n * (size_t)m->host.nr() * VJP_WORK_PER_RXN;
    if (!work) return fail(CRF_E_WORKSPACE, std::string(fn) + ": work is NULL");
    if (((uintptr_t)work & 15) != 0) return fail(CRF_E_WORKSPACE, std::string(fn) + ": work must be 16-byte aligned");
    if (work_bytes < need)
        return fail(CRF_E_WORKSPACE, std::string(fn) + ": work_bytes " + std::to_string(work_bytes) + " < " +
                                         std::to_string(need) + " needed");
    return CRF_OK;
}
}  // namespace

crf_status crf_wdot_fwd(const crf_mech *m, crf_precision prec, int64_t n, const double *T, const double *p,
                        int64_t ps, const double *Y, int64_t ld, double *wdot, double *hrr, double *mass_resid,
                        void *work, size_t work_bytes, crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_wdot_fwd");
    if (s == CRF_OK) s = check_prec(prec, "crf_wdot_fwd");
    if (s != CRF_OK) return s;
    if (n > 0 && !wdot) return fail(CRF_E_ARG, "crf_wdot_fwd: wdot must not be NULL");
    if (n > 0 && check_work(m, n, work, work_bytes, "crf_wdot_fwd") != CRF_OK) return CRF_E_WORKSPACE;
    if (check_device(m, "crf_wdot_fwd") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_wdot_fwd", [&] {
        return launch_wdot(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, wdot, hrr, mass_resid, (double *)work,
                           (hipStream_t)stream);
    });
}

crf_status crf_wdot_vjp(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                        const double *p, int64_t ps, const double *Y, int64_t ld, const double *u,
                        const double *u_hrr, double *gT, double *gY, const void *work, size_t work_bytes,
                        crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_wdot_vjp");
    if (s == CRF_OK) s = check_prec(prec, "crf_wdot_vjp");
    if (s != CRF_OK) return s;
    if (n > 0 && (!u || !gT || !gY)) return fail(CRF_E_ARG, "crf_wdot_vjp: u, gT and gY must not be NULL");
    if (n > 0 && work && check_work(m, n, work, work_bytes, "crf_wdot_vjp") != CRF_OK) return CRF_E_WORKSPACE;
    if (check_device(m, "crf_wdot_vjp") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_wdot_vjp", [&] {
        return launch_vjp(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, u, u_hrr, gT, gY,
                          (const double *)work, (hipStream_t)stream);
    });
}

crf_status crf_wdot_jvp(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                        const double *p, int64_t ps, const double *Y, int64_t ld, const double *vT,
                        const double *vY, double *jv_hrr, double *jv_w, double *wdot, crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_wdot_jvp");
    if (s == CRF_OK) s = check_prec(prec, "crf_wdot_jvp");
    if (s != CRF_OK) return s;
    if (n > 0 && (!vY || !jv_w)) return fail(CRF_E_ARG, "crf_wdot_jvp: vY and jv_w must not be NULL");
    if (check_device(m, "crf_wdot_jvp") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_wdot_jvp", [&] {
        return launch_jvp(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, vT, vY, jv_hrr, jv_w, wdot,
                          (hipStream_t)stream);
    });
}

crf_status crf_source(const crf_mech *m, crf_precision prec, int64_t n, const double *T, const double *p,
                      int64_t ps, const double *Y, int64_t ld, double dp0dt, double *dYdt, double *dTdt,
                      double *QT, double *hrr, crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_source");
    if (s == CRF_OK) s = check_prec(prec, "crf_source");
    if (s != CRF_OK) return s;
    if (!dYdt && !dTdt && !QT && !hrr) return fail(CRF_E_ARG, "crf_source: no output given");
    if (!std::isfinite(dp0dt)) return fail(CRF_E_ARG, "crf_source: dp0dt must be finite");
    if (check_device(m, "crf_source") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_source", [&] {
        return launch_source(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, dp0dt, dYdt, dTdt, QT, hrr,
                             (hipStream_t)stream);
    });
}

crf_status crf_reactor_step(const crf_mech *m, crf_precision prec, int64_t n, double *T, const double *p,
                            int64_t ps, double *Y, int64_t ld, double dt, int nsub, void *work, size_t work_bytes,
                            crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_reactor_step");
    if (s == CRF_OK) s = check_prec(prec, "crf_reactor_step");
    if (s != CRF_OK) return s;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CRF_E_ARG, "crf_reactor_step: dt must be positive and finite");
    if (nsub < 1 || nsub > 1000000) return fail(CRF_E_ARG, "crf_reactor_step: nsub must be in [1, 1000000]");
    if (n > 0) {
        const size_t need = reactor_work_bytes(m->host.ns(), prec == CRF_MIXED, n);
        if (!work) return fail(CRF_E_WORKSPACE, "crf_reactor_step: work is NULL");
        if (((uintptr_t)work & 255) != 0) return fail(CRF_E_WORKSPACE, "crf_reactor_step: work must be 256-byte aligned");
        if (work_bytes < need)
            return fail(CRF_E_WORKSPACE, "crf_reactor_step: work_bytes " + std::to_string(work_bytes) + " < " +
                                             std::to_string(need) + " needed");
    }
    if (check_device(m, "crf_reactor_step") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_reactor_step", [&] {
        return launch_reactor(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, dt, nsub, work, (hipStream_t)stream);
    });
}

crf_status crf_reactor_step_static(const crf_mech *m, crf_precision prec, int64_t n, double *T, const double *p,
                                   int64_t ps, double *Y, int64_t ld, double dt, int nsub, crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_reactor_step_static");
    if (s == CRF_OK) s = check_prec(prec, "crf_reactor_step_static");
    if (s != CRF_OK) return s;
    if (!(dt > 0.0) || !std::isfinite(dt))
        return fail(CRF_E_ARG, "crf_reactor_step_static: dt must be positive and finite");
    if (nsub < 1 || nsub > 1000000) return fail(CRF_E_ARG, "crf_reactor_step_static: nsub must be in [1, 1000000]");
    const size_t need = reactor_work_bytes(m->host.ns(), prec == CRF_MIXED, n);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(CRF_E_WORKSPACE, "crf_reactor_step_static: " + std::to_string(n) + " points need " +
                                         std::to_string(need) + " bytes of scratch, more than the static " +
                                         std::to_string(STATIC_SCRATCH_BYTES) + "; use crf_reactor_step");
    if (check_device(m, "crf_reactor_step_static") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_reactor_step_static", [&] {
        return launch_reactor_static(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, dt, nsub, (hipStream_t)stream);
    });
}

crf_status crf_wdot_jac(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                        const double *p, int64_t ps, const double *Y, int64_t ld, void *J, double *wdot,
                        crf_stream stream) {
    crf_status s = check_state(m, n, T, p, ps, Y, ld, "crf_wdot_jac");
    if (s == CRF_OK) s = check_prec(prec, "crf_wdot_jac");
    if (s != CRF_OK) return s;
    if (n > 0 && !J) return fail(CRF_E_ARG, "crf_wdot_jac: J must not be NULL");
    if (check_device(m, "crf_wdot_jac") != CRF_OK) return CRF_E_DEVICE;
    if (n == 0) return CRF_OK;
    return on_device(m, "crf_wdot_jac", [&] {
        return launch_jac(m->dev, prec == CRF_MIXED, n, T, p, ps, Y, ld, J, wdot, (hipStream_t)stream);
    });
}

crf_status crf_peak_rate(int kind, int64_t threads, int iters, double *out, crf_stream stream) {
    if (kind < 0 || kind > 4) return fail(CRF_E_ARG, "crf_peak_rate: kind must be 0..4");
    if (threads < 256 || threads % 256 != 0 || threads > ((int64_t)1 << 26))
        return fail(CRF_E_ARG, "crf_peak_rate: threads must be a multiple of 256 in [256, 2^26]");
    if (iters < 1 || !out) return fail(CRF_E_ARG, "crf_peak_rate: iters >= 1 and out required");
    const hipError_t e = launch_peak(kind, threads, iters, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(CRF_E_DEVICE, std::string("crf_peak_rate: launch failed: ") + hipGetErrorString(e));
    return CRF_OK;
}

}  // extern "C"
