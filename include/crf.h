/*
 * crf.h — C ABI of the MI355X per-grid-point thermochemistry library.
 *
 * The library evaluates, at every grid point, the chemistry terms that the
 * low-Mach reacting-flow solver of the nekCRF paper needs in each right-hand
 * side of its thermochemistry subsystem (Section 2, Eq. (1a)-(1d), Eq. (2)):
 * NASA-7 thermodynamics, net species production rates w_k and the heat-release
 * rate, mixture-averaged transport coefficients, and the derivatives of the
 * production rates (vector-Jacobian product and dense Jacobian) that a Newton
 * or Krylov iteration uses in place of difference quotients (Section 2).
 *
 * Conventions shared by every compute call
 * ---------------------------------------
 * Units: SI with kmol — T [K], p [Pa], C [kmol/m^3], w [kmol/(m^3 s)], hrr [W/m^3],
 *        mu [Pa s], lambda [W/(m K)], D [m^2/s], cp [J/(kmol K)], h and g [J/kmol].
 * State: n points; T[n]; p[i * p_stride] with p_stride 1 (per point) or 0 (one
 *        value for every point); mass fractions species-major,
 *        Y[k * ld + i] for species k < Ns and point i < n, ld >= n.
 *        Y is used as given (no renormalisation); every Y_k is an independent
 *        variable of the derivatives, p is held fixed.
 * Memory: every array argument is a DEVICE pointer on the mechanism's device,
 *        allocated and owned by the caller.  Per-species outputs use the same
 *        species-major layout and leading dimension ld as Y.  Outputs marked
 *        "nullable" may be NULL and are then neither computed nor written.
 *        The library allocates nothing but the mechanism tables.
 * Streams: compute calls enqueue kernels on `stream` (a hipStream_t; NULL is the
 *        null stream) and return without synchronising.
 * Errors: arguments are validated on the host before anything is launched; on a
 *        non-OK status nothing has been written and crf_last_error() describes
 *        the problem.  CRF_E_DEVICE reports a failed launch or device call.
 *        Physical-domain problems are not checked: T <= 0, non-finite inputs or
 *        negative Y propagate IEEE values.  Y_k = 0 is allowed and gives finite
 *        results (no division by concentrations anywhere).
 * Precision: CRF_FP64 computes everything in FP64.  CRF_MIXED computes the
 *        Arrhenius exponentials, the Troe blending and the transport fits and
 *        mixing rules in FP32 and keeps FP64 for the concentrations, the
 *        Gibbs-difference equilibrium constants, the forward-minus-reverse
 *        subtraction, the accumulation of w and the mass residual.  Outputs are
 *        FP64 buffers in both modes, except the Jacobian, which is FP32 in
 *        CRF_MIXED.
 * Threads: a loaded mechanism is read-only; concurrent calls on different
 *        streams are safe.
 */
#ifndef CRF_H
#define CRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct crf_mech crf_mech;   /* opaque: host copy and device tables of one mechanism */
typedef void *crf_stream;           /* a hipStream_t */

typedef enum {
    CRF_OK = 0,
    CRF_E_ARG = 1,          /* invalid argument (NULL, negative size, ld < n, bad enum ...) */
    CRF_E_PARSE = 2,        /* mechanism file unreadable or malformed */
    CRF_E_MECH = 3,         /* mechanism inconsistent (element balance, indices, ranges) */
    CRF_E_NOMEM = 4,        /* host or device allocation failed */
    CRF_E_DEVICE = 5,       /* device error, or a compute call on a host-only mechanism */
    CRF_E_UNSUPPORTED = 6,  /* valid file using a feature this library does not evaluate */
    CRF_E_WORKSPACE = 7     /* workspace missing, too small (crf_workspace_bytes) or misaligned */
} crf_status;

/* Operations that take a caller-allocated workspace (crf_workspace_bytes). */
typedef enum { CRF_OP_VJP = 1, CRF_OP_REACTOR = 2 } crf_op;

typedef enum { CRF_FP64 = 0, CRF_MIXED = 1 } crf_precision;

/* ---------------------------------------------------------------- mechanism */

/* Read a "crf-mech 1" text mechanism (species with element counts and NASA-7
 * coefficients, elementary / three-body / Troe-falloff reactions written with
 * integer stoichiometric coefficients, all reversible through K_c, and
 * cubic-in-ln(T) transport fits), validate it and upload its tables to
 * `device`.  device = -1 parses and validates only (no device is touched);
 * compute calls on such a mechanism return CRF_E_DEVICE.  Synchronous.
 * Validation: every reaction element-balanced, indices in range, no species on
 * both sides of a reaction, T_lo < T_mid < T_hi, positive atomic weights,
 * non-negative efficiencies, positive Troe T*** and T*, every diffusion pair
 * present.  On success *out owns everything; release it with crf_free_mech. */
crf_status crf_load_mech(const char *path, int device, crf_mech **out);

/* Free a mechanism.  The caller must have synchronised every stream that used it. NULL is a no-op. */
void crf_free_mech(crf_mech *m);

int crf_n_species(const crf_mech *m);     /* -1 for NULL */
int crf_n_reactions(const crf_mech *m);   /* -1 for NULL */
int crf_device(const crf_mech *m);        /* device the tables live on, -1 for host-only or NULL */

/* Which kernel crf_wdot_jac runs for this mechanism: "segmented" (one workgroup per
 * point, one reaction per thread, lockstep gather of the derivative sums; needs at
 * most 384 reactions, 64 species, 3 molecules per side, no optional rate forms and
 * 80 KB of LDS), "reaction-table (<reason>)" (each reaction evaluated once per point
 * into an LDS table, rows assembled from it in blocks; needs the table and 16 rows of
 * accumulators in 160 KB of LDS, FP32 table entries in the mixed mode) or
 * "row-block (<reason>)" (reactions re-evaluated per block of rows; any size).
 * Informational; the string is owned by the mechanism and valid until crf_free_mech.
 * "" for NULL. */
const char *crf_jac_plan(const crf_mech *m);

/* Message describing the last non-OK status returned on this thread ("" if none). */
const char *crf_last_error(void);
const char *crf_status_str(crf_status s);

/* ---------------------------------------------------------------- thermodynamics */

/* NASA-7 properties (Eq. (1b): c_p,k and h_k; Eq. (1d): rho), FP64.
 * Per species [k*ld + i] (each nullable): cp_k = R cp/R, h_k = R T h/(RT),
 * s_k = R s/R (standard state at p0), g_k = h_k - T s_k.
 * Per point [i] (each nullable): cp_mass = sum Y_k cp_k / W_k, h_mass = sum Y_k h_k / W_k,
 * rho = p Wbar / (R T), Wbar = 1 / sum (Y_k / W_k). */
crf_status crf_thermo(const crf_mech *m, int64_t n, const double *T, const double *p, int64_t p_stride,
                      const double *Y, int64_t ld,
                      double *cp_k, double *h_k, double *s_k, double *g_k,
                      double *cp_mass, double *h_mass, double *rho, double *Wbar, crf_stream stream);

/* ---------------------------------------------------------------- production rates */

/* Net production rates w_k = sum_i (nu''_ki - nu'_ki) q_i (the source of Eq. (1a)),
 * written to wdot[k*ld + i]; hrr[i] = -sum_k h_k w_k (the heat-release term of
 * Eq. (1b), positive when exothermic; nullable); mass_resid[i] = sum_k W_k w_k
 * (zero for an element-balanced mechanism, FP64 in both modes; nullable). */
crf_status crf_wdot(const crf_mech *m, crf_precision prec, int64_t n, const double *T, const double *p,
                    int64_t p_stride, const double *Y, int64_t ld,
                    double *wdot, double *hrr, double *mass_resid, crf_stream stream);

/* ---------------------------------------------------------------- transport */

/* Mixture-averaged transport without Soret/Dufour effects (Section 2, Eq. (2)):
 * mu[i] (Wilke), lambda[i] (Mathur-Saxena average), and the mixture diffusion
 * coefficients Dmix[k*ld + i] = (1 - Y_k) / sum_{j != k} X_j / D_jk of
 * V_k = -(D_k / X_k) grad X_k.  Each output nullable. */
crf_status crf_transport(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                         const double *p, int64_t p_stride, const double *Y, int64_t ld,
                         double *mu, double *lambda, double *Dmix, crf_stream stream);

/* ---------------------------------------------------------------- derivatives */

/* Bytes of workspace that operation `op` needs for n points (0 and CRF_E_ARG in
 * crf_last_error for invalid arguments).  CRF_OP_VJP: the rate intermediates that
 * crf_wdot_fwd stores and crf_wdot_vjp reuses, 32 bytes per reaction and point (k_f,
 * 1/K_c, dk_f/dT, dk_f/d[M], FP64 in both modes).  CRF_OP_REACTOR: the matrices and
 * stage vectors of crf_reactor_step (about 8 (Ns+1)^2 + 36 (Ns+1) bytes per point, plus
 * 4 (Ns+1)^2 with CRF_MIXED).  Whether to store them or to let the
 * VJP recompute them is the caller's choice against its memory budget; the Python
 * binding stores them while they fit in CRF_HBM_BUDGET bytes (unset: recompute). */
size_t crf_workspace_bytes(const crf_mech *m, crf_precision prec, int op, int64_t n);

/* Production rates as crf_wdot (wdot required, hrr and mass_resid nullable) that also
 * store, in the caller's workspace `work` (work_bytes >= crf_workspace_bytes(m, prec,
 * CRF_OP_VJP, n), 16-byte aligned, else CRF_E_WORKSPACE), the rate constants and their
 * derivatives of every reaction at every point, for a later crf_wdot_vjp at the same
 * state: the forward half of a reverse-mode step that keeps its intermediates. */
crf_status crf_wdot_fwd(const crf_mech *m, crf_precision prec, int64_t n, const double *T, const double *p,
                        int64_t p_stride, const double *Y, int64_t ld,
                        double *wdot, double *hrr, double *mass_resid, void *work, size_t work_bytes,
                        crf_stream stream);

/* Vector-Jacobian product of (hrr, w_1..w_Ns) with respect to (T, Y_1..Y_Ns) at
 * fixed p: gT[i] = u_hrr[i] dhrr/dT + sum_k u[k*ld+i] dw_k/dT and
 * gY[j*ld + i] = u_hrr[i] dhrr/dY_j + sum_k u[k*ld+i] dw_k/dY_j.
 * u_hrr nullable (treated as zero).
 * work == NULL (work_bytes ignored): every rate intermediate is recomputed.
 * Otherwise work must hold what crf_wdot_fwd stored for the same mechanism, precision,
 * n, T, p and Y (not checked: other contents give meaningless results) and
 * work_bytes >= crf_workspace_bytes(m, prec, CRF_OP_VJP, n), 16-byte aligned, else
 * CRF_E_WORKSPACE; the rate constants are then read, not re-evaluated. */
crf_status crf_wdot_vjp(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                        const double *p, int64_t p_stride, const double *Y, int64_t ld,
                        const double *u, const double *u_hrr, double *gT, double *gY,
                        const void *work, size_t work_bytes, crf_stream stream);

/* Jacobian-vector product (forward mode) of (hrr, w_1..w_Ns) with respect to
 * (T, Y_1..Y_Ns) at fixed p, along the tangent v = (vT, vY): the directional
 * derivative that the paper's Newton-GMRES iteration approximates by difference
 * quotients (Section 2), formed analytically:
 *   jv_w[k*ld + i] = dw_k/dT vT[i] + sum_j dw_k/dY_j vY[j*ld + i],
 *   jv_hrr[i]      = dhrr/dT vT[i] + sum_j dhrr/dY_j vY[j*ld + i].
 * vT nullable (treated as zero); vY required, same layout as Y.  jv_hrr and wdot
 * (the production rates of the same evaluation) nullable; jv_w required.  The
 * tangent sums over reactions are FP64 in both modes (the rates of progress and
 * their derivatives follow the precision mode). */
crf_status crf_wdot_jvp(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                        const double *p, int64_t p_stride, const double *Y, int64_t ld,
                        const double *vT, const double *vY, double *jv_hrr, double *jv_w,
                        double *wdot, crf_stream stream);

/* Point-wise chemistry source terms of the thermochemistry subsystem (Section 2,
 * Eq. (1a)-(1b)) and the point-wise part of the divergence constraint (Eq. (3)),
 * for a homogeneous mixture at each point (no transport terms):
 *   dYdt[k*ld + i] = W_k w_k / rho                        [1/s]
 *   dTdt[i]        = (hrr + dp0dt) / (rho c_p)            [K/s], c_p per unit mass
 *   QT[i]          = dTdt/T + sum_k (Wbar/W_k) dYdt_k - dp0dt/p   [1/s]
 *   hrr[i]         = -sum_k h_k w_k                       [W/m^3]
 * dp0dt is the rate of the (spatially uniform) thermodynamic pressure, 0 for an open
 * domain.  Every output nullable; at least one must be given. */
crf_status crf_source(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                      const double *p, int64_t p_stride, const double *Y, int64_t ld, double dp0dt,
                      double *dYdt, double *dTdt, double *QT, double *hrr, crf_stream stream);

/* Dense Jacobian of (hrr, w_1..w_Ns) with respect to (T, Y_1..Y_Ns) at fixed p,
 * for the Newton iteration of an implicit chemistry step (Section 2).  Point-major,
 * row-major per point: with N1 = Ns + 1, entry (r, c) of point i is
 * J[i * N1 * N1 + r * N1 + c]; row 0 = hrr, row 1 + k = w_k; column 0 = T,
 * column 1 + j = Y_j.  J holds doubles for CRF_FP64 and floats for CRF_MIXED.
 * wdot (nullable) receives the production rates of the same evaluation, [k*ld + i]
 * (with CRF_MIXED and the segmented kernel, summed in FP32).  Results are bitwise
 * reproducible run to run with the segmented kernel; the reaction-table and row-block
 * kernels sum a point's rows over several wavefronts with LDS atomics, reproducible to
 * rounding. */
crf_status crf_wdot_jac(const crf_mech *m, crf_precision prec, int64_t n, const double *T,
                        const double *p, int64_t p_stride, const double *Y, int64_t ld,
                        void *J, double *wdot, crf_stream stream);

/* ---------------------------------------------------------------- reactor step */

/* Advances every point, an adiabatic homogeneous mixture at constant pressure (the
 * thermochemistry subsystem of Section 2, Eq. (1a)-(1b), without transport terms; the
 * homogeneous autoignition of Section 3.1), by dt seconds: nsub substeps of the
 * two-stage L-stable Rosenbrock method ROS2 (Verwer, Spee, Blom and Hundsdorfer, 1999),
 *   (I - g h A) k1 = f(x),  (I - g h A) k2 = f(x + h k1) - 2 k1,  x <- x + 3/2 h k1 + 1/2 h k2,
 * with h = dt/nsub, g = 1 + 1/sqrt(2), x = (T, Y), f the source terms of crf_source
 * (dp0/dt = 0) and A = df/dx from the dense Jacobian of crf_wdot_jac (evaluated once per
 * substep), each point's linear systems solved by LU with partial pivoting.
 * T[n] and Y[k*ld + i] are read and overwritten in place; p is held fixed.
 * CRF_MIXED evaluates the rates and the Jacobian in the mixed mode (FP32 Jacobian
 * entries); the matrices, factorisation and updates are FP64 in both modes.
 * work: caller workspace of at least crf_workspace_bytes(m, prec, CRF_OP_REACTOR, n)
 * bytes, 256-byte aligned (else CRF_E_WORKSPACE); its contents on return are undefined.
 * dt > 0 finite and 1 <= nsub <= 1000000, else CRF_E_ARG.  No step-size control: a
 * singular Newton matrix or a step beyond the method's accuracy propagates IEEE values. */
crf_status crf_reactor_step(const crf_mech *m, crf_precision prec, int64_t n, double *T, const double *p,
                            int64_t p_stride, double *Y, int64_t ld, double dt, int nsub, void *work,
                            size_t work_bytes, crf_stream stream);

/* crf_reactor_step for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation,
 * with the workspace taken from a static scratch array of 128 MiB that the library holds
 * on each device it runs on until the process ends.  Allocates nothing (no hipMalloc or
 * hipFree, no allocating library call).  n is limited to what fits the 128 MiB
 * (crf_workspace_bytes(m, prec, CRF_OP_REACTOR, n) <= 134217728: about 5 000 points at 53
 * species in FP64); larger n returns CRF_E_WORKSPACE.  Every call on a device shares that
 * device's scratch (no part of it needs to start at zero; its last contents stay): calls
 * that overlap in time on one device, on different streams or threads, race and give
 * undefined results; serialise them. */
crf_status crf_reactor_step_static(const crf_mech *m, crf_precision prec, int64_t n, double *T, const double *p,
                                   int64_t p_stride, double *Y, int64_t ld, double dt, int nsub,
                                   crf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* CRF_H */
