// Internal definitions shared by the loader, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "crf.h"

namespace crf {

// Reaction kinds (bits 0-1 of the packed reaction info word).  RXN_TROE is every falloff
// reaction (Troe, Lindemann or SRI broadening, RxnVar flags).
enum : int { RXN_ELEMENTARY = 0, RXN_THREEBODY = 1, RXN_TROE = 2 };

// Optional rate forms and modifiers of a reaction (RxnVar.flags):
enum : int {
    VAR_PLOG = 1,          // rate: PLOG table at vtab[rate_off]: n, then n x (ln p, ln A, b, theta)
    VAR_CHEB = 2,          // rate: Chebyshev at vtab[rate_off]: nT, nP, 1/Tmin, 1/Tmax, log10 Pmin,
                           //       log10 Pmax, alpha[nT][nP]
    VAR_RATE_MASK = 3,
    VAR_LINDEMANN = 4,     // falloff broadening F = 1 (troe row: ln A0, b0, theta0)
    VAR_SRI = 8,           // falloff broadening SRI (troe row: ln A0, b0, theta0, a, b, c, d, e)
    VAR_REVERSE = 16,      // explicit reverse Arrhenius at vtab[rev_off]: ln A, b, theta
    VAR_IRREV = 32,        // no reverse reaction
    VAR_ORDERS = 64        // forward orders of reactant slots 0..2 at vtab[ord_off]
};
struct alignas(16) RxnVar { int flags, rate_off, rev_off, ord_off; };

// Slots per reaction: up to 3 distinct reactant species (slots 0-2) and up to 3
// distinct product species (slots 3-5).  Packed info word:
//   bits 0-1  kind
//   bits 2-3  number of reactant slots used
//   bits 4-5  number of product slots used
//   bits 6+2s coefficient (1..3) of slot s, s = 0..5
constexpr int MAX_SIDE = 3;
constexpr int SLOTS = 6;

// Largest mechanism the kernels evaluate: the lane-per-reaction kernels keep a few
// per-species arrays of every point in flight in LDS (at least 64 x ns bytes for one
// wavefront), and the row-block Jacobian one row of accumulators besides its species
// state.  Larger files are refused at load with CRF_E_UNSUPPORTED.
constexpr int MAX_SPECIES = 2048;
// Workspace of the stored-intermediate VJP: k_f, 1/K_c, dk_f/dT, dk_f/d[M] per reaction and point.
constexpr size_t VJP_WORK_PER_RXN = 4 * sizeof(double);
// Static device scratch of crf_reactor_step_static (per device, for the life of the process).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int MAX_DEVICES = 64;
// LDS of one compute unit (gfx950), the most one workgroup may request.
constexpr int CU_LDS_BYTES = 160 * 1024;

__host__ __device__ inline int info_kind(int w) { return w & 3; }
__host__ __device__ inline int info_nreac(int w) { return (w >> 2) & 3; }
__host__ __device__ inline int info_nprod(int w) { return (w >> 4) & 3; }
__host__ __device__ inline int info_nu(int w, int s) { return (w >> (6 + 2 * s)) & 3; }

// Per-reaction integer record, 8 ints (two 16-byte loads):
//   [0..5] species of slots 0..5 (-1 unused)
//   [6]    first third-body efficiency exception (index into eff_sp / eff_m1)
//   [7]    number of exceptions (bits 0-7) | troe index << 8
struct alignas(16) RxnInts { int v[8]; };

// Device tables of one mechanism; pointers into a single device allocation.
struct DevMech {
    int ns, nr, n_troe, n_exc;
    double R, p0;
    // species
    const double *W, *invW;
    const double *nasa;       // [ns][16]: Tmid, a_lo[7], a_hi[7], pad
    const double *mu_fit;     // [ns][4]
    const double *lam_fit;    // [ns][4]
    const double *w4;         // W^(1/4)
    const double *iw4;        // W^(-1/4)
    const double *wilke_c;    // [j][k]: (1/sqrt 8) (1 + W_k/W_j)^(-1/2)
    // binary-diffusion pairs as a round-robin schedule: each of tr_rounds rounds is a
    // perfect matching of the species (plus the dummy species ns when ns is odd), tr_slots
    // pairs per round
    const int *tr_jk;         // [round][slot]: j | k << 16 (the FP64 tables' pair order)
    const unsigned *tr_off;   // [prec][round][slot]: byte offsets of rows j and k in a point tile,
                              // 8 tt_rs(W) j | 8 tt_rs(W) k << 16, W the tile width of the FP64
                              // (prec 0) or mixed (prec 1) transport
    const double *tr_fit;     // [round][slot][4]: the pair's ln D fit (zeros for the dummy pair)
    const float *tr_fit32;    // the fits rounded to FP32 in the mixed tables' pair order (the
                              // mixed tile; the same order as tr_fit when both widths agree)
    int tr_rounds, tr_slots;
    // reactions
    const double *lnA, *b, *theta;
    const int *info;          // packed info word
    const int *rxn_order;     // processing order of the lane-per-reaction kernels: falloff, third-body, elementary
    const int *dnu_sum;       // sum_k (nu''_k - nu'_k)
    const RxnInts *ri;
    const double *troe;       // [n_troe][8]: lnA0, b0, theta0, alpha, 1/T3, 1/T1, T2, 0
    const int *eff_sp;        // [n_exc]
    const double *eff_m1;     // [n_exc] eps - 1
    const RxnVar *var;        // [nr] optional rate forms (all zero for a plain mechanism)
    const double *vtab;       // their parameters
    int n_var;                // reactions with a nonzero RxnVar
    // Segmented Jacobian plan (build_jac_plan in mech.cpp); jp_ok == 0 if the mechanism does not fit it
    const int *jp_thr;        // [JS_THREADS] per-thread reaction constants (JsThr)
    const unsigned *jp_recs;  // gather rounds, [JS_WAVES][JS_DMAX][64 lanes] uint2 (build_jac_plan)
    const int *jp_mrx;        // [jp_nm][2]: first efficiency exception, exception count of each [M] slot
    const int *jp_prog;       // [JS_WAVES][8]: gather rounds in use, first 32-bit word of the rounds
    int jp_ok, jp_nd, jp_sr, jp_lds;
    int jp_rmax;              // most gather rounds of a wavefront (at most JS_DMAX)
    int jp_off_a, jp_off_sp, jp_off_row, jp_off_p, jp_off_sc, jp_off_tp, jp_off_ex;  // LDS bytes
    int jp_off_tq, jp_off_ns, jp_off_iw, jp_off_mx, jp_off_mq, jp_nm;
    int jp_qb;                // first per-reaction (dT, q, d[M], sum) value among the d values
};

// Segmented Jacobian kernel (k_jac_seg): six wavefronts per workgroup, one reaction per
// thread, at most JS_DMAX gather rounds of JS_LD records per lane (streamed through
// registers, JS_DW rounds ahead).
constexpr int JS_WAVES = 6;
constexpr int JS_THREADS = 64 * JS_WAVES;
constexpr int JS_LD = 3;
constexpr int JS_DMAX = 24;
constexpr int JS_DW = 8;            // gather rounds whose records are in registers ahead of use
constexpr int JS_PWAVES = 3;        // wavefronts that form the heat-release row
constexpr int JS_EWAVES = 4;        // wavefronts that emit the Jacobian
constexpr int JS_EROWS = 10;        // most Jacobian rows one emitting thread writes
constexpr int JS_TP = 12;           // staged Troe constants per falloff reaction
constexpr int JS_TQ = 6;            // per-point temperature terms per falloff reaction
constexpr int JS_MAX_LDS = 80 * 1024;   // two workgroups per compute unit (160 KB of LDS)

// Per-thread constants of k_jac_seg (8 ints, two 16-byte loads).
struct alignas(16) JsThr {
    int r;        // reaction, -1 if the thread is idle
    int sp03;     // species of molecule slots 0..3, 8 bits each (ns = the unit dummy species)
    int sp45;     // slots 4, 5 (bits 0-15) | reactant molecules << 16 | product molecules << 19 | kind << 22
    int dpos;     // first derivative value of the reaction (index into the d values)
    int xpos;     // first efficiency-exception value (bits 0-15) | exception count << 16
    int exc0;     // first exception in eff_sp / eff_m1
    int troe;     // Troe parameter row (bits 0-15) | [M] slot << 16; 0xffff in either field if none
    int dnu;      // sum_k (nu''_k - nu'_k)
};

// Host copy of a parsed mechanism.
struct HostMech {
    double R = 0, p0 = 0;
    std::vector<std::string> elements;
    std::vector<double> aw;
    std::vector<std::string> names;
    std::vector<int> comp;               // [ns][ne]
    std::vector<double> W;
    std::vector<double> nasa;            // [ns][16]
    std::vector<double> mu_fit, lam_fit; // [ns][4]
    std::vector<double> dif_full;        // [ns][ns][4], symmetric
    std::vector<char> dif_seen;          // [ns][ns]
    std::vector<double> lnA, b, theta;
    std::vector<int> info, dnu_sum;
    std::vector<RxnInts> ri;
    std::vector<double> troe;            // [n_troe][8]
    std::vector<int> eff_sp;
    std::vector<double> eff_m1;
    std::vector<RxnVar> var;             // [nr]
    std::vector<double> vtab;
    int n_var = 0;
    // segmented Jacobian plan
    std::vector<JsThr> jp_thr;
    std::vector<unsigned> jp_recs;
    std::vector<int> jp_prog;
    int jp_ok = 0, jp_nd = 0, jp_sr = 0, jp_lds = 0, jp_rmax = 0;
    int jp_off_a = 0, jp_off_sp = 0, jp_off_row = 0, jp_off_p = 0, jp_off_sc = 0;
    int jp_off_tp = 0, jp_off_ex = 0, jp_off_tq = 0, jp_off_ns = 0, jp_off_iw = 0, jp_off_mx = 0, jp_off_mq = 0;
    int jp_nm = 0, jp_qb = 0;
    std::vector<int> jp_mrx;
    std::string jp_why;                  // why the plan is absent (for diagnostics)
    int ns() const { return (int)names.size(); }
    int nr() const { return (int)lnA.size(); }
};

}  // namespace crf

struct crf_mech {
    crf::HostMech host;
    crf::DevMech dev{};
    int device = -1;
    void *dev_buf = nullptr;
    std::string plan_text;   // what crf_jac_plan returns, fixed at load
};

namespace crf {

// Error reporting (thread-local message of the last failure).
crf_status fail(crf_status s, const std::string &msg);
void clear_error();

// Parsing / validation / upload (mech.cpp).
crf_status parse_mechanism(const char *path, HostMech &out);
void build_jac_plan(HostMech &h);
crf_status upload_mechanism(crf_mech *m, int device);

// LDS of the reaction-table Jacobian kernel (k_jac_rt): the species state {C, g/RT, h/RT,
// cp/R} (nsp each), the row scalars {tau, jtc, R, w} (nsp + 1 each), every reaction's
// enthalpy (nrp doubles) and 7 table values (d of six slots and d/d[M]; FP64, or FP32 in
// the mixed mode), then rb Jacobian rows of FP64 accumulators with two per-row scalars
// each.  The kernel takes the mechanism when 16 rows fit 160 KB and there are at most
// 511 species (one emitting thread per column).
struct JacRtLayout { size_t total; int rows; };
inline bool jac_rt_fits(int ns, int nr, bool mixed, JacRtLayout *out = nullptr) {
    const int nsp = ns | 1, n1 = ns + 1, sr = n1 | 1, nrp = (nr + 1) & ~1;
    const size_t fixed = (size_t)(4 * nsp + 4 * (nsp + 1) + nrp) * sizeof(double) +
                         (size_t)7 * nrp * (mixed ? sizeof(float) : sizeof(double)) + 16 +
                         16 * sizeof(double);   // per-wavefront partial sums of the state
    const size_t budget = CU_LDS_BYTES - 256, row_bytes = (size_t)(sr + 2) * sizeof(double);
    if (n1 > 512 || fixed + (size_t)16 * row_bytes > budget) return false;
    if (out) {
        int rb = (int)((budget - fixed) / row_bytes);
        if (rb >= n1) rb = n1;
        const int nblk = (n1 + rb - 1) / rb;
        rb = (n1 + nblk - 1) / nblk;
        out->rows = rb;
        out->total = fixed + (size_t)rb * row_bytes;
    }
    return true;
}

// Byte layout of the workspace of crf_reactor_step for n points (offsets of its regions; all
// regions 256-byte aligned).  FP64: the Newton matrix overwrites the Jacobian in place.
struct RosLayout {
    size_t J, M, wd, piv, k1, Tw, Yw, Ts, Ys, fT, fY, total;
};
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline RosLayout ros_layout(int ns, int mixed, int64_t n) {
    const size_t N = (size_t)ns + 1, nn = (size_t)n;
    RosLayout L{};
    size_t o = 0;
    L.J = o; o = align256(o + nn * N * N * (mixed ? sizeof(float) : sizeof(double)));
    if (mixed) { L.M = o; o = align256(o + nn * N * N * sizeof(double)); } else { L.M = L.J; }
    L.wd = o; o = align256(o + nn * ns * sizeof(double));
    L.piv = o; o = align256(o + nn * N * sizeof(int));
    L.k1 = o; o = align256(o + nn * N * sizeof(double));
    L.Tw = o; o = align256(o + nn * sizeof(double));
    L.Yw = o; o = align256(o + nn * ns * sizeof(double));
    L.Ts = o; o = align256(o + nn * sizeof(double));
    L.Ys = o; o = align256(o + nn * ns * sizeof(double));
    L.fT = o; o = align256(o + nn * sizeof(double));
    L.fY = o; o = align256(o + nn * ns * sizeof(double));
    L.total = o;
    return L;
}
inline size_t reactor_work_bytes(int ns, int mixed, int64_t n) { return n > 0 ? ros_layout(ns, mixed, n).total : 0; }

// Transport on point tiles of TT_P points, W wavefronts per workgroup, each wavefront
// owning TT_P / W points of the diffusion sums.  The row stride (doubles) of the tile's
// [species][point] arrays in LDS is TT_P + TT_P / W, so that the TT_P / W points of row j
// start at bank slot j mod W (32 banks of 4 bytes); the host orders the pairs of the
// schedule so that W consecutive pairs have distinct first and distinct second members mod W.
constexpr int TT_P = 16;
constexpr int tt_rs(int W) { return TT_P + TT_P / W; }
// LDS bytes of the tile kernel for `rows` species rows (species and the schedule's dummy).
inline size_t tile_transport_lds(int rows, bool mixed, int W) {
    return (size_t)rows * tt_rs(W) * (2 * sizeof(double) + (mixed ? sizeof(float) : sizeof(double))) +
           (size_t)(64 + 2 * TT_P + 4 * W * TT_P) * sizeof(double);
}
// Wavefronts per tile workgroup: 4 while four or more such workgroups fit a compute unit's
// LDS, else 8 while two or three do, else 16 (one); each width judged with its own row
// stride; 0 if the tile does not fit (the species-per-lane kernel).
inline int tile_transport_waves(int rows, bool mixed) {
    auto fit = [&](int W) { return (int)(CU_LDS_BYTES / tile_transport_lds(rows, mixed, W)); };
    const int W = fit(4) >= 4 ? 4 : (fit(8) >= 2 ? 8 : 16);
    const bool fits = tile_transport_lds(rows, mixed, W) <= (size_t)CU_LDS_BYTES;
    return fits && 8 * tt_rs(W) * rows <= 0xffff ? W : 0;   // 16-bit row offsets
}

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_thermo(const DevMech &m, int64_t n, const double *T, const double *p, int64_t ps,
                         const double *Y, int64_t ld, double *cp_k, double *h_k, double *s_k,
                         double *g_k, double *cp_mass, double *h_mass, double *rho, double *Wbar,
                         hipStream_t st);
hipError_t launch_wdot(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                       int64_t ps, const double *Y, int64_t ld, double *wdot, double *hrr,
                       double *rmass, double *work, hipStream_t st);
hipError_t launch_transport(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                            int64_t ps, const double *Y, int64_t ld, double *mu, double *lam,
                            double *Dmix, hipStream_t st);
hipError_t launch_vjp(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                      int64_t ps, const double *Y, int64_t ld, const double *u, const double *uh,
                      double *gT, double *gY, const double *work, hipStream_t st);
hipError_t launch_jvp(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                      int64_t ps, const double *Y, int64_t ld, const double *vT, const double *vY,
                      double *jh, double *jw, double *wdot, hipStream_t st);
hipError_t launch_source(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                         int64_t ps, const double *Y, int64_t ld, double dp0dt, double *dYdt,
                         double *dTdt, double *QT, double *hrr, hipStream_t st);
hipError_t launch_reactor(const DevMech &m, int mixed, int64_t n, double *T, const double *p, int64_t ps,
                          double *Y, int64_t ld, double dt, int nsub, void *work, hipStream_t st);
hipError_t launch_reactor_static(const DevMech &m, int mixed, int64_t n, double *T, const double *p, int64_t ps,
                                 double *Y, int64_t ld, double dt, int nsub, hipStream_t st);
hipError_t launch_peak(int kind, int64_t threads, int iters, double *out, hipStream_t st);
hipError_t launch_jac(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                      int64_t ps, const double *Y, int64_t ld, void *J, double *wdot, hipStream_t st);

}  // namespace crf
