// HIP kernels for gfx950 (CDNA4): per-point thermochemistry, production rates,
// transport, vector-Jacobian product and dense Jacobian.
//
// Work decomposition.  A mechanism has tens to thousands of reactions and tens
// to hundreds of species, and the chemistry of every grid point is independent.
// Each 64-wide wavefront therefore owns one grid point (or a few) at a time:
//   * state phase:    lanes = species (mixture state, NASA-7 polynomials);
//   * reaction phase: lanes = reactions (rate constants, falloff, equilibrium
//                     constants, rates of progress and their derivatives);
//   * output phase:   lanes = species / Jacobian columns.
// Per-point species arrays live in LDS ([species] per point, a few KB per wave),
// reaction constants are read from the mechanism tables (the same addresses for
// every wave, so they stay in L1/L2), and the sparse stoichiometric reductions
// (w_k = sum_i dnu_ki q_i and the Jacobian assembly) are scatters into LDS with
// native ds_add_f64 / ds_add_f32.  In the production-rate and VJP kernels every LDS
// address is owned by one wave, so the order of additions is fixed by the program and
// results are reproducible; the row-block Jacobian shares a point's rows between four
// wavefronts, so its sums are reproducible to rounding only.
//
// Thermodynamics (crf_thermo) is point-parallel instead: lane = point, species
// loop uniform, coefficients via scalar loads, fully coalesced stores.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "crf_internal.h"

namespace crf {

namespace {

constexpr int WAVE = 64;
constexpr double LN10 = 2.302585092994045684;
constexpr double INV_LN10 = 0.4342944819032518277;

// ------------------------------------------------------------------ helpers
// v from the lane `ctrl` selects (DPP), 0 where the source lane is outside the pattern or
// the lane is outside the row/bank masks; a double moves as two 32-bit halves.
template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, returned in every lane.  Data-parallel prefix steps through
// DPP (row shifts by 1, 2, 4, 8, then the row broadcasts of lanes 15 and 31), which stay
// in the VALU; lane 63 ends with the total, read back as a uniform value.  The order of
// additions is fixed, so the result is reproducible.
__device__ inline double wave_sum(double v) {
    v += dpp_f64<0x111, 0xf>(v);   // row_shr:1
    v += dpp_f64<0x112, 0xf>(v);   // row_shr:2
    v += dpp_f64<0x114, 0xf>(v);   // row_shr:4
    v += dpp_f64<0x118, 0xf>(v);   // row_shr:8
    v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Largest value over the 64 lanes (IEEE maxNum: NaN entries are passed over), in every
// lane; the same DPP pattern as wave_sum, so the reduction stays in the VALU.
__device__ inline double wave_max(double v) {
    v = fmax(v, dpp_f64<0x111, 0xf>(v));
    v = fmax(v, dpp_f64<0x112, 0xf>(v));
    v = fmax(v, dpp_f64<0x114, 0xf>(v));
    v = fmax(v, dpp_f64<0x118, 0xf>(v));
    v = fmax(v, dpp_f64<0x142, 0xa>(v));
    v = fmax(v, dpp_f64<0x143, 0xc>(v));
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Makes LDS writes of all lanes of this wave visible to all its lanes.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline double ipow(double x, int n) {   // n in 0..3
    return n == 1 ? x : n == 2 ? x * x : n == 3 ? x * x * x : 1.0;
}
__device__ inline double ipow_m1(double x, int n) {   // n * x^(n-1), n in 1..3
    return n == 1 ? 1.0 : n == 2 ? 2.0 * x : 3.0 * x * x;
}

template <class R> __device__ inline R exp_r(R x);
// e^x in FP64: Cody-Waite reduction x = k ln2 + f (ln2 split in a 32-bit head and a
// tail, so k ln2_hi is exact for |k| < 2^21), |f| <= ln2/2, then a degree-11
// polynomial interpolating e^f at the Chebyshev nodes of that interval (fitted in
// extended precision; about 2 ulp over the interval), scaled by 2^k.  Underflows to 0
// and overflows to +inf like e^x; NaN propagates.
__device__ inline double exp_fast(double x) {
    const double k = rint(x * 1.4426950408889634074);
    double f = fma(-k, 6.93147180369123816490e-01, x);
    f = fma(-k, 1.90821492927058770002e-10, f);
    double q = 2.51107961235593001e-08;
    q = fma(q, f, 2.76326740329670590e-07);
    q = fma(q, f, 2.75572379539371718e-06);
    q = fma(q, f, 2.48014853795884660e-05);
    q = fma(q, f, 1.98412698943924382e-04);
    q = fma(q, f, 1.38888889524247327e-03);
    q = fma(q, f, 8.33333333331670763e-03);
    q = fma(q, f, 4.16666666664875993e-02);
    q = fma(q, f, 1.66666666666666879e-01);
    q = fma(q, f, 5.00000000000001887e-01);
    q = fma(q, f, 1.0);
    q = fma(q, f, 1.0);
    return ldexp(q, (int)fmax(fmin(k, 2100.0), -2100.0));
}
template <> __device__ inline double exp_r<double>(double x) { return exp_fast(x); }
template <> __device__ inline float exp_r<float>(float x) { return __expf(x); }
template <class R> __device__ inline R log_r(R x);
template <> __device__ inline double log_r<double>(double x) { return log(x); }
template <> __device__ inline float log_r<float>(float x) { return __logf(x); }

// LDS access by byte offset from the start of the workgroup's LDS allocation (the
// kernels that use these declare no static LDS, so dynamic LDS starts at offset 0);
// saves the base-address add the compiler emits for the dynamic-LDS symbol.
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) f64x2 lds_f64x2;
__device__ inline double lds_ld(unsigned off) { return *(const lds_f64 *)(uintptr_t)off; }
__device__ inline f64x2 lds_ld2(unsigned off) { return *(const lds_f64x2 *)(uintptr_t)off; }
__device__ inline void lds_st(unsigned off, double v) { *(lds_f64 *)(uintptr_t)off = v; }
__device__ inline void lds_st2(unsigned off, f64x2 v) { *(lds_f64x2 *)(uintptr_t)off = v; }
typedef __attribute__((address_space(3))) float lds_f32;
__device__ inline float lds_ldf(unsigned off) { return *(const lds_f32 *)(uintptr_t)off; }
__device__ inline void lds_stf(unsigned off, float v) { *(lds_f32 *)(uintptr_t)off = v; }
// Gather values of k_jac_seg: FP64, or FP32 in the mixed mode (half the LDS bytes; a
// value's byte offset is then half the FP64 one)
template <bool MIXED> struct GatherT { typedef double type; };
template <> struct GatherT<true> { typedef float type; };

struct PointState {
    double T, lnT, invT, lnp0RT, rho, Wbar, Ctot, p;
    bool valid;
};

// NASA-7 evaluation for one species: cp/R, h/RT, s/R (g/RT = h/RT - s/R).
__device__ inline void nasa7(const double *c16, double T, double lnT, double invT, double &cpR,
                             double &hRT, double &sR) {
    const double *a = (T <= c16[0]) ? c16 + 1 : c16 + 8;
    const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3], a4 = a[4], a5 = a[5], a6 = a[6];
    cpR = a0 + T * (a1 + T * (a2 + T * (a3 + T * a4)));
    hRT = a0 + T * (a1 * 0.5 + T * (a2 * (1.0 / 3.0) + T * (a3 * 0.25 + T * (a4 * 0.2)))) + a5 * invT;
    sR = a0 * lnT + T * (a1 + T * (a2 * 0.5 + T * (a3 * (1.0 / 3.0) + T * (a4 * 0.25)))) + a6;
}

// Loads T, p and the mixture state of point i; lanes = species write the
// per-species LDS arrays.  Returns the point scalars (identical in every lane).
template <bool NEED_H, bool NEED_CP>
__device__ inline PointState load_point(const DevMech &m, int64_t i, int64_t n, const double *T,
                                        const double *p, int64_t ps, const double *Y, int64_t ld,
                                        double *C, double *gRT, double *hRT, double *cpR, bool store = true) {
    const int lane = threadIdx.x & (WAVE - 1);
    PointState s;
    s.valid = i < n;
    const int64_t ii = s.valid ? i : 0;
    s.T = T[ii];
    s.p = p[ii * ps];
    s.lnT = log(s.T);
    s.invT = 1.0 / s.T;
    s.lnp0RT = log(m.p0 / (m.R * s.T));
    double sy = 0.0;
    for (int k = lane; k < m.ns; k += WAVE) sy += Y[(int64_t)k * ld + ii] * m.invW[k];
    sy = wave_sum(sy);
    s.Wbar = 1.0 / sy;
    s.rho = s.p * s.Wbar / (m.R * s.T);
    double ct = 0.0;
    for (int k = lane; k < m.ns; k += WAVE) {
        const double c = s.rho * Y[(int64_t)k * ld + ii] * m.invW[k];
        double cp, h, sr;
        nasa7(m.nasa + 16 * k, s.T, s.lnT, s.invT, cp, h, sr);
        if (store) {
            C[k] = c;
            gRT[k] = h - sr;
            if (NEED_H) hRT[k] = h;
            if (NEED_CP) cpR[k] = cp;
        }
        ct += c;
    }
    s.Ctot = wave_sum(ct);
    return s;
}

// Everything one reaction contributes at one point.
struct RxnEval {
    double q;            // net rate of progress (incl. [M] for three-body)
    double d[SLOTS];     // dq/dC of the slot species (mass-action part)
    double mfac;         // dq/d[M] (three-body and falloff), else 0
    double t;            // dq/dT at fixed concentrations
    double sigma;        // sum_j C_j dq/dC_j over all species (incl. efficiency part)
    double invKc;        // 1 / K_c
};

// Rate constant of one reaction and its partial derivatives: the transcendental part
// of a reaction's evaluation (what the forward pass stores for the VJP to reuse).
struct RateK {
    double M;            // third-body concentration [M] (0 for elementary reactions)
    double kf;           // forward rate constant (falloff-blended), without the [M] factor
    double dkfT;         // dk_f/dT at fixed [M]
    double dkfM;         // dk_f/d[M] at fixed T (falloff only, else 0)
};

// [M] = Ctot + sum_exc (eps - 1) C_k of a third-body or falloff reaction.
__device__ inline double third_body(const DevMech &m, const RxnInts &ri, double Ctot, const double *C) {
    double M = Ctot;
    const int n_exc = ri.v[7] & 255;
    for (int e = 0; e < n_exc; ++e) M += m.eff_m1[ri.v[6] + e] * C[m.eff_sp[ri.v[6] + e]];
    return M;
}

// PLOG: ln k is linear in ln p between the two tabulated pressures that bracket p, and the
// end expressions apply beyond the table (t: n, then n x (ln p_j, ln A_j, b_j, theta_j)).
template <class Rt>
__device__ inline void plog_rate(const double *t, double lnp, Rt lnT, Rt invT, Rt &lnk, Rt &dlnk) {
    const int n = (int)t[0];
    const double *e = t + 1;
    int j = 0;
    while (j + 2 < n && lnp >= e[4 * (j + 1)]) ++j;
    const int j1 = n > 1 ? j + 1 : j;
    Rt w = 0;
    if (n > 1) {
        const double ww = (lnp - e[4 * j]) / (e[4 * j1] - e[4 * j]);
        w = (Rt)(ww < 0.0 ? 0.0 : ww > 1.0 ? 1.0 : ww);
    }
    const Rt l0 = (Rt)e[4 * j + 1] + (Rt)e[4 * j + 2] * lnT - (Rt)e[4 * j + 3] * invT;
    const Rt l1 = (Rt)e[4 * j1 + 1] + (Rt)e[4 * j1 + 2] * lnT - (Rt)e[4 * j1 + 3] * invT;
    const Rt d0 = ((Rt)e[4 * j + 2] + (Rt)e[4 * j + 3] * invT) * invT;
    const Rt d1 = ((Rt)e[4 * j1 + 2] + (Rt)e[4 * j1 + 3] * invT) * invT;
    lnk = ((Rt)1 - w) * l0 + w * l1;
    dlnk = ((Rt)1 - w) * d0 + w * d1;
}

// Chebyshev: log10 k = sum_t c_t T_t(Tr), c_t = sum_q alpha_tq T_q(Pr), with T_n the Chebyshev
// polynomials, Tr = (2/T - 1/Tmin - 1/Tmax)/(1/Tmax - 1/Tmin), Pr likewise in log10 p;
// T_t' = t U_(t-1) for the temperature derivative (t: nT, nP, 1/Tmin, 1/Tmax, log10 Pmin,
// log10 Pmax, alpha[nT][nP]).
template <class Rt>
__device__ inline void cheb_rate(const double *t, double log10p, Rt invT, Rt &lnk, Rt &dlnk) {
    const int nT = (int)t[0], nP = (int)t[1];
    const Rt iTmin = (Rt)t[2], iTmax = (Rt)t[3];
    const Rt Tr = ((Rt)2 * invT - iTmin - iTmax) / (iTmax - iTmin);
    const Rt dTr = (Rt)-2 * invT * invT / (iTmax - iTmin);
    const Rt Pr = (Rt)((2.0 * log10p - t[4] - t[5]) / (t[5] - t[4]));
    const double *al = t + 6;
    Rt tm1 = 0, t0 = 1, um2 = 0, um1 = 0;     // T_{t-1}, T_t; U_{t-2}, U_{t-1}
    Rt lg = 0, dlg = 0;
    for (int it = 0; it < nT; ++it) {
        Rt c = 0, pm1 = 0, p0 = 1;
        for (int iq = 0; iq < nP; ++iq) {
            c += (Rt)al[it * nP + iq] * p0;
            const Rt pn = iq == 0 ? Pr : (Rt)2 * Pr * p0 - pm1;
            pm1 = p0;
            p0 = pn;
        }
        lg += c * t0;
        dlg += c * (Rt)it * um1;                 // T_t' = t U_{t-1}
        const Rt tn = it == 0 ? Tr : (Rt)2 * Tr * t0 - tm1;
        const Rt un = it == 0 ? (Rt)1 : it == 1 ? (Rt)2 * Tr : (Rt)2 * Tr * um1 - um2;
        tm1 = t0;
        t0 = tn;
        um2 = um1;
        um1 = un;
    }
    lnk = lg * (Rt)LN10;
    dlnk = dlg * dTr * (Rt)LN10;
}

// Rate constant (with DERIV, its derivatives).  MIXED: Arrhenius exponentials and falloff
// blending in FP32.  Falloff broadening: Troe (Gilbert-Luther-Troe), Lindemann (F = 1) or
// SRI (F = d (a e^(-b/T) + e^(-T/c))^X T^e, X = 1/(1 + log10^2 P_r)); plain reactions may
// use a PLOG or Chebyshev rate instead of their Arrhenius expression.
template <bool MIXED, bool DERIV, bool VAR>
__device__ inline RateK rate_constant(const DevMech &m, const PointState &ps, const double *C, int kind,
                                      const RxnInts &ri, const RxnVar &var, double lnA, double bb, double th) {
    using Rt = typename std::conditional<MIXED, float, double>::type;
    const int vf = VAR ? var.flags : 0;      // optional rate forms compiled in only with VAR
    RateK k;
    k.M = kind != RXN_ELEMENTARY ? third_body(m, ri, ps.Ctot, C) : 0.0;
    const Rt lnT = (Rt)ps.lnT, invT = (Rt)ps.invT, T = (Rt)ps.T;
    Rt lnkinf = (Rt)lnA + (Rt)bb * lnT - (Rt)th * invT;
    Rt dlnkinf = ((Rt)bb + (Rt)th * invT) * invT;
    if (vf & VAR_PLOG) plog_rate<Rt>(m.vtab + var.rate_off, log(ps.p), lnT, invT, lnkinf, dlnkinf);
    else if (vf & VAR_CHEB) cheb_rate<Rt>(m.vtab + var.rate_off, log10(ps.p), invT, lnkinf, dlnkinf);
    const Rt kinf = exp_r<Rt>(lnkinf);
    Rt kf = kinf, dkf_dT = kinf * dlnkinf, dkf_dM = 0;
    if (kind == RXN_TROE) {
        const double *tp = m.troe + 8 * (ri.v[7] >> 8);
        const Rt lnA0 = (Rt)tp[0], b0 = (Rt)tp[1], th0 = (Rt)tp[2];
        const Rt lnk0 = lnA0 + b0 * lnT - th0 * invT;
        const Rt lnM = log_r<Rt>((Rt)k.M);
        const Rt lnPr = lnk0 - lnkinf + lnM;
        const Rt Pr = exp_r<Rt>(lnPr);
        const Rt lnfloor = MIXED ? (Rt)-85.19 : (Rt)-690.7755278982137;
        const Rt ell = (lnPr > lnfloor ? lnPr : lnfloor) * (Rt)INV_LN10;
        // broadening F, d log10 F / d log10 P_r and d log10 F / dT at fixed P_r
        Rt F = 1, dlogF_dell = 0, dlogF_dT = 0;
        if (vf & VAR_SRI) {
            const Rt a = (Rt)tp[3], b = (Rt)tp[4], c = (Rt)tp[5], d = (Rt)tp[6], e = (Rt)tp[7];
            const Rt X = (Rt)1 / ((Rt)1 + ell * ell);
            const Rt ea = exp_r<Rt>(-b * invT), ec = exp_r<Rt>(-T / c);
            const Rt S = a * ea + ec;
            const Rt lnS = log_r<Rt>(S);
            F = d * exp_r<Rt>(X * lnS + e * lnT);
            if (DERIV) {
                dlogF_dell = (Rt)-2 * ell * X * X * lnS * (Rt)INV_LN10;
                const Rt dS = a * b * invT * invT * ea - ec / c;
                dlogF_dT = (X * dS / S + e * invT) * (Rt)INV_LN10;
            }
        } else if (!(vf & VAR_LINDEMANN)) {
            const Rt alpha = (Rt)tp[3], iT3 = (Rt)tp[4], iT1 = (Rt)tp[5], T2 = (Rt)tp[6];
            const Rt e3 = exp_r<Rt>(-T * iT3), e1 = exp_r<Rt>(-T * iT1), e2 = exp_r<Rt>(-T2 * invT);
            const Rt Fc = ((Rt)1 - alpha) * e3 + alpha * e1 + e2;
            const Rt tiny = MIXED ? (Rt)1e-37 : (Rt)1e-300;
            const Rt lFc = log_r<Rt>(Fc > tiny ? Fc : tiny) * (Rt)INV_LN10;
            const Rt c = (Rt)-0.4 - (Rt)0.67 * lFc;
            const Rt nn = (Rt)0.75 - (Rt)1.27 * lFc;
            const Rt u = ell + c;
            const Rt den = nn - (Rt)0.14 * u;
            const Rt f1 = u / den;
            const Rt g = (Rt)1 / ((Rt)1 + f1 * f1);
            F = exp_r<Rt>(lFc * g * (Rt)LN10);
            if (DERIV) {
                const Rt idd = (Rt)1 / (den * den);
                const Rt df1_dell = nn * idd;
                const Rt df1_dlFc = ((Rt)-0.67 * den - u * ((Rt)-1.27 + (Rt)0.67 * (Rt)0.14)) * idd;
                dlogF_dell = -lFc * (Rt)2 * f1 * df1_dell * g * g;
                const Rt dlogF_dlFc = g - lFc * (Rt)2 * f1 * df1_dlFc * g * g;
                const Rt dFc = -((Rt)1 - alpha) * iT3 * e3 - alpha * iT1 * e1 + T2 * invT * invT * e2;
                dlogF_dT = dlogF_dlFc * dFc / (Fc * (Rt)LN10);
            }
        }
        const Rt Prp = (Rt)1 / ((Rt)1 + (Rt)1 / Pr);     // Pr/(1+Pr), safe for Pr -> 0, inf
        kf = kinf * Prp * F;
        if (DERIV) {
            const Rt dlnk0 = (b0 + th0 * invT) * invT;
            const Rt dlnPr = dlnk0 - dlnkinf;
            const Rt dlnF = dlogF_dell * dlnPr + (Rt)LN10 * dlogF_dT;
            const Rt ip1 = (Rt)1 / ((Rt)1 + Pr);
            dkf_dT = kf * (dlnkinf + dlnPr * ip1 + dlnF);
            const Rt k0 = exp_r<Rt>(lnk0);
            dkf_dM = k0 * F * ip1 * (ip1 + dlogF_dell);
        }
    }
    k.kf = (double)kf;
    k.dkfT = (double)dkf_dT;
    k.dkfM = (double)dkf_dM;
    return k;
}

// C^o and d(C^o)/dC for a reaction order o > 0 (integer orders as plain powers).
__device__ inline double order_pow(double c, double o) {
    return o == 1.0 ? c : o == 2.0 ? c * c : o == 3.0 ? c * c * c : (c > 0.0 ? pow(c, o) : 0.0);
}
__device__ inline double order_dpow(double c, double o) {
    return o == 1.0 ? 1.0 : o == 2.0 ? 2.0 * c : o == 3.0 ? 3.0 * c * c : o * pow(c, o - 1.0);
}

// Rate of progress of a reaction from its rate constant (and, with DERIV, its
// derivatives): equilibrium constant, concentration products, q, dq/dC of every slot,
// dq/dT at fixed C, dq/d[M].  All FP64.  The reverse rate constant is k_f/K_c, an explicit
// reverse Arrhenius expression, or 0 for an irreversible reaction; invKc_in >= 0 supplies
// 1/K_c (a stored value), a negative value forms it from the Gibbs sums of the slots.
// Non-integer forward orders replace the reactant coefficients in the forward product.
template <bool DERIV, bool VAR>
__device__ inline void reaction_rates(const DevMech &m, const RxnVar &var, const PointState &ps, const double *C,
                                      const double *gRT, const double *hRT, int info, const RxnInts &ri,
                                      int dnu_sum, const RateK &k, double invKc_in, RxnEval &o) {
    const int vf = VAR ? var.flags : 0;      // optional forms compiled in only with VAR
    const int kind = info_kind(info);
    const int nre = info_nreac(info), npr = info_nprod(info);
    const bool kc_form = !(vf & (VAR_REVERSE | VAR_IRREV));
    const double *ord = m.vtab + var.ord_off;
    // equilibrium constant: ln K_c = -sum dnu_k g_k/RT + dnu ln(p0/RT)
    double lnKc = (double)dnu_sum * ps.lnp0RT;
    double dlnKc = -(double)dnu_sum;
    double pf = 1.0, pr = 1.0;
    double Cs[SLOTS], Ps[SLOTS], Os[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
        const int kk = used ? ri.v[s] : 0;
        const int nu = used ? info_nu(info, s) : 0;
        const double sgn = s < MAX_SIDE ? -1.0 : 1.0;
        const double c = used ? C[kk] : 1.0;
        Cs[s] = c;
        Os[s] = (s < MAX_SIDE && used && (vf & VAR_ORDERS)) ? ord[s] : (double)nu;
        Ps[s] = (s < MAX_SIDE && (vf & VAR_ORDERS)) ? (used ? order_pow(c, Os[s]) : 1.0) : ipow(c, nu);
        if (used && kc_form) {
            if (invKc_in < 0.0) lnKc -= sgn * nu * gRT[kk];
            if (DERIV) dlnKc += sgn * nu * hRT[kk];
        }
        if (s < MAX_SIDE) pf *= Ps[s]; else pr *= Ps[s];
    }
    // 1/K_c in FP64 in both modes: near equilibrium q = k_f (prod_f - prod_r / K_c) is
    // decided by this factor, so its relative error becomes the error of q
    double invKc = 0.0, krd = 0.0, dkrT = 0.0;
    const double kfd = k.kf;
    if (vf & VAR_REVERSE) {
        const double *rv = m.vtab + var.rev_off;
        krd = exp_fast(rv[0] + rv[1] * ps.lnT - rv[2] * ps.invT);
        if (DERIV) dkrT = krd * (rv[1] + rv[2] * ps.invT) * ps.invT;
    } else if (kc_form) {
        invKc = invKc_in >= 0.0 ? invKc_in : exp_fast(-lnKc);
        krd = kfd * invKc;
        if (DERIV) dkrT = k.dkfT * invKc - krd * dlnKc * ps.invT;
    }
    o.invKc = invKc;
    const double fac = kind == RXN_THREEBODY ? k.M : 1.0;
    o.q = fac * (kfd * pf - krd * pr);
    if (DERIV) {
        o.t = fac * (k.dkfT * pf - dkrT * pr);
        o.mfac = kind == RXN_THREEBODY ? kfd * pf - krd * pr : kind == RXN_TROE ? k.dkfM * (pf - invKc * pr) : 0.0;
        double sig = 0.0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
            const int nu = used ? info_nu(info, s) : 1;
            // d(prod)/dC_s = (order) C_s^(order-1) * product of the other slots of the same side
            double other = 1.0;
            const int lo = s < MAX_SIDE ? 0 : MAX_SIDE;
#pragma unroll
            for (int t = 0; t < MAX_SIDE; ++t)
                if (lo + t != s) other *= Ps[lo + t];
            const double dp = ((s < MAX_SIDE && (vf & VAR_ORDERS)) ? order_dpow(Cs[s], Os[s])
                                                                           : ipow_m1(Cs[s], nu)) * other;
            const double d = used ? (s < MAX_SIDE ? fac * kfd * dp : -fac * krd * dp) : 0.0;
            o.d[s] = d;
            sig += d * Cs[s];
        }
        // efficiency part of sum_j C_j dq/dC_j: mfac * sum_j eps_j C_j = mfac * [M]
        o.sigma = sig + o.mfac * k.M;
    }
}

// Rate of progress of reaction `r` (and, with DERIV, its derivatives).
// MIXED: Arrhenius exponentials and Troe blending in FP32; everything else FP64.
template <bool MIXED, bool DERIV, bool VAR>
__device__ inline void eval_reaction(const DevMech &m, int r, const PointState &ps, const double *C,
                                     const double *gRT, const double *hRT, int info, const RxnInts &ri,
                                     double lnA, double bb, double th, int dnu_sum, RxnEval &o) {
    const RxnVar var = VAR ? m.var[r] : RxnVar{0, 0, 0, 0};
    const RateK k = rate_constant<MIXED, DERIV, VAR>(m, ps, C, info_kind(info), ri, var, lnA, bb, th);
    reaction_rates<DERIV, VAR>(m, var, ps, C, gRT, hRT, info, ri, dnu_sum, k, -1.0, o);
}

// ------------------------------------------------------------------ thermo
__global__ __launch_bounds__(256) void k_thermo(DevMech m, int64_t n, const double *__restrict__ T,
                                                const double *__restrict__ p, int64_t ps,
                                                const double *__restrict__ Y, int64_t ld,
                                                double *__restrict__ cp_k, double *__restrict__ h_k,
                                                double *__restrict__ s_k, double *__restrict__ g_k,
                                                double *__restrict__ cp_mass, double *__restrict__ h_mass,
                                                double *__restrict__ rho, double *__restrict__ Wbar) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double t = T[i], lnT = log(t), invT = 1.0 / t;
        double sy = 0.0;
        for (int k = 0; k < m.ns; ++k) sy += Y[(int64_t)k * ld + i] * m.invW[k];
        const double wbar = 1.0 / sy;
        double cpm = 0.0, hm = 0.0;
        for (int k = 0; k < m.ns; ++k) {
            double cp, h, sr;
            nasa7(m.nasa + 16 * k, t, lnT, invT, cp, h, sr);
            const double cpv = m.R * cp, hv = m.R * t * h, sv = m.R * sr;
            const int64_t o = (int64_t)k * ld + i;
            if (cp_k) cp_k[o] = cpv;
            if (h_k) h_k[o] = hv;
            if (s_k) s_k[o] = sv;
            if (g_k) g_k[o] = hv - t * sv;
            const double yw = Y[o] * m.invW[k];
            cpm += yw * cpv;
            hm += yw * hv;
        }
        if (cp_mass) cp_mass[i] = cpm;
        if (h_mass) h_mass[i] = hm;
        if (rho) rho[i] = p[i * ps] * wbar / (m.R * t);
        if (Wbar) Wbar[i] = wbar;
    }
}

// ------------------------------------------------------------------ wdot
// LDS per wave: PPW points x {C, g/RT, h/RT, w} x nsp doubles, plus cp/R with SRC.
// SRC: the point-wise chemistry source terms instead of w (outputs dYdt, dTdt, QT):
//   dY_k/dt = W_k w_k / rho,  dT/dt = (hrr + dp0/dt) / (rho c_p),
//   Q_T = (1/T) dT/dt + sum_k (Wbar/W_k) dY_k/dt - (dp0/dt)/p
// with c_p = sum_k Y_k cp_k / W_k = (R/rho) sum_k C_k cp_k/R and
// sum_k (Wbar/W_k) dY_k/dt = (Wbar/rho) sum_k w_k.
// STORE: also writes every reaction's (k_f, 1/K_c, dk_f/dT, dk_f/d[M]) to
// work[(i * nr + x) * 4 + 0..3] (x = the reaction's position in the processing order),
// the transcendental part of the rates that the stored-intermediate VJP reuses.
template <bool MIXED, int PPW, bool SRC, bool STORE, bool VAR>
__global__ __launch_bounds__(256, 3) void k_wdot(DevMech m, int64_t n, const double *__restrict__ T,
                                              const double *__restrict__ p, int64_t ps,
                                              const double *__restrict__ Y, int64_t ld,
                                              double *__restrict__ wdot, double *__restrict__ hrr,
                                              double *__restrict__ rmass, double *__restrict__ dTdt,
                                              double *__restrict__ QT, double dp0dt, int nsp,
                                              double *__restrict__ work) {
    constexpr int NA = SRC ? 5 : 4;
    extern __shared__ double lds[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    double *base = lds + (size_t)wave * PPW * NA * nsp;
    const int64_t n_groups = (n + PPW - 1) / PPW;
    for (int64_t g = (int64_t)blockIdx.x * wpb + wave; g < n_groups; g += (int64_t)gridDim.x * wpb) {
        PointState st[PPW];
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            double *C = base + (NA * q + 0) * nsp, *G = C + nsp, *H = G + nsp, *Wd = H + nsp, *CP = Wd + nsp;
            st[q] = load_point<true, SRC>(m, g * PPW + q, n, T, p, ps, Y, ld, C, G, H, SRC ? CP : nullptr);
            for (int k = lane; k < m.ns; k += WAVE) Wd[k] = 0.0;
        }
        wave_lds_sync();
        for (int x = lane; x < m.nr; x += WAVE) {
            const int r = m.rxn_order[x];
            const int info = m.info[r];
            const RxnInts ri = m.ri[r];
            const double lnA = m.lnA[r], bb = m.b[r], th = m.theta[r];
            const int dsum = m.dnu_sum[r];
            const int nre = info_nreac(info), npr = info_nprod(info);
#pragma unroll
            for (int q = 0; q < PPW; ++q) {
                double *C = base + (NA * q + 0) * nsp, *G = C + nsp, *Wd = C + 3 * nsp;
                RxnEval o;
                if constexpr (STORE) {
                    const RxnVar var = VAR ? m.var[r] : RxnVar{0, 0, 0, 0};
                    const RateK k = rate_constant<MIXED, true, VAR>(m, st[q], C, info_kind(info), ri, var, lnA, bb, th);
                    reaction_rates<false, VAR>(m, var, st[q], C, G, nullptr, info, ri, dsum, k, -1.0, o);
                    const int64_t i = g * PPW + q;
                    if (st[q].valid) {
                        f64x2 *w = (f64x2 *)(work + ((size_t)i * m.nr + x) * 4);
                        w[0] = f64x2{k.kf, o.invKc};
                        w[1] = f64x2{k.dkfT, k.dkfM};
                    }
                } else {
                    eval_reaction<MIXED, false, VAR>(m, r, st[q], C, G, nullptr, info, ri, lnA, bb, th, dsum, o);
                }
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
                    if (used) atomicAdd(&Wd[ri.v[s]], (s < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, s) * o.q);
                }
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            if (!st[q].valid) continue;
            const int64_t i = g * PPW + q;
            const double *C = base + (NA * q) * nsp, *H = C + 2 * nsp, *Wd = C + 3 * nsp, *CP = C + 4 * nsp;
            double hs = 0.0, ms = 0.0, cs = 0.0;
            const double irho = SRC ? 1.0 / st[q].rho : 0.0;
            for (int k = lane; k < m.ns; k += WAVE) {
                const double w = Wd[k];
                if (SRC) {
                    if (wdot) wdot[(int64_t)k * ld + i] = m.W[k] * w * irho;
                    cs += C[k] * CP[k];
                    ms += w;
                } else {
                    wdot[(int64_t)k * ld + i] = w;
                    ms += m.W[k] * w;
                }
                hs += H[k] * w;
            }
            hs = wave_sum(hs);
            ms = wave_sum(ms);
            if (SRC) {
                cs = wave_sum(cs);
                if (lane == 0) {
                    const double hr = -m.R * st[q].T * hs;
                    const double cpm = m.R * cs * irho;                       // J/(kg K)
                    const double dt = (hr + dp0dt) * irho / cpm;
                    if (hrr) hrr[i] = hr;
                    if (dTdt) dTdt[i] = dt;
                    if (QT) QT[i] = dt * st[q].invT + st[q].Wbar * irho * ms - dp0dt / st[q].p;
                }
            } else if (lane == 0) {
                if (hrr) hrr[i] = -m.R * st[q].T * hs;
                if (rmass) rmass[i] = ms;
            }
        }
    }
}

// ------------------------------------------------------------------ VJP
// LDS per wave: {C, g/RT, h/RT, cp/R, u, gC, w} x nsp doubles (one point at a time).
// STORED: the rate constants and their derivatives come from the forward pass's work
// array (k_wdot with STORE) instead of being recomputed; the rest (concentration
// products, equilibrium-constant derivative, chain rule) is formed here.
template <bool MIXED, bool STORED, bool VAR>
__global__ __launch_bounds__(256, 3) void k_vjp(DevMech m, int64_t n, const double *__restrict__ T,
                                             const double *__restrict__ p, int64_t ps,
                                             const double *__restrict__ Y, int64_t ld,
                                             const double *__restrict__ u, const double *__restrict__ uh,
                                             double *__restrict__ gT, double *__restrict__ gY, int nsp,
                                             const double *__restrict__ work) {
    extern __shared__ double lds[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    double *C = lds + (size_t)wave * 7 * nsp, *G = C + nsp, *H = G + nsp, *CP = H + nsp, *U = CP + nsp,
           *GC = U + nsp, *Wd = GC + nsp;
    for (int64_t i = (int64_t)blockIdx.x * wpb + wave; i < n; i += (int64_t)gridDim.x * wpb) {
        wave_lds_sync();
        const PointState st = load_point<true, true>(m, i, n, T, p, ps, Y, ld, C, G, H, CP);
        const double uhr = uh ? uh[i] : 0.0;
        for (int k = lane; k < m.ns; k += WAVE) {
            U[k] = u[(int64_t)k * ld + i];
            GC[k] = 0.0;
            Wd[k] = 0.0;
        }
        wave_lds_sync();
        double a_tau = 0.0, a_t = 0.0, a_sig = 0.0;
        const double RT = m.R * st.T;
        for (int x = lane; x < m.nr; x += WAVE) {
            const int r = m.rxn_order[x];
            const int info = m.info[r];
            const RxnInts ri = m.ri[r];
            RxnEval o;
            if constexpr (STORED) {
                const f64x2 *w = (const f64x2 *)(work + ((size_t)i * m.nr + x) * 4);
                const f64x2 a = w[0], b = w[1];
                RateK k;
                k.M = info_kind(info) != RXN_ELEMENTARY ? third_body(m, ri, st.Ctot, C) : 0.0;
                k.kf = a.x;
                k.dkfT = b.x;
                k.dkfM = b.y;
                reaction_rates<true, VAR>(m, VAR ? m.var[r] : RxnVar{0, 0, 0, 0}, st, C, G, H, info, ri, m.dnu_sum[r], k, a.y, o);
            } else {
                eval_reaction<MIXED, true, VAR>(m, r, st, C, G, H, info, ri, m.lnA[r], m.b[r], m.theta[r],
                                                m.dnu_sum[r], o);
            }
            const int nre = info_nreac(info), npr = info_nprod(info);
            // ubar = sum_k dnu_k (u_k - u_hrr h_k)   (the hrr row is -sum_k h_k w_k)
            double ub = 0.0;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
                if (!used) continue;
                const int k = ri.v[s];
                const double dn = (s < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, s);
                ub += dn * (U[k] - uhr * RT * H[k]);
                if (uh) atomicAdd(&Wd[k], dn * o.q);
            }
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
                if (used) atomicAdd(&GC[ri.v[s]], ub * o.d[s]);
            }
            if (o.mfac != 0.0) {
                const int n_exc = ri.v[7] & 255;
                for (int e = 0; e < n_exc; ++e)
                    atomicAdd(&GC[m.eff_sp[ri.v[6] + e]], ub * o.mfac * m.eff_m1[ri.v[6] + e]);
            }
            a_tau += ub * o.mfac;
            a_t += ub * o.t;
            a_sig += ub * o.sigma;
        }
        a_tau = wave_sum(a_tau);
        a_t = wave_sum(a_t);
        a_sig = wave_sum(a_sig);
        wave_lds_sync();
        // R = sum_j (gC_j + tau) C_j ;  gY_j = (rho (gC_j + tau) - Wbar R) / W_j ;  gT = t - R/T - u_hrr sum cp w
        double cpw = 0.0;
        for (int k = lane; k < m.ns; k += WAVE) cpw += CP[k] * Wd[k];
        cpw = wave_sum(cpw) * m.R;
        const double Rsum = a_sig;   // sum_i ubar_i sigma_i already includes the efficiency part
        for (int k = lane; k < m.ns; k += WAVE)
            gY[(int64_t)k * ld + i] = (st.rho * (GC[k] + a_tau) - st.Wbar * Rsum) * m.invW[k];
        if (lane == 0) gT[i] = a_t - Rsum * st.invT - uhr * cpw;
    }
}

// ------------------------------------------------------------------ JVP
// Forward-mode derivative along v = (vT, vY): the tangent of the concentrations is
//   dC_k = rho vY_k / W_k - C_k s,   s = vT / T + Wbar sum_j vY_j / W_j
// (dC_k/dT = -C_k/T and dC_k/dY_j = delta_kj rho/W_k - C_k Wbar/W_j), that of [M] the
// efficiency-weighted sum of dC; every reaction contributes
//   dq = (dq/dT)_C vT + sum_slots (dq/dC_s) dC_s + (dq/d[M]) d[M]
// to dw_k = sum_i dnu_ki dq_i, and d hrr = -sum_k h_k dw_k - vT sum_k cp_k w_k.
// LDS per wave: PPW points x {C, g/RT, h/RT, cp/R, dC, dw, w} x nsp doubles.
template <bool MIXED, int PPW, bool VAR>
__global__ __launch_bounds__(256, 3) void k_jvp(DevMech m, int64_t n, const double *__restrict__ T,
                                             const double *__restrict__ p, int64_t ps,
                                             const double *__restrict__ Y, int64_t ld,
                                             const double *__restrict__ vT, const double *__restrict__ vY,
                                             double *__restrict__ jh, double *__restrict__ jw,
                                             double *__restrict__ wdot, int nsp) {
    constexpr int NA = 7;
    extern __shared__ double lds[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    const bool need_w = jh != nullptr || wdot != nullptr;
    double *base = lds + (size_t)wave * PPW * NA * nsp;
    const int64_t n_groups = (n + PPW - 1) / PPW;
    for (int64_t g = (int64_t)blockIdx.x * wpb + wave; g < n_groups; g += (int64_t)gridDim.x * wpb) {
        PointState st[PPW];
        double dct[PPW], vt[PPW];
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            double *C = base + (NA * q + 0) * nsp, *G = C + nsp, *H = G + nsp, *CP = H + nsp, *DC = CP + nsp,
                   *DW = DC + nsp, *Wd = DW + nsp;
            const int64_t i = g * PPW + q;
            st[q] = load_point<true, true>(m, i, n, T, p, ps, Y, ld, C, G, H, CP);
            const int64_t ii = st[q].valid ? i : 0;
            vt[q] = vT ? vT[ii] : 0.0;
            double sv = 0.0;
            for (int k = lane; k < m.ns; k += WAVE) sv += vY[(int64_t)k * ld + ii] * m.invW[k];
            const double s = vt[q] * st[q].invT + st[q].Wbar * wave_sum(sv);
            double dsum = 0.0;
            for (int k = lane; k < m.ns; k += WAVE) {
                // C[k] was written by this lane (same k), so no synchronisation is needed
                const double dc = st[q].rho * vY[(int64_t)k * ld + ii] * m.invW[k] - C[k] * s;
                DC[k] = dc;
                DW[k] = 0.0;
                Wd[k] = 0.0;
                dsum += dc;
            }
            dct[q] = wave_sum(dsum);
        }
        wave_lds_sync();
        for (int x = lane; x < m.nr; x += WAVE) {
            const int r = m.rxn_order[x];
            const int info = m.info[r];
            const RxnInts ri = m.ri[r];
            const double lnA = m.lnA[r], bb = m.b[r], th = m.theta[r];
            const int dsum = m.dnu_sum[r];
            const int nre = info_nreac(info), npr = info_nprod(info);
            const int n_exc = ri.v[7] & 255;
#pragma unroll
            for (int q = 0; q < PPW; ++q) {
                double *C = base + (NA * q + 0) * nsp, *G = C + nsp, *H = G + nsp, *DC = H + 2 * nsp,
                       *DW = DC + nsp, *Wd = DW + nsp;
                RxnEval o;
                eval_reaction<MIXED, true, VAR>(m, r, st[q], C, G, H, info, ri, lnA, bb, th, dsum, o);
                double dq = o.t * vt[q];
                if (o.mfac != 0.0) {
                    double dM = dct[q];
                    for (int e = 0; e < n_exc; ++e) dM += m.eff_m1[ri.v[6] + e] * DC[m.eff_sp[ri.v[6] + e]];
                    dq += o.mfac * dM;
                }
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
                    if (used) dq += o.d[s] * DC[ri.v[s]];
                }
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    const bool used = s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr;
                    if (!used) continue;
                    const double dn = (s < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, s);
                    atomicAdd(&DW[ri.v[s]], dn * dq);
                    if (need_w) atomicAdd(&Wd[ri.v[s]], dn * o.q);
                }
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            if (!st[q].valid) continue;
            const int64_t i = g * PPW + q;
            const double *H = base + (NA * q + 2) * nsp, *CP = H + nsp, *DW = CP + 2 * nsp, *Wd = DW + nsp;
            double hs = 0.0, cs = 0.0;
            for (int k = lane; k < m.ns; k += WAVE) {
                const double d = DW[k];
                jw[(int64_t)k * ld + i] = d;
                if (wdot) wdot[(int64_t)k * ld + i] = Wd[k];
                hs += H[k] * d;
                cs += CP[k] * Wd[k];
            }
            if (jh) {
                hs = wave_sum(hs);
                cs = wave_sum(cs);
                if (lane == 0) jh[i] = -m.R * st[q].T * hs - vt[q] * m.R * cs;
            }
        }
    }
}

// ------------------------------------------------------------------ Jacobian
// Rows 0..Ns of the Jacobian (row 0 = hrr) are assembled in blocks of `rb` rows:
// S[(row - r0) * sr + j] = sum_i dnu_row,i dq_i/dC_j (mass-action and efficiency
// exceptions; row 0 uses -sum_k h_k dnu_ki), then
//   J[row][T]   = jtc[row] - R[row]/T (- sum_k cp_k w_k for row 0)
//   J[row][Y_j] = (rho (S[row][j] + tau[row]) - Wbar R[row]) / W_j
// with tau = sum_i dnu_i dq_i/d[M] (the efficiency-1 part of every column),
// R = sum_i dnu_i sum_j C_j dq_i/dC_j, jtc = sum_i dnu_i dq_i/dT at fixed C.
// With 53 species the whole matrix is one block; larger mechanisms repeat the
// reaction pass per block instead of exceeding one wavefront's LDS.
// One workgroup of KJ_WAVES wavefronts per point shares the LDS: {C, g/RT, h/RT, cp/R} x nsp
// and {tau, jtc, R, w} x (nsp+1) doubles, plus rb x sr FP64 accumulators (the mixed mode
// stores J in FP32).  The wavefronts split the reactions of every pass; the rows of a
// block accumulate through LDS atomics.
constexpr int KJ_WAVES = 4;
template <bool MIXED, bool VAR>
__global__ __launch_bounds__(KJ_WAVES * 64) void k_jac(DevMech m, int64_t n, const double *__restrict__ T,
                                                       const double *__restrict__ p, int64_t ps,
                                                       const double *__restrict__ Y, int64_t ld,
                                                       void *__restrict__ Jv, double *__restrict__ wdot, int nsp,
                                                       int sr, int rb) {
    using Out = typename std::conditional<MIXED, float, double>::type;
    using Acc = double;     // accumulate in FP64 in both modes; the mixed mode stores FP32
    extern __shared__ double lds[];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    constexpr int NT = KJ_WAVES * WAVE;
    const int ns = m.ns, n1 = ns + 1;
    double *C = lds, *G = C + nsp, *H = G + nsp, *CP = H + nsp;
    double *TAU = CP + nsp, *JTC = TAU + (nsp + 1), *RC = JTC + (nsp + 1), *Wd = RC + (nsp + 1);
    Acc *S = (Acc *)(Wd + (nsp + 1));
    Out *J = (Out *)Jv;
    const float inv_n1 = 1.0f / (float)n1;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        __syncthreads();
        // every wavefront forms the point scalars; wavefront 0 stores the species arrays
        const PointState st = load_point<true, true>(m, i, n, T, p, ps, Y, ld, C, G, H, CP, wave == 0);
        for (int k = tid; k <= ns; k += NT) { TAU[k] = 0.0; JTC[k] = 0.0; RC[k] = 0.0; Wd[k] = 0.0; }
        const double RT = m.R * st.T;
        Out *Jp = J + (size_t)i * n1 * n1;
        for (int r0 = 0; r0 < n1; r0 += rb) {
            const int r1 = r0 + rb < n1 ? r0 + rb : n1;
            const bool first = r0 == 0;
            for (int e = tid; e < (r1 - r0) * sr; e += NT) S[e] = (Acc)0;
            __syncthreads();
            for (int x = tid; x < m.nr; x += NT) {
                const int r = m.rxn_order[x];
                const int info = m.info[r];
                const RxnInts ri = m.ri[r];
                RxnEval o;
                eval_reaction<MIXED, true, VAR>(m, r, st, C, G, H, info, ri, m.lnA[r], m.b[r], m.theta[r],
                                                m.dnu_sum[r], o);
                const int nre = info_nreac(info), npr = info_nprod(info);
                double dh = 0.0;   // reaction enthalpy sum_k dnu_k h_k
#pragma unroll
                for (int a = 0; a < SLOTS; ++a) {
                    const bool used = a < MAX_SIDE ? a < nre : (a - MAX_SIDE) < npr;
                    if (!used) continue;
                    const int k = ri.v[a];
                    const double dn = (a < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, a);
                    dh += dn * RT * H[k];
                    if (first) {
                        atomicAdd(&Wd[1 + k], dn * o.q);
                        atomicAdd(&JTC[1 + k], dn * o.t);
                        atomicAdd(&RC[1 + k], dn * o.sigma);
                        if (o.mfac != 0.0) atomicAdd(&TAU[1 + k], dn * o.mfac);
                    }
                    const int row = 1 + k;
                    if (row >= r0 && row < r1) {
                        Acc *Srow = S + (row - r0) * sr;
#pragma unroll
                        for (int b = 0; b < SLOTS; ++b) {
                            const bool ub = b < MAX_SIDE ? b < nre : (b - MAX_SIDE) < npr;
                            if (ub) atomicAdd(&Srow[ri.v[b]], (Acc)(dn * o.d[b]));
                        }
                    }
                }
                if (first) {   // hrr row: -dh times the reaction's derivatives
#pragma unroll
                    for (int b = 0; b < SLOTS; ++b) {
                        const bool ub = b < MAX_SIDE ? b < nre : (b - MAX_SIDE) < npr;
                        if (ub) atomicAdd(&S[ri.v[b]], (Acc)(-dh * o.d[b]));
                    }
                }
                if (o.mfac != 0.0) {
                    const int n_exc = ri.v[7] & 255;
                    for (int e = 0; e < n_exc; ++e) {
                        const int ke = m.eff_sp[ri.v[6] + e];
                        const double me = o.mfac * m.eff_m1[ri.v[6] + e];
                        if (first) atomicAdd(&S[ke], (Acc)(-dh * me));
                        for (int a = 0; a < SLOTS; ++a) {
                            const bool used = a < MAX_SIDE ? a < nre : (a - MAX_SIDE) < npr;
                            const int row = used ? 1 + ri.v[a] : -1;
                            if (row < r0 || row >= r1) continue;
                            const double dn = (a < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, a);
                            atomicAdd(&S[(row - r0) * sr + ke], (Acc)(dn * me));
                        }
                    }
                }
            }
            __syncthreads();
            if (first && wave == 0) {
                // row 0 scalars: tau_0, jtc_0, R_0 = -sum_k h_k (...)_k; sum cp_k w_k (in Wd[0])
                double t0 = 0.0, j0 = 0.0, q0 = 0.0, cw = 0.0;
                for (int k = lane; k < ns; k += WAVE) {
                    const double hk = RT * H[k];
                    t0 -= hk * TAU[1 + k];
                    j0 -= hk * JTC[1 + k];
                    q0 -= hk * RC[1 + k];
                    cw += m.R * CP[k] * Wd[1 + k];
                }
                t0 = wave_sum(t0); j0 = wave_sum(j0); q0 = wave_sum(q0); cw = wave_sum(cw);
                if (lane == 0) { TAU[0] = t0; JTC[0] = j0; RC[0] = q0; Wd[0] = cw; }
            }
            if (first) __syncthreads();
            // emission of rows r0..r1-1: two consecutive entries per thread, 2 NT per pass
            const int e_lo = r0 * n1, e_hi = r1 * n1;
            // paired stores need a 2-element-aligned address (e0 has the parity of e_lo)
            const bool vec_ok = (((uintptr_t)(Jp + e_lo)) & (2 * sizeof(Out) - 1)) == 0;
            for (int e0 = e_lo + 2 * tid; e0 < e_hi; e0 += 2 * NT) {
                Out v[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int e = e0 + t;
                    double x = 0.0;
                    if (e < e_hi) {
                        // row = e / n1 from a float estimate, corrected to the exact quotient
                        int row = (int)(((float)e + 0.5f) * inv_n1);
                        int c = e - row * n1;
                        if (c < 0) { row -= 1; c += n1; }
                        if (c >= n1) { row += 1; c -= n1; }
                        const double Rr = RC[row];
                        if (c == 0) {
                            x = JTC[row] - Rr * st.invT;
                            if (row == 0) x -= Wd[0];
                        } else {
                            x = (st.rho * ((double)S[(row - r0) * sr + c - 1] + TAU[row]) - st.Wbar * Rr) * m.invW[c - 1];
                        }
                    }
                    v[t] = (Out)x;
                }
                if (vec_ok && e0 + 1 < e_hi) {
                    typedef Out Out2 __attribute__((ext_vector_type(2)));
                    Out2 vv = {v[0], v[1]};
                    *(Out2 *)(Jp + e0) = vv;
                } else {
                    Jp[e0] = v[0];
                    if (e0 + 1 < e_hi) Jp[e0 + 1] = v[1];
                }
            }
            __syncthreads();
        }
        if (wdot)
            for (int k = tid; k < ns; k += NT) wdot[(int64_t)k * ld + i] = Wd[1 + k];
    }
}

// ------------------------------------------------------------------ Jacobian (reaction table)
// For mechanisms the segmented kernel does not take (more than 64 species or 384
// reactions, optional rate forms): one workgroup of WAVES wavefronts per point.  Each
// reaction is evaluated once per point; its derivative data (dq/dC of its slots and
// dq/d[M], FP64, or FP32 in the mixed mode) go to a table in LDS, its reaction enthalpy
// sum_k dnu_k h_k beside them, and the row scalars (tau, J_T at fixed C, R, w) are summed
// at once.  The Jacobian rows are then assembled in blocks of `rb` rows from the table
// (as in k_jac, without re-evaluating the reactions), and emitted.  The row accumulators
// are FP64 LDS atomics, so results are reproducible to rounding (not bitwise).
// LDS: {C, g/RT, h/RT, cp/R} x nsp and {tau, jtc, R, w} x (nsp+1) doubles, the enthalpy of
// every reaction (nrp doubles), the table (7 x nrp values), rb x sr FP64 accumulators, two
// per-row scalars of the block and one partial sum per wavefront.  WAVES is 16 for mechanisms with more reactions than
// 8 wavefronts have lanes, else 8 (two workgroups per compute unit).
template <bool MIXED, bool VAR, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_jac_rt(DevMech m, int64_t n, const double *__restrict__ T,
                                                          const double *__restrict__ p, int64_t ps,
                                                          const double *__restrict__ Y, int64_t ld,
                                                          void *__restrict__ Jv, double *__restrict__ wdot, int nsp,
                                                          int sr, int rb, int nrp) {
    using Out = typename std::conditional<MIXED, float, double>::type;
    using Vt = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    constexpr int NT = WAVES * WAVE;
    const int ns = m.ns, n1 = ns + 1, nr = m.nr;
    double *C = lds, *G = C + nsp, *H = G + nsp, *CP = H + nsp;
    double *TAU = CP + nsp, *JTC = TAU + (nsp + 1), *RC = JTC + (nsp + 1), *Wd = RC + (nsp + 1);
    double *DH = Wd + (nsp + 1);
    Vt *TB = (Vt *)(DH + nrp);                      // [7][nrp]: d[0..5], mfac
    double *S = (double *)(TB + 7 * (size_t)nrp + (MIXED ? (7 * nrp) & 1 : 0));
    Out *J = (Out *)Jv;
    double *AL = S + (size_t)rb * sr, *JT = AL + rb;    // per-row scalars of the current block
    double *RED = JT + rb;                              // per-wavefront partial sums of Y_k / W_k
    // the next point's T, p and Y_k (thread k), requested while the current point is computed
    double nT = 0.0, np = 0.0, ny = 0.0;
    auto prefetch = [&](int64_t j) {
        const int64_t jj = j < n ? j : n - 1;
        nT = T[jj];
        np = p[jj * ps];
        ny = tid < ns ? Y[(int64_t)tid * ld + jj] : 0.0;
    };
    if ((int64_t)blockIdx.x < n) prefetch(blockIdx.x);
    for (int e = tid; e < rb * sr; e += NT) S[e] = 0.0;   // the emission zeroes what it reads
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        __syncthreads();
        // state, one species per thread: sum Y_k / W_k over the workgroup (wavefront sums added
        // in a fixed order), then W, rho, C_k = rho Y_k / W_k, Ctot = rho sum Y_k / W_k and NASA-7
        PointState st;
        st.valid = true;
        st.T = nT;
        st.p = np;
        const double yw = tid < ns ? ny * m.invW[tid] : 0.0;
        prefetch(i + gridDim.x);
        st.lnT = log(st.T);
        st.invT = 1.0 / st.T;
        st.lnp0RT = log(m.p0 / (m.R * st.T));
        const double ws = wave_sum(yw);
        if (lane == 0) RED[wave] = ws;
        for (int k = tid; k <= ns; k += NT) { TAU[k] = 0.0; JTC[k] = 0.0; RC[k] = 0.0; Wd[k] = 0.0; }
        __syncthreads();
        double sy = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sy += RED[w];
        st.Wbar = 1.0 / sy;
        st.rho = st.p * st.Wbar / (m.R * st.T);
        st.Ctot = st.rho * sy;
        if (tid < ns) {
            double cp, h, sr_;
            nasa7(m.nasa + 16 * tid, st.T, st.lnT, st.invT, cp, h, sr_);
            C[tid] = st.rho * yw;
            G[tid] = h - sr_;
            H[tid] = h;
            CP[tid] = cp;
        }
        const double RT = m.R * st.T;
        __syncthreads();
        // every reaction once: table entries and the row scalars
        for (int x = tid; x < nr; x += NT) {
            const int r = m.rxn_order[x];
            const int info = m.info[r];
            const RxnInts ri = m.ri[r];
            RxnEval o;
            eval_reaction<MIXED, true, VAR>(m, r, st, C, G, H, info, ri, m.lnA[r], m.b[r], m.theta[r], m.dnu_sum[r], o);
            const int nre = info_nreac(info), npr = info_nprod(info);
            double dh = 0.0;
#pragma unroll
            for (int a = 0; a < SLOTS; ++a) {
                const bool used = a < MAX_SIDE ? a < nre : (a - MAX_SIDE) < npr;
                TB[a * nrp + x] = (Vt)(used ? o.d[a] : 0.0);
                if (!used) continue;
                const int k = ri.v[a];
                const double dn = (a < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, a);
                dh += dn * RT * H[k];
                atomicAdd(&Wd[1 + k], dn * o.q);
                atomicAdd(&JTC[1 + k], dn * o.t);
                atomicAdd(&RC[1 + k], dn * o.sigma);
                if (o.mfac != 0.0) atomicAdd(&TAU[1 + k], dn * o.mfac);
            }
            TB[6 * nrp + x] = (Vt)o.mfac;
            DH[x] = dh;
        }
        __syncthreads();
        if (wave == 0) {
            // row 0 scalars: tau_0, jtc_0, R_0 = -sum_k h_k (...)_k; sum cp_k w_k (in Wd[0])
            double t0 = 0.0, j0 = 0.0, q0 = 0.0, cw = 0.0;
            for (int k = lane; k < ns; k += WAVE) {
                const double hk = RT * H[k];
                t0 -= hk * TAU[1 + k];
                j0 -= hk * JTC[1 + k];
                q0 -= hk * RC[1 + k];
                cw += m.R * CP[k] * Wd[1 + k];
            }
            t0 = wave_sum(t0); j0 = wave_sum(j0); q0 = wave_sum(q0); cw = wave_sum(cw);
            if (lane == 0) { TAU[0] = t0; JTC[0] = j0; RC[0] = q0; Wd[0] = cw; }
        }
        Out *Jp = J + (size_t)i * n1 * n1;
        for (int r0 = 0; r0 < n1; r0 += rb) {
            const int r1 = r0 + rb < n1 ? r0 + rb : n1;
            const bool first = r0 == 0;
            for (int x = tid; x < nr; x += NT) {
                const int r = m.rxn_order[x];
                const int info = m.info[r];
                const RxnInts ri = m.ri[r];
                const int nre = info_nreac(info), npr = info_nprod(info);
                double d[SLOTS];
#pragma unroll
                for (int b = 0; b < SLOTS; ++b) d[b] = (double)TB[b * nrp + x];
                const double mf = (double)TB[6 * nrp + x], dh = DH[x];
                bool any = first;
#pragma unroll
                for (int a = 0; a < SLOTS; ++a) {
                    const bool used = a < MAX_SIDE ? a < nre : (a - MAX_SIDE) < npr;
                    const int row = used ? 1 + ri.v[a] : -1;
                    any |= row >= r0 && row < r1;
                }
                if (!any) continue;
#pragma unroll
                for (int a = 0; a < SLOTS; ++a) {
                    const bool used = a < MAX_SIDE ? a < nre : (a - MAX_SIDE) < npr;
                    if (!used) continue;
                    const int row = 1 + ri.v[a];
                    if (row < r0 || row >= r1) continue;
                    const double dn = (a < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, a);
                    double *Srow = S + (size_t)(row - r0) * sr;
#pragma unroll
                    for (int b = 0; b < SLOTS; ++b) {
                        const bool ub = b < MAX_SIDE ? b < nre : (b - MAX_SIDE) < npr;
                        if (ub) atomicAdd(&Srow[ri.v[b]], dn * d[b]);
                    }
                }
                if (first) {   // hrr row: -dh times the reaction's derivatives
#pragma unroll
                    for (int b = 0; b < SLOTS; ++b) {
                        const bool ub = b < MAX_SIDE ? b < nre : (b - MAX_SIDE) < npr;
                        if (ub) atomicAdd(&S[ri.v[b]], -dh * d[b]);
                    }
                }
                if (mf != 0.0) {
                    const int n_exc = ri.v[7] & 255;
                    for (int e = 0; e < n_exc; ++e) {
                        const int ke = m.eff_sp[ri.v[6] + e];
                        const double me = mf * m.eff_m1[ri.v[6] + e];
                        if (first) atomicAdd(&S[ke], -dh * me);
                        for (int a = 0; a < SLOTS; ++a) {
                            const bool used = a < MAX_SIDE ? a < nre : (a - MAX_SIDE) < npr;
                            const int row = used ? 1 + ri.v[a] : -1;
                            if (row < r0 || row >= r1) continue;
                            const double dn = (a < MAX_SIDE ? -1.0 : 1.0) * info_nu(info, a);
                            atomicAdd(&S[(size_t)(row - r0) * sr + ke], dn * me);
                        }
                    }
                }
            }
            __syncthreads();
            // emission of rows r0..r1-1: thread = (row phase, column), rows strided by the phase
            // count; per-row scalars formed once: AL[row] = rho tau - Wbar R, JT[row] = J_T of the row
            for (int row = r0 + tid; row < r1; row += NT) {
                const double Rr = RC[row];
                AL[row - r0] = st.rho * TAU[row] - st.Wbar * Rr;
                JT[row - r0] = JTC[row] - Rr * st.invT - (row == 0 ? Wd[0] : 0.0);
            }
            __syncthreads();
            {
                const int nph = NT / n1;                 // row phases (n1 <= NT)
                const int ph = tid / n1, c = tid - ph * n1;
                if (ph < nph) {
                    const double iw = c > 0 ? m.invW[c - 1] : 0.0;
                    const double rho = st.rho;
                    // rows in batches whose LDS reads are issued together (a row past the block's
                    // end reads its last row and stores nothing); each accumulator is read once,
                    // by its owner, which zeroes it for the next block
                    const int nq = (r1 - r0 + nph - 1) / nph;
                    constexpr int EB = 4;
                    for (int q0 = 0; q0 < nq; q0 += EB) {
                        int rr[EB];
                        double sv[EB], al[EB], jt[EB];
#pragma unroll
                        for (int b = 0; b < EB; ++b) {
                            const int row = r0 + ph + (q0 + b) * nph;
                            rr[b] = (row < r1 ? row : r1 - 1) - r0;
                            sv[b] = S[(size_t)rr[b] * sr + (c > 0 ? c - 1 : 0)];
                            al[b] = AL[rr[b]];
                            jt[b] = JT[rr[b]];
                        }
#pragma unroll
                        for (int b = 0; b < EB; ++b) {
                            const double v = c == 0 ? jt[b] : (rho * sv[b] + al[b]) * iw;
                            if (r0 + ph + (q0 + b) * nph < r1) {
                                Jp[(size_t)(r0 + rr[b]) * n1 + c] = (Out)v;
                                if (c > 0) S[(size_t)rr[b] * sr + c - 1] = 0.0;
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (wdot)
            for (int k = tid; k < ns; k += NT) wdot[(int64_t)k * ld + i] = Wd[1 + k];
    }
}

// ------------------------------------------------------------------ Jacobian (segmented gather)
// One workgroup of JS_THREADS threads (6 wavefronts) per point, persistent over an
// XCD-aware strided sequence of points; thread t owns one reaction for the workgroup's lifetime
// (its constants stay in registers).  The mechanism's Troe parameters and efficiency
// exceptions are staged in LDS once.  Per point, separated by workgroup barriers:
//   B  threads = reactions: rate of progress and all its derivatives into the per-point
//      reaction data (d values and quads, layout in build_jac_plan); each thread then
//      loads its wavefront's gather records into registers;
//   C  gather rounds (build_jac_plan) into the FP64 accumulator matrix
//      A[k][0..3] = (dw_k/dT at fixed C, w_k, tau_k, R_k), A[k][5 + j] = the mass-action
//      and efficiency-exception part of dw_k/dC_j; entries that no reaction reaches stay
//      zero from the workgroup's start;
//   D  hrr row partial sums -RT sum_k h_k A[k][c] (JS_PWAVES wavefronts split the
//      species), the row scalars alpha_k = rho tau_k - Wbar R_k and J_T of each row,
//      sum_k cp_k w_k and w_k to global memory (wavefront 3); meanwhile wavefronts 4 and
//      5 form the NEXT point's state (NASA-7 polynomials; C_k, Wbar, rho from the
//      prefetched T, p, Y) in the other half of the double-buffered state arrays;
//   E  emission, each thread a fixed pair of columns over a strided set of rows:
//        J[row][T]   = A[row][0] - R_row/T (- sum_k cp_k w_k on row 0)
//        J[row][Y_j] = (rho A[row][5 + j] + alpha_row) / W_j
// No LDS atomics: every LDS word has one writer per phase, and every sum is taken in
// an order fixed by the plan, so results are bitwise reproducible.
// VAR: the reaction may carry an optional form (RxnVar var; tables in vtab, SRI constants in
// TP): a PLOG or Chebyshev rate, Lindemann or SRI broadening, an explicit reverse rate or
// none (irreversible).  Non-integer orders are not taken (the plan refuses them).
template <bool MIXED, bool VAR>
__device__ inline void jac_seg_reaction(int r, unsigned sp03, unsigned sp45, int dpos, int xpos, int n_exc,
                                        int exc0, int troe, int dnu, double lnA, double bb, double th,
                                        const double *SP, const double *SC, const double *TQ, int nt,
                                        const double *MQ, const double *EXm, typename GatherT<MIXED>::type *RDd,
                                        int qb, const RxnVar &var, const double *vtab, const double *TP) {
    using Rt = typename std::conditional<MIXED, float, double>::type;
    const int vf = VAR ? var.flags : 0;
    const int nfm = (sp45 >> 16) & 7, nrm = (sp45 >> 19) & 7, kind = (sp45 >> 22) & 3;
    const double lnT = SC[5], invT = SC[6], lnp0RT = SC[7];
    // third-body concentration [M] and its logarithm (formed with the state)
    double M = 0.0, lnMd = 0.0;
    if (kind != RXN_ELEMENTARY) {
        const double2 mq = *(const double2 *)(MQ + 2 * (troe >> 16));
        M = mq.x;
        lnMd = mq.y;
    }
    troe &= 0xffff;
    // forward rate constant (Arrhenius; Lindemann-Troe blending for falloff reactions,
    // whose temperature-only terms come from jac_seg_troe_t)
    const Rt rlnT = (Rt)lnT, rinvT = (Rt)invT;
    Rt lnkinf = (Rt)lnA + (Rt)bb * rlnT - (Rt)th * rinvT;
    Rt dlnkinf = ((Rt)bb + (Rt)th * rinvT) * rinvT;
    if constexpr (VAR) {
        if (vf & VAR_PLOG) plog_rate<Rt>(vtab + var.rate_off, log(SC[1]), rlnT, rinvT, lnkinf, dlnkinf);
        else if (vf & VAR_CHEB) cheb_rate<Rt>(vtab + var.rate_off, log10(SC[1]), rinvT, lnkinf, dlnkinf);
    }
    const Rt kinf = exp_r<Rt>(lnkinf);
    Rt kf = kinf, dkf_dT = kinf * dlnkinf, dkf_dM = 0;
    if (VAR && kind == RXN_TROE && (vf & (VAR_LINDEMANN | VAR_SRI))) {
        // Lindemann (F = 1) or SRI broadening, with the temperature terms of k0/kinf from TQ
        const double *tq = TQ + troe;
        const Rt lnkr = (Rt)tq[2 * nt], dlnPr = (Rt)tq[3 * nt], k0 = (Rt)tq[4 * nt];
        const Rt lnPr = lnkr + (Rt)lnMd;
        const Rt Pr = exp_r<Rt>(lnPr);
        Rt F = 1, dlogF_dell = 0, dlnF = 0;
        if (vf & VAR_SRI) {
            const double *tp = TP + troe;   // a, b, c, d, e at constants 3..7
            const Rt a = (Rt)tp[3 * nt], b = (Rt)tp[4 * nt], c = (Rt)tp[5 * nt], d = (Rt)tp[6 * nt], e = (Rt)tp[7 * nt];
            const Rt T = (Rt)SC[0];
            const Rt lnfloor = MIXED ? (Rt)-85.19 : (Rt)-690.7755278982137;
            const Rt ell = (lnPr > lnfloor ? lnPr : lnfloor) * (Rt)INV_LN10;
            const Rt X = (Rt)1 / ((Rt)1 + ell * ell);
            const Rt ea = exp_r<Rt>(-b * rinvT), ec = exp_r<Rt>(-T / c);
            const Rt S = a * ea + ec;
            const Rt lnS = log_r<Rt>(S);
            F = d * exp_r<Rt>(X * lnS + e * rlnT);
            dlogF_dell = (Rt)-2 * ell * X * X * lnS * (Rt)INV_LN10;
            const Rt dS = a * b * rinvT * rinvT * ea - ec / c;
            dlnF = dlogF_dell * dlnPr + X * dS / S + e * rinvT;   // LN10 d log10 F / dT at fixed P_r
        }
        const Rt Prp = (Rt)1 / ((Rt)1 + (Rt)1 / Pr);
        kf = kinf * Prp * F;
        const Rt ip1 = (Rt)1 / ((Rt)1 + Pr);
        dkf_dT = kf * (dlnkinf + dlnPr * ip1 + dlnF);
        dkf_dM = k0 * F * ip1 * (ip1 + dlogF_dell);
    } else if (kind == RXN_TROE) {
        const double *tq = TQ + troe;   // [term][falloff reaction]
        const Rt lFc = (Rt)tq[0], dlFc = (Rt)tq[nt], lnkr = (Rt)tq[2 * nt], dlnPr = (Rt)tq[3 * nt], k0 = (Rt)tq[4 * nt];
        // P_r capped where P_r / (1 + P_r) = 1 to the working precision (P_r stays finite):
        // in FP64 (k0/kinf) [M] with k0/kinf formed with the point's state (an FP64
        // exponential fewer on the falloff wavefront), in FP32 e^(ln P_r)
        const Rt lnceil = MIXED ? (Rt)80 : (Rt)700;
        const Rt lnPr0 = lnkr + (Rt)lnMd;
        const Rt lnPr = lnPr0 < lnceil ? lnPr0 : lnceil;
        Rt Pr;
        if constexpr (MIXED) {
            Pr = exp_r<Rt>(lnPr);
        } else {
            const Rt Pr0 = (Rt)tq[5 * nt] * (Rt)M;
            Pr = Pr0 < (Rt)1.0e304 ? Pr0 : (Rt)1.0e304;   // about e^700
        }
        const Rt cc = (Rt)-0.4 - (Rt)0.67 * lFc;
        const Rt nn = (Rt)0.75 - (Rt)1.27 * lFc;
        const Rt lnfloor = MIXED ? (Rt)-85.19 : (Rt)-690.7755278982137;
        const Rt ell = (lnPr > lnfloor ? lnPr : lnfloor) * (Rt)INV_LN10;
        const Rt u = ell + cc;
        const Rt den = nn - (Rt)0.14 * u;
        // one reciprocal for 1/den, f1 = u/den and 1/(1 + f1^2) = den^2/(den^2 + u^2)
        const Rt d2 = den * den, s2 = d2 + u * u;
        const Rt rr = (Rt)1 / (den * s2);
        const Rt iden = s2 * rr;
        const Rt f1 = u * iden;
        const Rt gg = d2 * den * rr;
        const Rt F = exp_r<Rt>(lFc * gg * (Rt)LN10);
        const Rt ip1 = (Rt)1 / ((Rt)1 + Pr);
        const Rt Prp = Pr * ip1;
        kf = kinf * Prp * F;
        const Rt idd = iden * iden;
        const Rt df1_dell = nn * idd;
        const Rt df1_dlFc = ((Rt)-0.67 * den - u * ((Rt)-1.27 + (Rt)0.67 * (Rt)0.14)) * idd;
        const Rt dlogF_dell = -lFc * (Rt)2 * f1 * df1_dell * gg * gg;
        const Rt dlogF_dlFc = gg - lFc * (Rt)2 * f1 * df1_dlFc * gg * gg;
        const Rt dlnF = dlogF_dell * dlnPr + (Rt)LN10 * dlogF_dlFc * dlFc;
        dkf_dT = kf * (dlnkinf + dlnPr * ip1 + dlnF);
        dkf_dM = k0 * F * ip1 * (ip1 + dlogF_dell);
    }
    __builtin_amdgcn_sched_barrier(0);   // the slot loads below start after the rate constant
    double c[SLOTS], g[SLOTS], h[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const unsigned k = s < 4 ? (sp03 >> (8 * s)) & 255u : (sp45 >> (8 * (s - 4))) & 255u;
        const double2 cg = *(const double2 *)(SP + 4 * k);
        c[s] = cg.x;
        g[s] = cg.y;
        h[s] = SP[4 * k + 2];
    }
    // equilibrium constant and rates of progress (FP64)
    const double lnKc = (double)dnu * lnp0RT - ((g[3] + g[4] + g[5]) - (g[0] + g[1] + g[2]));
    const double dlnKc = ((h[3] + h[4] + h[5]) - (h[0] + h[1] + h[2]) - (double)dnu) * invT;
    const double kfd = (double)kf;
    const double fac = kind == RXN_THREEBODY ? M : 1.0;
    const double pf = c[0] * c[1] * c[2], pr = c[3] * c[4] * c[5];
    double fk, fr, t, mf;
    if (VAR && (vf & (VAR_REVERSE | VAR_IRREV))) {
        // explicit reverse Arrhenius expression (independent of [M]) or no reverse reaction
        double kr = 0.0, dkrT = 0.0;
        if (vf & VAR_REVERSE) {
            const double *rv = vtab + var.rev_off;
            kr = exp_fast(rv[0] + rv[1] * lnT - rv[2] * invT);
            dkrT = kr * (rv[1] + rv[2] * invT) * invT;
        }
        fk = fac * kfd;
        fr = fac * kr;
        t = fac * ((double)dkf_dT * pf - dkrT * pr);
        mf = kind == RXN_THREEBODY ? kfd * pf - kr * pr : kind == RXN_TROE ? (double)dkf_dM * pf : 0.0;
    } else {
        const double invKc = exp_fast(-lnKc);   // FP64 in both modes (it decides q near equilibrium)
        fk = fac * kfd;
        fr = fk * invKc;
        const double bracket = pf - invKc * pr;
        t = fac * (double)dkf_dT * bracket + fr * pr * dlnKc;
        mf = kind == RXN_THREEBODY ? kfd * bracket : kind == RXN_TROE ? (double)dkf_dM * bracket : 0.0;
    }
    const double qf = fk * pf, qr = fr * pr;
    const double sig = (double)nfm * qf - (double)nrm * qr + mf * M;
    if constexpr (MIXED) {   // 16-byte aligned (qb a multiple of 4)
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        *(f32x4 *)(RDd + qb + 4 * r) = f32x4{(float)t, (float)(qf - qr), (float)mf, (float)sig};
    } else {
        double2 *qd = (double2 *)(RDd + qb + 4 * r);
        qd[0] = double2{t, qf - qr};
        qd[1] = double2{mf, sig};
    }
    // dq/dC of each molecule slot: the product of the other slots of its side
    const double dv[SLOTS] = {fk * c[1] * c[2], fk * c[0] * c[2], fk * c[0] * c[1],
                              -fr * c[4] * c[5], -fr * c[3] * c[5], -fr * c[3] * c[4]};
    typename GatherT<MIXED>::type *pos = RDd + 1 + dpos;
#pragma unroll
    for (int s = 0; s < MAX_SIDE; ++s)
        if (s < nfm) pos[s] = dv[s];
#pragma unroll
    for (int s = 0; s < MAX_SIDE; ++s)
        if (s < nrm) pos[nfm + s] = dv[MAX_SIDE + s];
    for (int e = 0; e < n_exc; ++e) RDd[1 + xpos + e] = mf * EXm[exc0 + e];
}

// Temperature-only terms of the falloff reactions at temperature Tt (lane j = falloff
// reaction j), in two halves that run on different wavefronts:
//   jac_seg_troe_fc: log10 Fcent and its T-derivative (TQ[0], TQ[1]);
//   jac_seg_troe_k:  ln(k0/kinf), its T-derivative, k0 and, in FP64, k0/kinf (TQ[2..5]).
template <bool MIXED>
__device__ inline void jac_seg_troe_fc(int lane, int n_troe, double Tt, const double *TP, double *TQ) {
    using Rt = typename std::conditional<MIXED, float, double>::type;
    for (int j = lane; j < n_troe; j += WAVE) {
        const double *tp = TP + j;      // [constant][falloff reaction]: lanes read adjacent words
        const Rt T = (Rt)Tt, invT = (Rt)1 / T;
        const Rt alpha = (Rt)tp[3 * n_troe], iT3 = (Rt)tp[4 * n_troe], iT1 = (Rt)tp[5 * n_troe], T2 = (Rt)tp[6 * n_troe];
        const Rt e3 = exp_r<Rt>(-T * iT3), e1 = exp_r<Rt>(-T * iT1), e2 = exp_r<Rt>(-T2 * invT);
        const Rt Fc = ((Rt)1 - alpha) * e3 + alpha * e1 + e2;
        const Rt tiny = MIXED ? (Rt)1e-37 : (Rt)1e-300;
        const Rt dFc = -((Rt)1 - alpha) * iT3 * e3 - alpha * iT1 * e1 + T2 * invT * invT * e2;
        double *tq = TQ + j;
        tq[0] = (double)(log_r<Rt>(Fc > tiny ? Fc : tiny) * (Rt)INV_LN10);
        tq[n_troe] = (double)(dFc / (Fc * (Rt)LN10));
    }
}

template <bool MIXED>
__device__ inline void jac_seg_troe_k(int lane, int n_troe, double lnT_, double invT_, const double *TP, double *TQ) {
    using Rt = typename std::conditional<MIXED, float, double>::type;
    for (int j = lane; j < n_troe; j += WAVE) {
        const double *tp = TP + j;
        const Rt lnT = (Rt)lnT_, invT = (Rt)invT_;
        const Rt lnA0 = (Rt)tp[0], b0 = (Rt)tp[n_troe], th0 = (Rt)tp[2 * n_troe];
        const Rt lnA = (Rt)tp[8 * n_troe], bb = (Rt)tp[9 * n_troe], th = (Rt)tp[10 * n_troe];
        const Rt lnk0 = lnA0 + b0 * lnT - th0 * invT;
        const Rt lnkinf = lnA + bb * lnT - th * invT;
        double *tq = TQ + j;
        tq[2 * n_troe] = (double)(lnk0 - lnkinf);
        tq[3 * n_troe] = (double)((b0 + th0 * invT) * invT - (bb + th * invT) * invT);
        tq[4 * n_troe] = (double)exp_r<Rt>(lnk0);
        if constexpr (!MIXED) tq[5 * n_troe] = exp_r<Rt>(lnk0 - lnkinf);
    }
}

// State phase of k_jac_seg for one point: wavefront `wy` (lane = species) forms C_k,
// Wbar, rho and Ctot from the prefetched Y, p, T; wavefront `wy - 1` evaluates the
// NASA-7 polynomials (coefficients staged in LDS) and the T-functions.  Writes
// SP[k][C, g/RT, h/RT, cp/R] and SC.
template <bool MIXED>
__device__ inline void jac_seg_state(int ns, double R, double lnp0R, int wave, int wy, int lane, double Tt,
                                     double pp, double yk, const double *NS, const double *IW, const int *MX,
                                     int n_m, const double *EXm, const int *EXs, int n_troe, const double *TP,
                                     double *SP, double *SC, double *MQ, double *TQ) {
    if (wave == wy) {
        const bool has = lane < ns;
        // static tables first (their LDS latency then overlaps the mixture sums): 1/W of this
        // lane's species and the efficiency exceptions of [M] slot `lane`, up to four of them
        // (the unused ones point at the unit dummy species with a zero coefficient)
        const double iw = has ? IW[lane] : 0.0;
        int2 mx0 = make_int2(0, 0);
        if (lane < n_m) mx0 = *(const int2 *)(MX + 2 * lane);
        int ek[4];
        double em[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool on = e < mx0.y;
            ek[e] = on ? EXs[mx0.x + e] : ns;
            em[e] = on ? EXm[mx0.x + e] : 0.0;
        }
        const double yw = has ? yk * iw : 0.0;
        const double wbar = 1.0 / wave_sum(yw);
        const double rho = pp * wbar / (R * Tt);
        const double cv = rho * yw;
        if (has) SP[4 * lane] = cv;
        const double ct = wave_sum(cv);
        if (lane == 0) {
            SC[1] = pp;
            SC[2] = rho;
            SC[3] = wbar;
            SC[4] = ct;
        }
        // [M] = Ctot + sum_exc (eps - 1) C_k of every third-body / falloff reaction, and
        // ln [M] of the falloff ones (slots 0 .. n_troe - 1)
        wave_lds_sync();
        for (int j = lane; j < n_m; j += WAVE) {
            double M = ct;
            if (j == lane && mx0.y <= 4) {
                M += em[0] * SP[4 * ek[0]] + em[1] * SP[4 * ek[1]] + em[2] * SP[4 * ek[2]] + em[3] * SP[4 * ek[3]];
                double lnM = 0.0;
                if (j < n_troe) lnM = MIXED ? (double)__logf((float)M) : log(M);
                *(double2 *)(MQ + 2 * j) = double2{M, lnM};
                continue;
            }
            const int2 mx = *(const int2 *)(MX + 2 * j);
            int e = 0;
            for (; e + 4 <= mx.y; e += 4) {   // the exceptions' loads issued together
                const int k0 = EXs[mx.x + e], k1 = EXs[mx.x + e + 1], k2 = EXs[mx.x + e + 2], k3 = EXs[mx.x + e + 3];
                const double c0 = SP[4 * k0], c1 = SP[4 * k1], c2 = SP[4 * k2], c3 = SP[4 * k3];
                M += EXm[mx.x + e] * c0 + EXm[mx.x + e + 1] * c1 + EXm[mx.x + e + 2] * c2 + EXm[mx.x + e + 3] * c3;
            }
            for (; e < mx.y; ++e) M += EXm[mx.x + e] * SP[4 * EXs[mx.x + e]];
            double lnM = 0.0;
            if (j < n_troe) lnM = MIXED ? (double)__logf((float)M) : log(M);
            *(double2 *)(MQ + 2 * j) = double2{M, lnM};
        }
    } else if (wave == wy - 1) {
        // both ranges' coefficients are requested at once, then one is selected
        double c15[15];
        if (lane < ns) {
#pragma unroll
            for (int q = 0; q < 15; ++q) c15[q] = NS[q * ns + lane];   // coefficient-major: no bank conflicts
        }
        const double lnT = log(Tt), invT = 1.0 / Tt;
        if (lane < ns) {
            const bool low = Tt <= c15[0];   // the temperature range's 7 coefficients
            double b[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) b[q] = low ? c15[1 + q] : c15[8 + q];
            const double cp = b[0] + Tt * (b[1] + Tt * (b[2] + Tt * (b[3] + Tt * b[4])));
            const double hh = b[0] + Tt * (b[1] * 0.5 + Tt * (b[2] * (1.0 / 3.0) + Tt * (b[3] * 0.25 + Tt * (b[4] * 0.2)))) +
                              b[5] * invT;
            const double sr_ = b[0] * lnT + Tt * (b[1] + Tt * (b[2] * 0.5 + Tt * (b[3] * (1.0 / 3.0) + Tt * (b[4] * 0.25)))) + b[6];
            SP[4 * lane + 1] = hh - sr_;
            SP[4 * lane + 2] = hh;
            SP[4 * lane + 3] = cp;
        }
        if (lane == 0) {
            SC[0] = Tt;
            SC[5] = lnT;
            SC[6] = invT;
            SC[7] = lnp0R - lnT;
        }
        jac_seg_troe_k<MIXED>(lane, n_troe, lnT, invT, TP, TQ);
    }
}

template <bool MIXED, int DMAX, bool VAR>
__global__ __launch_bounds__(JS_THREADS, 3) void k_jac_seg(DevMech m, int64_t n, const double *__restrict__ T,
                                                          const double *__restrict__ p, int64_t ps,
                                                          const double *__restrict__ Y, int64_t ld,
                                                          void *__restrict__ Jv, double *__restrict__ wdot) {
    using Out = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ __align__(16) unsigned char lds_b[];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int ns = m.ns, n1 = ns + 1, sr = m.jp_sr, n_troe = m.n_troe;
    constexpr int WY = JS_WAVES - 1;        // wavefront that forms the mixture state
    constexpr int WT = JS_PWAVES;           // wavefront that forms the falloff temperature terms
    using Acc = typename GatherT<MIXED>::type;
    constexpr unsigned VB = sizeof(Acc);                // bytes per gather value
    Acc *RDd = (Acc *)lds_b;
    Acc *A = (Acc *)(lds_b + m.jp_off_a / (8 / VB));  // the accumulators' index space
    double *SP0 = (double *)(lds_b + m.jp_off_sp);
    double *ROW = (double *)(lds_b + m.jp_off_row);
    double *P = (double *)(lds_b + m.jp_off_p);
    double *SC0 = (double *)(lds_b + m.jp_off_sc);
    double *TP = (double *)(lds_b + m.jp_off_tp);
    double *TQ0 = (double *)(lds_b + m.jp_off_tq);
    double *NS = (double *)(lds_b + m.jp_off_ns);
    double *IW = (double *)(lds_b + m.jp_off_iw);
    double *EXm = (double *)(lds_b + m.jp_off_ex);
    int *EXs = (int *)(EXm + m.n_exc);
    int *MX = (int *)(lds_b + m.jp_off_mx);
    double *MQ0 = (double *)(lds_b + m.jp_off_mq);
    const int n_m = m.jp_nm;
    Out *J = (Out *)Jv;
    // ---- workgroup set-up: zero accumulators and the no-op entries, the unit dummy
    // species in both state buffers, the Troe and efficiency tables
    for (int e = tid; e < ns * sr + 4; e += JS_THREADS) A[e] = 0.0;
    if (tid == 0) RDd[0] = 0.0;
    if (tid < 4) {
        SP0[4 * ns + tid] = tid == 0 ? 1.0 : 0.0;
        SP0[4 * (ns + 1) + 4 * ns + tid] = tid == 0 ? 1.0 : 0.0;
    }
    for (int e = tid; e < 8 * n_troe; e += JS_THREADS) TP[(e % 8) * n_troe + e / 8] = m.troe[e];   // [q][j]
    for (int e = tid; e < m.n_exc; e += JS_THREADS) {
        EXm[e] = m.eff_m1[e];
        EXs[e] = m.eff_sp[e];
    }
    for (int e = tid; e < 16 * ns; e += JS_THREADS) NS[(e & 15) * ns + (e >> 4)] = m.nasa[e];   // [q][k]
    for (int e = tid; e < ns; e += JS_THREADS) IW[e] = m.invW[e];
    for (int e = tid; e < 2 * n_m; e += JS_THREADS) MX[e] = m.jp_mrx[e];
    const double lnp0R = log(m.p0 / m.R);
    // this thread's reaction
    const int4 ta = ((const int4 *)m.jp_thr)[2 * tid], tb = ((const int4 *)m.jp_thr)[2 * tid + 1];
    const int r = ta.x;
    const unsigned sp03 = (unsigned)ta.y, sp45 = (unsigned)ta.z;
    const int dpos = ta.w, xpos = tb.x & 0xffff, n_exc = (tb.x >> 16) & 0xffff, exc0 = tb.y, troe = tb.z, dnu = tb.w;
    // in the mixed mode, wavefronts holding falloff reactions have the longest rate phase (it
    // bounds the rate + emission phase): they issue first on their SIMD while it runs (in
    // FP64 the emitting wavefronts are as long, and the priority gains nothing)
    const bool falloff_wave = MIXED && __builtin_amdgcn_ballot_w64(r >= 0 && (troe & 0xffff) != 0xffff) != 0;
    double lnA = 0.0, bb = 0.0, th = 0.0;
    const RxnVar var = (VAR && r >= 0) ? m.var[r] : RxnVar{0, 0, 0, 0};
    if (r >= 0) {
        lnA = m.lnA[r];
        bb = m.b[r];
        th = m.theta[r];
        const int ti = troe & 0xffff;
        if (ti != 0xffff) {   // the high-pressure Arrhenius constants beside the Troe constants
            TP[8 * n_troe + ti] = lnA;
            TP[9 * n_troe + ti] = bb;
            TP[10 * n_troe + ti] = th;
        }
    }
    // gather program of this wavefront (uniform)
    const int *prog = m.jp_prog + 8 * wave;
    const uint2 *drec = (const uint2 *)(m.jp_recs + __builtin_amdgcn_readfirstlane(prog[1]));
    const int qb = m.jp_qb;
    // emission mapping: a pair of columns (c0, c0 + 1) and a row phase per thread, on
    // wavefronts 0..JS_EWAVES-1, whose rate phase that follows is the shortest (the
    // third-body and falloff reactions sit on the last wavefronts)
    const int npair = (n1 + 1) / 2;
    const int rphase = JS_EWAVES * WAVE / npair;
    const int pc0 = 2 * (tid % npair), pr0 = tid / npair;
    const bool pon = tid < JS_EWAVES * WAVE && pr0 < rphase && pr0 < n1;
    // with an even row length and a J aligned to a pair, every emitted pair is one aligned
    // vector store (point-major rows of n1 values)
    const bool evec = n1 % 2 == 0 && (((uintptr_t)Jv) & (2 * sizeof(Out) - 1)) == 0;
    // this workgroup's points: i = slot, slot + G, ... (G = gridDim.x).  Workgroups are
    // dispatched round-robin over the 8 XCDs, so the slots of one XCD's workgroups are a
    // contiguous run of G/8 points: the 16 points of a 128-byte line of the species-major Y
    // (and of w) are handled at the same time on one XCD and meet in its L2
    const int64_t G = gridDim.x;
    const int64_t slot = (G % 8 == 0) ? (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : (int64_t)blockIdx.x;
    // state of the first point into buffer 0; prefetch of the second (indices clamped; a
    // repeat of the last point past the end is never used)
    double pf_T = 0.0, pf_p = 0.0, pf_Y = 0.0;
    __syncthreads();   // staged tables complete
    if (n > 0) {
        const int64_t i0 = min(slot, n - 1), i1 = min(i0 + G, n - 1);
        const int ky = min(lane, ns - 1);
        if (wave >= WY - 1)
            jac_seg_state<MIXED>(ns, m.R, lnp0R, wave, WY, lane, T[i0], p[i0 * ps], Y[(int64_t)ky * ld + i0], NS,
                                 IW, MX, n_m, EXm, EXs, n_troe, TP, SP0, SC0, MQ0, TQ0);
        else if (wave == WT)
            jac_seg_troe_fc<MIXED>(lane, n_troe, T[i0], TP, TQ0);
        pf_T = T[i1];
        pf_p = p[i1 * ps];
        pf_Y = Y[(int64_t)ky * ld + i1];
    }
    __syncthreads();
    int buf = 0;
    for (int64_t i = slot; i < n; i += G, buf ^= 1) {
        const double *SP = SP0 + buf * 4 * (ns + 1);
        double *SC = SC0 + buf * 16;
        // ---- B
        if (falloff_wave) __builtin_amdgcn_s_setprio(2);
        if (r >= 0)
            jac_seg_reaction<MIXED, VAR>(r, sp03, sp45, dpos, xpos, n_exc, exc0, troe, dnu, lnA, bb, th, SP, SC,
                                         TQ0, n_troe, MQ0, EXm, RDd, qb, var, m.vtab, TP);
        if (falloff_wave) __builtin_amdgcn_s_setprio(0);
        const double Tt = SC[0], rho = SC[2], wbar = SC[3], invT = SC[6];
        // this wavefront's gather records (the same for every point; L1/L2 resident); every
        // wavefront runs DMAX rounds (the plan pads with no-op rounds), so the gather
        // below is straight-line code
        uint2 dr[DMAX];
#pragma unroll
        for (int q = 0; q < (JS_DW < DMAX ? JS_DW : DMAX); ++q) dr[q] = drec[q * 64 + lane];   // the first window;
        __syncthreads();                                                 // the rest streams in below
        // ---- C: software-pipelined without branches: round q + 1's values are read before
        // round q's store; the plan puts an empty round between levels, so a level's reads
        // follow the previous level's stores in program order (LDS executes a wavefront's
        // operations in order)
        {
            // a record holds 8 x the value's index (FP64 byte offset) over its 3-bit coefficient
            auto cf = [](unsigned rec) { return (Acc)(int)__builtin_amdgcn_sbfe((int)rec, 0, 3); };
            auto ld = [](unsigned rec8) -> Acc {
                if constexpr (MIXED) return lds_ldf(rec8 >> 1);
                else return lds_ld(rec8);
            };
            Acc v0 = ld((dr[0].x >> 16) & 0xfff8u);
            Acc v1 = ld(dr[0].y & 0xfff8u);
            Acc v2 = ld((dr[0].y >> 16) & 0xfff8u);
#pragma unroll
            for (int q = 0; q < DMAX; ++q) {
                if (q + JS_DW < DMAX) dr[q + JS_DW < DMAX ? q + JS_DW : q] = drec[(q + JS_DW) * 64 + lane];
                const uint2 w = dr[q];
                const Acc acc = fma(cf(w.y >> 16), v2, fma(cf(w.y), v1, cf(w.x >> 16) * v0));
                if (q + 1 < DMAX) {
                    const uint2 wn = dr[q + 1 < DMAX ? q + 1 : q];
                    v0 = ld((wn.x >> 16) & 0xfff8u);
                    v1 = ld(wn.y & 0xfff8u);
                    v2 = ld((wn.y >> 16) & 0xfff8u);
                }
                if constexpr (MIXED) lds_stf(4u * (w.x & 0xffffu), acc);
                else lds_st(8u * (w.x & 0xffffu), acc);
                __builtin_amdgcn_sched_barrier(0);   // keeps the record stream JS_DW rounds ahead
            }
        }
        __syncthreads();
        // ---- D (and the next point's state on wavefronts WY - 1, WY)
        if (wave < JS_PWAVES) {
            const double mRT = -m.R * Tt;
            for (int cc = lane; cc < ns + 5; cc += WAVE) {
                double s0 = 0.0, s1 = 0.0;
                int k = wave;
#pragma unroll 4
                for (; k + JS_PWAVES < ns; k += 2 * JS_PWAVES) {
                    s0 += SP[4 * k + 2] * A[k * sr + cc];
                    s1 += SP[4 * (k + JS_PWAVES) + 2] * A[(k + JS_PWAVES) * sr + cc];
                }
                if (k < ns) s0 += SP[4 * k + 2] * A[k * sr + cc];
                P[wave * sr + cc] = mRT * (s0 + s1);
            }
        } else if (wave == JS_PWAVES) {
            double cwp = 0.0;
            for (int k = lane; k < ns; k += WAVE) {
                double2 q01, q23;
                if constexpr (MIXED) {   // 8-byte aligned pairs (sr even)
                    typedef float f32x2 __attribute__((ext_vector_type(2)));
                    const f32x2 a01 = *(const f32x2 *)(A + k * sr), a23 = *(const f32x2 *)(A + k * sr + 2);
                    q01 = double2{a01.x, a01.y};
                    q23 = double2{a23.x, a23.y};
                } else {
                    q01 = *(const double2 *)(A + k * sr);
                    q23 = *(const double2 *)(A + k * sr + 2);
                }
                *(double2 *)(ROW + 2 * k) = double2{rho * q23.x - wbar * q23.y, q01.x - q23.y * invT};
                cwp += SP[4 * k + 3] * q01.y;
                if (wdot) wdot[(int64_t)k * ld + i] = q01.y;
            }
            const double cw = wave_sum(cwp) * m.R;
            if (lane == 0) SC[8] = cw;
            jac_seg_troe_fc<MIXED>(lane, n_troe, pf_T, TP, TQ0);
        } else {
            // state of point i + G (past the end: a repeat of the last point, unused)
            double *SPn = SP0 + (buf ^ 1) * 4 * (ns + 1), *SCn = SC0 + (buf ^ 1) * 16;
            jac_seg_state<MIXED>(ns, m.R, lnp0R, wave, WY, lane, pf_T, pf_p, pf_Y, NS, IW, MX, n_m, EXm, EXs,
                                 n_troe, TP, SPn, SCn, MQ0, TQ0);
        }
        {   // prefetch of point i + 2G, in straight-line code on every wavefront
            const int64_t i2 = min(i + 2 * G, n - 1);
            pf_T = T[i2];
            pf_p = p[i2 * ps];
            pf_Y = Y[(int64_t)min(lane, ns - 1) * ld + i2];
        }
        __syncthreads();
        // ---- E
        Out *Jp = J + (size_t)i * n1 * n1;
        if (pon) {
            const double iw0 = pc0 >= 1 ? IW[pc0 - 1] : 0.0, iw1 = pc0 < ns ? IW[pc0] : 0.0;
            auto emit = [&](int row, double a0, double a1, double al, double jt) {
                const Out v0 = (Out)(pc0 == 0 ? jt : (rho * a0 + al) * iw0);
                const Out v1 = (Out)((rho * a1 + al) * iw1);
                Out *dst = Jp + row * n1 + pc0;
                if (pc0 + 1 < n1) {
                    if ((((uintptr_t)dst) & (2 * sizeof(Out) - 1)) == 0) {
                        typedef Out Out2 __attribute__((ext_vector_type(2)));
                        *(Out2 *)dst = Out2{v0, v1};
                    } else {
                        dst[0] = v0;
                        dst[1] = v1;
                    }
                } else {
                    dst[0] = v0;
                }
            };
            if (pr0 == 0) {   // the heat-release row: sum of the partial rows
                double pv[JS_PWAVES][5];
#pragma unroll
                for (int w = 0; w < JS_PWAVES; ++w) {
                    const double *Pw = P + w * sr;
                    pv[w][0] = Pw[0];
                    pv[w][1] = Pw[2];
                    pv[w][2] = Pw[3];
                    pv[w][3] = Pw[4 + pc0];
                    pv[w][4] = pc0 + 1 < n1 ? Pw[5 + pc0] : 0.0;
                }
                const double cw = SC[8];
                double t0 = 0.0, tau0 = 0.0, R0 = 0.0, a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int w = 0; w < JS_PWAVES; ++w) {
                    t0 += pv[w][0];
                    tau0 += pv[w][1];
                    R0 += pv[w][2];
                    a0 += pv[w][3];
                    a1 += pv[w][4];
                }
                emit(0, a0, a1, rho * tau0 - wbar * R0, t0 - cw - R0 * invT);
            }
            typedef Acc Acc2 __attribute__((ext_vector_type(2)));
            if (evec) {
                // every pair whole and aligned, and no branch in the loop: a row outside
                // 1 .. n1 - 1 is clamped onto a row whose owner (same column pair) stores the
                // identical value, so every iteration is two LDS reads and one vector store
                typedef Out Out2 __attribute__((ext_vector_type(2)));
                const int nq = (n1 + rphase - 1) / rphase;
                constexpr int EB = 3;   // rows whose reads are issued together
                for (int q = 0; q < nq; q += EB) {
                    int row[EB];
                    Acc2 av[EB];
                    f64x2 rw[EB];
#pragma unroll
                    for (int b = 0; b < EB; ++b) {
                        const int rr = pr0 + (q + b) * rphase;
                        row[b] = rr < 1 ? 1 : (rr < n1 ? rr : n1 - 1);
                        av[b] = *(const Acc2 *)(A + (row[b] - 1) * sr + 4 + pc0);
                        rw[b] = *(const f64x2 *)(ROW + 2 * (row[b] - 1));
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int b = 0; b < EB; ++b) {
                        const Out v0 = (Out)(pc0 == 0 ? rw[b].y : (rho * (double)av[b].x + rw[b].x) * iw0);
                        const Out v1 = (Out)((rho * (double)av[b].y + rw[b].x) * iw1);
                        *(Out2 *)(Jp + row[b] * n1 + pc0) = Out2{v0, v1};
                    }
                }
            } else {
#pragma unroll 2
                for (int q = 0; q < JS_EROWS; ++q) {
                    const int row = pr0 + q * rphase;
                    if (row >= 1 && row < n1) {
                        const Acc2 av = *(const Acc2 *)(A + (row - 1) * sr + 4 + pc0);   // aligned pair
                        const f64x2 rw = *(const f64x2 *)(ROW + 2 * (row - 1));
                        emit(row, av.x, av.y, rw.x, rw.y);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ transport
// LDS per wave: PPW points x {X, mu, W^(1/4)/sqrt(mu), isum} x nsp doubles (isum: sum_j X_j / D_jk).
template <bool MIXED, int PPW>
__global__ __launch_bounds__(256) void k_transport(DevMech m, int64_t n, const double *__restrict__ T,
                                                   const double *__restrict__ p, int64_t ps,
                                                   const double *__restrict__ Y, int64_t ld,
                                                   double *__restrict__ mu, double *__restrict__ lam,
                                                   double *__restrict__ Dmix, int nsp) {
    using Rt = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ double lds[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    const int ns = m.ns;
    double *base = lds + (size_t)wave * PPW * 4 * nsp;
    const int64_t n_groups = (n + PPW - 1) / PPW;
    for (int64_t g = (int64_t)blockIdx.x * wpb + wave; g < n_groups; g += (int64_t)gridDim.x * wpb) {
        double lnT[PPW], lnp0p[PPW], lam_out[PPW];
        bool valid[PPW];
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            const int64_t i = g * PPW + q;
            valid[q] = i < n;
            const int64_t ii = valid[q] ? i : 0;
            double *X = base + (4 * q) * nsp, *MU = X + nsp, *SMU = MU + nsp, *IS = SMU + nsp;
            const double t = T[ii];
            lnT[q] = log(t);
            lnp0p[q] = log(m.p0 / p[ii * ps]);
            double sy = 0.0;
            for (int k = lane; k < ns; k += WAVE) sy += Y[(int64_t)k * ld + ii] * m.invW[k];
            const double wbar = 1.0 / wave_sum(sy);
            double sxl = 0.0, sxil = 0.0;
            const Rt L = (Rt)lnT[q];
            for (int k = lane; k < ns; k += WAVE) {
                const double x = wbar * Y[(int64_t)k * ld + ii] * m.invW[k];
                const double *a = m.mu_fit + 4 * k, *b = m.lam_fit + 4 * k;
                const double muk = (double)exp_r<Rt>((Rt)a[0] + L * ((Rt)a[1] + L * ((Rt)a[2] + L * (Rt)a[3])));
                const double lk = (double)exp_r<Rt>((Rt)b[0] + L * ((Rt)b[1] + L * ((Rt)b[2] + L * (Rt)b[3])));
                X[k] = x;
                MU[k] = muk;
                SMU[k] = m.w4[k] / sqrt(muk);   // W_k^(1/4) / sqrt(mu_k)
                IS[k] = 0.0;
                sxl += x * lk;
                sxil += x / lk;
            }
            if (lane == 0) {   // the dummy species of the pair schedule
                X[ns] = 0.0;
                IS[ns] = 0.0;
            }
            sxl = wave_sum(sxl);
            sxil = wave_sum(sxil);
            lam_out[q] = 0.5 * (sxl + 1.0 / sxil);
        }
        wave_lds_sync();
        // binary diffusion, sum_j X_j / D_jk, on the round-robin schedule: half a wavefront
        // per point takes one round (a perfect matching of the species) at a time, 32 pairs
        // at a time; every species is touched once per round, so plain read-modify-writes
        // suffice, in a fixed order
        static_assert(PPW == 2, "one point per half wavefront");
        if (Dmix) {
            const int q = lane >> 5, sl = lane & 31;
            double *X = base + (4 * q) * nsp, *IS = X + 3 * nsp;
            const Rt L = (Rt)(q ? lnT[PPW - 1] : lnT[0]), lp = (Rt)(q ? lnp0p[PPW - 1] : lnp0p[0]);
            for (int r = 0; r < m.tr_rounds; ++r)
                for (int sc = sl; sc < m.tr_slots; sc += 32) {
                    const int e = r * m.tr_slots + sc;
                    const int jk = m.tr_jk[e];
                    const int j = jk & 0xffff, k = jk >> 16;
                    const double *c = m.tr_fit + 4 * e;
                    const Rt c0 = (Rt)c[0], c1 = (Rt)c[1], c2 = (Rt)c[2], c3 = (Rt)c[3];
                    const double invD = (double)exp_r<Rt>(-(c0 + L * (c1 + L * (c2 + L * c3))) - lp);
                    const double xj = X[j], xk = X[k];
                    IS[k] += xj * invD;
                    IS[j] += xk * invD;
                }
        }
        wave_lds_sync();
        // Wilke: denominator_k = sum_j X_j Phi_kj, Phi_kj = c_jk (1 + sqrt(mu_k/mu_j) (W_j/W_k)^(1/4))^2,
        // with the factor written as 1 + a_k b_j, a_k = sqrt(mu_k) / W_k^(1/4), b_j = SMU[j]; the
        // wavefront's points share each c_jk load
        double num[PPW];
#pragma unroll
        for (int q = 0; q < PPW; ++q) num[q] = 0.0;
        if (mu) {
            for (int k = lane; k < ns; k += WAVE) {
                const double iw4k = m.iw4[k];
                Rt ak[PPW], den[PPW];
#pragma unroll
                for (int q = 0; q < PPW; ++q) {
                    ak[q] = (Rt)(sqrt(base[(4 * q + 1) * nsp + k]) * iw4k);
                    den[q] = 0;
                }
#pragma unroll 2
                for (int j = 0; j < ns; ++j) {
                    const Rt c = (Rt)m.wilke_c[(size_t)j * ns + k];
#pragma unroll
                    for (int q = 0; q < PPW; ++q) {
                        const Rt f = (Rt)1 + ak[q] * (Rt)base[(4 * q + 2) * nsp + j];
                        den[q] += (Rt)base[(4 * q) * nsp + j] * c * f * f;
                    }
                }
#pragma unroll
                for (int q = 0; q < PPW; ++q)
                    num[q] += base[(4 * q) * nsp + k] * base[(4 * q + 1) * nsp + k] / (double)den[q];
            }
#pragma unroll
            for (int q = 0; q < PPW; ++q) num[q] = wave_sum(num[q]);
        }
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            const int64_t i = g * PPW + q;
            const double *IS = base + (4 * q + 3) * nsp;
            if (!valid[q]) continue;
            if (Dmix)
                for (int k = lane; k < ns; k += WAVE)
                    Dmix[(int64_t)k * ld + i] = (1.0 - Y[(int64_t)k * ld + i]) / IS[k];
            if (lane == 0) {
                if (mu) mu[i] = num[q];
                if (lam) lam[i] = lam_out[q];
            }
        }
    }
}

// ------------------------------------------------------------------ transport, point tiles
// Sixteen points per workgroup of W wavefronts, one tile per workgroup.  LDS holds, per
// species row of the tile (row stride tt_rs(W) doubles; the host orders the pairs of a round so
// that the rows one part of an instruction touches fall on different banks): Xs_k = Y_k / W_k, the diffusion sums
// IS_k = sum_j Xs_j / D_jk and a_k = sqrt(mu_k) / W_k^(1/4); b_k = 1 / a_k and
// mu_k = (a_k W_k^(1/4))^2 are formed where they are used, which keeps the tile small enough
// for six workgroups per compute unit (53 species, FP64).  The mole fractions are
// X = Wbar Xs; Wbar cancels from Wilke's quotient and is applied to the conductivity and
// diffusion sums at the end.
//   * setup: thread = (point, species group); the 16 points of a species row are adjacent
//     in Y, so each group of 16 lanes reads one 128-byte line;
//   * diffusion: each wavefront owns 16/W points and runs every round of the pair schedule on
//     them, 64 W/16 pairs per instruction.  A round touches each species once, so the LDS
//     additions of one instruction never meet, and only the owning wavefront adds into a
//     point's sums, in program order: the result is reproducible bit for bit;
//   * Wilke: den_k = sum_j X_j c_jk (1 + a_k b_j)^2 with a_k = sqrt(mu_k) / W_k^(1/4) is
//     D1_k + a_k (2 D2_k + a_k D3_k) with D1 = Xs C, D2 = (Xs b) C, D3 = (Xs b^2) C:
//     three [16 x Ns] x [Ns x Ns] products on the matrix cores (16x16x4 MFMA, FP64, or FP32
//     in the mixed mode), tiles of 16 species columns dealt to the wavefronts, C = wilke_c
//     read from L2 once per tile of points.  mu = sum_k Xs_k mu_k / den~_k (Wbar cancels).
// 2^(j/64), j = 0..63, each the double nearest to its exact value.
__constant__ double EXP2_J64[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0
};

// e^x in FP64 by the table-driven method of Tang (ACM TOMS 15, 1989): x = (64 m + j) ln2/64 + r,
// |r| <= ln2/128 (ln2/64 split as in exp_fast, so kf ln2_hi/64 is exact), then
// e^x = 2^m 2^(j/64) e^r with e^r from its degree-5 Taylor polynomial (truncation below 4e-17
// relative) and 2^(j/64) from `tab` (EXP2_J64 staged in LDS).  About 1.5 ulp; fewer
// instructions than exp_fast, whose eleven polynomial coefficients the fused multiply-adds
// consume one register copy each.
__device__ inline double exp_tab(double x, const double *tab) {
    const double kf = fmin(fmax(rint(x * 92.332482616893657), -140000.0), 140000.0);
    double r = fma(-kf, 6.93147180369123816490e-01 / 64.0, x);
    r = fma(-kf, 1.90821492927058770002e-10 / 64.0, r);
    const int k = (int)kf;
    const double q = fma(r, fma(r, fma(r, fma(r, fma(r, 1.0 / 120.0, 1.0 / 24.0), 1.0 / 6.0), 0.5), 1.0), 1.0);
    return ldexp(tab[k & 63] * q, k >> 6);
}

template <bool MIXED> struct TileMfma;
template <> struct TileMfma<false> {
    typedef double V __attribute__((ext_vector_type(4)));
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // row of the product held in register r of `lane` (its column is lane % 16)
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct TileMfma<true> {
    typedef float V __attribute__((ext_vector_type(4)));
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Sum over the 16 lanes that share lane / 16 (butterfly, fixed order).
__device__ inline double row16_sum(double v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool MIXED, int W>
__global__ __launch_bounds__(W * WAVE) __attribute__((amdgpu_waves_per_eu(4))) void k_transport_tile(DevMech m, int64_t n, const double *__restrict__ T,
                                                             const double *__restrict__ p, int64_t ps,
                                                             const double *__restrict__ Y, int64_t ld,
                                                             double *__restrict__ mu, double *__restrict__ lam,
                                                             double *__restrict__ Dmix, int rows) {
    using Rt = typename std::conditional<MIXED, float, double>::type;
    using MM = TileMfma<MIXED>;
    constexpr int NT = W * WAVE;
    constexpr int PW = TT_P / W;                 // points per wavefront in the diffusion phase
    constexpr int G = WAVE / PW;                 // pairs per wavefront instruction
    constexpr int NG = NT / TT_P;                // species groups of the setup and output phases
    constexpr int RS = tt_rs(W);                 // row stride of the species rows
    extern __shared__ double lds[];
    double *XS = lds;                            // [rows][RS]
    double *IS = XS + rows * RS;              // [rows][RS]
    double *E2 = IS + rows * RS;              // 2^(j/64) for exp_tab
    double *PT = E2 + 64;                        // lnT[16], ln(p0/p)[16], sums[W][16][3], num[W][16]
    double *SUMS = PT + 2 * TT_P, *NUM = SUMS + 3 * W * TT_P;
    Rt *AA = (Rt *)(NUM + W * TT_P);             // [rows][RS]
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid & (WAVE - 1);
    const int ns = m.ns;
    if (!MIXED && tid < 64) E2[tid] = EXP2_J64[tid];
    {
        const int64_t i0 = (int64_t)blockIdx.x * TT_P;
        {   // setup
            const int mm = tid % TT_P, g = tid / TT_P;
            const int64_t i = i0 + mm < n ? i0 + mm : n - 1;
            const double L = log(T[i]);
            const Rt Lr = (Rt)L;
            if (g == 0) {
                PT[mm] = L;
                PT[TT_P + mm] = log(m.p0 / p[i * ps]);
            }
            double sx = 0.0, sxl = 0.0, sxil = 0.0;
            for (int k = g; k < rows; k += NG) {
                double x = 0.0;
                Rt ak = 0;
                if (k < ns) {
                    x = Y[(int64_t)k * ld + i] * m.invW[k];
                    const double *a = m.mu_fit + 4 * k, *c = m.lam_fit + 4 * k;
                    const Rt muk = exp_r<Rt>((Rt)a[0] + Lr * ((Rt)a[1] + Lr * ((Rt)a[2] + Lr * (Rt)a[3])));
                    const double lk = (double)exp_r<Rt>((Rt)c[0] + Lr * ((Rt)c[1] + Lr * ((Rt)c[2] + Lr * (Rt)c[3])));
                    ak = (Rt)(sqrt((double)muk) * m.iw4[k]);
                    sx += x;
                    sxl += x * lk;
                    sxil += x / lk;
                }
                XS[k * RS + mm] = x;
                IS[k * RS + mm] = 0.0;
                AA[k * RS + mm] = ak;
            }
            // the wavefront's four species groups of a point: lanes mm, mm + 16, mm + 32, mm + 48
            sx += __shfl_xor(sx, 16);
            sx += __shfl_xor(sx, 32);
            sxl += __shfl_xor(sxl, 16);
            sxl += __shfl_xor(sxl, 32);
            sxil += __shfl_xor(sxil, 16);
            sxil += __shfl_xor(sxil, 32);
            if (lane < TT_P) {
                double *s = SUMS + 3 * (wave * TT_P + lane);
                s[0] = sx;
                s[1] = sxl;
                s[2] = sxil;
            }
        }
        __syncthreads();
        if (Dmix) {   // binary diffusion sums of the wavefront's own points
            const int q = lane % PW, sg = lane / PW, mm = wave * PW + q;
            const Rt L = (Rt)PT[mm], lp = (Rt)PT[TT_P + mm];
            // byte addresses of this point's column in the species rows (pair offsets add to them)
            const unsigned xs_b = (unsigned)((const char *)(XS + mm) - (const char *)lds);
            const unsigned is_b = (unsigned)((const char *)(IS + mm) - (const char *)lds);
            const int slots = m.tr_slots, passes = (slots + G - 1) / G, total = m.tr_rounds * passes;
            // one pass = G pairs of one round (lanes past the round's end idle); the next pass's
            // pair offsets and fit coefficients are loaded while this pass computes
            int r = 0, t = 0;
            bool ok_n = sg < slots;
            int e_n = ok_n ? sg : 0;
            const unsigned *offs = m.tr_off + (MIXED ? m.tr_rounds * m.tr_slots : 0);
            unsigned off_n = offs[e_n];
            Rt cn[4];
            auto load_fit = [&](int e) {
                if constexpr (MIXED) {
                    const float4 c = *(const float4 *)(m.tr_fit32 + 4 * e);
                    cn[0] = c.x; cn[1] = c.y; cn[2] = c.z; cn[3] = c.w;
                } else {
                    const double2 a = *(const double2 *)(m.tr_fit + 4 * e);
                    const double2 b = *(const double2 *)(m.tr_fit + 4 * e + 2);
                    cn[0] = a.x; cn[1] = a.y; cn[2] = b.x; cn[3] = b.y;
                }
            };
            load_fit(e_n);
            for (int it = 0; it < total; ++it) {
                const bool ok = ok_n;
                const unsigned off = off_n;
                const Rt c0 = cn[0], c1 = cn[1], c2 = cn[2], c3 = cn[3];
                if (++t == passes) { t = 0; ++r; }
                if (it + 1 < total) {
                    const int s = sg + t * G;
                    ok_n = s < slots;
                    e_n = r * slots + (ok_n ? s : 0);
                    off_n = offs[e_n];
                    load_fit(e_n);
                }
                if (ok) {
                    const unsigned oj = off & 0xffffu, ok16 = off >> 16;
                    const Rt arg = -(c0 + L * (c1 + L * (c2 + L * c3))) - lp;
                    double invD;
                    if constexpr (MIXED) invD = (double)exp_r<Rt>(arg);
                    else invD = exp_tab(arg, E2);
                    const double xj = lds_ld(xs_b + oj), xk = lds_ld(xs_b + ok16);
                    atomicAdd((double *)((char *)lds + is_b + ok16), xj * invD);
                    atomicAdd((double *)((char *)lds + is_b + oj), xk * invD);
                }
            }
        }
        if (mu) {     // Wilke on the matrix cores
            double num[4] = {0.0, 0.0, 0.0, 0.0};
            const int ntiles = (ns + 15) / 16, ksteps = (ns + 3) / 4;
            const int mrow = lane & 15, kin = lane >> 4;
            for (int nt = wave; nt < ntiles; nt += W) {
                const int kc = nt * 16 + (lane & 15);      // this lane's product column (species k)
                typename MM::V d1 = {0, 0, 0, 0}, d2 = {0, 0, 0, 0}, d3 = {0, 0, 0, 0};
                Rt u1n = 0, bjn = 0, cn = 0;     // operands of the next K step, loaded a step ahead
                auto load_k = [&](int ks) {
                    const int j = ks * 4 + kin;
                    u1n = 0; bjn = 0; cn = 0;
                    if (j < ns) {
                        u1n = (Rt)XS[j * RS + mrow];
                        bjn = (Rt)1 / AA[j * RS + mrow];
                        if (kc < ns) cn = (Rt)m.wilke_c[(size_t)j * ns + kc];
                    }
                };
                load_k(0);
                for (int ks = 0; ks < ksteps; ++ks) {
                    const Rt u1 = u1n, bj = bjn, c = cn;
                    if (ks + 1 < ksteps) load_k(ks + 1);
                    const Rt u2 = u1 * bj, u3 = u2 * bj;
                    d1 = MM::mma(u1, c, d1);
                    d2 = MM::mma(u2, c, d2);
                    d3 = MM::mma(u3, c, d3);
                }
                if (kc < ns) {
                    const Rt w4k = (Rt)m.w4[kc];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int o = kc * RS + MM::row(lane, r);
                        const Rt a = AA[o];
                        const Rt den = d1[r] + a * ((Rt)2 * d2[r] + a * d3[r]);
                        const Rt sq = a * w4k;   // sqrt(mu_k)
                        num[r] += XS[o] * (double)(sq * sq) / (double)den;
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double s = row16_sum(num[r]);
                if ((lane & 15) == 0) NUM[wave * TT_P + MM::row(lane, r)] = s;
            }
        }
        __syncthreads();
        {   // outputs
            const int mm = tid % TT_P, g = tid / TT_P;
            const int64_t i = i0 + mm;
            if (i < n) {
                double sx = 0.0, sxl = 0.0, sxil = 0.0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const double *s = SUMS + 3 * (w * TT_P + mm);
                    sx += s[0];
                    sxl += s[1];
                    sxil += s[2];
                }
                const double wbar = 1.0 / sx;
                if (Dmix)
                    for (int k = g; k < ns; k += NG)
                        Dmix[(int64_t)k * ld + i] = (1.0 - Y[(int64_t)k * ld + i]) / (wbar * IS[k * RS + mm]);
                if (g == 0) {
                    if (lam) lam[i] = 0.5 * (wbar * sxl + 1.0 / (wbar * sxil));
                    if (mu) {
                        double s = 0.0;
#pragma unroll
                        for (int w = 0; w < W; ++w) s += NUM[w * TT_P + mm];
                        mu[i] = s;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ reactor step (ROS2)
// Constant-pressure adiabatic reactor, x = (T, Y), dx/dt = f(x) = (hrr/(rho c_p), W_k w_k/rho),
// one two-stage Rosenbrock (ROS2) substep of size h:
//   (I - gamma h A) k1 = f(x),  (I - gamma h A) k2 = f(x + h k1) - 2 k1,
//   x <- x + 3/2 h k1 + 1/2 h k2,  gamma = 1 + 1/sqrt(2),
// with A = df/dx formed from the Jacobian J of (hrr, w) by the chain rule through
// rho(T, Y) and c_p(T, Y).  k_ros_lu: one workgroup per point forms M = I - gamma h A, factors
// it (LU with partial pivoting, the row of largest magnitude, lowest index on ties),
// solves for k1 and writes the stage state x + h k1; k_ros_finish solves for k2 with the
// stored factors and updates x in place.  The matrix lives in LDS when it fits (a copy
// of the factors goes to the workspace for k_ros_finish), else in the workspace itself.
constexpr int ROS_THREADS = 256;
constexpr double ROS_GAMMA = 1.7071067811865475244;

// Sum over the workgroup (ROS_THREADS threads); `red` holds ROS_THREADS / WAVE doubles.
__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int wave = threadIdx.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < ROS_THREADS / WAVE; ++w) s += red[w];
    return s;
}

// LU factorisation with partial pivoting of the N x N row-major matrix A (lda = N), in
// place; piv[k] = the row swapped with row k at step k.  All ROS_THREADS threads take part.
__device__ inline void lu_factor(double *A, int N, int *piv) {
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    for (int k = 0; k < N; ++k) {
        if (tid < WAVE) {   // pivot search on wavefront 0: largest |A[r][k]|, lowest r on ties
            double best = -1.0;
            int br = k;
            for (int r = k + lane; r < N; r += WAVE) {
                const double a = fabs(A[(size_t)r * N + k]);
                if (a > best) { best = a; br = r; }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ob = __shfl_xor(best, off);
                const int orr = __shfl_xor(br, off);
                if (ob > best || (ob == best && orr < br)) { best = ob; br = orr; }
            }
            if (lane == 0) piv[k] = br;
        }
        __syncthreads();
        const int pr = piv[k];
        if (pr != k)
            for (int c = tid; c < N; c += ROS_THREADS) {
                const double a = A[(size_t)k * N + c];
                A[(size_t)k * N + c] = A[(size_t)pr * N + c];
                A[(size_t)pr * N + c] = a;
            }
        __syncthreads();
        const double inv = 1.0 / A[(size_t)k * N + k];
        for (int r = k + 1 + tid; r < N; r += ROS_THREADS) A[(size_t)r * N + k] *= inv;
        __syncthreads();
        const int m = N - k - 1;
        for (int e = tid; e < m * m; e += ROS_THREADS) {
            const int r = k + 1 + e / m, c = k + 1 + e % m;
            A[(size_t)r * N + c] = fma(-A[(size_t)r * N + k], A[(size_t)k * N + c], A[(size_t)r * N + c]);
        }
        __syncthreads();
    }
}

// Solves (LU) x = P b in place in b (LDS, N values) with the factors of lu_factor.
__device__ inline void lu_solve(const double *A, int N, const int *piv, double *b) {
    const int tid = threadIdx.x;
    if (tid == 0)
        for (int k = 0; k < N; ++k) {
            const int pr = piv[k];
            if (pr != k) { const double t = b[k]; b[k] = b[pr]; b[pr] = t; }
        }
    __syncthreads();
    for (int k = 0; k < N; ++k) {          // forward: unit lower triangle
        const double bk = b[k];
        for (int r = k + 1 + tid; r < N; r += ROS_THREADS) b[r] = fma(-A[(size_t)r * N + k], bk, b[r]);
        __syncthreads();
    }
    for (int k = N - 1; k >= 0; --k) {     // backward: upper triangle
        if (tid == 0) b[k] = b[k] / A[(size_t)k * N + k];
        __syncthreads();
        const double bk = b[k];
        for (int r = tid; r < k; r += ROS_THREADS) b[r] = fma(-A[(size_t)r * N + k], bk, b[r]);
        __syncthreads();
    }
}

// LDS of k_ros_lu: per-point vectors {f, drho/rho, dcp/cp, row scale, w} x N1, N1 pivots,
// ROS_THREADS/WAVE reduction slots, then the N1 x N1 matrix when it fits.
template <bool JF32>
__global__ __launch_bounds__(ROS_THREADS) void k_ros_lu(DevMech m, int64_t n, const double *__restrict__ T,
                                                        const double *__restrict__ p, int64_t ps,
                                                        const double *__restrict__ Y, int64_t ld,
                                                        const void *__restrict__ Jv, const double *__restrict__ wd,
                                                        double h, double *__restrict__ Mbuf, int *__restrict__ pivg,
                                                        double *__restrict__ k1g, double *__restrict__ Ts,
                                                        double *__restrict__ Ys, int mat_in_lds) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int ns = m.ns, N = ns + 1;
    double *F = lds, *DR = F + N, *DC = DR + N, *RS = DC + N, *WV = RS + N;
    double *red = WV + N;
    int *piv = (int *)(red + ROS_THREADS / WAVE);
    double *AL = (double *)(piv + ((N + 1) & ~1));
    using Jt = typename std::conditional<JF32, float, double>::type;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const double t = T[i], pp = p[i * ps], invT = 1.0 / t;
        // mixture: Wbar, rho, c_p, dc_p/dT, hrr = -R T sum_k (h_k/RT) w_k
        double syw = 0.0, scp = 0.0, sdcp = 0.0, shw = 0.0;
        for (int k = tid; k < ns; k += ROS_THREADS) {
            const double *c16 = m.nasa + 16 * k;
            const double *a = (t <= c16[0]) ? c16 + 1 : c16 + 8;
            const double cpR = a[0] + t * (a[1] + t * (a[2] + t * (a[3] + t * a[4])));
            const double dcpR = a[1] + t * (2.0 * a[2] + t * (3.0 * a[3] + t * 4.0 * a[4]));
            const double hRT = a[0] + t * (a[1] * 0.5 + t * (a[2] * (1.0 / 3.0) + t * (a[3] * 0.25 + t * (a[4] * 0.2)))) +
                               a[5] * invT;
            const double yw = Y[(int64_t)k * ld + i] * m.invW[k];
            const double w = wd[(int64_t)k * n + i];
            syw += yw;
            scp += yw * cpR;
            sdcp += yw * dcpR;
            shw += hRT * w;
            WV[1 + k] = w;
            DC[1 + k] = cpR * m.invW[k];                     // d c_p/dY_k / R
        }
        syw = block_sum(syw, red);
        scp = block_sum(scp, red);
        sdcp = block_sum(sdcp, red);
        shw = block_sum(shw, red);
        const double wbar = 1.0 / syw, rho = pp * wbar / (m.R * t);
        const double cp = m.R * scp, hrr = -m.R * t * shw;
        const double fT = hrr / (rho * cp);
        for (int c = tid; c < N; c += ROS_THREADS) {
            if (c == 0) {
                F[0] = fT;
                DR[0] = -invT;                               // (d rho/dT)/rho
                DC[0] = sdcp / scp;                          // (d c_p/dT)/c_p
                RS[0] = 1.0 / (rho * cp);
                WV[0] = 0.0;
            } else {
                F[c] = m.W[c - 1] * WV[c] / rho;
                DR[c] = -wbar * m.invW[c - 1];               // (d rho/dY_j)/rho
                DC[c] = DC[c] / scp;                         // (d c_p/dY_j)/c_p
                RS[c] = m.W[c - 1] / rho;
            }
        }
        __syncthreads();
        // M = I - gamma h A
        double *A = mat_in_lds ? AL : Mbuf + (size_t)i * N * N;
        const Jt *Jp = (const Jt *)Jv + (size_t)i * N * N;
        const double gh = ROS_GAMMA * h;
        for (int e = tid; e < N * N; e += ROS_THREADS) {
            const int r = e / N, c = e - r * N;
            const double j = (double)Jp[e];
            const double a = r == 0 ? RS[0] * j - fT * (DR[c] + DC[c]) : RS[r] * (j - WV[r] * DR[c]);
            A[e] = (r == c ? 1.0 : 0.0) - gh * a;
        }
        __syncthreads();
        lu_factor(A, N, piv);
        double *b = RS;                                      // reuse: right-hand side f
        for (int c = tid; c < N; c += ROS_THREADS) b[c] = F[c];
        __syncthreads();
        lu_solve(A, N, piv, b);
        for (int c = tid; c < N; c += ROS_THREADS) {
            k1g[(size_t)i * N + c] = b[c];
            pivg[(size_t)i * N + c] = piv[c];
            if (c == 0) Ts[i] = t + h * b[0];
            else Ys[(int64_t)(c - 1) * n + i] = Y[(int64_t)(c - 1) * ld + i] + h * b[c];
        }
        if (mat_in_lds)
            for (int e = tid; e < N * N; e += ROS_THREADS) Mbuf[(size_t)i * N * N + e] = A[e];
        __syncthreads();
    }
}

// Second stage: k2 = (LU)^-1 (f(x_s) - 2 k1), x <- x + 3/2 h k1 + 1/2 h k2 (T, Y in place).
__global__ __launch_bounds__(ROS_THREADS) void k_ros_finish(DevMech m, int64_t n, double *__restrict__ T,
                                                            double *__restrict__ Y, int64_t ld,
                                                            const double *__restrict__ Mbuf,
                                                            const int *__restrict__ pivg,
                                                            const double *__restrict__ k1g,
                                                            const double *__restrict__ fTs,
                                                            const double *__restrict__ fYs, double h) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int ns = m.ns, N = ns + 1;
    double *b = lds;
    int *piv = (int *)(b + N);
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        for (int c = tid; c < N; c += ROS_THREADS) {
            const double f = c == 0 ? fTs[i] : fYs[(int64_t)(c - 1) * n + i];
            b[c] = f - 2.0 * k1g[(size_t)i * N + c];
            piv[c] = pivg[(size_t)i * N + c];
        }
        __syncthreads();
        lu_solve(Mbuf + (size_t)i * N * N, N, piv, b);
        for (int c = tid; c < N; c += ROS_THREADS) {
            const double dx = 1.5 * h * k1g[(size_t)i * N + c] + 0.5 * h * b[c];
            if (c == 0) T[i] += dx;
            else Y[(int64_t)(c - 1) * ld + i] += dx;
        }
        __syncthreads();
    }
}

// Wave-per-point forms of the two reactor kernels for N = Ns + 1 <= NM (NM = 16, 40 or 56): lane r
// holds row r of the Newton matrix in registers, so the factorisation needs no barrier and
// moves no rows.  Partial pivoting by selection: at step k the not yet selected row with the
// largest |M_rk| (lowest lane on ties) is selected, its entries are broadcast through scalar
// registers (readlane), and every other unselected row takes l = M_rk / M_pk and
// M_rj -= l M_pj (the same operations as a factorisation with row exchanges).  Lane r keeps
// its multipliers for the steps before its own selection step s_r and the U row of step s_r
// after it (with 1/U_kk stored on the diagonal); the factors and s_r go to the workspace for
// the second stage.  The solution of
// step k's unknown (column k) is formed on the lane selected at step k.  Every loop over the
// row is expanded at compile time (static_for), so that each element of the row array has a
// constant index from the start and is kept in a register.
template <int I, int E, class F>
__device__ __attribute__((always_inline)) inline void static_for(F &&f) {
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}

__device__ inline double lane_bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// The lane selected at step k (the step indices of the lanes are a permutation of 0..N-1).
__device__ inline int lane_of_step(int step, int k) {
    return __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(step == k)));
}

// Solves with the factors held in a[] (see above): b is row r's right-hand side on entry,
// and on return lane s^-1(k) holds unknown k.
template <int NM>
__device__ __attribute__((always_inline)) inline double ros_solve_w(const double (&a)[NM], int step, int N,
                                                                   double b) {
    static_for<0, NM>([&](auto kc) __attribute__((always_inline)) {   // forward: unit lower factor
        constexpr int k = decltype(kc)::value;
        if (k < N) {
            const double yk = lane_bcast(b, lane_of_step(step, k));
            if (step > k) b = fma(-a[k], yk, b);
        }
    });
    static_for<0, NM>([&](auto ic) __attribute__((always_inline)) {   // backward: upper factor
        constexpr int k = NM - 1 - decltype(ic)::value;
        if (k < N) {
            const int pv = lane_of_step(step, k);
            const double xk = lane_bcast(b, pv) * lane_bcast(a[k], pv);   // 1/U_kk is stored
            if (step == k) b = xk;
            else if (step < k) b = fma(-a[k], xk, b);
        }
    });
    return b;
}

template <bool JF32, int NM>
__global__ __launch_bounds__(256) void k_ros_lu_w(DevMech m, int64_t n, const double *__restrict__ T,
                                                  const double *__restrict__ p, int64_t ps,
                                                  const double *__restrict__ Y, int64_t ld,
                                                  const void *Jv, const double *__restrict__ wd,
                                                  double h, double *Mbuf, int *__restrict__ stepg,
                                                  double *__restrict__ k1g, double *__restrict__ Ts,
                                                  double *__restrict__ Ys) {
    using Jt = typename std::conditional<JF32, float, double>::type;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;                    // whole wavefronts
    const int ns = m.ns, N = ns + 1;
    const double t = T[i], pp = p[i * ps], invT = 1.0 / t;
    // mixture (lane c = 1 + species k): Wbar, rho, c_p, dc_p/dT, hrr = -R T sum_k (h_k/RT) w_k
    const int k = lane - 1;
    const bool sp = lane >= 1 && lane < N;
    double yw = 0.0, cpy = 0.0, dcpy = 0.0, hw = 0.0, w = 0.0, cpw = 0.0;
    if (sp) {
        const double *c16 = m.nasa + 16 * k;
        const double *ca = (t <= c16[0]) ? c16 + 1 : c16 + 8;
        const double cpR = ca[0] + t * (ca[1] + t * (ca[2] + t * (ca[3] + t * ca[4])));
        const double dcpR = ca[1] + t * (2.0 * ca[2] + t * (3.0 * ca[3] + t * 4.0 * ca[4]));
        const double hRT = ca[0] + t * (ca[1] * 0.5 + t * (ca[2] * (1.0 / 3.0) + t * (ca[3] * 0.25 + t * (ca[4] * 0.2)))) +
                           ca[5] * invT;
        yw = Y[(int64_t)k * ld + i] * m.invW[k];
        w = wd[(int64_t)k * n + i];
        cpy = yw * cpR;
        dcpy = yw * dcpR;
        hw = hRT * w;
        cpw = cpR * m.invW[k];
    }
    const double syw = wave_sum(yw), scp = wave_sum(cpy), sdcp = wave_sum(dcpy), shw = wave_sum(hw);
    const double wbar = 1.0 / syw, rho = pp * wbar / (m.R * t);
    const double cp = m.R * scp, hrr = -m.R * t * shw;
    const double fT = hrr / (rho * cp);
    // per column c (lane c): (d rho/dx_c)/rho and (d c_p/dx_c)/c_p; per row r (lane r): f_r,
    // the row scale and w_r
    double F = 0.0, DR = 0.0, DC = 0.0, RS = 0.0, WV = 0.0;
    if (lane == 0) {
        F = fT; DR = -invT; DC = sdcp / scp; RS = 1.0 / (rho * cp);
    } else if (sp) {
        F = m.W[k] * w / rho; DR = -wbar * m.invW[k]; DC = cpw / scp; RS = m.W[k] / rho; WV = w;
    }
    const double DRC = DR + DC;
    // row `lane` of M = I - gamma h A (identity rows and columns beyond N)
    const double gh = ROS_GAMMA * h;
    const Jt *Jr = (const Jt *)Jv + (size_t)i * N * N + (size_t)(lane < N ? lane : 0) * N;
    double a[NM];
    static_for<0, NM>([&](auto cc) __attribute__((always_inline)) {
        constexpr int c = decltype(cc)::value;
        double v = lane == c ? 1.0 : 0.0;
        if (c < N) {
            const double dr = lane_bcast(DR, c), drc = lane_bcast(DRC, c);
            if (lane < N) {
                const double j = (double)Jr[c];
                const double ar = lane == 0 ? RS * j - fT * drc : RS * (j - WV * dr);
                v -= gh * ar;
            }
        }
        a[c] = v;
        if constexpr ((c & 7) == 7) __builtin_amdgcn_sched_barrier(0);   // bounds the loads in flight
    });
    // factorisation
    int step = NM;
    bool live = lane < N;
    static_for<0, NM>([&](auto kc) __attribute__((always_inline)) {
        constexpr int kk = decltype(kc)::value;
        if (kk < N) {
            // pivot: the largest |M_rk| (DPP reduction), the lowest such lane (ballot); a column
            // of NaNs selects the lowest unselected lane
            const double key = live ? fabs(a[kk]) : -1.0;
            const double mx = wave_max(key);
            unsigned long long sel = __ballot(live && key == mx);
            if (sel == 0) sel = __ballot(live);
            const int pv = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(sel));
            const double inv = 1.0 / lane_bcast(a[kk], pv);
            if (lane == pv) {   // the selected row keeps 1/U_kk in place of U_kk
                step = kk;
                live = false;
                a[kk] = inv;
            }
            if (live) {   // the padding columns of real rows are zero, so they stay unchanged
                const double l = a[kk] * inv;
                a[kk] = l;
                static_for<kk + 1, NM>([&](auto jc) __attribute__((always_inline)) {
                    constexpr int j = decltype(jc)::value;
                    a[j] = fma(-l, lane_bcast(a[j], pv), a[j]);
                });
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // one step at a time: bounds the live registers
    });
    // stage 1: k1 = M^-1 f; the lane selected at step c holds component c
    const double x = ros_solve_w<NM>(a, step, N, F);
    if (lane < N) {
        const int c = step;
        k1g[(size_t)i * N + c] = x;
        if (c == 0) Ts[i] = t + h * x;
        else Ys[(int64_t)(c - 1) * n + i] = Y[(int64_t)(c - 1) * ld + i] + h * x;
        // column-major (lane-contiguous) factors; in FP64 Mbuf is the Jacobian's storage, whose
        // rows this wavefront read above
        double *Mc = Mbuf + (size_t)i * N * N + lane;
        static_for<0, NM>([&](auto cc) __attribute__((always_inline)) {
            constexpr int c2 = decltype(cc)::value;
            if (c2 < N) Mc[(size_t)c2 * N] = a[c2];
        });
        stepg[(size_t)i * N + lane] = step;
    }
}

// Second stage, wave per point: k2 = M^-1 (f(x_s) - 2 k1), x <- x + 3/2 h k1 + 1/2 h k2.
template <int NM>
__global__ __launch_bounds__(256) void k_ros_finish_w(DevMech m, int64_t n, double *__restrict__ T,
                                                      double *__restrict__ Y, int64_t ld,
                                                      const double *__restrict__ Mbuf,
                                                      const int *__restrict__ stepg,
                                                      const double *__restrict__ k1g,
                                                      const double *__restrict__ fTs,
                                                      const double *__restrict__ fYs, double h) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;
    const int N = m.ns + 1;
    double a[NM];
    int step = NM;
    double b = 0.0;
    const double *Mc = Mbuf + (size_t)i * N * N + (lane < N ? lane : 0);   // column-major factors
    static_for<0, NM>([&](auto cc) __attribute__((always_inline)) {
        constexpr int c = decltype(cc)::value;
        a[c] = (c < N && lane < N) ? Mc[(size_t)c * N] : 0.0;
    });
    if (lane < N) {
        step = stepg[(size_t)i * N + lane];
        const double f = lane == 0 ? fTs[i] : fYs[(int64_t)(lane - 1) * n + i];
        b = f - 2.0 * k1g[(size_t)i * N + lane];
    }
    const double x = ros_solve_w<NM>(a, step, N, b);
    if (lane < N) {
        const int c = step;
        const double dx = 1.5 * h * k1g[(size_t)i * N + c] + 0.5 * h * x;
        if (c == 0) T[i] += dx;
        else Y[(int64_t)(c - 1) * ld + i] += dx;
    }
}

// ------------------------------------------------------------------ peak-rate probes
// Throughput probes for the roofline denominators: every thread runs 8 independent
// chains of `iters` operations of one kind (0: exp_fast (FP64), 1: exp of the device
// library (FP64), 2: __expf (v_exp_f32), 3: FP64 FMA, 4: FP32 FMA); out[thread] keeps the
// result alive.  Operations = threads x iters x 8.
__global__ __launch_bounds__(256) void k_peak(int kind, int iters, double *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double d[8];
    float f[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        d[c] = -1e-3 * (double)((t + c) & 1023);
        f[c] = (float)d[c];
    }
    if (kind == 0) {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < 8; ++c) d[c] = exp_fast(d[c]) - 1.0;
    } else if (kind == 1) {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < 8; ++c) d[c] = exp(d[c]) - 1.0;
    } else if (kind == 2) {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < 8; ++c) f[c] = __expf(f[c]) - 1.0f;
    } else if (kind == 3) {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < 8; ++c) d[c] = fma(d[c], 0.999999, 1e-9);
    } else {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < 8; ++c) f[c] = fmaf(f[c], 0.999999f, 1e-9f);
    }
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += d[c] + (double)f[c];
    out[t] = acc;
}

int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        cached[dev] = cu;
    }
    return cached[dev];
}

inline unsigned grid_for(int64_t work_items, int per_block, int blocks_per_cu) {
    const int64_t need = (work_items + per_block - 1) / per_block;
    const int64_t cap = (int64_t)device_cu_count() * blocks_per_cu;
    return (unsigned)(need < cap ? (need > 0 ? need : 1) : cap);
}

inline int pad_odd(int x) { return x | 1; }

// Wavefronts per workgroup (up to 4) of a kernel whose wavefronts each need `per_wave`
// bytes of dynamic LDS: as many as one compute unit's LDS holds.  Raises the kernel's
// dynamic-LDS limit (64 KB by default) to what the workgroup uses.  The loader refuses
// mechanisms for which even one wavefront would not fit.
hipError_t lds_waves(const void *fn, size_t per_wave, int &wpb, size_t &shm) {
    wpb = 4;
    while (wpb > 1 && (size_t)wpb * per_wave > (size_t)CU_LDS_BYTES) --wpb;
    shm = (size_t)wpb * per_wave;
    if (shm > (size_t)CU_LDS_BYTES) return hipErrorInvalidValue;
    if (shm > 64 * 1024) return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    return hipSuccess;
}

}  // namespace

hipError_t launch_peak(int kind, int64_t threads, int iters, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_peak, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, kind, iters, out);
    return hipGetLastError();
}

hipError_t launch_thermo(const DevMech &m, int64_t n, const double *T, const double *p, int64_t ps,
                         const double *Y, int64_t ld, double *cp_k, double *h_k, double *s_k, double *g_k,
                         double *cp_mass, double *h_mass, double *rho, double *Wbar, hipStream_t st) {
    hipLaunchKernelGGL(k_thermo, dim3(grid_for(n, 256, 16)), dim3(256), 0, st, m, n, T, p, ps, Y, ld, cp_k,
                       h_k, s_k, g_k, cp_mass, h_mass, rho, Wbar);
    return hipGetLastError();
}

template <bool SRC, bool STORE, bool VAR>
hipError_t launch_wdot_tv(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                          const double *Y, int64_t ld, double *wdot, double *hrr, double *rmass, double *dTdt,
                          double *QT, double dp0dt, double *work, hipStream_t st) {
    constexpr int PPW = 2;
    constexpr int NA = SRC ? 5 : 4;
    const int nsp = pad_odd(m.ns);
    const void *fn = mixed ? (const void *)k_wdot<true, PPW, SRC, STORE, VAR> : (const void *)k_wdot<false, PPW, SRC, STORE, VAR>;
    int WPB = 4;
    size_t shm = 0;
    const hipError_t e = lds_waves(fn, (size_t)PPW * NA * nsp * sizeof(double), WPB, shm);
    if (e != hipSuccess) return e;
    const int64_t groups = (n + PPW - 1) / PPW;
    const dim3 grid(grid_for(groups, WPB, 16)), block(WPB * WAVE);
    if (mixed)
        hipLaunchKernelGGL((k_wdot<true, PPW, SRC, STORE, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, wdot, hrr,
                           rmass, dTdt, QT, dp0dt, nsp, work);
    else
        hipLaunchKernelGGL((k_wdot<false, PPW, SRC, STORE, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, wdot, hrr,
                           rmass, dTdt, QT, dp0dt, nsp, work);
    return hipGetLastError();
}

// Mechanisms with optional rate forms run the instances that evaluate them (VAR); the
// others run instances without that code (fewer registers, no per-reaction form record).
template <bool SRC, bool STORE>
hipError_t launch_wdot_t(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                         const double *Y, int64_t ld, double *wdot, double *hrr, double *rmass, double *dTdt,
                         double *QT, double dp0dt, double *work, hipStream_t st) {
    if (m.n_var)
        return launch_wdot_tv<SRC, STORE, true>(m, mixed, n, T, p, ps, Y, ld, wdot, hrr, rmass, dTdt, QT, dp0dt, work,
                                                st);
    return launch_wdot_tv<SRC, STORE, false>(m, mixed, n, T, p, ps, Y, ld, wdot, hrr, rmass, dTdt, QT, dp0dt, work, st);
}

hipError_t launch_wdot(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                       const double *Y, int64_t ld, double *wdot, double *hrr, double *rmass, double *work,
                       hipStream_t st) {
    if (work)
        return launch_wdot_t<false, true>(m, mixed, n, T, p, ps, Y, ld, wdot, hrr, rmass, nullptr, nullptr, 0.0,
                                          work, st);
    return launch_wdot_t<false, false>(m, mixed, n, T, p, ps, Y, ld, wdot, hrr, rmass, nullptr, nullptr, 0.0,
                                       nullptr, st);
}

hipError_t launch_source(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                         const double *Y, int64_t ld, double dp0dt, double *dYdt, double *dTdt, double *QT,
                         double *hrr, hipStream_t st) {
    return launch_wdot_t<true, false>(m, mixed, n, T, p, ps, Y, ld, dYdt, hrr, nullptr, dTdt, QT, dp0dt, nullptr,
                                      st);
}

template <bool VAR>
hipError_t launch_vjp_v(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                        const double *Y, int64_t ld, const double *u, const double *uh, double *gT, double *gY,
                        const double *work, hipStream_t st) {
    const int nsp = pad_odd(m.ns);
    // the stored values already carry the forward pass's precision: one stored instance
    const void *fn = work ? (const void *)k_vjp<false, true, VAR>
                          : (mixed ? (const void *)k_vjp<true, false, VAR> : (const void *)k_vjp<false, false, VAR>);
    int WPB = 4;
    size_t shm = 0;
    const hipError_t e = lds_waves(fn, (size_t)7 * nsp * sizeof(double), WPB, shm);
    if (e != hipSuccess) return e;
    const dim3 grid(grid_for(n, WPB, 16)), block(WPB * WAVE);
    if (work)
        hipLaunchKernelGGL((k_vjp<false, true, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, u, uh, gT, gY, nsp,
                           work);
    else if (mixed)
        hipLaunchKernelGGL((k_vjp<true, false, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, u, uh, gT, gY, nsp,
                           work);
    else
        hipLaunchKernelGGL((k_vjp<false, false, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, u, uh, gT, gY, nsp,
                           work);
    return hipGetLastError();
}

hipError_t launch_vjp(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                      const double *Y, int64_t ld, const double *u, const double *uh, double *gT, double *gY,
                      const double *work, hipStream_t st) {
    return m.n_var ? launch_vjp_v<true>(m, mixed, n, T, p, ps, Y, ld, u, uh, gT, gY, work, st)
                   : launch_vjp_v<false>(m, mixed, n, T, p, ps, Y, ld, u, uh, gT, gY, work, st);
}

template <bool VAR>
hipError_t launch_jvp_v(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                        const double *Y, int64_t ld, const double *vT, const double *vY, double *jh, double *jw,
                        double *wdot, hipStream_t st) {
    // one point per wavefront: the two-point form needed more than the 168 VGPRs of three
    // waves per SIMD and spilled to scratch (and its mixed-mode build returned NaN on the
    // mechanism with PLOG/Chebyshev/SRI reactions, which this form does not)
    const int nsp = pad_odd(m.ns);
    const size_t per_point = (size_t)7 * nsp * sizeof(double);
    const void *fn = mixed ? (const void *)k_jvp<true, 1, VAR> : (const void *)k_jvp<false, 1, VAR>;
    int WPB = 4;
    size_t shm = 0;
    const hipError_t e = lds_waves(fn, per_point, WPB, shm);
    if (e != hipSuccess) return e;
    const dim3 grid(grid_for(n, WPB, 16)), block(WPB * WAVE);
    if (mixed)
        hipLaunchKernelGGL((k_jvp<true, 1, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, vT, vY, jh, jw, wdot, nsp);
    else
        hipLaunchKernelGGL((k_jvp<false, 1, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, vT, vY, jh, jw, wdot, nsp);
    return hipGetLastError();
}

hipError_t launch_jvp(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                      const double *Y, int64_t ld, const double *vT, const double *vY, double *jh, double *jw,
                      double *wdot, hipStream_t st) {
    return m.n_var ? launch_jvp_v<true>(m, mixed, n, T, p, ps, Y, ld, vT, vY, jh, jw, wdot, st)
                   : launch_jvp_v<false>(m, mixed, n, T, p, ps, Y, ld, vT, vY, jh, jw, wdot, st);
}

template <int DMAX, bool VAR>
hipError_t launch_jac_seg(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                          const double *Y, int64_t ld, void *J, double *wdot, hipStream_t st) {
    const dim3 grid(grid_for(n, 1, 2)), block(JS_THREADS);
    const void *fn = mixed ? (const void *)k_jac_seg<true, DMAX, VAR> : (const void *)k_jac_seg<false, DMAX, VAR>;
    // more than 64 KB of dynamic LDS per workgroup has to be allowed explicitly
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, m.jp_lds);
    if (e != hipSuccess) return e;
    if (mixed)
        hipLaunchKernelGGL((k_jac_seg<true, DMAX, VAR>), grid, block, m.jp_lds, st, m, n, T, p, ps, Y, ld, J, wdot);
    else
        hipLaunchKernelGGL((k_jac_seg<false, DMAX, VAR>), grid, block, m.jp_lds, st, m, n, T, p, ps, Y, ld, J, wdot);
    return hipGetLastError();
}

// The reaction-table kernel with WAVES wavefronts per workgroup: as many resident
// workgroups per compute unit as its registers and LDS allow, each persistent over points.
template <bool VAR, int WAVES>
hipError_t launch_jac_rt(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                         const double *Y, int64_t ld, void *J, double *wdot, int nsp, int sr, const JacRtLayout &lay,
                         int nrp, hipStream_t st) {
    const void *fn = mixed ? (const void *)k_jac_rt<true, VAR, WAVES> : (const void *)k_jac_rt<false, VAR, WAVES>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.total);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WAVES * WAVE, lay.total);
    if (e != hipSuccess) return e;
    const dim3 grid(grid_for(n, 1, per_cu > 1 ? per_cu : 1)), block(WAVES * WAVE);
    if (mixed)
        hipLaunchKernelGGL((k_jac_rt<true, VAR, WAVES>), grid, block, lay.total, st, m, n, T, p, ps, Y, ld, J, wdot, nsp,
                           sr, lay.rows, nrp);
    else
        hipLaunchKernelGGL((k_jac_rt<false, VAR, WAVES>), grid, block, lay.total, st, m, n, T, p, ps, Y, ld, J, wdot, nsp,
                           sr, lay.rows, nrp);
    return hipGetLastError();
}

// The kernels for mechanisms the segmented plan does not take: the reaction table when it
// fits the LDS, else the row blocks that re-evaluate the reactions per block.
template <bool VAR>
hipError_t launch_jac_general(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                              const double *Y, int64_t ld, void *J, double *wdot, hipStream_t st) {
    const int nsp = pad_odd(m.ns);
    const int n1 = m.ns + 1;
    const int sr = pad_odd(n1);
    const size_t acc = sizeof(double);
    JacRtLayout lay;
    if (jac_rt_fits(m.ns, m.nr, mixed != 0, &lay)) {
        // reaction table in LDS: each reaction evaluated once per point
        const int nrp = (m.nr + 1) & ~1;
        return m.nr > 8 * WAVE ? launch_jac_rt<VAR, 16>(m, mixed, n, T, p, ps, Y, ld, J, wdot, nsp, sr, lay, nrp, st)
                               : launch_jac_rt<VAR, 8>(m, mixed, n, T, p, ps, Y, ld, J, wdot, nsp, sr, lay, nrp, st);
    }
    const size_t fixed = (size_t)(4 * nsp + 4 * (nsp + 1)) * sizeof(double);
    // rows per block: as many as fit one compute unit's LDS (one workgroup per point)
    const size_t budget = CU_LDS_BYTES - 256;
    int rb = (int)((budget > fixed ? budget - fixed : 0) / ((size_t)sr * acc));
    if (rb >= n1) rb = n1;
    if (rb < 1) return hipErrorInvalidValue;
    const size_t shm = fixed + (size_t)rb * sr * acc;
    const void *fn = mixed ? (const void *)k_jac<true, VAR> : (const void *)k_jac<false, VAR>;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    const dim3 grid(grid_for(n, 1, 1)), block(KJ_WAVES * WAVE);
    if (mixed)
        hipLaunchKernelGGL((k_jac<true, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, J, wdot, nsp, sr, rb);
    else
        hipLaunchKernelGGL((k_jac<false, VAR>), grid, block, shm, st, m, n, T, p, ps, Y, ld, J, wdot, nsp, sr, rb);
    return hipGetLastError();
}

hipError_t launch_jac(const DevMech &m, int mixed, int64_t n, const double *T, const double *p, int64_t ps,
                      const double *Y, int64_t ld, void *J, double *wdot, hipStream_t st) {
    if (m.jp_ok && m.jp_lds <= JS_MAX_LDS) {
        // the instance with the fewest gather rounds that covers the plan (every wavefront
        // runs that many rounds in straight-line code; the plan pads with no-op rounds)
        const int r = m.jp_rmax;
        if (m.n_var) {   // mechanisms with optional rate forms: fewer instances
            if (r <= 8) return launch_jac_seg<8, true>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
            if (r <= 12) return launch_jac_seg<12, true>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
            if (r <= 16) return launch_jac_seg<16, true>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
            return launch_jac_seg<JS_DMAX, true>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        }
        if (r <= 6) return launch_jac_seg<6, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 8) return launch_jac_seg<8, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 10) return launch_jac_seg<10, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 11) return launch_jac_seg<11, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 12) return launch_jac_seg<12, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 13) return launch_jac_seg<13, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 14) return launch_jac_seg<14, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 15) return launch_jac_seg<15, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 16) return launch_jac_seg<16, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 18) return launch_jac_seg<18, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 20) return launch_jac_seg<20, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        if (r <= 22) return launch_jac_seg<22, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
        return launch_jac_seg<JS_DMAX, false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
    }
    return m.n_var ? launch_jac_general<true>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st)
                   : launch_jac_general<false>(m, mixed, n, T, p, ps, Y, ld, J, wdot, st);
}

// Copies the state (T, Y with leading dimension lds) to (T, Y with leading dimension ldd).
__global__ __launch_bounds__(256) void k_state_copy(int64_t n, int ns, const double *__restrict__ Ts,
                                                    const double *__restrict__ Ysrc, int64_t lds_,
                                                    double *__restrict__ Td, double *__restrict__ Yd, int64_t ldd) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * (ns + 1);
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, i = e - c * n;
        if (c == 0) Td[i] = Ts[i];
        else Yd[(c - 1) * ldd + i] = Ysrc[(c - 1) * lds_ + i];
    }
}

hipError_t launch_reactor(const DevMech &m, int mixed, int64_t n, double *T, const double *p, int64_t ps, double *Y,
                          int64_t ld, double dt, int nsub, void *work, hipStream_t st) {
    const int ns = m.ns, N = ns + 1;
    const RosLayout L = ros_layout(ns, mixed, n);
    char *w = (char *)work;
    void *Jb = w + L.J;
    double *Mb = (double *)(w + L.M), *wd = (double *)(w + L.wd), *k1 = (double *)(w + L.k1);
    int *piv = (int *)(w + L.piv);
    double *Tw = (double *)(w + L.Tw), *Yw = (double *)(w + L.Yw), *Ts = (double *)(w + L.Ts);
    double *Ys = (double *)(w + L.Ys), *fT = (double *)(w + L.fT), *fY = (double *)(w + L.fY);
    const dim3 cgrid(grid_for(n * N, 256, 8)), cblock(256);
    hipLaunchKernelGGL(k_state_copy, cgrid, cblock, 0, st, n, ns, T, Y, ld, Tw, Yw, (int64_t)n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t vec_lds = (size_t)(5 * N + ROS_THREADS / WAVE) * sizeof(double) + (size_t)((N + 1) & ~1) * sizeof(int);
    const size_t mat_lds = (size_t)N * N * sizeof(double);
    const int in_lds = vec_lds + mat_lds <= (size_t)64 * 1024;
    const size_t shm = vec_lds + (in_lds ? mat_lds : 0);
    const void *fn = mixed ? (const void *)k_ros_lu<true> : (const void *)k_ros_lu<false>;
    if (shm > (size_t)CU_LDS_BYTES) return hipErrorInvalidValue;
    if (shm > 64 * 1024) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    const dim3 grid(grid_for(n, 1, 8)), block(ROS_THREADS);
    const size_t fshm = (size_t)N * sizeof(double) + (size_t)N * sizeof(int);
    const double h = dt / nsub;
    // up to 56 unknowns: a wavefront per point with the matrix in registers
    const dim3 wgrid((unsigned)((n + 3) / 4)), wblock(4 * WAVE);
    for (int s = 0; s < nsub; ++s) {
        e = launch_jac(m, mixed, n, Tw, p, ps, Yw, n, Jb, wd, st);
        if (e != hipSuccess) return e;
        if (N <= 56) {
#define CRF_ROS_W(NMX)                                                                                              \
    do {                                                                                                            \
        if (mixed)                                                                                                  \
            hipLaunchKernelGGL((k_ros_lu_w<true, NMX>), wgrid, wblock, 0, st, m, n, Tw, p, ps, Yw, (int64_t)n, Jb, wd, \
                               h, Mb, piv, k1, Ts, Ys);                                                             \
        else                                                                                                        \
            hipLaunchKernelGGL((k_ros_lu_w<false, NMX>), wgrid, wblock, 0, st, m, n, Tw, p, ps, Yw, (int64_t)n, Jb,    \
                               wd, h, Mb, piv, k1, Ts, Ys);                                                         \
        e = hipGetLastError();                                                                                      \
        if (e != hipSuccess) return e;                                                                              \
        e = launch_source(m, mixed, n, Ts, p, ps, Ys, n, 0.0, fY, fT, nullptr, nullptr, st);                        \
        if (e != hipSuccess) return e;                                                                              \
        hipLaunchKernelGGL((k_ros_finish_w<NMX>), wgrid, wblock, 0, st, m, n, Tw, Yw, (int64_t)n, Mb, piv, k1, fT,    \
                           fY, h);                                                                                  \
    } while (0)
            if (N <= 16) CRF_ROS_W(16);
            else if (N <= 40) CRF_ROS_W(40);
            else CRF_ROS_W(56);
#undef CRF_ROS_W
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            continue;
        }
        if (mixed)
            hipLaunchKernelGGL((k_ros_lu<true>), grid, block, shm, st, m, n, Tw, p, ps, Yw, (int64_t)n, Jb, wd, h, Mb,
                               piv, k1, Ts, Ys, in_lds);
        else
            hipLaunchKernelGGL((k_ros_lu<false>), grid, block, shm, st, m, n, Tw, p, ps, Yw, (int64_t)n, Jb, wd, h, Mb,
                               piv, k1, Ts, Ys, in_lds);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_source(m, mixed, n, Ts, p, ps, Ys, n, 0.0, fY, fT, nullptr, nullptr, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_ros_finish, grid, block, fshm, st, m, n, Tw, Yw, (int64_t)n, Mb, piv, k1, fT, fY, h);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_state_copy, cgrid, cblock, 0, st, n, ns, Tw, Yw, (int64_t)n, T, Y, ld);
    return hipGetLastError();
}

// Scratch of the allocation-free reactor entry point (crf_reactor_step_static): one copy per
// device, held for the life of the process.  Host code never uses the array's name as an
// address (on the host it is a stand-in symbol): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is passed to
// the kernels like a caller's workspace.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void **out) {
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_reactor_static(const DevMech &m, int mixed, int64_t n, double *T, const double *p, int64_t ps,
                                 double *Y, int64_t ld, double dt, int nsub, hipStream_t st) {
    if (reactor_work_bytes(m.ns, mixed, n) > STATIC_SCRATCH_BYTES) return hipErrorInvalidValue;
    void *work = nullptr;
    const hipError_t e = static_scratch(&work);
    if (e != hipSuccess) return e;
    return launch_reactor(m, mixed, n, T, p, ps, Y, ld, dt, nsub, work, st);
}

hipError_t launch_transport(const DevMech &m, int mixed, int64_t n, const double *T, const double *p,
                            int64_t ps, const double *Y, int64_t ld, double *mu, double *lam, double *Dmix,
                            hipStream_t st) {
    // Point tiles while a tile's species rows fit one compute unit's LDS: 4 wavefronts per
    // workgroup while four or more workgroups fit, else 8 (two or three) or 16 (one).
    const int rows = m.ns + 1;
    const int W = tile_transport_waves(rows, mixed != 0);
    if (W) {
        const size_t tshm = tile_transport_lds(rows, mixed, W);
        const void *fn = nullptr;
        if (W == 4) fn = mixed ? (const void *)k_transport_tile<true, 4> : (const void *)k_transport_tile<false, 4>;
        else if (W == 8) fn = mixed ? (const void *)k_transport_tile<true, 8> : (const void *)k_transport_tile<false, 8>;
        else fn = mixed ? (const void *)k_transport_tile<true, 16> : (const void *)k_transport_tile<false, 16>;
        if (tshm > 64 * 1024) {
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tshm);
            if (e != hipSuccess) return e;
        }
        const int64_t tiles = (n + TT_P - 1) / TT_P;
        const dim3 grid((unsigned)tiles), block(W * WAVE);
#define CRF_TT_LAUNCH(MX, WW) hipLaunchKernelGGL((k_transport_tile<MX, WW>), grid, block, tshm, st, m, n, T, p, ps, Y, ld, mu, lam, Dmix, rows)
        if (W == 4) { if (mixed) CRF_TT_LAUNCH(true, 4); else CRF_TT_LAUNCH(false, 4); }
        else if (W == 8) { if (mixed) CRF_TT_LAUNCH(true, 8); else CRF_TT_LAUNCH(false, 8); }
        else { if (mixed) CRF_TT_LAUNCH(true, 16); else CRF_TT_LAUNCH(false, 16); }
#undef CRF_TT_LAUNCH
        return hipGetLastError();
    }
    // larger mechanisms: two points per wavefront, per-point species arrays in LDS
    constexpr int PPW = 2;
    const int nsp = pad_odd(m.ns + 1);   // room for the dummy species of the pair schedule
    const void *fn = mixed ? (const void *)k_transport<true, PPW> : (const void *)k_transport<false, PPW>;
    int WPB = 4;
    size_t shm = 0;
    const hipError_t e = lds_waves(fn, (size_t)PPW * 4 * nsp * sizeof(double), WPB, shm);
    if (e != hipSuccess) return e;
    const int64_t groups = (n + PPW - 1) / PPW;
    const dim3 grid(grid_for(groups, WPB, 16)), block(WPB * WAVE);
    if (mixed)
        hipLaunchKernelGGL((k_transport<true, PPW>), grid, block, shm, st, m, n, T, p, ps, Y, ld, mu, lam, Dmix, nsp);
    else
        hipLaunchKernelGGL((k_transport<false, PPW>), grid, block, shm, st, m, n, T, p, ps, Y, ld, mu, lam, Dmix, nsp);
    return hipGetLastError();
}

}  // namespace crf
