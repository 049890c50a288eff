// Device-side building blocks of the TENO5-LAD Euler right-hand side
// (Peng et al., arXiv:2003.09145) for gfx950.
//
// Every function here evaluates its formula in one fixed operation order
// (no FMA contraction: the library is built with -ffp-contract=off), so that
// the GPU result is reproducible bit for bit and every cutoff decision is a
// deterministic function of the input state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "teno_index.hpp"

namespace teno {

// Scheme parameters as the kernels see them (copied from teno_grid).
struct SchemeParams {
    double gamma;
    double ct_fixed;
    double H;
    double eps;
    int32_t scheme;  // 0 LAD, 1 fixed C_T, 2 linear (all stencils kept), 3 TENO5-A
    int32_t Bl, Bu;
    int32_t kA_nan;  // TENO5-A: exponent taken by a non-finite sensor, floor(a1 - a2)
    int32_t theta_cut;  // LAD: 1 sets theta = 0 where max chi~ > H (eq 3.2, cut form)
    double bu_bl;    // LAD: (double)(B_u - B_l) (host-converted)
    double a1, a2;   // TENO5-A: alpha_1, alpha_2 of eq 2.16
    double cr;       // TENO5-A: C_r of eq 2.17
    double epsA;     // TENO5-A: 0.9 C_r / (1 - 0.9 C_r) xi^2 of eq 2.18 (host-evaluated)
};

// Ladder array of Sec. 3 eq 3.3 as decimal literals: kLadder[k] = 10^-k, so
// C_T = Lad(m) = kLadder[m] (eq 3.4).
__constant__ const double kLadder[21] = {
    1e0,  1e-1,  1e-2,  1e-3,  1e-4,  1e-5,  1e-6,  1e-7,  1e-8,  1e-9, 1e-10,
    1e-11, 1e-12, 1e-13, 1e-14, 1e-15, 1e-16, 1e-17, 1e-18, 1e-19, 1e-20};

// Coefficients of Sec. 2: the FP64 quotients of the printed integer ratios.
constexpr double kB13_12 = 13.0 / 12.0;  // eq 2.9-2.11
constexpr double kB1_4 = 0.25;
constexpr double kC1_3 = 1.0 / 3.0;      // eq 2.4-2.6
constexpr double kC7_6 = 7.0 / 6.0;
constexpr double kC11_6 = 11.0 / 6.0;
constexpr double kC1_6 = 1.0 / 6.0;
constexpr double kC5_6 = 5.0 / 6.0;
constexpr double kLin0 = 0.1, kLin1 = 0.6, kLin2 = 0.3;  // linear weights

// ---------------------------------------------------------------------------
// Correctly rounded FP64 division and square root.
//
// The compiler's FP64 a / b sequence on gfx950 is faithful but not always
// correctly rounded (for instance 0.3499999999999998 / 0.12499999999999993
// returns 2.8 instead of 2.8000000000000003), and the method's cutoff
// decisions must match an IEEE-754 evaluation bit for bit.  Both wrappers take
// the hardware result q (within one ulp), form the remainder with one FMA --
// exact, because the remainder of a faithful quotient (a - q b) or root
// (x - s^2) is representable -- and move q to its neighbour when the exact
// value lies beyond the midpoint (ties to even for the quotient; a square
// root of a double is never a midpoint).  Operands are restricted to
// [2^-900, 2^900] in magnitude for the correction (no under/overflow in the
// remainder); outside it the hardware value is returned.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double step_toward(double q, bool up) {
    const long long bits = __double_as_longlong(q);
    return __longlong_as_double(bits + (((q > 0.0) == up) ? 1ll : -1ll));
}

__device__ __forceinline__ bool in_safe_range(double v) {
    const double av = fabs(v);
    return av >= 0x1p-900 && av <= 0x1p900;
}

// Sufficient test that q = RN(a / b) given r = RN(a - q b): |a/b - q| <
// ulp(q)/2 with both neighbours of q one ulp away makes q the nearest
// double.  q = mq 2^eq with |mq| in (1/2, 1) excludes zero, powers of two,
// infinities and NaN; ulp(q)/2 |b| = |b| 2^(eq - 54) is computed exactly when
// it is a normal number (checked; for a subnormal q the bound is smaller than
// the true half-ulp, which only makes the test stricter); and rounding is
// monotone, so |r| below the bound implies the exact remainder is below it,
// whether or not r itself is exact.  Signed zeros and operands outside the
// normal range therefore never pass and take the exact path.
__device__ __forceinline__ bool quotient_is_nearest(double q, double b, double r) {
    int eq;
    const double mq = frexp(q, &eq);
    const double hb = ldexp(fabs(b), eq - 54);
    return fabs(r) < hb && hb >= 0x1p-1000 && fabs(mq) > 0.5;
}

__device__ __forceinline__ double cr_div(double a, double b) {
    const double q = a / b;
    const double r = __builtin_fma(-q, b, a);  // a - q b, exact in the safe range
    if (quotient_is_nearest(q, b, r)) return q;
    if (!(in_safe_range(a) && in_safe_range(b) && in_safe_range(q))) return q;
    if (r == 0.0) return q;
    const bool up = (r > 0.0) == (b > 0.0);     // true quotient above q
    const double qn = step_toward(q, up);
    const double h = 0.5 * ((qn - q) * b);      // remainder at the midpoint, exact
    const double ar = fabs(r), ah = fabs(h);
    if (ar > ah) return qn;
    if (ar == ah) return (__double_as_longlong(q) & 1ll) ? qn : q;
    return q;
}

__device__ __forceinline__ double cr_sqrt_exact(double x) {
    const double s = sqrt(x);
    if (!(x >= 0x1p-900 && x <= 0x1p900)) return s;
    const double r = __builtin_fma(-s, s, x);  // x - s^2, exact
    if (r == 0.0) return s;
    const bool up = r > 0.0;
    const double sn = step_toward(s, up);
    const double sg = s * (sn - s);             // exact: the gap is a power of two
    if (up) return (r > sg) ? sn : s;
    return (r <= sg) ? sn : s;
}

// sqrt(x) correctly rounded.  In the safe range the root comes from the
// hardware reciprocal square root refined by one Goldschmidt and two Newton
// steps (no scaling is needed there) and is accepted when
// |x - s^2| < ulp(s) (s - ulp(s)): a root error of half an ulp or more would
// make |x - s^2| >= ulp(s) (s - ulp(s)/4), and rounding is monotone, so the
// accepted s is the nearest double (s not a power of two, both neighbours one
// ulp away; the bound is exact and normal).  Everything else takes the exact
// neighbour test on the compiler's root.
// Fast phase: *s is the refined root (for x outside the safe range, any
// value); true when it is certified.  The exact phase is cr_sqrt_exact.
__device__ __forceinline__ bool sqrt_fast(double x, double* sout) {
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y;
    double h = 0.5 * y;
    const double e = __builtin_fma(-h, s, 0.5);
    s = __builtin_fma(s, e, s);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-s, s, x);
    s = __builtin_fma(d, h, s);
    d = __builtin_fma(-s, s, x);
    s = __builtin_fma(d, h, s);
    const double r = __builtin_fma(-s, s, x);
    int es;
    const double ms = frexp(s, &es);
    const double u = ldexp(1.0, es - 53);  // ulp(s)
    *sout = s;
    return (x >= 0x1p-900 && x <= 0x1p900) && fabs(r) < ldexp(s - u, es - 53) && ms > 0.5;
}
__device__ __forceinline__ double cr_sqrt(double x) {
    double s;
    if (sqrt_fast(x, &s)) return s;
    return cr_sqrt_exact(x);
}

// Reciprocal to within a few ulp: hardware estimate plus two Newton steps.
__device__ __forceinline__ double rcp_nr(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-b, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Correctly rounded a / b from rb = rcp_nr(b): q0 = a rb, one Markstein step
// q1 = q0 + (a - q0 b) rb (faithful), then the exact-remainder correction of
// cr_div.  Outside the safe range it defers to cr_div.
//
// Split in two phases so that several independent divisions share one
// (rarely taken) correction branch: div_r_fast forms q1 and its remainder and
// reports whether the fast test already certifies q1; div_r_fix corrects a
// quotient the test did not certify.
__device__ __forceinline__ bool div_r_fast(double a, double b, double rb, double* q, double* r) {
    const double q0 = a * rb;
    const double e = __builtin_fma(-q0, b, a);
    *q = __builtin_fma(e, rb, q0);
    *r = __builtin_fma(-*q, b, a);  // exact in the safe range
    return quotient_is_nearest(*q, b, *r);
}
__device__ __forceinline__ double div_r_fix(double a, double b, double q, double r) {
    if (!(in_safe_range(a) && in_safe_range(b) && in_safe_range(q))) return cr_div(a, b);
    if (r == 0.0) return q;
    const bool up = (r > 0.0) == (b > 0.0);
    const double qn = step_toward(q, up);
    const double h = 0.5 * ((qn - q) * b);
    const double ar = fabs(r), ah = fabs(h);
    if (ar > ah) return qn;
    if (ar == ah) return (__double_as_longlong(q) & 1ll) ? qn : q;
    return q;
}
__device__ __forceinline__ double cr_div_r(double a, double b, double rb) {
    double q, r;
    if (div_r_fast(a, b, rb, &q, &r)) return q;
    return div_r_fix(a, b, q, r);
}
// q[i] = a[i] / b correctly rounded for N independent dividends.
template <int N>
__device__ __forceinline__ void cr_div_r_n(const double (&a)[N], double b, double rb,
                                           double (&q)[N]) {
    double r[N];
    bool ok[N];
    bool all = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        ok[i] = div_r_fast(a[i], b, rb, &q[i], &r[i]);
        all = all && ok[i];
    }
    if (!all) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (!ok[i]) q[i] = div_r_fix(a[i], b, q[i], r[i]);
    }
}

// TENO weights of eq 2.15 for each cutoff mask, omega_k = delta_k c_k / D with
// D = (delta_0 c_0 + delta_1 c_1) + delta_2 c_2, folded at compile time in
// IEEE round-to-nearest (the same operations and order as the runtime form).
constexpr double omega_of(int mask, int k) {
    const double d0 = (double)(mask & 1), d1 = (double)((mask >> 1) & 1),
                 d2 = (double)((mask >> 2) & 1);
    const double D = (d0 * 0.1 + d1 * 0.6) + d2 * 0.3;
    const double dk = (k == 0) ? d0 : (k == 1) ? d1 : d2;
    const double ck = (k == 0) ? 0.1 : (k == 1) ? 0.6 : 0.3;
    return mask == 0 ? 0.0 : (dk * ck) / D;
}
__constant__ const double kOmega[8][3] = {
    {omega_of(0, 0), omega_of(0, 1), omega_of(0, 2)},
    {omega_of(1, 0), omega_of(1, 1), omega_of(1, 2)},
    {omega_of(2, 0), omega_of(2, 1), omega_of(2, 2)},
    {omega_of(3, 0), omega_of(3, 1), omega_of(3, 2)},
    {omega_of(4, 0), omega_of(4, 1), omega_of(4, 2)},
    {omega_of(5, 0), omega_of(5, 1), omega_of(5, 2)},
    {omega_of(6, 0), omega_of(6, 1), omega_of(6, 2)},
    {omega_of(7, 0), omega_of(7, 1), omega_of(7, 2)}};

// Decision constants of one launch.  The LAD ladder index m = B_l +
// floor(theta (B_u - B_l)), theta = 1 / (1 + x / H) with x = max_k chi~_k
// (eq 3.1-3.4), is formed from an approximate x and theta and trusted when
// y = theta (B_u - B_l) lies farther than ymarg from an integer: the literal
// chain of correctly rounded operations differs from it by a few ulp.
struct DecisionConsts {
    double inv_h;          // 1 / H
    double nthr_d;         // B_u - B_l
    double ymarg;          // kDecisionMargin (B_u - B_l)
    double ct_hi;          // largest C_T the scheme can use (10^-B_l or C_T)
    double ct_lo;          // smallest C_T (10^-B_u or C_T)
    int32_t nthr;          // B_u - B_l
    int32_t literal;       // 1: evaluate every decision with the literal formula
    int32_t need_m;        // 1: the ladder index is wanted (decision dumps)
    int32_t pad_;
    // Smooth-stencil bound: when tau <= smooth_t (min_k beta_k + eps), every
    // chi~_k = tau / (beta_k + eps) is at most smooth_t (to rounding), so each
    // gamma_k of eq 2.8 lies in [1, (1 + smooth_t)^6] and every chi_k is at
    // least 1 / (1 + 2 (1 + smooth_t)^6), which the host chooses above the
    // largest cutoff ct_hi: all three stencils are kept, whatever the ladder
    // index.  Negative: no such bound (never satisfied).
    double smooth_t;
    // host products of the margins below: ct_hi (1 + margin) and ct_lo (1 -
    // margin) (kept out of the kernels' loops, where the compiler would
    // re-form them for every characteristic field)
    double hi_fac, lo_fac;
    // cut form of theta: max chi~ above h_hi = H (1 + margin) is certainly over
    // H (m = B_l), at or above h_lo = H (1 - margin) it is not trusted; NaN for
    // the printed form, so that neither test holds
    double h_hi, h_lo;
};

// Relative margin inside which an approximate decision value is not trusted
// (the approximate path differs from the literal one by < 200 ulp).
constexpr double kDecisionMargin = 0x1p-40;

// The literal decision of eq 2.8-2.14 / eq 3.1-3.4 (oracle operation order,
// correctly rounded divisions).  Returns m | (mask << 5).
// TENO5-A cutoff of eq 2.16-2.18 on the reconstruction's own values (a..e) =
// (f_{i-2} .. f_{i+2}): sensors eta_j at j = i-1, i, i+1 (eq 2.18, denominator
// df_{j+1/2}^2 + df_{j-1/2}^2), eta_{i+1/2} = their minimum, m = 1 - min(1,
// eta / C_r), g = (1 - m)^4 (1 + 4 m), beta = alpha_1 - alpha_2 (1 - g),
// C_T = 10^-floor(beta).  Operation order of the oracle; *k = floor(beta).
__device__ __forceinline__ double teno5a_cutoff(const SchemeParams& S, double a, double b,
                                                double c, double d, double e, int* k) {
    const double df0 = b - a, df1 = c - b, df2 = d - c, df3 = e - d;
    // 2 x and 4 x are exact, so the fused forms below round exactly as the
    // oracle's product-then-add
    const double eta0 =
        cr_div(__builtin_fma(2.0, fabs(df1 * df0), S.epsA), (df1 * df1 + df0 * df0) + S.epsA);
    const double eta1 =
        cr_div(__builtin_fma(2.0, fabs(df2 * df1), S.epsA), (df2 * df2 + df1 * df1) + S.epsA);
    const double eta2 =
        cr_div(__builtin_fma(2.0, fabs(df3 * df2), S.epsA), (df3 * df3 + df2 * df2) + S.epsA);
    double eh = eta0;
    if (eta1 < eh) eh = eta1;
    if (eta2 < eh) eh = eta2;
    const double q = cr_div(eh, S.cr);
    const double mA = 1.0 - (q < 1.0 ? q : 1.0);
    const double om = 1.0 - mA;
    const double om2 = om * om;
    const double g = (om2 * om2) * __builtin_fma(4.0, mA, 1.0);
    const double bA = S.a1 - S.a2 * (1.0 - g);
    const int kk = (bA >= 0.0) ? (int)floor(bA) : S.kA_nan;
    *k = kk;
    return kLadder[kk];
}

// A5: the launch runs TENO5-A (scheme 3); its cutoff code is compiled only
// into the A5 instantiations, so the other schemes' kernels do not carry it.
template <bool A5>
__device__ __forceinline__ uint32_t teno5_decide_literal(const SchemeParams& S, double beta0,
                                                      double beta1, double beta2, double a,
                                                      double b, double c, double d, double e) {
    const double tau = fabs(beta2 - beta0);
    const double t0 = cr_div(tau, beta0 + S.eps);
    const double t1 = cr_div(tau, beta1 + S.eps);
    const double t2 = cr_div(tau, beta2 + S.eps);
    double y, y2;
    y = 1.0 + t0;
    y2 = y * y;
    const double g0 = (y2 * y2) * y2;
    y = 1.0 + t1;
    y2 = y * y;
    const double g1 = (y2 * y2) * y2;
    y = 1.0 + t2;
    y2 = y * y;
    const double g2 = (y2 * y2) * y2;
    const double sum = (g0 + g1) + g2;
    const double chi0 = cr_div(g0, sum);
    const double chi1 = cr_div(g1, sum);
    const double chi2 = cr_div(g2, sum);
    double ct = 0.0;
    int m = 0;
    if (S.scheme == 0) {
        double x = t0;
        if (t1 > x) x = t1;
        if (t2 > x) x = t2;
        if (S.theta_cut && x > S.H) {
            m = S.Bl;  // theta = 0: the stencil counts as discontinuous
        } else {
            const double theta = cr_div(1.0, 1.0 + cr_div(x, S.H));
            if (theta >= 0.0)
                m = S.Bl + (int)floor(theta * S.bu_bl);
            else
                m = S.Bl;
        }
        ct = kLadder[m];
    } else if (A5) {
        ct = teno5a_cutoff(S, a, b, c, d, e, &m);
    } else {
        ct = S.ct_fixed;
    }
    const uint32_t mask = (chi0 < ct ? 0u : 1u) | (chi1 < ct ? 0u : 2u) | (chi2 < ct ? 0u : 4u);
    return (uint32_t)m | (mask << 5);
}

// One scalar TENO5 reconstruction of the face value from (a..e) =
// (f_{i-2} .. f_{i+2}): smoothness indicators (eq 2.9-2.12), scale
// separation (eq 2.8, 2.13), cutoff (eq 2.14) with C_T from the LAD mapping
// (eq 3.1-3.4), weights (eq 2.15) and combination (eq 2.4-2.7).
//
// The cutoff flags and the ladder index are discrete functions of the
// literal formula.  They are first evaluated with approximate reciprocals;
// if any decision value lies within kDecisionMargin of its threshold (or is
// not finite) the lane re-evaluates the literal formula, so the decisions
// equal the literal ones exactly.  The flux itself is the literal
// combination with the eq 2.15 weights of the chosen mask.
// *code receives m | (mask << 5).
template <bool A5>
__device__ __forceinline__ double teno5_rec_fast(const SchemeParams& S, const DecisionConsts& K,
                                                 const double* __restrict__ omega_lds,
                                                 double a, double b, double c, double d,
                                                 double e, uint32_t* code) {
    // sums of products as fused multiply-adds, in the oracle's order; a - 2 b
    // and a - 4 b are single roundings either way (2 b and 4 b are exact for
    // |b| below 2^1021), so they are fused here too
    const double s01 = __builtin_fma(-2.0, b, a) + c;
    const double s02 = __builtin_fma(3.0, c, __builtin_fma(-4.0, b, a));
    const double s11 = __builtin_fma(-2.0, c, b) + d;
    const double s12 = b - d;
    const double s21 = __builtin_fma(-2.0, d, c) + e;
    const double s22 = __builtin_fma(3.0, c, __builtin_fma(-4.0, d, e));
    const double beta0 = __builtin_fma(kB13_12 * s01, s01, kB1_4 * (s02 * s02));
    const double beta1 = __builtin_fma(kB13_12 * s11, s11, kB1_4 * (s12 * s12));
    const double beta2 = __builtin_fma(kB13_12 * s21, s21, kB1_4 * (s22 * s22));

    uint32_t cd;
    if (S.scheme == 2) {
        cd = 7u << 5;
    } else {
        bool sure = K.literal == 0;
        uint32_t m = 0, mask = 7u;
        const double tau = fabs(beta2 - beta0);
        const double be0 = beta0 + S.eps, be1 = beta1 + S.eps, be2 = beta2 + S.eps;
        // Smooth test tau <= smooth_t (min_k beta_k + eps), one compare per
        // stencil: x -> RN(x + eps) and x -> RN(smooth_t x) are monotone
        // (smooth_t > 0; a negative smooth_t fails every form), so the rounded
        // bound at the smallest beta_k is the smallest of the three bounds.
        // A NaN beta_k fails its compare, and it needs a NaN stencil value,
        // which makes beta_0 or beta_2 NaN and so tau NaN as well.
        const bool smooth = tau <= K.smooth_t * be0 && tau <= K.smooth_t * be1 &&
                            tau <= K.smooth_t * be2;
        if (sure && K.need_m == 0 && smooth) {
            // smooth stencil: all kept (no reciprocal, no gamma_k)
        } else if (sure) {
            // Approximate gamma_k (eq 2.8) from approximate chi~_k = tau / (beta_k + eps).
            const double t0 = tau * rcp_nr(be0);
            const double t1 = tau * rcp_nr(be1);
            const double t2 = tau * rcp_nr(be2);
            double y, y2;
            y = 1.0 + t0;
            y2 = y * y;
            const double g0 = (y2 * y2) * y2;
            y = 1.0 + t1;
            y2 = y * y;
            const double g1 = (y2 * y2) * y2;
            y = 1.0 + t2;
            y2 = y * y;
            const double g2 = (y2 * y2) * y2;
            const double sum = (g0 + g1) + g2;
            // chi_k = g_k / sum against the extreme cutoffs: a flag that is the
            // same for every rung of the ladder needs no ladder index.  TENO5-A
            // evaluates its cutoff exactly and uses it for both bounds.
            double chi_hi = K.ct_hi, chi_lo = K.ct_lo;
            if (A5) {
                int kA;
                chi_hi = chi_lo = teno5a_cutoff(S, a, b, c, d, e, &kA);
                m = (uint32_t)kA;
            }
            const double hi = (A5 ? chi_hi * (1.0 + kDecisionMargin) : K.hi_fac) * sum;
            const double lo = (A5 ? chi_lo * (1.0 - kDecisionMargin) : K.lo_fac) * sum;
            const bool k0 = g0 >= hi, k1 = g1 >= hi, k2 = g2 >= hi;
            const bool c0 = g0 < lo, c1 = g1 < lo, c2 = g2 < lo;
            sure = isfinite(sum) && (k0 || c0) && (k1 || c1) && (k2 || c2);
            mask = (k0 ? 1u : 0u) | (k1 ? 2u : 0u) | (k2 ? 4u : 0u);
            if (S.scheme == 0 && (K.need_m || !sure)) {
                // ladder index from approximate x and theta.  A NaN t_k makes
                // sum NaN, which already sends the lane to the literal
                // formula; the clamp keeps the table index in range for any x.
                const double x = fmax(fmax(t0, t1), t2);
                const double y = rcp_nr(__builtin_fma(x, K.inv_h, 1.0)) * K.nthr_d;
                const double fl = floor(y);
                const double fr = y - fl;
                bool msure =
                    K.nthr == 0 || (isfinite(x) && fr > K.ymarg && fr < 1.0 - K.ymarg);
                m = (uint32_t)S.Bl + (uint32_t)(int)fmin(fmax(fl, 0.0), K.nthr_d);
                // cut form of theta: x certainly over H gives B_l; x within
                // the margin of H takes the literal formula
                if (x > K.h_hi) {
                    m = (uint32_t)S.Bl;
                    msure = true;
                } else if (x >= K.h_lo) {
                    msure = false;
                }
                if (!sure) {
                    const double ct = kLadder[m];
                    const double rs = rcp_nr(sum);
                    const double x0 = g0 * rs, x1 = g1 * rs, x2 = g2 * rs;
                    const double band = kDecisionMargin * ct;
                    sure = isfinite(sum) && fabs(x0 - ct) > band && fabs(x1 - ct) > band &&
                           fabs(x2 - ct) > band;
                    mask = (x0 < ct ? 0u : 1u) | (x1 < ct ? 0u : 2u) | (x2 < ct ? 0u : 4u);
                }
                sure = sure && msure;
            }
        }
        cd = m | (mask << 5);
        if (!sure) cd = teno5_decide_literal<A5>(S, beta0, beta1, beta2, a, b, c, d, e);
    }
    *code = cd;
    const uint32_t mask = cd >> 5;
    const double f0 = __builtin_fma(kC11_6, c, __builtin_fma(kC1_3, a, -kC7_6 * b));
    const double f1 = __builtin_fma(kC1_3, d, __builtin_fma(-kC1_6, b, kC5_6 * c));
    const double f2 = __builtin_fma(-kC1_6, e, __builtin_fma(kC1_3, c, kC5_6 * d));
    const double* w = omega_lds + 3 * mask;
    return __builtin_fma(w[2], f2, __builtin_fma(w[0], f0, w[1] * f1));
}

// Local component order of a sweep along DIR: rho, normal momentum, the
// tangential momenta in increasing axis order, E.
template <int ND, int DIR>
struct LocalOrder {
    static constexpr int NC = ND + 2;
    __device__ static constexpr int nat(int q) {
        // q = 0 -> 0; q = 1 -> 1 + DIR; q = 2..ND -> tangential axes; q = NC-1 -> NC-1
        return q == 0 ? 0
               : q == 1 ? 1 + DIR
               : q == NC - 1 ? NC - 1
               : 1 + ((q - 2) < DIR ? (q - 2) : (q - 1));
    }
    // tangential axis index of local tangential slot k = 1 .. ND-1
    __device__ static constexpr int tan_axis(int k) { return (k - 1) < DIR ? (k - 1) : k; }
};

}  // namespace teno
