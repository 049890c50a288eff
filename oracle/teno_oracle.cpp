/*
 * TENO5-LAD reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what the GPU path computes:
 * the semi-discrete Euler right-hand side with characteristic-wise TENO5
 * reconstruction of global Lax-Friedrichs split fluxes, the locally adaptive
 * cutoff C_T of Peng, Li, Shen, Liu and Zhang (arXiv:2003.09145, "An
 * efficient targeted ENO scheme with local adaptive dissipation for
 * compressible flow simulation"), and SSP-RK3 time stepping.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  The product path never does, and this file
 * shares no code, header or table with it.
 *
 * Build: g++ -O2 -ffp-contract=off -mfma -fopenmp (never -ffast-math), so every
 * + - * / sqrt below is exactly one IEEE-754 binary64 operation, evaluated in
 * the order written (left to right unless parenthesised), and every fmadd is
 * one correctly rounded fused multiply-add (std::fma).
 *
 * The scalar type is a template parameter so that a forward-mode dual number
 * can run through the same code (Jacobian-vector products for the adjoint
 * checks).  Every discrete decision (cutoff flags, ladder index, max) is taken
 * on real parts only.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - the characteristic projection uses the Roe average of the two cells next
 *    to the face and the standard Euler eigenvectors normalised as below;
 *  - "global" Lax-Friedrichs: one alpha per direction per RHS evaluation,
 *    the max over interior cells of |u_d| + c, shared by all fields;
 *  - the f^- reconstruction uses the mirrored stencil (i+3 ... i-1);
 *  - the chi-tilde of the LAD function and gamma_k share one epsilon;
 *  - 3D time step: dt = sigma / (a_x/dx + a_y/dy + a_z/dz);
 *  - ghost cells: periodic wrap, zero-gradient copy, or mirror with the
 *    normal momentum negated (reflecting wall), 3 per side; with per-side
 *    boundaries also a fixed state, chosen along the boundary by a split
 *    that may move in time (evaluated at the stage times t, t + dt,
 *    t + dt/2);
 *  - the gravity source of the Rayleigh-Taylor problem is added after the
 *    flux differences;
 *  - the LAD sensor theta of eq 3.2 as printed, 1 / (1 + x / H) with x the
 *    largest chi-tilde_k, or (theta_form 1) that form cut to 0 wherever
 *    x > H: Sec. 3 calls such a stencil discontinuous and gives theta = 0
 *    for a discontinuity, while the printed form is 1/2 at x = H;
 *  - rounding of the sums of products (the paper fixes none).  The file
 *    builds in two modes:
 *      default: the smoothness indicators (eq 2.9-2.11), candidate fluxes
 *        (eq 2.4-2.6), their weighted sum (eq 2.7), the global
 *        Lax-Friedrichs split (F +- alpha U) / 2, the characteristic
 *        projection onto the left eigenvectors and the back-projection R f^
 *        use fused multiply-adds, in the order written below;
 *      ORACLE_LITERAL: no fused operation anywhere.  Each formula is the
 *        plain product-then-sum of its printed form, left to right:
 *        beta_0 = 13/12 (a - 2b + c)^2 + 1/4 (a - 4b + 3c)^2,
 *        f_0 = (1/3 a - 7/6 b) + 11/6 c, f_1 = (-1/6 b + 5/6 c) + 1/3 d,
 *        f_2 = (1/3 c + 5/6 d) - 1/6 e, f^ = (w_0 f_0 + w_1 f_1) + w_2 f_2;
 *        the projection first (w_j = L U_j, g_j = L F_j, summed over the
 *        components in order), then the split v+- = (g_j +- alpha w_j) / 2;
 *        F^ = R (f^+ + f^-) summed over the fields in order.
 *    Both modes are the same method; they differ only in rounding, which is
 *    what a comparison between them measures.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

extern "C" {

/* Problem description passed from Python (ctypes mirror in oracle/__init__.py). */
typedef struct {
    int32_t ndim;       /* 1, 2 or 3                                        */
    int32_t n[3];       /* cells along x, y, z (unused axes: 1)              */
    double dx[3];       /* uniform spacing per axis                         */
    int32_t bc[3];      /* 0 periodic, 1 zero-gradient, 2 reflecting        */
    int32_t scheme;     /* 0 TENO5-LAD, 1 TENO5 fixed C_T, 2 linear upwind5,
                           3 TENO5-A (adaptive C_T of eq 2.16-2.18)         */
    double gamma;       /* ratio of specific heats                          */
    double ct_fixed;    /* C_T of scheme 1                                  */
    double H;           /* LAD intensity threshold (Sec. 3, eq 3.2)         */
    int32_t Bl, Bu;     /* LAD magnitude bounds (Sec. 3, eq 3.1)            */
    double eps;         /* epsilon of eq 2.8 / eq 3.2                       */
    double a1, a2;      /* TENO5-A: alpha_1, alpha_2 of eq 2.16             */
    double cr, xi;      /* TENO5-A: C_r of eq 2.17, xi of eq 2.18           */
    /* Boundaries that differ per end, along the boundary or in time, and a
     * gravity source (the 2D workloads of Sec. 4.3).  Used when has_ext. */
    int32_t has_ext;
    int32_t side_kind[3][2][2];    /* [axis][end][a, b]: 0 periodic, 1 zero-gradient,
                                      2 reflecting, 3 fixed state                     */
    int32_t side_axis[3][2];       /* axis of the split coordinate, -1: kind a only  */
    double side_split[3][2][2];    /* split position = split0 + rate * t           */
    double side_state[3][2][2][5]; /* conserved fixed states (natural order)        */
    double gravity[3];             /* momentum += rho g, energy += m . g            */
    double time;                   /* time of or_rhs evaluations                    */
    int32_t theta_form;            /* LAD theta of eq 3.2: 0 as printed; 1 also
                                      theta = 0 where max chi-tilde exceeds H      */
} OrParams;

}  // extern "C"

namespace {

/* ------------------------------------------------------------------------ */
/* Forward-mode dual number (value, one tangent).                           */
/* ------------------------------------------------------------------------ */
struct Dual {
    double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual operator/(double a, Dual b) {
    double q = a / b.v;
    return {q, -q * b.d / b.v};
}
inline Dual dsqrt(Dual a) {
    double s = std::sqrt(a.v);
    return {s, a.d / (2.0 * s)};
}
inline double dsqrt(double a) { return std::sqrt(a); }
/* a b + c with one rounding of the value; tangents by the product rule */
inline double fmadd(double a, double b, double c) { return std::fma(a, b, c); }
inline Dual fmadd(Dual a, Dual b, Dual c) {
    return {std::fma(a.v, b.v, c.v), (a.d * b.v + a.v * b.d) + c.d};
}
inline Dual fmadd(double a, Dual b, Dual c) { return {std::fma(a, b.v, c.v), a * b.d + c.d}; }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
template <class T> inline T from_double(double x);
template <> inline double from_double<double>(double x) { return x; }
template <> inline Dual from_double<Dual>(double x) { return {x, 0.0}; }

/* ------------------------------------------------------------------------ */
/* Constants: FP64 quotients of the integer literals printed in the paper.   */
/* ------------------------------------------------------------------------ */
const double K13_12 = 13.0 / 12.0;  /* eq 2.9-2.11 */
const double K1_4 = 0.25;           /* eq 2.9-2.11 */
const double T1_3 = 1.0 / 3.0;      /* eq 2.4-2.6, eq 4.3 */
const double T7_6 = 7.0 / 6.0;
const double T11_6 = 11.0 / 6.0;
const double T1_6 = 1.0 / 6.0;
const double T5_6 = 5.0 / 6.0;
const double T2_3 = 2.0 / 3.0;      /* eq 4.3 */
const double C_LIN[3] = {0.1, 0.6, 0.3};  /* linear weights, Sec. 2 */
const double SCALE_C = 1.0;          /* C of eq 2.8 (q = 6 is the multiply chain) */

/* The Ladder array of eq 3.3, written as decimal literals (never pow):
 * POW10NEG[k] = 10^-k.  C_T = Lad(m) = POW10NEG[m] (eq 3.4). */
const double POW10NEG[21] = {1e0,   1e-1,  1e-2,  1e-3,  1e-4,  1e-5,  1e-6,
                             1e-7,  1e-8,  1e-9,  1e-10, 1e-11, 1e-12, 1e-13,
                             1e-14, 1e-15, 1e-16, 1e-17, 1e-18, 1e-19, 1e-20};

/* ------------------------------------------------------------------------ */
/* Scalar TENO5-LAD decision (Sec. 2 eq 2.8-2.14, Sec. 3 eq 3.1-3.4).       */
/* Decisions depend on real values only.                                    */
/* ------------------------------------------------------------------------ */
struct Decision {
    int m;     /* ladder exponent, C_T = 10^-m (0 for non-LAD schemes) */
    int mask;  /* bit k = delta_k of eq 2.14 */
};

struct DecisionTrace {  /* intermediate values, for the pin tests */
    double beta[3], tau, t[3], gam[3], chi[3], x, theta, ct;
    int m, mask;
};

Decision teno_decide(const OrParams& P, double a, double b, double c, double d,
                     double e, DecisionTrace* tr) {
    /* Jiang-Shu smoothness indicators, eq 2.9-2.11, on (f_{i-2} .. f_{i+2}) =
     * (a, b, c, d, e). */
    double beta[3];
#ifdef ORACLE_LITERAL
    double s01 = (a - 2.0 * b) + c;
    double s02 = (a - 4.0 * b) + 3.0 * c;
    double s11 = (b - 2.0 * c) + d;
    double s12 = b - d;
    double s21 = (c - 2.0 * d) + e;
    double s22 = (3.0 * c - 4.0 * d) + e;
    beta[0] = K13_12 * (s01 * s01) + K1_4 * (s02 * s02);
    beta[1] = K13_12 * (s11 * s11) + K1_4 * (s12 * s12);
    beta[2] = K13_12 * (s21 * s21) + K1_4 * (s22 * s22);
#else
    double s01 = (a - 2.0 * b) + c;
    double s02 = fmadd(3.0, c, a - 4.0 * b);
    double s11 = (b - 2.0 * c) + d;
    double s12 = b - d;
    double s21 = (c - 2.0 * d) + e;
    double s22 = fmadd(3.0, c, e - 4.0 * d);
    beta[0] = fmadd(K13_12 * s01, s01, K1_4 * (s02 * s02));
    beta[1] = fmadd(K13_12 * s11, s11, K1_4 * (s12 * s12));
    beta[2] = fmadd(K13_12 * s21, s21, K1_4 * (s22 * s22));
#endif
    /* Global smoothness indicator tau_5 = |beta_2 - beta_0|, eq 2.12. */
    double tau = std::fabs(beta[2] - beta[0]);
    /* chi-tilde_k = tau / (beta_k + eps) (eq 3.2), which is also the ratio
     * inside eq 2.8; gamma_k = (C + chi-tilde_k)^6 as a multiply chain. */
    double t[3], gam[3];
    for (int k = 0; k < 3; ++k) {
        t[k] = tau / (beta[k] + P.eps);
        double y = SCALE_C + t[k];
        double y2 = y * y;
        gam[k] = (y2 * y2) * y2;
    }
    /* Normalisation, eq 2.13. */
    double S = (gam[0] + gam[1]) + gam[2];
    double chi[3];
    for (int k = 0; k < 3; ++k) chi[k] = gam[k] / S;

    /* Cutoff value. */
    double ct = 0.0, x = 0.0, theta = 0.0;
    int m = 0;
    if (P.scheme == 0) {
        /* LAD, eq 3.1-3.2: theta = 1 / (1 + max_k chi-tilde_k / H),
         * m = B_l + floor(theta (B_u - B_l)), C_T = Lad(m) (eq 3.4). */
        x = t[0];
        if (t[1] > x) x = t[1];
        if (t[2] > x) x = t[2];
        /* theta_form 1: Sec. 3 calls a stencil whose largest chi-tilde is over
         * H discontinuous, and theta is 0 for a discontinuity; the printed
         * form would give 1/2 at x = H, so this form sets theta = 0 there. */
        if (P.theta_form == 1 && x > P.H)
            theta = 0.0;
        else
            theta = 1.0 / (1.0 + x / P.H);
        /* A NaN theta only arises from a non-physical stencil (flagged by the
         * positivity status); it takes the most dissipative rung B_l. */
        if (theta >= 0.0)
            m = P.Bl + (int)std::floor(theta * (double)(P.Bu - P.Bl));
        else
            m = P.Bl;
        ct = POW10NEG[m];
    } else if (P.scheme == 1) {
        ct = P.ct_fixed;
    } else if (P.scheme == 3) {
        /* TENO5-A, eq 2.16-2.18.  The sensor of eq 2.18 at the stencil points
         * j = i-1, i, i+1 uses df_{j+1/2} = f_{j+1} - f_j and df_{j-1/2}; its
         * denominator is read as df_{j+1/2}^2 + df_{j-1/2}^2 (the printed
         * formula repeats df_{i+1/2}).  epsilon = 0.9 C_r / (1 - 0.9 C_r) xi^2. */
        double epsA = ((0.9 * P.cr) / (1.0 - 0.9 * P.cr)) * (P.xi * P.xi);
        double df[4] = {b - a, c - b, d - c, e - d};
        double eta[3];
        for (int j = 0; j < 3; ++j) {
            double dm = df[j], dp = df[j + 1];
            eta[j] = (2.0 * std::fabs(dp * dm) + epsA) / ((dp * dp + dm * dm) + epsA);
        }
        /* eq 2.17: eta_{i+1/2} = min of the three, m = 1 - min(1, eta / C_r) */
        double eh = eta[0];
        if (eta[1] < eh) eh = eta[1];
        if (eta[2] < eh) eh = eta[2];
        double q = eh / P.cr;
        double mA = 1.0 - (q < 1.0 ? q : 1.0);
        /* eq 2.16: g(m) = (1 - m)^4 (1 + 4 m), beta = alpha_1 - alpha_2 (1 - g),
         * C_T = 10^-floor(beta) */
        double om = 1.0 - mA;
        double om2 = om * om;
        double g = (om2 * om2) * (1.0 + 4.0 * mA);
        double bA = P.a1 - P.a2 * (1.0 - g);
        /* a NaN sensor (non-finite stencil) takes the largest cutoff */
        if (bA >= 0.0)
            m = (int)std::floor(bA);
        else
            m = (int)std::floor(P.a1 - P.a2);
        x = eh;
        theta = bA;
        ct = POW10NEG[m];
    }
    /* Cutoff, eq 2.14 (a tie chi_k == C_T keeps the stencil). */
    int mask = 0;
    for (int k = 0; k < 3; ++k) {
        int delta = (P.scheme == 2) ? 1 : ((chi[k] < ct) ? 0 : 1);
        mask |= delta << k;
    }
    if (tr) {
        for (int k = 0; k < 3; ++k) {
            tr->beta[k] = beta[k];
            tr->t[k] = t[k];
            tr->gam[k] = gam[k];
            tr->chi[k] = chi[k];
        }
        tr->tau = tau;
        tr->x = x;
        tr->theta = theta;
        tr->ct = ct;
        tr->m = m;
        tr->mask = mask;
    }
    return Decision{m, mask};
}

/* TENO5 flux from the cutoff flags: candidate fluxes eq 2.4-2.6, weights
 * eq 2.15, combination eq 2.7.  Linear in (a..e) once the mask is fixed. */
template <class T>
T teno_flux(int mask, T a, T b, T c, T d, T e) {
#ifdef ORACLE_LITERAL
    T f0 = (T1_3 * a - T7_6 * b) + T11_6 * c;
    T f1 = (-T1_6 * b + T5_6 * c) + T1_3 * d;
    T f2 = (T1_3 * c + T5_6 * d) - T1_6 * e;
#else
    T f0 = fmadd(T11_6, c, fmadd(T1_3, a, -T7_6 * b));
    T f1 = fmadd(T1_3, d, fmadd(-T1_6, b, T5_6 * c));
    T f2 = fmadd(-T1_6, e, fmadd(T1_3, c, T5_6 * d));
#endif
    double dl[3];
    for (int k = 0; k < 3; ++k) dl[k] = (double)((mask >> k) & 1);
    double D = (dl[0] * C_LIN[0] + dl[1] * C_LIN[1]) + dl[2] * C_LIN[2];
    double w[3];
    for (int k = 0; k < 3; ++k) w[k] = (dl[k] * C_LIN[k]) / D;
#ifdef ORACLE_LITERAL
    return (w[0] * f0 + w[1] * f1) + w[2] * f2;
#else
    return fmadd(w[2], f2, fmadd(w[0], f0, w[1] * f1));
#endif
}

template <class T>
T teno_rec(const OrParams& P, T a, T b, T c, T d, T e, Decision* dec) {
    Decision q = teno_decide(P, val(a), val(b), val(c), val(d), val(e), nullptr);
    if (dec) *dec = q;
    return teno_flux<T>(q.mask, a, b, c, d, e);
}

/* ------------------------------------------------------------------------ */
/* Euler physics (Sec. 4.2 eq 4.7 and its 2D/3D analogue).                  */
/* Natural component order: rho, rho u_x, [rho u_y], [rho u_z], E.          */
/* ------------------------------------------------------------------------ */
template <class T>
struct Prim {
    T rho, u[3], p, H;
};

template <class T>
Prim<T> primitives(const OrParams& P, const T* U) {
    int nd = P.ndim, nc = nd + 2;
    Prim<T> w;
    w.rho = U[0];
    for (int k = 0; k < 3; ++k) w.u[k] = from_double<T>(0.0);
    for (int k = 0; k < nd; ++k) w.u[k] = U[1 + k] / w.rho;
    T mu = U[1] * w.u[0];
    for (int k = 1; k < nd; ++k) mu = mu + U[1 + k] * w.u[k];
    T ke = 0.5 * mu;
    T E = U[nc - 1];
    w.p = (P.gamma - 1.0) * (E - ke);
    w.H = (E + w.p) / w.rho;
    return w;
}

/* Flux along axis d, natural component order. */
template <class T>
void euler_flux(const OrParams& P, int d, const T* U, const Prim<T>& w, T* F) {
    int nd = P.ndim, nc = nd + 2;
    F[0] = U[1 + d];
    for (int k = 0; k < nd; ++k) {
        if (k == d)
            F[1 + k] = U[1 + k] * w.u[d] + w.p;
        else
            F[1 + k] = U[1 + k] * w.u[d];
    }
    F[nc - 1] = (U[nc - 1] + w.p) * w.u[d];
}

/* Local component order for a sweep along d: rho, normal momentum, the
 * tangential momenta in increasing axis order, E.  perm[local] = natural. */
void local_perm(int ndim, int d, int* perm) {
    int nc = ndim + 2;
    perm[0] = 0;
    perm[1] = 1 + d;
    int j = 2;
    for (int k = 0; k < ndim; ++k)
        if (k != d) perm[j++] = 1 + k;
    perm[nc - 1] = nc - 1;
}

/* Roe average between cells L and R and the eigenvectors of the flux Jacobian
 * along d at that state, in local component order.  Lm[s][c]: row s = left
 * eigenvector of field s; Rm[c][s]: column s = right eigenvector.  Fields:
 * 0 = u_n - c, 1 = entropy, 2.. = shear (one per tangential axis), last =
 * u_n + c.  L R = I. */
template <class T>
void roe_eigen(const OrParams& P, int d, const T* UL, const T* UR, T Lm[5][5],
               T Rm[5][5]) {
    int nd = P.ndim, nc = nd + 2;
    Prim<T> wl = primitives(P, UL), wr = primitives(P, UR);
    T rl = dsqrt(wl.rho), rr = dsqrt(wr.rho);
    T wsum = 1.0 / (rl + rr);
    T u[3];
    for (int k = 0; k < nd; ++k) u[k] = (rl * wl.u[k] + rr * wr.u[k]) * wsum;
    T Hb = (rl * wl.H + rr * wr.H) * wsum;
    T q2 = u[0] * u[0];
    for (int k = 1; k < nd; ++k) q2 = q2 + u[k] * u[k];
    T c2 = (P.gamma - 1.0) * (Hb - 0.5 * q2);
    T c = dsqrt(c2);
    T ci = 1.0 / c;
    T b1 = (P.gamma - 1.0) / c2;
    T b2 = (0.5 * q2) * b1;

    int perm[5];
    local_perm(nd, d, perm);
    T ul[3];  /* velocities in local order: ul[0] normal, then tangentials */
    for (int k = 0; k < nd; ++k) ul[k] = u[perm[1 + k] - 1];
    T un = ul[0];

    T zero = from_double<T>(0.0), one = from_double<T>(1.0);
    for (int s = 0; s < 5; ++s)
        for (int q = 0; q < 5; ++q) {
            Lm[s][q] = zero;
            Rm[s][q] = zero;
        }
    int last = nc - 1;
    /* Right eigenvectors (columns). */
    Rm[0][0] = one;
    Rm[1][0] = un - c;
    for (int k = 1; k < nd; ++k) Rm[1 + k][0] = ul[k];
    Rm[last][0] = Hb - un * c;

    Rm[0][1] = one;
    Rm[1][1] = un;
    for (int k = 1; k < nd; ++k) Rm[1 + k][1] = ul[k];
    Rm[last][1] = 0.5 * q2;

    for (int k = 1; k < nd; ++k) {
        int s = 1 + k;
        Rm[1 + k][s] = one;
        Rm[last][s] = ul[k];
    }

    Rm[0][last] = one;
    Rm[1][last] = un + c;
    for (int k = 1; k < nd; ++k) Rm[1 + k][last] = ul[k];
    Rm[last][last] = Hb + un * c;

    /* Left eigenvectors (rows). */
    Lm[0][0] = 0.5 * (b2 + un * ci);
    Lm[0][1] = 0.5 * (-(b1 * un) - ci);
    for (int k = 1; k < nd; ++k) Lm[0][1 + k] = 0.5 * (-(b1 * ul[k]));
    Lm[0][last] = 0.5 * b1;

    Lm[1][0] = 1.0 - b2;
    Lm[1][1] = b1 * un;
    for (int k = 1; k < nd; ++k) Lm[1][1 + k] = b1 * ul[k];
    Lm[1][last] = -b1;

    for (int k = 1; k < nd; ++k) {
        int s = 1 + k;
        Lm[s][0] = -ul[k];
        Lm[s][1 + k] = one;
    }

    Lm[last][0] = 0.5 * (b2 - un * ci);
    Lm[last][1] = 0.5 * (-(b1 * un) + ci);
    for (int k = 1; k < nd; ++k) Lm[last][1 + k] = 0.5 * (-(b1 * ul[k]));
    Lm[last][last] = 0.5 * b1;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers.                                                            */
/* ------------------------------------------------------------------------ */
inline int64_t ncells(const OrParams& P) {
    return (int64_t)P.n[0] * P.n[1] * P.n[2];
}
inline int64_t cell_index(const OrParams& P, int x, int y, int z) {
    return ((int64_t)z * P.n[1] + y) * P.n[0] + x;
}

/* Ghost synthesis along axis d for local position j of a line (Sec. 4:
 * periodic, zero-gradient, reflecting).  Returns the source cell position
 * along the axis and whether the normal momentum is negated. */
inline int ghost_source(int bc, int n, int j, bool* flip) {
    *flip = false;
    if (j >= 0 && j < n) return j;
    if (bc == 0) return ((j % n) + n) % n;
    if (bc == 1) return j < 0 ? 0 : n - 1;
    *flip = true;
    return j < 0 ? -1 - j : 2 * n - 1 - j;
}

/* Load the conserved state of line cell j (natural order) into out[] at time
 * t.  With per-side boundaries, a ghost cell takes the kind of its end: kind
 * a where the split coordinate (the cell centre (i + 1/2) dx along the split
 * axis, on the line) lies below split0 + rate t, else kind b; a fixed kind
 * supplies its stored state. */
template <class T>
void load_cell(const OrParams& P, const T* U, int d, const int base[3], int j,
               T* out, double t) {
    int nc = P.ndim + 2;
    int64_t N = ncells(P);
    bool flip;
    int kind = P.bc[d];
    if (P.has_ext && (j < 0 || j >= P.n[d])) {
        int end = j < 0 ? 0 : 1;
        int ax = P.side_axis[d][end];
        int which = 0;  /* 0: kind a, 1: kind b */
        if (ax >= 0) {
            double coord = ((double)base[ax] + 0.5) * P.dx[ax];
            double split = P.side_split[d][end][0] + P.side_split[d][end][1] * t;
            if (!(coord < split)) which = 1;
        }
        kind = P.side_kind[d][end][which];
        if (kind == 3) {
            for (int q = 0; q < nc; ++q) out[q] = from_double<T>(P.side_state[d][end][which][q]);
            return;
        }
    }
    int src = ghost_source(kind, P.n[d], j, &flip);
    int pos[3] = {base[0], base[1], base[2]};
    pos[d] = src;
    int64_t ci = cell_index(P, pos[0], pos[1], pos[2]);
    for (int q = 0; q < nc; ++q) out[q] = U[q * N + ci];
    if (flip) out[1 + d] = -out[1 + d];
}

/* ------------------------------------------------------------------------ */
/* Face flux (Sec. 2 eq 2.2 with characteristic TENO5-LAD, Sec. 4).         */
/* ------------------------------------------------------------------------ */
/* st[j][q] (j = 0..5) holds cells i-2 .. i+3 around face i+1/2, natural
 * order.  Writes the numerical flux F^ (natural order) and, if dec != null,
 * the 2*nc decisions in the order (field s, sign +, sign -). */
template <class T>
void face_flux(const OrParams& P, int d, T st[6][5], double alpha, T* Fhat,
               Decision* dec, double* Fmag = nullptr) {
    int nd = P.ndim, nc = nd + 2;
    int perm[5];
    local_perm(nd, d, perm);
    /* Cell fluxes F_j and states U_j of the stencil in local order. */
    T Uloc[6][5], Floc[6][5];
    for (int j = 0; j < 6; ++j) {
        Prim<T> w = primitives(P, st[j]);
        T F[5];
        euler_flux(P, d, st[j], w, F);
        for (int q = 0; q < nc; ++q) {
            Uloc[j][q] = st[j][perm[q]];
            Floc[j][q] = F[perm[q]];
        }
    }
#ifndef ORACLE_LITERAL
    /* Global Lax-Friedrichs splitting of the cell fluxes first:
     * f^{+-}_j = 1/2 (F_j +- alpha U_j). */
    T fp[6][5], fm[6][5];
    for (int j = 0; j < 6; ++j)
        for (int q = 0; q < nc; ++q) {
            fp[j][q] = 0.5 * fmadd(alpha, Uloc[j][q], Floc[j][q]);
            fm[j][q] = 0.5 * fmadd(-alpha, Uloc[j][q], Floc[j][q]);
        }
#endif
    /* Characteristic projection at the Roe state of cells i and i+1. */
    T Lm[5][5], Rm[5][5];
    roe_eigen(P, d, st[2], st[3], Lm, Rm);
    T fh[5];
    for (int s = 0; s < nc; ++s) {
        /* Projected split fluxes v^{+-}_j = l_s . (F_j +- alpha U_j) / 2. */
        T vp[6], vm[6];
        for (int j = 0; j < 6; ++j) {
#ifdef ORACLE_LITERAL
            /* projection first (w_j = l_s . U_j, g_j = l_s . F_j), then the split */
            T wj = Lm[s][0] * Uloc[j][0];
            T gj = Lm[s][0] * Floc[j][0];
            for (int q = 1; q < nc; ++q) {
                wj = wj + Lm[s][q] * Uloc[j][q];
                gj = gj + Lm[s][q] * Floc[j][q];
            }
            vp[j] = 0.5 * (gj + alpha * wj);
            vm[j] = 0.5 * (gj - alpha * wj);
#else
            T ap = Lm[s][0] * fp[j][0];
            T am = Lm[s][0] * fm[j][0];
            for (int q = 1; q < nc; ++q) {
                ap = fmadd(Lm[s][q], fp[j][q], ap);
                am = fmadd(Lm[s][q], fm[j][q], am);
            }
            vp[j] = ap;
            vm[j] = am;
#endif
        }
        Decision dp, dm;
        /* f^+ on cells i-2..i+2; f^- on the mirrored stencil i+3..i-1. */
        T rp = teno_rec<T>(P, vp[0], vp[1], vp[2], vp[3], vp[4], &dp);
        T rm = teno_rec<T>(P, vm[5], vm[4], vm[3], vm[2], vm[1], &dm);
        fh[s] = rp + rm;
        if (dec) {
            dec[2 * s] = dp;
            dec[2 * s + 1] = dm;
        }
    }
    /* Back to conserved variables: F^ = R f^. */
    for (int q = 0; q < nc; ++q) {
        T acc = Rm[q][0] * fh[0];
#ifdef ORACLE_LITERAL
        for (int s = 1; s < nc; ++s) acc = acc + Rm[q][s] * fh[s];
#else
        for (int s = 1; s < nc; ++s) acc = fmadd(Rm[q][s], fh[s], acc);
#endif
        Fhat[perm[q]] = acc;
        if (Fmag) {  /* sum_s |R_qs f^_s|: the terms the back-projection adds */
            double m = 0.0;
            for (int s = 0; s < nc; ++s) m += std::fabs(val(Rm[q][s]) * val(fh[s]));
            Fmag[perm[q]] = m;
        }
    }
}

inline uint8_t encode_decision(Decision q) {
    return (uint8_t)(q.m | (q.mask << 5));
}

/* Number of lines along axis d and the base position of line l. */
inline int64_t nlines(const OrParams& P, int d) { return ncells(P) / P.n[d]; }
inline void line_base(const OrParams& P, int d, int64_t l, int base[3]) {
    int a = (d == 0) ? 1 : 0;           /* first non-swept axis */
    int b = (d == 2) ? 1 : 2;           /* second non-swept axis */
    base[d] = 0;
    base[a] = (int)(l % P.n[a]);
    base[b] = (int)(l / P.n[a]);
}

/* ------------------------------------------------------------------------ */
/* Global Lax-Friedrichs speeds (Sec. 4): alpha_d = max_i (|u_d| + c).      */
/* status: 0 ok, 3 if some cell has rho <= 0, p <= 0 or a non-finite value. */
/* ------------------------------------------------------------------------ */
void lf_alpha(const OrParams& P, const double* U, double alpha[3], int* status) {
    int nd = P.ndim, nc = nd + 2;
    int64_t N = ncells(P);
    alpha[0] = alpha[1] = alpha[2] = 0.0;
    int bad = 0;
    for (int64_t i = 0; i < N; ++i) {
        double q[5];
        for (int c = 0; c < nc; ++c) q[c] = U[c * N + i];
        Prim<double> w = primitives(P, q);
        double cs = std::sqrt((P.gamma * w.p) / w.rho);
        if (!(w.rho > 0.0) || !(w.p > 0.0) || !std::isfinite(cs)) bad = 1;
        for (int k = 0; k < nd; ++k) {
            double s = std::fabs(w.u[k]) + cs;
            if (s > alpha[k]) alpha[k] = s;
        }
    }
    if (status) *status = bad ? 3 : 0;
}

/* ------------------------------------------------------------------------ */
/* Semi-discrete RHS, eq 2.2 summed over directions x, y, z in that order:  */
/* dUdt = 0 - dF_x/dx - dF_y/dy - dF_z/dz.                                   */
/* dump (nullable): per direction d, per line, per face phi = i+1 in        */
/* [0, n_d], 2*nc decision bytes (m | mask << 5).                           */
/* ------------------------------------------------------------------------ */
template <class T>
void rhs_impl(const OrParams& P, const T* U, const double alpha[3], T* out,
              uint8_t* dump, double t, double* flux_abs = nullptr,
              double* flux_max = nullptr) {
    int nd = P.ndim, nc = nd + 2;
    int64_t N = ncells(P);
    for (int64_t i = 0; i < (int64_t)nc * N; ++i) out[i] = from_double<T>(0.0);
    int64_t dump_off = 0;
    for (int d = 0; d < nd; ++d) {
        int n = P.n[d];
        int64_t L = nlines(P, d);
        double dxd = P.dx[d];
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t l = 0; l < L; ++l) {
            int base[3];
            line_base(P, d, l, base);
            /* The line with 3 ghost cells per side. */
            std::vector<T> ext((size_t)(n + 6) * 5);
            for (int j = -3; j < n + 3; ++j)
                load_cell(P, U, d, base, j, &ext[(size_t)(j + 3) * 5], t);
            std::vector<T> fl((size_t)(n + 1) * 5);
            std::vector<double> fmag(flux_max ? (size_t)(n + 1) * 5 : 0);
            for (int phi = 0; phi <= n; ++phi) {  /* face i+1/2, i = phi-1 */
                T st[6][5];
                for (int j = 0; j < 6; ++j)
                    for (int q = 0; q < nc; ++q) st[j][q] = ext[(size_t)(phi + j) * 5 + q];
                Decision dec[10];
                face_flux(P, d, st, alpha[d], &fl[(size_t)phi * 5], dump ? dec : nullptr,
                          flux_max ? &fmag[(size_t)phi * 5] : nullptr);
                if (dump) {
                    uint8_t* o = dump + dump_off + ((size_t)l * (n + 1) + phi) * 2 * nc;
                    for (int k = 0; k < 2 * nc; ++k) o[k] = encode_decision(dec[k]);
                }
            }
            for (int i = 0; i < n; ++i) {
                int pos[3] = {base[0], base[1], base[2]};
                pos[d] = i;
                int64_t ci = cell_index(P, pos[0], pos[1], pos[2]);
                for (int q = 0; q < nc; ++q) {
                    T diff = fl[(size_t)(i + 1) * 5 + q] - fl[(size_t)i * 5 + q];
                    out[q * N + ci] = out[q * N + ci] - diff / dxd;
                }
            }
            if (flux_abs) {
                /* sum over the line's faces of |F^| / dx and max of
                 * sum_s |R_qs f^_s| / dx (magnitudes for rounding bounds; not
                 * part of the method) */
                double loc[5] = {0, 0, 0, 0, 0}, mx[5] = {0, 0, 0, 0, 0};
                for (int phi = 0; phi <= n; ++phi)
                    for (int q = 0; q < nc; ++q) {
                        loc[q] += std::fabs(val(fl[(size_t)phi * 5 + q])) / dxd;
                        double a = fmag[(size_t)phi * 5 + q] / dxd;
                        if (a > mx[q]) mx[q] = a;
                    }
#pragma omp critical
                for (int q = 0; q < nc; ++q) {
                    flux_abs[q] += loc[q];
                    if (mx[q] > flux_max[q]) flux_max[q] = mx[q];
                }
            }
        }
        dump_off += L * (int64_t)(n + 1) * 2 * nc;
    }
    /* Gravity source (Sec. 4.3, Rayleigh-Taylor): rho g_d on each momentum
     * component, m . g on the energy, added after the flux differences. */
    if (P.has_ext) {
        for (int64_t i = 0; i < N; ++i) {
            for (int dd = 0; dd < nd; ++dd)
                out[(1 + dd) * N + i] = out[(1 + dd) * N + i] + U[i] * P.gravity[dd];
            T sE = U[1 * N + i] * P.gravity[0];
            for (int dd = 1; dd < nd; ++dd) sE = sE + U[(1 + dd) * N + i] * P.gravity[dd];
            out[(nc - 1) * N + i] = out[(nc - 1) * N + i] + sE;
        }
    }
}

/* RHS of single cells (same arithmetic, only the two faces of each cell per
 * direction), for spot checks of large grids. */
void rhs_cells_impl(const OrParams& P, const double* U, const double alpha[3],
                    int64_t ncell, const int64_t* cells, double* out,
                    uint8_t* dump) {
    int nd = P.ndim, nc = nd + 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < ncell; ++s) {
        int64_t ci = cells[s];
        int pos[3];
        pos[0] = (int)(ci % P.n[0]);
        pos[1] = (int)((ci / P.n[0]) % P.n[1]);
        pos[2] = (int)(ci / ((int64_t)P.n[0] * P.n[1]));
        double r[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < nd; ++d) {
            int base[3] = {pos[0], pos[1], pos[2]};
            base[d] = 0;
            int i = pos[d];
            double fl[2][5];
            for (int side = 0; side < 2; ++side) {
                int phi = i + side;  /* face i-1/2 (phi = i) and i+1/2 */
                double st[6][5];
                for (int j = 0; j < 6; ++j) load_cell(P, U, d, base, phi - 3 + j, st[j], P.time);
                Decision dec[10];
                face_flux(P, d, st, alpha[d], fl[side], dump ? dec : nullptr);
                if (dump) {
                    uint8_t* o = dump + ((s * nd + d) * 2 + side) * 2 * nc;
                    for (int k = 0; k < 2 * nc; ++k) o[k] = encode_decision(dec[k]);
                }
            }
            for (int q = 0; q < nc; ++q) r[q] = r[q] - (fl[1][q] - fl[0][q]) / P.dx[d];
        }
        if (P.has_ext) {
            int64_t N = ncells(P);
            for (int dd = 0; dd < nd; ++dd) r[1 + dd] = r[1 + dd] + U[ci] * P.gravity[dd];
            double sE = U[1 * N + ci] * P.gravity[0];
            for (int dd = 1; dd < nd; ++dd) sE = sE + U[(1 + dd) * N + ci] * P.gravity[dd];
            r[nc - 1] = r[nc - 1] + sE;
        }
        for (int q = 0; q < nc; ++q) out[s * nc + q] = r[q];
    }
}

/* Time step from the LF speeds of u^n (Sec. 4, eq dt1 / eq dt2; 3D: the
 * harmonic extension), clipped so that t + dt does not pass t_end. */
double cfl_dt(const OrParams& P, const double alpha[3], double cfl, double t,
              double t_end) {
    double dt;
    if (P.ndim == 1) {
        dt = cfl * P.dx[0] / alpha[0];
    } else if (P.ndim == 2) {
        double dtx = P.dx[0] / alpha[0];
        double dty = P.dx[1] / alpha[1];
        dt = cfl * (dtx * dty) / (dtx + dty);
    } else {
        dt = cfl / ((alpha[0] / P.dx[0] + alpha[1] / P.dx[1]) + alpha[2] / P.dx[2]);
    }
    if (t + dt > t_end) dt = t_end - t;
    return dt;
}

}  // namespace

/* ======================================================================== */
/* C interface (ctypes).                                                    */
/* ======================================================================== */
extern "C" {

int or_version(void) { return 1; }

/* 1 for the ORACLE_LITERAL build (no fused multiply-adds), else 0. */
int or_literal(void) {
#ifdef ORACLE_LITERAL
    return 1;
#else
    return 0;
#endif
}

/* Scalar reconstruction with its intermediate values.  v[5] = (f_{i-2}..f_{i+2}).
 * out9 = beta0..2, tau, x, theta, ct, chi0, chi1 ... (see below). */
double or_rec(const OrParams* P, const double* v, int32_t* m, int32_t* mask,
              double* trace /* nullable, 17 doubles */) {
    DecisionTrace tr;
    teno_decide(*P, v[0], v[1], v[2], v[3], v[4], &tr);
    double f = teno_flux<double>(tr.mask, v[0], v[1], v[2], v[3], v[4]);
    if (m) *m = tr.m;
    if (mask) *mask = tr.mask;
    if (trace) {
        double* o = trace;
        for (int k = 0; k < 3; ++k) *o++ = tr.beta[k];
        *o++ = tr.tau;
        for (int k = 0; k < 3; ++k) *o++ = tr.t[k];
        for (int k = 0; k < 3; ++k) *o++ = tr.gam[k];
        for (int k = 0; k < 3; ++k) *o++ = tr.chi[k];
        *o++ = tr.x;
        *o++ = tr.theta;
        *o++ = tr.ct;
    }
    return f;
}

/* Eigenvectors at the Roe state of UL, UR (natural order in, local order out). */
void or_eigen(const OrParams* P, int d, const double* UL, const double* UR,
              double* Lout /* 25 */, double* Rout /* 25 */) {
    double Lm[5][5], Rm[5][5];
    roe_eigen<double>(*P, d, UL, UR, Lm, Rm);
    for (int s = 0; s < 5; ++s)
        for (int q = 0; q < 5; ++q) {
            Lout[s * 5 + q] = Lm[s][q];
            Rout[s * 5 + q] = Rm[s][q];
        }
}

int or_alpha(const OrParams* P, const double* U, double* alpha3) {
    int st;
    lf_alpha(*P, U, alpha3, &st);
    return st;
}

/* dUdt = L(U).  alpha3 (nullable): frozen LF speeds; computed from U if null.
 * Returns the positivity status of U. */
int or_rhs(const OrParams* P, const double* U, const double* alpha3,
           double* dUdt, uint8_t* dump) {
    double a[3];
    int st = 0;
    lf_alpha(*P, U, a, &st);
    if (alpha3) {
        a[0] = alpha3[0];
        a[1] = alpha3[1];
        a[2] = alpha3[2];
    }
    rhs_impl<double>(*P, U, a, dUdt, dump, P->time);
    return st;
}

/* dUdt = L(U) as or_rhs; flux_abs[q] = sum over axes d and faces f of
 * |F^_f,q| / dx_d (the magnitudes behind the rounding of the flux
 * differences) and flux_max[q] = max over them of sum_s |R_qs f^_s| / dx_d
 * (those behind the rounding of the back-projection), for error bounds. */
int or_rhs_fluxabs(const OrParams* P, const double* U, double* dUdt, double* flux_abs,
                   double* flux_max) {
    double a[3];
    int st = 0;
    lf_alpha(*P, U, a, &st);
    for (int q = 0; q < 5; ++q) flux_abs[q] = flux_max[q] = 0.0;
    rhs_impl<double>(*P, U, a, dUdt, nullptr, P->time, flux_abs, flux_max);
    return st;
}

int or_rhs_cells(const OrParams* P, const double* U, const double* alpha3,
                 int64_t ncell, const int64_t* cells, double* out, uint8_t* dump) {
    rhs_cells_impl(*P, U, alpha3, ncell, cells, out, dump);
    return 0;
}

/* Jacobian-vector product of L at U with alpha frozen at alpha3 and the
 * cutoff decisions frozen at those of U: JV = dL/dU . V. */
int or_rhs_jvp(const OrParams* P, const double* U, const double* V,
               const double* alpha3, double* dUdt, double* JV) {
    int64_t tot = ncells(*P) * (P->ndim + 2);
    std::vector<Dual> X((size_t)tot), Y((size_t)tot);
    for (int64_t i = 0; i < tot; ++i) X[(size_t)i] = Dual{U[i], V[i]};
    rhs_impl<Dual>(*P, X.data(), alpha3, Y.data(), nullptr, P->time);
    for (int64_t i = 0; i < tot; ++i) {
        if (dUdt) dUdt[i] = Y[(size_t)i].v;
        JV[i] = Y[(size_t)i].d;
    }
    return 0;
}

/* One SSP-RK3 step (Sec. 4 eq 4.1-4.3) in place.
 * replay = 0: dt from the LF speeds of U (clipped to t_end); the speeds of
 *             every stage and dt are written to alpha9 [stage][dir] and *dt.
 * replay = 1: dt and alpha9 are inputs (frozen), nothing is recomputed.
 * Returns the worst positivity status seen. */
int or_step(const OrParams* P, double* U, double cfl, double* t, double t_end,
            int replay, double* dt, double* alpha9) {
    int64_t tot = ncells(*P) * (P->ndim + 2);
    std::vector<double> U1((size_t)tot), U2((size_t)tot), Lv((size_t)tot);
    int status = 0, st;
    double a[3];
    /* Stage 1. */
    if (replay) {
        for (int k = 0; k < 3; ++k) a[k] = alpha9[k];
    } else {
        lf_alpha(*P, U, a, &st);
        status |= st;
        *dt = cfl_dt(*P, a, cfl, *t, t_end);
        for (int k = 0; k < 3; ++k) alpha9[k] = a[k];
    }
    double h = *dt;
    /* stage times t, t + h, t + h/2 (for time-dependent boundaries) */
    rhs_impl<double>(*P, U, a, Lv.data(), nullptr, *t);
    for (int64_t i = 0; i < tot; ++i) U1[(size_t)i] = U[i] + h * Lv[(size_t)i];
    /* Stage 2. */
    if (replay) {
        for (int k = 0; k < 3; ++k) a[k] = alpha9[3 + k];
    } else {
        lf_alpha(*P, U1.data(), a, &st);
        status |= st;
        for (int k = 0; k < 3; ++k) alpha9[3 + k] = a[k];
    }
    rhs_impl<double>(*P, U1.data(), a, Lv.data(), nullptr, *t + h);
    for (int64_t i = 0; i < tot; ++i)
        U2[(size_t)i] = (0.75 * U[i] + 0.25 * U1[(size_t)i]) + 0.25 * (h * Lv[(size_t)i]);
    /* Stage 3. */
    if (replay) {
        for (int k = 0; k < 3; ++k) a[k] = alpha9[6 + k];
    } else {
        lf_alpha(*P, U2.data(), a, &st);
        status |= st;
        for (int k = 0; k < 3; ++k) alpha9[6 + k] = a[k];
    }
    rhs_impl<double>(*P, U2.data(), a, Lv.data(), nullptr, *t + 0.5 * h);
    for (int64_t i = 0; i < tot; ++i)
        U[i] = (T1_3 * U[i] + T2_3 * U2[(size_t)i]) + T2_3 * (h * Lv[(size_t)i]);
    *t = *t + h;
    return status;
}

/* Forward-mode derivative of nsteps replayed RK3 steps: (U, V) -> (U_K, V_K)
 * with dt[k] and alpha[k][3][3] frozen (recorded by a forward run). */
int or_run_jvp(const OrParams* P, double* U, double* V, int64_t nsteps,
               const double* dts, const double* alphas) {
    int64_t tot = ncells(*P) * (P->ndim + 2);
    std::vector<Dual> X((size_t)tot), X1((size_t)tot), X2((size_t)tot), Lv((size_t)tot);
    for (int64_t i = 0; i < tot; ++i) X[(size_t)i] = Dual{U[i], V[i]};
    double t = P->time;
    for (int64_t k = 0; k < nsteps; ++k) {
        double h = dts[k];
        const double* a = alphas + 9 * k;
        rhs_impl<Dual>(*P, X.data(), a, Lv.data(), nullptr, t);
        for (int64_t i = 0; i < tot; ++i) X1[(size_t)i] = X[(size_t)i] + h * Lv[(size_t)i];
        rhs_impl<Dual>(*P, X1.data(), a + 3, Lv.data(), nullptr, t + h);
        for (int64_t i = 0; i < tot; ++i)
            X2[(size_t)i] = (0.75 * X[(size_t)i] + 0.25 * X1[(size_t)i]) + 0.25 * (h * Lv[(size_t)i]);
        rhs_impl<Dual>(*P, X2.data(), a + 6, Lv.data(), nullptr, t + 0.5 * h);
        for (int64_t i = 0; i < tot; ++i)
            X[(size_t)i] = (T1_3 * X[(size_t)i] + T2_3 * X2[(size_t)i]) + T2_3 * (h * Lv[(size_t)i]);
        t = t + h;
    }
    for (int64_t i = 0; i < tot; ++i) {
        U[i] = X[(size_t)i].v;
        V[i] = X[(size_t)i].d;
    }
    return 0;
}

/* nvec independent forward-mode derivatives of the same replayed run: the
 * tangents V[k] (k < nvec, each ncell * nc doubles) are advanced in place
 * from the common start U, one OpenMP thread per tangent. */
int or_run_jvp_batch(const OrParams* P, const double* U, double* V, int64_t nvec,
                     int64_t nsteps, const double* dts, const double* alphas) {
    int64_t tot = ncells(*P) * (P->ndim + 2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nvec; ++k) {
        std::vector<double> Uk(U, U + tot);
        or_run_jvp(P, Uk.data(), V + k * tot, nsteps, dts, alphas);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Scalar linear advection u_t + u_x = 0, periodic (Sec. 4.1 eq 4.4).        */
/* f = u, global LF with alpha = 1: f^+ = u, f^- = 0.                        */
/* ------------------------------------------------------------------------ */
void or_advect_rhs(const OrParams* P, int n, double dx, const double* u,
                   double* out) {
    std::vector<double> fp((size_t)n + 6), fm((size_t)n + 6), fl((size_t)n + 1);
    for (int j = -3; j < n + 3; ++j) {
        double uj = u[((j % n) + n) % n];
        fp[(size_t)(j + 3)] = 0.5 * (uj + 1.0 * uj);
        fm[(size_t)(j + 3)] = 0.5 * (uj - 1.0 * uj);
    }
    for (int phi = 0; phi <= n; ++phi) {
        const double* a = &fp[(size_t)phi];
        const double* b = &fm[(size_t)phi];
        double rp = teno_rec<double>(*P, a[0], a[1], a[2], a[3], a[4], nullptr);
        double rm = teno_rec<double>(*P, b[5], b[4], b[3], b[2], b[1], nullptr);
        fl[(size_t)phi] = rp + rm;
    }
    for (int i = 0; i < n; ++i) out[i] = 0.0 - (fl[(size_t)i + 1] - fl[(size_t)i]) / dx;
}

/* RK3 with constant dt (last step clipped to t_end); u in place.
 * Returns the number of steps taken. */
int64_t or_advect_run(const OrParams* P, int n, double dx, double dt,
                      double t_end, double* u) {
    std::vector<double> L((size_t)n), u1((size_t)n), u2((size_t)n);
    double t = 0.0;
    int64_t steps = 0;
    while (t < t_end) {
        double h = dt;
        if (t + h > t_end) h = t_end - t;
        or_advect_rhs(P, n, dx, u, L.data());
        for (int i = 0; i < n; ++i) u1[(size_t)i] = u[i] + h * L[(size_t)i];
        or_advect_rhs(P, n, dx, u1.data(), L.data());
        for (int i = 0; i < n; ++i)
            u2[(size_t)i] = (0.75 * u[i] + 0.25 * u1[(size_t)i]) + 0.25 * (h * L[(size_t)i]);
        or_advect_rhs(P, n, dx, u2.data(), L.data());
        for (int i = 0; i < n; ++i)
            u[i] = (T1_3 * u[i] + T2_3 * u2[(size_t)i]) + T2_3 * (h * L[(size_t)i]);
        t = t + h;
        ++steps;
    }
    return steps;
}

}  // extern "C"
