// Discrete adjoint of the TENO5-LAD Euler right-hand side and of one SSP-RK3
// step (Peng et al., arXiv:2003.09145, Sec. 2-4).
//
// With the cutoff flags delta_k (eq 2.14) and the Lax-Friedrichs speeds held
// fixed, the weights omega_k of eq 2.15 are constants and every face flux is a
// smooth function of its six stencil cells.  For a cotangent lambda of
// dU/dt = L(U), summation by parts of eq 2.2 gives
//     <lambda, L(U)> = sum over faces f = i+1/2 of <mu_f, F^_f>,
//     mu_f = (lambda_{i+1} - lambda_i) / dx   (lambda = 0 outside the line),
// so A(U)^T lambda is the sum over faces of J_f^T mu_f, J_f the Jacobian of
// the face flux with respect to its stencil.  Pass A (one thread per face)
// recomputes the forward face -- the cutoff decisions come out identical to
// the forward pass because the same arithmetic is evaluated -- and
// back-propagates mu_f through the back-projection, the frozen-weight
// reconstruction, the characteristic projection, the Roe average and
// eigenvectors and the flux splitting, writing 6 x ncomp stencil
// contributions.  Pass B (one thread per cell) gathers the contributions of
// every face whose stencil holds the cell or one of its ghost images, in a
// fixed order, so the result is deterministic without floating-point
// atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_face.hpp"
#include "teno_host.hpp"

namespace teno {

// Derivatives of the three candidate fluxes of eq 2.4-2.6 with respect to
// (a, b, c, d, e) = (f_{i-2} .. f_{i+2}).
__device__ __forceinline__ double cand_coef(const double* w, int m) {
    constexpr double c13 = 1.0 / 3.0, c76 = 7.0 / 6.0, c116 = 11.0 / 6.0, c16 = 1.0 / 6.0,
                     c56 = 5.0 / 6.0;
    switch (m) {
        case 0: return w[0] * c13;
        case 1: return -(w[0] * c76) - w[1] * c16;
        case 2: return (w[0] * c116 + w[1] * c56) + w[2] * c13;
        case 3: return w[1] * c13 + w[2] * c56;
        default: return -(w[2] * c16);
    }
}

template <int ND, int DIR, bool A5>
__device__ __forceinline__ void face_adjoint(const double (&q)[6][ND + 2], double alpha,
                                             double gm1, const SchemeParams& S,
                                             const DecisionConsts& K,
                                             const double* __restrict__ omega,
                                             const double* mu_nat, double (&gq)[6][ND + 2]) {
    constexpr int NC = ND + 2;
    using LO = LocalOrder<ND, DIR>;
    // ---- forward: primitives, fluxes and split fluxes of the six cells ----
    double rho[6], u[6][ND], p[6], H[6], sr[6], fp[6][NC], fm[6][NC];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        rho[j] = q[j][0];
        const double rr = rcp_nr(rho[j]);
#pragma unroll
        for (int k = 0; k < ND; ++k) u[j][k] = cr_div_r(q[j][1 + k], rho[j], rr);
        double mu = q[j][1] * u[j][0];
#pragma unroll
        for (int k = 1; k < ND; ++k) mu = mu + q[j][1 + k] * u[j][k];
        p[j] = gm1 * (q[j][NC - 1] - 0.5 * mu);
        H[j] = cr_div_r(q[j][NC - 1] + p[j], rho[j], rr);
        sr[j] = cr_sqrt(rho[j]);
        double F[NC];
        F[0] = q[j][1 + DIR];
#pragma unroll
        for (int k = 0; k < ND; ++k)
            F[1 + k] = (k == DIR) ? q[j][1 + k] * u[j][DIR] + p[j] : q[j][1 + k] * u[j][DIR];
        F[NC - 1] = (q[j][NC - 1] + p[j]) * u[j][DIR];
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) {
            const int g = LO::nat(qq);
            fp[j][qq] = 0.5 * (F[g] + alpha * q[j][g]);
            fm[j][qq] = 0.5 * (F[g] - alpha * q[j][g]);
        }
    }
    // ---- Roe average and eigenvectors (local order) ------------------------
    const double rl = sr[2], rr = sr[3];
    const double rsum = rl + rr;
    const double w = cr_div_r(1.0, rsum, rcp_nr(rsum));
    double Sk[ND], ub[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        Sk[k] = rl * u[2][k] + rr * u[3][k];
        ub[k] = Sk[k] * w;
    }
    const double SH = rl * H[2] + rr * H[3];
    const double Hb = SH * w;
    double q2 = ub[0] * ub[0];
#pragma unroll
    for (int k = 1; k < ND; ++k) q2 = q2 + ub[k] * ub[k];
    const double c2 = gm1 * (Hb - 0.5 * q2);
    const double cs = cr_sqrt(c2);
    const double ci = cr_div_r(1.0, cs, rcp_nr(cs));
    const double b1 = cr_div_r(gm1, c2, rcp_nr(c2));
    const double b2 = (0.5 * q2) * b1;
    const double un = ub[DIR];
    double ut[ND > 1 ? ND - 1 : 1];
#pragma unroll
    for (int k = 1; k < ND; ++k) ut[k - 1] = ub[LO::tan_axis(k)];
    double L[NC][NC], R[NC][NC];
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) L[a][b] = R[a][b] = 0.0;
    const double unci = un * ci, b1un = b1 * un, unc = un * cs;
    L[0][0] = 0.5 * (b2 + unci);
    L[0][1] = 0.5 * (-b1un - ci);
    L[NC - 1][0] = 0.5 * (b2 - unci);
    L[NC - 1][1] = 0.5 * (-b1un + ci);
    L[1][0] = 1.0 - b2;
    L[1][1] = b1un;
#pragma unroll
    for (int k = 1; k < ND; ++k) {
        const double b1ut = b1 * ut[k - 1];
        L[0][1 + k] = 0.5 * (-b1ut);
        L[NC - 1][1 + k] = 0.5 * (-b1ut);
        L[1][1 + k] = b1ut;
        L[1 + k][0] = -ut[k - 1];
        L[1 + k][1 + k] = 1.0;
        R[1 + k][0] = ut[k - 1];
        R[1 + k][1] = ut[k - 1];
        R[1 + k][NC - 1] = ut[k - 1];
        R[1 + k][1 + k] = 1.0;
        R[NC - 1][1 + k] = ut[k - 1];
    }
    L[0][NC - 1] = 0.5 * b1;
    L[NC - 1][NC - 1] = 0.5 * b1;
    L[1][NC - 1] = -b1;
    R[0][0] = 1.0;
    R[0][1] = 1.0;
    R[0][NC - 1] = 1.0;
    R[1][0] = un - cs;
    R[1][1] = un;
    R[1][NC - 1] = un + cs;
    R[NC - 1][0] = Hb - unc;
    R[NC - 1][1] = 0.5 * q2;
    R[NC - 1][NC - 1] = Hb + unc;

    // ---- forward reconstruction: frozen masks and the field fluxes ---------
    uint32_t mask[NC][2];
    double fh[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        double rsg[2];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            double v[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int j = sg ? 5 - m : m;
                const double* f = sg ? fm[j] : fp[j];
                double acc = L[s][0] * f[0];
#pragma unroll
                for (int c = 1; c < NC; ++c) acc = acc + L[s][c] * f[c];
                v[m] = acc;
            }
            uint32_t code;
            rsg[sg] = teno5_rec_fast<A5>(S, K, omega, v[0], v[1], v[2], v[3], v[4], &code);
            mask[s][sg] = code >> 5;
        }
        fh[s] = rsg[0] + rsg[1];
    }

    // ---- reverse ---------------------------------------------------------
    double mul[NC];
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) mul[qq] = mu_nat[LO::nat(qq)];
    double fpb[6][NC], fmb[6][NC], Lb[NC][NC];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) fpb[j][c] = fmb[j][c] = 0.0;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) Lb[a][b] = 0.0;
    double un_b = 0.0, cs_b = 0.0, ci_b = 0.0, b1_b = 0.0, b2_b = 0.0, Hb_b = 0.0, q2_b = 0.0;
    double ut_b[ND > 1 ? ND - 1 : 1];
#pragma unroll
    for (int k = 0; k < ND - 1; ++k) ut_b[k] = 0.0;

#pragma unroll
    for (int s = 0; s < NC; ++s) {
        // F^ = R fh: cotangent of fh_s and of R[:, s]
        double nu = 0.0;
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) nu += R[qq][s] * mul[qq];
        const bool acoustic = (s == 0 || s == NC - 1);
        const double sgn = (s == 0) ? -1.0 : 1.0;
        if (acoustic) {
            un_b += mul[1] * fh[s];
            cs_b += sgn * mul[1] * fh[s];
            Hb_b += mul[NC - 1] * fh[s];
            un_b += sgn * cs * mul[NC - 1] * fh[s];
            cs_b += sgn * un * mul[NC - 1] * fh[s];
#pragma unroll
            for (int k = 1; k < ND; ++k) ut_b[k - 1] += mul[1 + k] * fh[s];
        } else if (s == 1) {
            un_b += mul[1] * fh[s];
            q2_b += 0.5 * mul[NC - 1] * fh[s];
#pragma unroll
            for (int k = 1; k < ND; ++k) ut_b[k - 1] += mul[1 + k] * fh[s];
        } else {
            ut_b[s - 2] += mul[NC - 1] * fh[s];
        }
        // frozen-weight reconstruction of f+ (cells 0..4) and f- (cells 5..1)
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const double* wts = omega + 3 * mask[s][sg];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int j = sg ? 5 - m : m;
                const double vb = nu * cand_coef(wts, m);
                const double* f = sg ? fm[j] : fp[j];
                double* fb = sg ? fmb[j] : fpb[j];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    fb[c] += L[s][c] * vb;
                    Lb[s][c] += f[c] * vb;
                }
            }
        }
    }
    // left eigenvector entries -> Roe scalars
    {
        const double a00 = Lb[0][0], a01 = Lb[0][1], l00 = Lb[NC - 1][0], l01 = Lb[NC - 1][1];
        b2_b += 0.5 * a00 + 0.5 * l00 - Lb[1][0];
        un_b += 0.5 * ci * (a00 - l00) - 0.5 * b1 * (a01 + l01) + b1 * Lb[1][1];
        ci_b += 0.5 * un * (a00 - l00) - 0.5 * a01 + 0.5 * l01;
        b1_b += -0.5 * un * (a01 + l01) + un * Lb[1][1] + 0.5 * (Lb[0][NC - 1] + Lb[NC - 1][NC - 1]) -
                Lb[1][NC - 1];
#pragma unroll
        for (int k = 1; k < ND; ++k) {
            const double t = -0.5 * (Lb[0][1 + k] + Lb[NC - 1][1 + k]) + Lb[1][1 + k];
            b1_b += ut[k - 1] * t;
            ut_b[k - 1] += b1 * t - Lb[1 + k][0];
        }
    }
    // derived scalars
    q2_b += 0.5 * b1 * b2_b;
    b1_b += 0.5 * q2 * b2_b;
    double c2_b = -(b1 / c2) * b1_b;
    cs_b += -(ci * ci) * ci_b;
    c2_b += cs_b / (2.0 * cs);
    Hb_b += gm1 * c2_b;
    q2_b += -0.5 * gm1 * c2_b;
    double ub_b[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) ub_b[k] = 2.0 * ub[k] * q2_b;
    ub_b[DIR] += un_b;
#pragma unroll
    for (int k = 1; k < ND; ++k) ub_b[LO::tan_axis(k)] += ut_b[k - 1];
    // Roe average -> cells 2 and 3
    double w_b = SH * Hb_b;
    const double SH_b = w * Hb_b;
    double u_b[6][ND], p_b[6], H_b[6], sr_b[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        p_b[j] = H_b[j] = sr_b[j] = 0.0;
#pragma unroll
        for (int k = 0; k < ND; ++k) u_b[j][k] = 0.0;
    }
    H_b[2] += rl * SH_b;
    H_b[3] += rr * SH_b;
    double rl_b = H[2] * SH_b, rr_b = H[3] * SH_b;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        w_b += Sk[k] * ub_b[k];
        const double Sk_b = w * ub_b[k];
        u_b[2][k] += rl * Sk_b;
        u_b[3][k] += rr * Sk_b;
        rl_b += u[2][k] * Sk_b;
        rr_b += u[3][k] * Sk_b;
    }
    rl_b += -(w * w) * w_b;
    rr_b += -(w * w) * w_b;
    sr_b[2] += rl_b;
    sr_b[3] += rr_b;
    // split fluxes -> fluxes and states; fluxes and primitives -> states
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double Fb[NC];
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) {
            const int g = LO::nat(qq);
            Fb[g] = 0.5 * (fpb[j][qq] + fmb[j][qq]);
            gq[j][g] = 0.5 * alpha * (fpb[j][qq] - fmb[j][qq]);
        }
        const double E = q[j][NC - 1];
        double m_b[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) m_b[k] = 0.0;
        double E_b = 0.0, rho_b = 0.0;
        // flux along DIR
        m_b[DIR] += Fb[0];
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            m_b[k] += u[j][DIR] * Fb[1 + k];
            u_b[j][DIR] += q[j][1 + k] * Fb[1 + k];
        }
        p_b[j] += Fb[1 + DIR];
        E_b += u[j][DIR] * Fb[NC - 1];
        p_b[j] += u[j][DIR] * Fb[NC - 1];
        u_b[j][DIR] += (E + p[j]) * Fb[NC - 1];
        // H = (E + p) / rho
        E_b += H_b[j] / rho[j];
        p_b[j] += H_b[j] / rho[j];
        rho_b += -H[j] * H_b[j] / rho[j];
        // sqrt(rho)
        rho_b += sr_b[j] / (2.0 * sr[j]);
        // p = (gamma - 1) (E - |m|^2 / (2 rho))
        double uu = 0.0;
#pragma unroll
        for (int k = 0; k < ND; ++k) uu += u[j][k] * u[j][k];
        E_b += gm1 * p_b[j];
        rho_b += 0.5 * gm1 * uu * p_b[j];
#pragma unroll
        for (int k = 0; k < ND; ++k) m_b[k] += -gm1 * u[j][k] * p_b[j];
        // u_k = m_k / rho
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            m_b[k] += u_b[j][k] / rho[j];
            rho_b += -u[j][k] * u_b[j][k] / rho[j];
        }
        gq[j][0] += rho_b;
#pragma unroll
        for (int k = 0; k < ND; ++k) gq[j][1 + k] += m_b[k];
        gq[j][NC - 1] += E_b;
    }
}

struct AdjArgs {
    const double* U;
    const double* lam;
    const double* alpha;  // 3 device doubles
    double* G;            // [ncols][ftot][6][NC]
    double* out;
    int64_t ncell, line_step, stride, col_step, ftot, ncols;
    int32_t n, bc, accumulate;
    double dx;
    SchemeParams sch;
    DecisionConsts dk;
};

template <int ND, int DIR, bool A5>
__global__ __launch_bounds__(64) void k_adj_faces(AdjArgs A) {
    constexpr int NC = ND + 2;
    __shared__ double omega[24];
    if (threadIdx.x < 24) omega[threadIdx.x] = kOmega[threadIdx.x / 3][threadIdx.x % 3];
    __syncthreads();
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= A.ncols * A.ftot) return;
    const int64_t col = id / A.ftot, F = id - col * A.ftot;
    const int n = A.n;
    const int64_t b = F / (n + 1);
    const int phi = (int)(F - b * (n + 1));
    const int64_t base = col * A.col_step + b * A.line_step;
    double q[6][NC];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        bool flip;
        const int src = ghost_src(A.bc, n, phi - 3 + m, &flip);
        const int64_t cell = base + (int64_t)src * A.stride;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[m][c] = A.U[c * A.ncell + cell];
        if (flip) q[m][1 + DIR] = -q[m][1 + DIR];
    }
    double mu[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double lr = (phi <= n - 1) ? A.lam[c * A.ncell + base + (int64_t)phi * A.stride] : 0.0;
        const double ll = (phi >= 1) ? A.lam[c * A.ncell + base + (int64_t)(phi - 1) * A.stride] : 0.0;
        mu[c] = (lr - ll) / A.dx;
    }
    double gq[6][NC];
    face_adjoint<ND, DIR, A5>(q, A.alpha[DIR], A.sch.gamma - 1.0, A.sch, A.dk, omega, mu, gq);
    double* Gp = A.G + id * 6 * NC;
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int c = 0; c < NC; ++c) Gp[m * NC + c] = gq[m][c];
}

template <int ND, int DIR>
__global__ __launch_bounds__(256) void k_adj_cells(AdjArgs A) {
    constexpr int NC = ND + 2;
    const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (cell >= A.ncell) return;
    // (column, line, position) of the cell along DIR
    int64_t col, b;
    int i;
    if (DIR == 0) {
        col = 0;
        b = cell / A.n;
        i = (int)(cell - b * A.n);
    } else {
        col = cell % A.ncols;
        const int64_t rest = cell / A.ncols;  // (z, y) for DIR 1: y fastest
        if (DIR == 1) {
            i = (int)(rest % A.n);
            b = rest / A.n;
        } else {  // DIR 2: rest = z ny + y, lines ordered by y
            const int64_t ny = A.stride / A.ncols;
            b = rest % ny;
            i = (int)(rest / ny);
        }
    }
    const int n = A.n;
    // images of the cell on its line: itself and the ghost cells it supplies
    int img[7];
    bool flp[7];
    int nimg = 0;
    img[nimg] = i;
    flp[nimg++] = false;
    if (A.bc == TENO_BC_PERIODIC) {
        if (i >= n - 3) { img[nimg] = i - n; flp[nimg++] = false; }
        if (i <= 2) { img[nimg] = i + n; flp[nimg++] = false; }
    } else if (A.bc == TENO_BC_TRANSMISSIVE) {
        if (i == 0) { img[nimg] = -1; flp[nimg++] = false; img[nimg] = -2; flp[nimg++] = false; img[nimg] = -3; flp[nimg++] = false; }
        if (i == n - 1) { img[nimg] = n; flp[nimg++] = false; img[nimg] = n + 1; flp[nimg++] = false; img[nimg] = n + 2; flp[nimg++] = false; }
    } else {
        if (i <= 2) { img[nimg] = -1 - i; flp[nimg++] = true; }
        if (i >= n - 3) { img[nimg] = 2 * n - 1 - i; flp[nimg++] = true; }
    }
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const double* Gl = A.G + (col * A.ftot + b * (n + 1)) * 6 * NC;
    for (int t = 0; t < nimg; ++t) {
        for (int m = 0; m < 6; ++m) {
            const int phi = img[t] + 3 - m;
            if (phi < 0 || phi > n) continue;
            const double* Gp = Gl + ((int64_t)phi * 6 + m) * NC;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double v = Gp[c];
                acc[c] += (flp[t] && c == 1 + DIR) ? -v : v;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double* o = A.out + c * A.ncell + cell;
        *o = A.accumulate ? *o + acc[c] : acc[c];
    }
}

// Elementwise combinations of the RK3 transpose (dt read from the device).
__global__ void k_adj_combo(int which, int64_t n, const double* dtp, const double* lam,
                            const double* l2, const double* l1, const double* T, double* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = *dtp;
    if (which == 2) {
        out[i] = (2.0 / 3.0) * lam[i] + (2.0 / 3.0) * (h * T[i]);
    } else if (which == 1) {
        out[i] = 0.25 * l2[i] + 0.25 * (h * T[i]);
    } else {
        out[i] = (((1.0 / 3.0) * lam[i] + 0.75 * l2[i]) + l1[i]) + h * T[i];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int64_t adj_faces(const teno_grid* g, int d) {
    const int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
    return ncell / g->n[d] * (g->n[d] + 1);
}

static size_t adj_G_bytes(const teno_grid* g) {
    int64_t mx = 0;
    for (int d = 0; d < g->ndim; ++d) {
        const int64_t f = adj_faces(g, d);
        if (f > mx) mx = f;
    }
    return (size_t)mx * 6 * (g->ndim + 2) * sizeof(double);
}

static size_t adj_state_bytes(const teno_grid* g) {
    return (size_t)(g->ndim + 2) * g->n[0] * g->n[1] * g->n[2] * sizeof(double);
}

static size_t adj_ws_bytes(const teno_grid* g) {
    return 6 * adj_state_bytes(g) + adj_G_bytes(g) + 256;
}

template <int ND, int DIR>
static hipError_t launch_adj(AdjArgs A, hipStream_t st) {
    const int64_t nf = A.ncols * A.ftot;
    if (A.sch.scheme == TENO_SCHEME_TENO5A)
        hipLaunchKernelGGL((k_adj_faces<ND, DIR, true>), dim3((unsigned)((nf + 63) / 64)), dim3(64), 0,
                           st, A);
    else
        hipLaunchKernelGGL((k_adj_faces<ND, DIR, false>), dim3((unsigned)((nf + 63) / 64)), dim3(64),
                           0, st, A);
    hipLaunchKernelGGL((k_adj_cells<ND, DIR>), dim3((unsigned)((A.ncell + 255) / 256)), dim3(256), 0, st,
                       A);
    return hipGetLastError();
}

static hipError_t rhs_adjoint_impl(const teno_grid* g, const double* U, const double* alpha,
                                   const double* lam, double* out, double* G, hipStream_t st) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    for (int d = 0; d < g->ndim; ++d) {
        AdjArgs A;
        memset(&A, 0, sizeof(A));
        A.U = U;
        A.lam = lam;
        A.alpha = alpha;
        A.G = G;
        A.out = out;
        A.ncell = (int64_t)nx * ny * nz;
        A.n = g->n[d];
        A.bc = g->bc[d];
        A.dx = g->dx[d];
        A.accumulate = d > 0;
        A.sch = scheme_of(g);
        A.dk = decision_consts(g, false);
        int64_t lines;
        if (d == 0) {
            A.ncols = 1; A.col_step = 0; A.line_step = nx; A.stride = 1; lines = (int64_t)ny * nz;
        } else if (d == 1) {
            A.ncols = nx; A.col_step = 1; A.line_step = (int64_t)nx * ny; A.stride = nx; lines = nz;
        } else {
            A.ncols = nx; A.col_step = 1; A.line_step = nx; A.stride = (int64_t)nx * ny; lines = ny;
        }
        A.ftot = lines * (A.n + 1);
        hipError_t e = hipErrorInvalidValue;
        switch (g->ndim * 4 + d) {
            case 4: e = launch_adj<1, 0>(A, st); break;
            case 8: e = launch_adj<2, 0>(A, st); break;
            case 9: e = launch_adj<2, 1>(A, st); break;
            case 12: e = launch_adj<3, 0>(A, st); break;
            case 13: e = launch_adj<3, 1>(A, st); break;
            case 14: e = launch_adj<3, 2>(A, st); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace teno

using namespace teno;

// forward sweeps of one RK stage with frozen speeds (defined in teno_kernels.hip)
namespace teno {
hipError_t stage_frozen(const teno_grid* g, const double* Uin, const double* Un, double* Uout,
                        double* R, const double* alpha, const double* dtp, int rk, hipStream_t st);
}

extern "C" {

size_t teno_adjoint_workspace_bytes(const teno_grid* g) {
    if (validate(g) != TENO_OK) return 0;
    return adj_ws_bytes(g);
}

int teno_rhs_adjoint(const teno_grid* g, const double* U, const double* alpha, const double* lam,
                     double* gradU, void* ws, size_t ws_bytes, void* stream) {
    if (validate(g) != TENO_OK || U == nullptr || alpha == nullptr || lam == nullptr ||
        gradU == nullptr || ws == nullptr || ws_bytes < adj_ws_bytes(g) ||
        g->boundary_dev != nullptr)
        return TENO_ERR_ARG;
    double* G = (double*)((char*)ws + 6 * adj_state_bytes(g));
    return rhs_adjoint_impl(g, U, alpha, lam, gradU, G, (hipStream_t)stream) == hipSuccess
               ? TENO_OK
               : TENO_ERR_DEVICE;
}

int teno_step_adjoint(const teno_grid* g, const double* Un, const teno_ctrl* ctrl, double* lam,
                      void* ws, size_t ws_bytes, void* stream) {
    if (validate(g) != TENO_OK || Un == nullptr || ctrl == nullptr || lam == nullptr ||
        ws == nullptr || ws_bytes < adj_ws_bytes(g) || g->boundary_dev != nullptr)
        return TENO_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const size_t sb = adj_state_bytes(g);
    char* w = (char*)ws;
    double* U1 = (double*)w;
    double* U2 = (double*)(w + sb);
    double* L2 = (double*)(w + 2 * sb);
    double* L1 = (double*)(w + 3 * sb);
    double* T = (double*)(w + 4 * sb);
    double* R = (double*)(w + 5 * sb);
    double* G = (double*)(w + 6 * sb);
    const double* dtp = &ctrl->dt;
    // stage states of the step with its recorded dt and speeds
    if (stage_frozen(g, Un, Un, U1, R, &ctrl->alpha[0][0], dtp, 1, st) != hipSuccess ||
        stage_frozen(g, U1, Un, U2, R, &ctrl->alpha[1][0], dtp, 2, st) != hipSuccess)
        return TENO_ERR_DEVICE;
    const int64_t n = (int64_t)(g->ndim + 2) * g->n[0] * g->n[1] * g->n[2];
    const unsigned blocks = (unsigned)((n + 255) / 256);
    // transpose of eq 4.3, 4.2, 4.1
    if (rhs_adjoint_impl(g, U2, &ctrl->alpha[2][0], lam, T, G, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_adj_combo, dim3(blocks), dim3(256), 0, st, 2, n, dtp, lam, L2, L1, T, L2);
    if (rhs_adjoint_impl(g, U1, &ctrl->alpha[1][0], L2, T, G, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_adj_combo, dim3(blocks), dim3(256), 0, st, 1, n, dtp, lam, L2, L1, T, L1);
    if (rhs_adjoint_impl(g, Un, &ctrl->alpha[0][0], L1, T, G, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_adj_combo, dim3(blocks), dim3(256), 0, st, 0, n, dtp, lam, L2, L1, T, lam);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

}  // extern "C"
