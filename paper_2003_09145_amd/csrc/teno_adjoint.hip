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
// the face flux with respect to its stencil.
//
// Pass A (k_adj_chunk, one wave per chunk of 64 consecutive faces of a
// column's face stream, the layout of the forward sweep) stages the chunk's
// cells with the forward sweep's own stage_cell and evaluates each face's
// Roe average and cutoff decisions with the forward face code, so the frozen
// masks are those of the forward pass bit for bit.  Each face then pulls mu_f
// back through the back-projection, the frozen-weight reconstruction and the
// characteristic projection to cotangents of its six cells' split fluxes and
// of the Roe average (linear in mu_f), which are summed per staged cell in
// LDS in a fixed order.  One lane per staged cell then applies the cell's
// own Jacobian (fluxes, primitives, sqrt(rho), H) once and writes the chunk's
// partial gradient of that cell.  Pass B (k_adj_gather, one thread per cell)
// adds the partials of the at most two chunks that touch each image of the
// cell (the cell itself and the ghost cells it supplies), in a fixed order,
// so the result is deterministic without floating-point atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_face.hpp"
#include "teno_host.hpp"

namespace teno {

constexpr int kAdjChunk = 64;  // faces per pass-A chunk (one wave)

// Derivative of the frozen-weight reconstruction sum_k omega_k q_k (eq
// 2.4-2.6, 2.15) with respect to its m-th stencil value (a .. e = v_0 .. v_4)
// for the weights w of one cutoff mask.
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

struct AdjArgs {
    const double* U;
    const double* lam;
    const double* alpha;  // 3 device doubles
    double* P;            // chunk partials [chunk k][NC][cap][ncols]
    double* out;
    int64_t ncell, line_step, stride, col_step, ftot, ncols;
    int64_t kchunks;      // chunks per column
    int32_t n, bc, accumulate, cap;
    // multiply-and-shift division by n + 1, n + 6, ncols, n and the line count
    // of a DIR-2 column (dividends < 2^31); div32: every cell, face and ext
    // index is below 2^31
    uint32_t m1, s1, m6, s6, mc, sc, mn, sn, mb, sb;
    int32_t div32;
    int32_t nb;  // lines of a DIR-2 column (ny)
    double dx;
    SchemeParams sch;
    DecisionConsts dk;
};

// Stencil cell jq - 3 of the extended line numbering (n + 6 cells per line,
// three ghost cells at each end) starting from line be0: its line, its
// interior source cell and whether the ghost image flips the normal momentum.
__device__ __forceinline__ int64_t ext_source(const AdjArgs& A, int64_t colbase, int64_t be0,
                                              int jq, bool* flip) {
    const int np6 = A.n + 6;
    const int bw = div_by(jq, A.m6, A.s6);
    const int j = jq - bw * np6 - 3;
    const int src = ghost_src(A.bc, A.n, j, flip);
    return colbase + (be0 + bw) * A.line_step + (int64_t)src * A.stride;
}

template <int ND, int DIR, bool A5>
__global__ __launch_bounds__(64) void k_adj_chunk(AdjArgs A) {
    constexpr int NC = ND + 2;
    constexpr int NV = 2 * NC + ND + 2;  // f+ (NC), f- (NC), sqrt(rho), u (ND), H
    using LO = LocalOrder<ND, DIR>;
    extern __shared__ double smem[];
    const int cap = A.cap;
    double* omega = smem;       // 24: eq 2.15 weights per cutoff mask
    double* ctab = smem + 24;   // 40: cand_coef per (mask, stencil value)
    double* ext = smem + 64;    // NV x cap staged rows (forward quantities)
    double* acc = ext + (size_t)NV * cap;  // NV x cap cotangents: F (NC, local),
                                           // U (NC, local), sqrt(rho), u (ND), H
    const int lane = threadIdx.x;
    if (lane < 24) omega[lane] = kOmega[lane / 3][lane % 3];
    if (lane < 40) ctab[lane] = cand_coef(&kOmega[lane / 5][0], lane % 5);

    const int64_t chunk = xcd_logical_block(blockIdx.x, gridDim.x);
    int64_t col = 0, k = chunk;
    if (DIR != 0) {  // columns fastest, as in the forward sweep
        k = div_by((int)chunk, A.mc, A.sc);  // chunk < kchunks ncols < 2^31
        col = chunk - k * A.ncols;
    }
    const int n = A.n;
    const int64_t np1 = n + 1, np6 = n + 6;
    const int64_t colbase = col * A.col_step;
    const int64_t F0 = k * kAdjChunk;
    const int64_t F = F0 + lane;
    const bool valid = F < A.ftot;
    const int64_t Fc = valid ? F : F0;
    const int64_t bl0 = A.div32 ? (int64_t)div_by((int)F0, A.m1, A.s1) : F0 / np1;
    const int phi0 = (int)(F0 - bl0 * np1);
    const int tq = phi0 + (int)(Fc - F0);
    const int wraps = div_by(tq, A.m1, A.s1);
    const int64_t bl = bl0 + wraps;             // line of this lane's face
    const int phi = tq - wraps * (int)np1;      // face index in the line
    const int64_t e_lo = F0 + 5 * bl0;
    int64_t Flast = F0 + kAdjChunk - 1;
    if (Flast > A.ftot - 1) Flast = A.ftot - 1;
    const int count = (int)(Flast + 5 * (A.div32 ? (int64_t)div_by((int)Flast, A.m1, A.s1)
                                                  : Flast / np1) + 6 - e_lo);
    const int64_t be0 = A.div32 ? (int64_t)div_by((int)e_lo, A.m6, A.s6) : e_lo / np6;
    const int je0 = (int)(e_lo - be0 * np6);
    const double alpha = A.alpha[DIR];
    const double gm1 = A.sch.gamma - 1.0;

    // ---- stage the chunk's cells exactly as the forward sweep does ---------
    // conserved state of staged cell idx as stored (ghost flip not applied)
    auto load_ext = [&](int idx, double* q, bool* flip) {
        const int64_t cell = ext_source(A, colbase, be0, je0 + idx, flip);
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = A.U[c * A.ncell + cell];
    };
    {
        // one cell ahead: the next cell's loads are in flight meanwhile
        int idx = lane;
        double qn[NC];
        bool fn = false;
        if (idx < count) load_ext(idx, qn, &fn);
        while (idx < count) {
            double q[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = qn[c];
            const bool flip = fn;
            const int cur = idx;
            idx += 64;
            if (idx < count) load_ext(idx, qn, &fn);
            if (flip) q[1 + DIR] = -q[1 + DIR];
            stage_cell<ND, DIR>(q, alpha, gm1, ext, cap, cur);
#pragma unroll
            for (int r = 0; r < NV; ++r) acc[(size_t)r * cap + cur] = 0.0;
        }
    }
    __syncthreads();

    if (valid) {
        const int o = (int)(Fc + 5 * bl - e_lo);  // ext offset of the face's cell i-2
        // cotangent of the face flux (local order)
        const int64_t lbase = colbase + bl * A.line_step;
        double mul[NC];
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) {
            const int64_t c = LO::nat(qq);
            const double lr = (phi <= n - 1) ? A.lam[c * A.ncell + lbase + (int64_t)phi * A.stride] : 0.0;
            const double ll = (phi >= 1) ? A.lam[c * A.ncell + lbase + (int64_t)(phi - 1) * A.stride] : 0.0;
            mul[qq] = (lr - ll) / A.dx;
        }
        const FaceRoe<ND> R = face_roe<ND, DIR>(ext, cap, o, gm1);

        // forward: frozen cutoff masks, and the cotangent of the right
        // eigenvectors through F^ = R fh (R[:, s] depends on un, cs, Hb, q2, ut)
        double un_b = 0.0, cs_b = 0.0, Hb_b = 0.0, q2_b = 0.0, ci_b = 0.0, b1_b = 0.0, b2_b = 0.0;
        double ut_b[ND > 1 ? ND - 1 : 1];
#pragma unroll
        for (int kk = 0; kk < ND - 1; ++kk) ut_b[kk] = 0.0;
        uint32_t masks = 0;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            double Lr[NC];
            left_row<ND>(R, s, Lr);
            double fh = 0.0;
#pragma unroll 1
            for (int sg = 0; sg < 2; ++sg) {
                __asm__ __volatile__("" ::: "memory");
                uint32_t code;
                const double r = char_rec<ND, A5>(ext, cap, o, s, sg, Lr, A.sch, A.dk, omega, &code);
                masks |= (code >> 5) << (3 * (2 * s + sg));
                fh = sg ? fh + r : r;
            }
            if (s == 0 || s == NC - 1) {
                const double sgn = (s == 0) ? -1.0 : 1.0;
                un_b += mul[1] * fh + sgn * R.cs * mul[NC - 1] * fh;
                cs_b += sgn * mul[1] * fh + sgn * R.un * mul[NC - 1] * fh;
                Hb_b += mul[NC - 1] * fh;
#pragma unroll
                for (int kk = 1; kk < ND; ++kk) ut_b[kk - 1] += mul[1 + kk] * fh;
            } else if (s == 1) {
                un_b += mul[1] * fh;
                q2_b += 0.5 * mul[NC - 1] * fh;
#pragma unroll
                for (int kk = 1; kk < ND; ++kk) ut_b[kk - 1] += mul[1 + kk] * fh;
            } else {
#pragma unroll
                for (int kk = 1; kk < ND; ++kk)
                    if (s == 1 + kk) ut_b[kk - 1] += mul[NC - 1] * fh;
            }
        }

        // nu_s = (R^T mu)_s: the cotangent of the characteristic flux fh_s
        double nu[NC];
        {
            double tsum = 0.0;
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) tsum += R.ut[kk - 1] * mul[1 + kk];
            nu[0] = mul[0] + (R.un - R.cs) * mul[1] + tsum + (R.Hb - R.unc) * mul[NC - 1];
            nu[1] = mul[0] + R.un * mul[1] + tsum + R.hq2 * mul[NC - 1];
            nu[NC - 1] = mul[0] + (R.un + R.cs) * mul[1] + tsum + (R.Hb + R.unc) * mul[NC - 1];
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) nu[1 + kk] = mul[1 + kk] + R.ut[kk - 1] * mul[NC - 1];
        }
        double Lrow[NC][NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) left_row<ND>(R, s, Lrow[s]);

        // Stencil cell j of the face (0 .. 5 = i-2 .. i+3): the reconstruction
        // of f+ holds it as value j (j <= 4), that of f- as value 5 - j
        // (j >= 1).  a_s, b_s are the cotangents of those projected values;
        // the split-flux cotangents are L^T a and L^T b, added to the cell's
        // accumulators as F-bar = (f+bar + f-bar)/2 and U-bar = alpha (f+bar -
        // f-bar)/2.  Lanes hold distinct cells at each j, and a wave's LDS
        // operations complete in order, so the sums need no atomics.
        double Lb[NC][NC];  // cotangent of the left eigenvector entries
#pragma unroll
        for (int s = 0; s < NC; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) Lb[s][c] = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int jp = j <= 4 ? j : 4, jm = j >= 1 ? 5 - j : 0;
            double a[NC], b[NC];
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const uint32_t mp = (masks >> (6 * s)) & 7u, mm = (masks >> (6 * s + 3)) & 7u;
                a[s] = (j <= 4) ? nu[s] * ctab[mp * 5 + jp] : 0.0;
                b[s] = (j >= 1) ? nu[s] * ctab[mm * 5 + jm] : 0.0;
            }
            double* cf = acc + o + j;
            const double* fpj = ext + o + j;
            const double* fmj = ext + (size_t)NC * cap + o + j;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double pb = 0.0, mb = 0.0;
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const bool shear = !(s == 0 || s == NC - 1) && s != 1;
                    if (!shear) {
                        pb += Lrow[s][c] * a[s];
                        mb += Lrow[s][c] * b[s];
                    } else if (c == 0) {
                        pb += Lrow[s][0] * a[s];
                        mb += Lrow[s][0] * b[s];
                    } else if (c == s) {
                        pb += a[s];
                        mb += b[s];
                    }
                }
                cf[(size_t)c * cap] += 0.5 * (pb + mb);
                cf[(size_t)(NC + c) * cap] += (0.5 * alpha) * (pb - mb);
                const double fp = fpj[(size_t)c * cap], fm = fmj[(size_t)c * cap];
#pragma unroll
                for (int s = 0; s < NC; ++s) {
                    const bool shear = !(s == 0 || s == NC - 1) && s != 1;
                    if (!shear || c == 0) Lb[s][c] += fp * a[s] + fm * b[s];
                }
            }
            __asm__ __volatile__("" ::: "memory");
        }

        // left eigenvector entries -> Roe scalars
        {
            const double a00 = Lb[0][0], a01 = Lb[0][1], l00 = Lb[NC - 1][0], l01 = Lb[NC - 1][1];
            b2_b += 0.5 * a00 + 0.5 * l00 - Lb[1][0];
            un_b += 0.5 * R.ci * (a00 - l00) - 0.5 * R.b1 * (a01 + l01) + R.b1 * Lb[1][1];
            ci_b += 0.5 * R.un * (a00 - l00) - 0.5 * a01 + 0.5 * l01;
            b1_b += -0.5 * R.un * (a01 + l01) + R.un * Lb[1][1] +
                    0.5 * (Lb[0][NC - 1] + Lb[NC - 1][NC - 1]) - Lb[1][NC - 1];
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) {
                const double t = -0.5 * (Lb[0][1 + kk] + Lb[NC - 1][1 + kk]) + Lb[1][1 + kk];
                b1_b += R.ut[kk - 1] * t;
                ut_b[kk - 1] += R.b1 * t - Lb[1 + kk][0];
            }
        }
        // derived scalars: b2 = b1 q2 / 2, b1 = gm1 / c2, ci = 1 / cs, cs = sqrt(c2),
        // c2 = gm1 (Hb - q2 / 2), q2 = |ub|^2
        q2_b += 0.5 * R.b1 * b2_b;
        b1_b += 0.5 * R.q2 * b2_b;
        double c2_b = -(R.b1 / R.c2) * b1_b;
        cs_b += -(R.ci * R.ci) * ci_b;
        c2_b += cs_b / (2.0 * R.cs);
        Hb_b += gm1 * c2_b;
        q2_b += -0.5 * gm1 * c2_b;
        double ub_b[ND];
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) ub_b[kk] = 2.0 * R.ub[kk] * q2_b;
        ub_b[DIR] += un_b;
#pragma unroll
        for (int kk = 1; kk < ND; ++kk) ub_b[LO::tan_axis(kk)] += ut_b[kk - 1];
        // Roe average of cells o+2 (weight rl) and o+3 (rr), w = 1 / (rl + rr)
        const double* uu = ext + (size_t)(2 * NC + 1) * cap;
        const double* hh = ext + (size_t)(2 * NC + 1 + ND) * cap;
        const double w = R.wsum, rl = R.rl, rr = R.rr;
        const double SH = rl * hh[o + 2] + rr * hh[o + 3];
        double w_b = SH * Hb_b;
        const double SH_b = w * Hb_b;
        double rl_b = hh[o + 2] * SH_b, rr_b = hh[o + 3] * SH_b;
        double ul_b[ND], ur_b[ND];
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            const double u2 = uu[(size_t)kk * cap + o + 2], u3 = uu[(size_t)kk * cap + o + 3];
            w_b += (rl * u2 + rr * u3) * ub_b[kk];
            const double Sk_b = w * ub_b[kk];
            ul_b[kk] = rl * Sk_b;
            ur_b[kk] = rr * Sk_b;
            rl_b += u2 * Sk_b;
            rr_b += u3 * Sk_b;
        }
        rl_b += -(w * w) * w_b;
        rr_b += -(w * w) * w_b;
        double* cr = acc + (size_t)(2 * NC) * cap + o;
        cr[2] += rl_b;
        cr[(size_t)(1 + ND) * cap + 2] += rl * SH_b;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) cr[(size_t)(1 + kk) * cap + 2] += ul_b[kk];
        __asm__ __volatile__("" ::: "memory");
        cr[3] += rr_b;
        cr[(size_t)(1 + ND) * cap + 3] += rr * SH_b;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) cr[(size_t)(1 + kk) * cap + 3] += ur_b[kk];
    }
    // the first staged cell of the per-cell phase is loaded before the barrier
    int idx3 = lane;
    double qn3[NC];
    bool fn3 = false;
    if (idx3 < count) load_ext(idx3, qn3, &fn3);
    __syncthreads();

    // ---- per staged cell: the cell's own Jacobian, once ---------------------
    while (idx3 < count) {
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = qn3[c];
        const bool flip = fn3;
        const int idx = idx3;
        idx3 += 64;
        if (idx3 < count) load_ext(idx3, qn3, &fn3);
        if (flip) q[1 + DIR] = -q[1 + DIR];
        const double rho = q[0], ri = 1.0 / rho, E = q[NC - 1];
        double u[ND], uu2 = 0.0;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            u[kk] = q[1 + kk] * ri;
            uu2 += u[kk] * u[kk];
        }
        const double p = gm1 * (E - 0.5 * rho * uu2);
        const double H = (E + p) * ri;
        double Fb[NC], gq[NC];
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) {
            Fb[LO::nat(qq)] = acc[(size_t)qq * cap + idx];
            gq[LO::nat(qq)] = acc[(size_t)(NC + qq) * cap + idx];
        }
        const double sr_b = acc[(size_t)(2 * NC) * cap + idx];
        const double H_b = acc[(size_t)(2 * NC + 1 + ND) * cap + idx];
        double u_b[ND], m_b[ND];
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            u_b[kk] = acc[(size_t)(2 * NC + 1 + kk) * cap + idx];
            m_b[kk] = 0.0;
        }
        double E_b = 0.0, rho_b = 0.0, p_b = 0.0;
        // flux along DIR: (m_d, m u_d + p e_d, (E + p) u_d)
        m_b[DIR] += Fb[0];
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            m_b[kk] += u[DIR] * Fb[1 + kk];
            u_b[DIR] += q[1 + kk] * Fb[1 + kk];
        }
        p_b += Fb[1 + DIR];
        E_b += u[DIR] * Fb[NC - 1];
        p_b += u[DIR] * Fb[NC - 1];
        u_b[DIR] += (E + p) * Fb[NC - 1];
        // H = (E + p) / rho
        E_b += H_b * ri;
        p_b += H_b * ri;
        rho_b += -H * H_b * ri;
        // sqrt(rho)
        rho_b += sr_b / (2.0 * sqrt(rho));
        // p = (gamma - 1) (E - |m|^2 / (2 rho))
        E_b += gm1 * p_b;
        rho_b += 0.5 * gm1 * uu2 * p_b;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) m_b[kk] += -gm1 * u[kk] * p_b;
        // u_k = m_k / rho
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            m_b[kk] += u_b[kk] * ri;
            rho_b += -u[kk] * u_b[kk] * ri;
        }
        gq[0] += rho_b;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) gq[1 + kk] += m_b[kk];
        gq[NC - 1] += E_b;
        if (flip) gq[1 + DIR] = -gq[1 + DIR];  // ghost image: back to the source's frame
#pragma unroll
        for (int c = 0; c < NC; ++c)
            A.P[((k * NC + c) * cap + idx) * A.ncols + col] = gq[c];
    }
}

// Pass B: every cell adds the chunk partials of its images along DIR.
template <int ND, int DIR>
__global__ __launch_bounds__(256) void k_adj_gather(AdjArgs A) {
    constexpr int NC = ND + 2;
    const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (cell >= A.ncell) return;
    // (column, line, position) of the cell along DIR
    int64_t col, b;
    int i;
    if (A.div32) {
        if (DIR == 0) {
            col = 0;
            b = div_by((int)cell, A.mn, A.sn);
            i = (int)(cell - b * A.n);
        } else {
            const int64_t rest = div_by((int)cell, A.mc, A.sc);  // (z, y) for DIR 1: y fastest
            col = cell - rest * A.ncols;
            const int64_t hi = div_by((int)rest, DIR == 1 ? A.mn : A.mb, DIR == 1 ? A.sn : A.sb);
            const int64_t lo = rest - hi * (DIR == 1 ? A.n : A.nb);
            if (DIR == 1) {
                i = (int)lo;
                b = hi;
            } else {  // DIR 2: rest = z ny + y, lines ordered by y
                b = lo;
                i = (int)hi;
            }
        }
    } else if (DIR == 0) {
        col = 0;
        b = cell / A.n;
        i = (int)(cell - b * A.n);
    } else {
        col = cell % A.ncols;
        const int64_t rest = cell / A.ncols;
        if (DIR == 1) {
            i = (int)(rest % A.n);
            b = rest / A.n;
        } else {
            const int64_t ny = A.stride / A.ncols;
            b = rest % ny;
            i = (int)(rest / ny);
        }
    }
    const int n = A.n;
    // images of the cell on its line: itself and the ghost cells it supplies
    int img[7];
    int nimg = 0;
    img[nimg++] = i;
    if (A.bc == TENO_BC_PERIODIC) {
        if (i >= n - 3) img[nimg++] = i - n;
        if (i <= 2) img[nimg++] = i + n;
    } else if (A.bc == TENO_BC_TRANSMISSIVE) {
        if (i == 0) { img[nimg++] = -1; img[nimg++] = -2; img[nimg++] = -3; }
        if (i == n - 1) { img[nimg++] = n; img[nimg++] = n + 1; img[nimg++] = n + 2; }
    } else {
        if (i <= 2) img[nimg++] = -1 - i;
        if (i >= n - 3) img[nimg++] = 2 * n - 1 - i;
    }
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const int64_t np1 = n + 1;
    for (int t = 0; t < nimg; ++t) {
        // extended cell e of line b is in the stencils of faces e-5 .. e
        const int e = img[t] + 3;
        const int64_t E = b * (n + 6) + e;
        const int64_t Fa = b * np1 + (e - 5 > 0 ? e - 5 : 0);
        const int64_t Fz = b * np1 + (e < n ? e : n);
        const int64_t ka = Fa / kAdjChunk, kz = Fz / kAdjChunk;
        for (int64_t kk = ka; kk <= kz; ++kk) {
            const int64_t F0 = kk * kAdjChunk;
            const int64_t slot =
                E - (F0 + 5 * (A.div32 ? (int64_t)div_by((int)F0, A.m1, A.s1) : F0 / np1));
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += A.P[((kk * NC + c) * A.cap + slot) * A.ncols + col];
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
// Launch geometry of one axis: faces of a column, columns, and the chunk
// partial buffer (chunks per column x NC x cap x columns doubles).
struct AdjAxis {
    int64_t ncols, col_step, line_step, stride, ftot, kchunks;
    int cap;
};

static AdjAxis adj_axis(const teno_grid* g, int d) {
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    AdjAxis X;
    int64_t lines;
    if (d == 0) {
        X.ncols = 1; X.col_step = 0; X.line_step = nx; X.stride = 1; lines = ny * nz;
    } else if (d == 1) {
        X.ncols = nx; X.col_step = 1; X.line_step = nx * ny; X.stride = nx; lines = nz;
    } else {
        X.ncols = nx; X.col_step = 1; X.line_step = nx; X.stride = nx * ny; lines = ny;
    }
    X.ftot = lines * (g->n[d] + 1);
    X.kchunks = (X.ftot + kAdjChunk - 1) / kAdjChunk;
    X.cap = ext_cap_for(g->n[d]);
    return X;
}

static size_t adj_P_bytes(const teno_grid* g) {
    size_t mx = 0;
    for (int d = 0; d < g->ndim; ++d) {
        const AdjAxis X = adj_axis(g, d);
        const size_t b = (size_t)X.kchunks * (g->ndim + 2) * X.cap * X.ncols * sizeof(double);
        if (b > mx) mx = b;
    }
    return mx;
}

static size_t adj_state_bytes(const teno_grid* g) {
    return (size_t)(g->ndim + 2) * g->n[0] * g->n[1] * g->n[2] * sizeof(double);
}

static size_t adj_ws_bytes(const teno_grid* g) {
    return 6 * adj_state_bytes(g) + adj_P_bytes(g) + 256;
}

template <int ND, int DIR>
static hipError_t launch_adj(AdjArgs A, hipStream_t st) {
    constexpr int NV = 2 * (ND + 2) + ND + 2;
    const int64_t nblk = A.kchunks * A.ncols;
    const size_t lds = (size_t)(64 + 2 * NV * A.cap) * sizeof(double);
    if (A.sch.scheme == TENO_SCHEME_TENO5A)
        hipLaunchKernelGGL((k_adj_chunk<ND, DIR, true>), dim3((unsigned)nblk), dim3(64), lds, st, A);
    else
        hipLaunchKernelGGL((k_adj_chunk<ND, DIR, false>), dim3((unsigned)nblk), dim3(64), lds, st, A);
    hipLaunchKernelGGL((k_adj_gather<ND, DIR>), dim3((unsigned)((A.ncell + 255) / 256)), dim3(256), 0,
                       st, A);
    return hipGetLastError();
}

static hipError_t rhs_adjoint_impl(const teno_grid* g, const double* U, const double* alpha,
                                   const double* lam, double* out, double* P, hipStream_t st) {
    for (int d = 0; d < g->ndim; ++d) {
        const AdjAxis X = adj_axis(g, d);
        AdjArgs A;
        memset(&A, 0, sizeof(A));
        A.U = U;
        A.lam = lam;
        A.alpha = alpha;
        A.P = P;
        A.out = out;
        A.ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
        A.n = g->n[d];
        A.bc = g->bc[d];
        A.dx = g->dx[d];
        A.accumulate = d > 0;
        A.cap = X.cap;
        A.sch = scheme_of(g);
        A.dk = decision_consts(g, false);
        A.ncols = X.ncols;
        A.col_step = X.col_step;
        A.line_step = X.line_step;
        A.stride = X.stride;
        A.ftot = X.ftot;
        A.kchunks = X.kchunks;
        if (A.kchunks * A.ncols > (int64_t(1) << 31) - 64) return hipErrorInvalidValue;
        const int64_t nb = (d == 2) ? A.stride / A.ncols : 1;  // lines of a DIR-2 column
        const DivMagic d1 = div_magic((uint32_t)(A.n + 1)), d6 = div_magic((uint32_t)(A.n + 6)),
                       dc = div_magic((uint32_t)A.ncols), dn = div_magic((uint32_t)A.n),
                       db = div_magic((uint32_t)nb);
        A.m1 = d1.m; A.s1 = d1.sh; A.m6 = d6.m; A.s6 = d6.sh; A.mc = dc.m; A.sc = dc.sh;
        A.mn = dn.m; A.sn = dn.sh; A.mb = db.m; A.sb = db.sh;
        A.nb = (int32_t)nb;
        // largest index: a cell, or an ext index ftot + 5 lines (+ a chunk's tail)
        const int64_t lines = A.ftot / (A.n + 1);
        A.div32 = (A.ncell < (int64_t(1) << 31) && A.ftot + 6 * lines + 128 < (int64_t(1) << 31)) ? 1 : 0;
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
    double* P = (double*)((char*)ws + 6 * adj_state_bytes(g));
    return rhs_adjoint_impl(g, U, alpha, lam, gradU, P, (hipStream_t)stream) == hipSuccess
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
    double* P = (double*)(w + 6 * sb);
    const double* dtp = &ctrl->dt;
    // stage states of the step with its recorded dt and speeds
    if (stage_frozen(g, Un, Un, U1, R, &ctrl->alpha[0][0], dtp, 1, st) != hipSuccess ||
        stage_frozen(g, U1, Un, U2, R, &ctrl->alpha[1][0], dtp, 2, st) != hipSuccess)
        return TENO_ERR_DEVICE;
    const int64_t n = (int64_t)(g->ndim + 2) * g->n[0] * g->n[1] * g->n[2];
    const unsigned blocks = (unsigned)((n + 255) / 256);
    // transpose of eq 4.3, 4.2, 4.1
    if (rhs_adjoint_impl(g, U2, &ctrl->alpha[2][0], lam, T, P, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_adj_combo, dim3(blocks), dim3(256), 0, st, 2, n, dtp, lam, L2, L1, T, L2);
    if (rhs_adjoint_impl(g, U1, &ctrl->alpha[1][0], L2, T, P, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_adj_combo, dim3(blocks), dim3(256), 0, st, 1, n, dtp, lam, L2, L1, T, L1);
    if (rhs_adjoint_impl(g, Un, &ctrl->alpha[0][0], L1, T, P, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_adj_combo, dim3(blocks), dim3(256), 0, st, 0, n, dtp, lam, L2, L1, T, lam);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

}  // extern "C"
