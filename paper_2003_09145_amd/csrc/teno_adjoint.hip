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
// partial gradient of that cell.  Pass B (k_adj_gather, one thread per cell,
// once for all axes) adds the partials of the at most two chunks that touch
// each image of the cell along each axis (the cell itself and the ghost
// cells it supplies), in a fixed order, so the result is deterministic
// without floating-point atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_face.hpp"
#include "teno_host.hpp"

namespace teno {

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

// The reverse-mode arithmetic below is not held to the forward path's
// bit-for-bit order (its bar is a relative error against the oracle's forward
// mode), so its sums of products are fused multiply-adds.
__device__ __forceinline__ double fmad(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

// Derivatives of the all-kept (mask 7) reconstruction with respect to its
// stencil values v_0 .. v_4: cand_coef on the mask-7 weights.
__device__ __forceinline__ constexpr double lin_coef(int m) {
    return m == 0   ? omega_of(7, 0) * (1.0 / 3.0)
           : m == 1 ? -(omega_of(7, 0) * (7.0 / 6.0)) - omega_of(7, 1) * (1.0 / 6.0)
           : m == 2 ? (omega_of(7, 0) * (11.0 / 6.0) + omega_of(7, 1) * (5.0 / 6.0)) +
                          omega_of(7, 2) * (1.0 / 3.0)
           : m == 3 ? omega_of(7, 1) * (1.0 / 3.0) + omega_of(7, 2) * (5.0 / 6.0)
                    : -(omega_of(7, 2) * (1.0 / 6.0));
}

// Reverse sums of one face over its stencil cells j = 0 .. 5 (cells i-2 ..
// i+3).  The reconstruction of f+ holds cell j as value j (j <= 4), that of
// f- as value 5 - j (j >= 1); a_s, b_s are the cotangents of those projected
// values of characteristic field s: nu_s times the derivative of the
// frozen-weight reconstruction.  LM (compile time): the fields whose masks
// are 7 for both signs on every face of the wave; their reconstruction is the
// linear one for all of them, so their part of the sums factors through one
// linear reconstruction per component (rev_read_fold) and through
// g = sum_s L[s, :] nu_s (rev_acc).

// Folds the cotangent x = Lb[s, :] of row s of the left eigenvector matrix
// into the cotangents of the Roe scalars it is built from (rows of
// left_row: acoustic 0.5 (b2 +- un ci, -b1 un -+ ci, -b1 ut, b1), entropy
// (1 - b2, b1 un, b1 ut, -b1), shear (-ut, unit)).  Linear in x, so the rows
// can be folded one at a time.
template <int ND>
__device__ __forceinline__ void fold_row(int s, const double* x, const FaceRoe<ND>& R,
                                         double& un_b, double& ci_b, double& b1_b,
                                         double& b2_b, double* ut_b) {
    constexpr int NC = ND + 2;
    if (s == 0 || s == NC - 1) {
        const double sg = (s == 0) ? 0.5 : -0.5;
        b2_b = fmad(0.5, x[0], b2_b);
        un_b = fmad(sg * R.ci, x[0], fmad(-0.5 * R.b1, x[1], un_b));
        ci_b = fmad(sg * R.un, x[0], fmad(-sg, x[1], ci_b));
        b1_b = fmad(-0.5 * R.un, x[1], fmad(0.5, x[NC - 1], b1_b));
#pragma unroll
        for (int kk = 1; kk < ND; ++kk) {
            b1_b = fmad(-0.5 * R.ut[kk - 1], x[1 + kk], b1_b);
            ut_b[kk - 1] = fmad(-0.5 * R.b1, x[1 + kk], ut_b[kk - 1]);
        }
    } else if (s == 1) {
        b2_b -= x[0];
        un_b = fmad(R.b1, x[1], un_b);
        b1_b = fmad(R.un, x[1], b1_b - x[NC - 1]);
#pragma unroll
        for (int kk = 1; kk < ND; ++kk) {
            b1_b = fmad(R.ut[kk - 1], x[1 + kk], b1_b);
            ut_b[kk - 1] = fmad(R.b1, x[1 + kk], ut_b[kk - 1]);
        }
    } else if (s >= 2) {
        ut_b[s - 2] -= x[0];
    }
}

// Read phase of the reverse sums: Lb[s, c] = sum_j f+_j[c] a_s + f-_j[c] b_s
// (the cotangent of the left eigenvector entries), folded row by row into
// the Roe-scalar cotangents.  Linear fields: one linear reconstruction h of
// f+ and f- per component, Lb[s, :] = nu_s h.  The others one field at a
// time, re-reading the stencil, so that no more than one row is live.
template <int ND, int LM>
__device__ __forceinline__ void rev_read_fold(const double* __restrict__ ext, int cap, int o,
                                              uint32_t masks, const double (&nu)[ND + 2],
                                              const double* __restrict__ ctab,
                                              const FaceRoe<ND>& R, double& un_b, double& ci_b,
                                              double& b1_b, double& b2_b, double* ut_b) {
    constexpr int NC = ND + 2;
    const double* fp0 = ext + o;
    const double* fm0 = ext + (size_t)NC * cap + o;
    if (LM != 0) {
        double h[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c] = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (j <= 4) h[c] = fmad(lin_coef(j), fp0[(size_t)c * cap + j], h[c]);
                if (j >= 1) h[c] = fmad(lin_coef(5 - j), fm0[(size_t)c * cap + j], h[c]);
            }
        }
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            if (!(LM & (1 << s))) continue;
            double x[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = nu[s] * h[c];
            fold_row<ND>(s, x, R, un_b, ci_b, b1_b, b2_b, ut_b);
        }
    }
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (LM & (1 << s)) continue;
        // each field reads the stencil afresh (the compiler would otherwise
        // hold all of it in registers across the fields)
        __asm__ __volatile__("" ::: "memory");
        const bool shear = !(s == 0 || s == NC - 1) && s != 1;
        const uint32_t mp = (masks >> (6 * s)) & 7u, mm = (masks >> (6 * s + 3)) & 7u;
        double x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double a = (j <= 4) ? nu[s] * ctab[mp * 5 + (j <= 4 ? j : 4)] : 0.0;
            const double b = (j >= 1) ? nu[s] * ctab[mm * 5 + (j >= 1 ? 5 - j : 0)] : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (shear && c != 0) continue;
                x[c] = fmad(fp0[(size_t)c * cap + j], a, fmad(fm0[(size_t)c * cap + j], b, x[c]));
            }
        }
        fold_row<ND>(s, x, R, un_b, ci_b, b1_b, b2_b, ut_b);
    }
}

// Accumulation of L^T a and L^T b into the stencil cells' cotangent rows as
// F-bar = (f+bar + f-bar)/2 and U-bar = alpha (f+bar - f-bar)/2.  Lanes hold
// distinct cells at each j, and a wave's LDS operations complete in order,
// so the sums need no atomics.
template <int ND, int LM>
__device__ __forceinline__ void rev_acc(double* __restrict__ acc, int cap, int o, uint32_t masks,
                                        const double (&nu)[ND + 2],
                                        const double (&Lrow)[ND + 2][ND + 2],
                                        const double* __restrict__ ctab, double alpha) {
    constexpr int NC = ND + 2;
    double g[NC];  // sum over the linear fields of L[s, :] nu_s
#pragma unroll
    for (int c = 0; c < NC; ++c) g[c] = 0.0;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (!(LM & (1 << s))) continue;
        const bool shear = !(s == 0 || s == NC - 1) && s != 1;
        if (!shear) {
#pragma unroll
            for (int c = 0; c < NC; ++c) g[c] = fmad(Lrow[s][c], nu[s], g[c]);
        } else {
            g[0] = fmad(Lrow[s][0], nu[s], g[0]);
            g[s] += nu[s];
        }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const int jp = j <= 4 ? j : 4, jm = j >= 1 ? 5 - j : 0;
        const double cp = (j <= 4) ? lin_coef(jp) : 0.0, cm = (j >= 1) ? lin_coef(jm) : 0.0;
        double a[NC], b[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            if (LM & (1 << s)) continue;
            const uint32_t mp = (masks >> (6 * s)) & 7u, mm = (masks >> (6 * s + 3)) & 7u;
            a[s] = (j <= 4) ? nu[s] * ctab[mp * 5 + jp] : 0.0;
            b[s] = (j >= 1) ? nu[s] * ctab[mm * 5 + jm] : 0.0;
        }
        double* cf = acc + o + j;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double pb = (LM != 0 && j <= 4) ? cp * g[c] : 0.0;
            double mb = (LM != 0 && j >= 1) ? cm * g[c] : 0.0;
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                if (LM & (1 << s)) continue;
                const bool shear = !(s == 0 || s == NC - 1) && s != 1;
                if (!shear) {
                    pb = fmad(Lrow[s][c], a[s], pb);
                    mb = fmad(Lrow[s][c], b[s], mb);
                } else if (c == 0) {
                    pb = fmad(Lrow[s][0], a[s], pb);
                    mb = fmad(Lrow[s][0], b[s], mb);
                } else if (c == s) {
                    pb += a[s];
                    mb += b[s];
                }
            }
            cf[(size_t)c * cap] = fmad(0.5, pb + mb, cf[(size_t)c * cap]);
            cf[(size_t)(NC + c) * cap] = fmad(0.5 * alpha, pb - mb, cf[(size_t)(NC + c) * cap]);
        }
        __asm__ __volatile__("" ::: "memory");
    }
}

struct AdjArgs {
    const double* U;
    const double* lam;
    const double* alpha;  // 3 device doubles
    double* P;            // chunk partials of the axis [chunk k][NC][cap][ncols]
    AdjGeom G;            // geometry of the axis (teno_index.hpp)
    double dx;
    SchemeParams sch;
    DecisionConsts dk;
};

// CAPC: the LDS row stride when it is known at compile time (ext_cap_for(n)
// = 74 for every n >= 63), so that every row of a staged cell is an immediate
// offset from one address; 0: taken from the geometry.
template <int ND, int DIR, bool A5, int CAPC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_adj_chunk(AdjArgs A) {
    constexpr int NC = ND + 2;
    constexpr int NV = 2 * NC + ND + 2;  // f+ (NC), f- (NC), sqrt(rho), u (ND), H
    using LO = LocalOrder<ND, DIR>;
    extern __shared__ double smem[];
    const AdjGeom& G = A.G;
    const int cap = CAPC ? CAPC : G.cap;
    double* omega = smem;       // 24: eq 2.15 weights per cutoff mask
    double* ctab = smem + 24;   // 40: cand_coef per (mask, stencil value)
    double* ext = smem + 64;    // NV x cap staged rows (forward quantities)
    // NV x cap cotangents: F (NC, local), U (NC, local), sqrt(rho), u (ND), H.
    // They reuse the staged rows: every read of those rows comes first in
    // program order, and the chunk is one wave, whose LDS operations
    // complete in order.
    double* acc = ext;
    const int lane = threadIdx.x;
    if (lane < 24) omega[lane] = kOmega[lane / 3][lane % 3];
    if (lane < 40) ctab[lane] = cand_coef(&kOmega[lane / 5][0], lane % 5);

    // columns fastest for y and z, as in the forward sweep
    const AdjChunk C = adj_chunk(G, DIR, xcd_logical_block(blockIdx.x, gridDim.x));
    const int n = G.n;
    const int64_t k = C.k, col = C.col, colbase = C.colbase;
    const bool valid = C.F0 + lane < G.ftot;
    int64_t bl;  // line of this lane's face
    int phi, o;  // face index in the line; staged offset of its cell i-2
    adj_lane_face(G, C, valid ? lane : 0, &bl, &phi, &o);
    const int count = C.count;
    const double alpha = A.alpha[DIR];
    const double gm1 = A.sch.gamma - 1.0;

    // ---- stage the chunk's cells exactly as the forward sweep does ---------
    // conserved state of staged cell idx as stored (ghost flip not applied)
    auto load_ext = [&](int idx, double* q, bool* flip) {
        const int64_t cell = adj_staged_cell(G, C, idx, flip);
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = A.U[c * G.ncell + cell];
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
        }
    }
    __syncthreads();

    // Per face, held from the read phase to the accumulation phase: the
    // frozen masks, nu = R^T mu, the left eigenvector rows (formed after the
    // read phase's peak), and the Roe cotangents of the face's two cells
    // (sqrt(rho), u, H of cells o+2, o+3).
    uint32_t masks = 0;
    double nu[NC];
    double Lrow[NC][NC];
    double roe_l[ND + 2], roe_r[ND + 2];
    int rmode = 0;  // 2: every field linear on the wave; 1: all but the entropy field

    if (valid) {
        // cotangent of the face flux (local order)
        const int64_t lbase = colbase + bl * G.line_step;
        double mul[NC];
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) {
            const int64_t c = LO::nat(qq);
            const double lr = (phi <= n - 1) ? A.lam[c * G.ncell + lbase + (int64_t)phi * G.stride] : 0.0;
            const double ll = (phi >= 1) ? A.lam[c * G.ncell + lbase + (int64_t)(phi - 1) * G.stride] : 0.0;
            mul[qq] = (lr - ll) / A.dx;
        }
        const FaceRoe<ND> R = face_roe<ND, DIR>(ext, cap, o, gm1);

        // forward: frozen cutoff masks, and the cotangent of the right
        // eigenvectors through F^ = R fh (R[:, s] depends on un, cs, Hb, q2, ut)
        double un_b = 0.0, cs_b = 0.0, Hb_b = 0.0, q2_b = 0.0, ci_b = 0.0, b1_b = 0.0, b2_b = 0.0;
        double ut_b[ND > 1 ? ND - 1 : 1];
#pragma unroll
        for (int kk = 0; kk < ND - 1; ++kk) ut_b[kk] = 0.0;
        const double csm = R.cs * mul[NC - 1];      // acoustic terms of R^T mu
        const double m1u = fmad(R.un, mul[NC - 1], mul[1]);
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
                // d/d(un, cs, Hb) of mu . R[:, s] fh with R[:, s] = (1, un -+ cs,
                // ut, Hb -+ un cs)
                const double sfh = (s == 0) ? -fh : fh;
                un_b = fmad(mul[1], fh, fmad(csm, sfh, un_b));
                cs_b = fmad(m1u, sfh, cs_b);
                Hb_b = fmad(mul[NC - 1], fh, Hb_b);
#pragma unroll
                for (int kk = 1; kk < ND; ++kk) ut_b[kk - 1] = fmad(mul[1 + kk], fh, ut_b[kk - 1]);
            } else if (s == 1) {
                un_b = fmad(mul[1], fh, un_b);
                q2_b = fmad(0.5 * mul[NC - 1], fh, q2_b);
#pragma unroll
                for (int kk = 1; kk < ND; ++kk) ut_b[kk - 1] = fmad(mul[1 + kk], fh, ut_b[kk - 1]);
            } else {
#pragma unroll
                for (int kk = 1; kk < ND; ++kk)
                    if (s == 1 + kk) ut_b[kk - 1] = fmad(mul[NC - 1], fh, ut_b[kk - 1]);
            }
        }

        // nu_s = (R^T mu)_s: the cotangent of the characteristic flux fh_s
        {
            double t0 = mul[0];  // mu_0 + ut . mu_t
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) t0 = fmad(R.ut[kk - 1], mul[1 + kk], t0);
            nu[0] = fmad(R.Hb - R.unc, mul[NC - 1], fmad(R.un - R.cs, mul[1], t0));
            nu[1] = fmad(R.hq2, mul[NC - 1], fmad(R.un, mul[1], t0));
            nu[NC - 1] = fmad(R.Hb + R.unc, mul[NC - 1], fmad(R.un + R.cs, mul[1], t0));
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) nu[1 + kk] = fmad(R.ut[kk - 1], mul[NC - 1], mul[1 + kk]);
        }
        // the reverse sums over the stencil, specialized on the fields whose
        // reconstruction is linear on the whole wave (a wave-uniform choice)
        constexpr uint32_t kAllKept = (1u << (6 * NC)) - 1u;
        rmode = __all(masks == kAllKept) ? 2 : __all((masks | (63u << 6)) == kAllKept) ? 1 : 0;
        if (rmode == 2)
            rev_read_fold<ND, (1 << NC) - 1>(ext, cap, o, masks, nu, ctab, R, un_b, ci_b, b1_b,
                                             b2_b, ut_b);
        else if (rmode == 1)
            rev_read_fold<ND, ((1 << NC) - 1) & ~2>(ext, cap, o, masks, nu, ctab, R, un_b, ci_b,
                                                    b1_b, b2_b, ut_b);
        else
            rev_read_fold<ND, 0>(ext, cap, o, masks, nu, ctab, R, un_b, ci_b, b1_b, b2_b, ut_b);
        // derived scalars: b2 = b1 q2 / 2, b1 = gm1 / c2, ci = 1 / cs, cs = sqrt(c2),
        // c2 = gm1 (Hb - q2 / 2), q2 = |ub|^2
        q2_b = fmad(0.5 * R.b1, b2_b, q2_b);
        b1_b = fmad(0.5 * R.q2, b2_b, b1_b);
        cs_b = fmad(-(R.ci * R.ci), ci_b, cs_b);
        // c2_b = -(b1 / c2) b1_b + cs_b / (2 cs), with 1 / cs = ci
        const double c2_b = fmad(-(R.b1 / R.c2), b1_b, (0.5 * R.ci) * cs_b);
        Hb_b = fmad(gm1, c2_b, Hb_b);
        q2_b = fmad(-0.5 * gm1, c2_b, q2_b);
        double ub_b[ND];
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) ub_b[kk] = (2.0 * R.ub[kk]) * q2_b;
        ub_b[DIR] += un_b;
#pragma unroll
        for (int kk = 1; kk < ND; ++kk) ub_b[LO::tan_axis(kk)] += ut_b[kk - 1];
        // Roe average of cells o+2 (weight rl) and o+3 (rr), w = 1 / (rl + rr)
        const double* uu = ext + (size_t)(2 * NC + 1) * cap;
        const double* hh = ext + (size_t)(2 * NC + 1 + ND) * cap;
        const double w = R.wsum, rl = R.rl, rr = R.rr;
        const double SH = fmad(rl, hh[o + 2], rr * hh[o + 3]);
        double w_b = SH * Hb_b;
        const double SH_b = w * Hb_b;
        double rl_b = hh[o + 2] * SH_b, rr_b = hh[o + 3] * SH_b;
        double ul_b[ND], ur_b[ND];
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            const double u2 = uu[(size_t)kk * cap + o + 2], u3 = uu[(size_t)kk * cap + o + 3];
            w_b = fmad(fmad(rl, u2, rr * u3), ub_b[kk], w_b);
            const double Sk_b = w * ub_b[kk];
            ul_b[kk] = rl * Sk_b;
            ur_b[kk] = rr * Sk_b;
            rl_b = fmad(u2, Sk_b, rl_b);
            rr_b = fmad(u3, Sk_b, rr_b);
        }
        rl_b = fmad(-(w * w), w_b, rl_b);
        rr_b = fmad(-(w * w), w_b, rr_b);
        roe_l[0] = rl_b;
        roe_r[0] = rr_b;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            roe_l[1 + kk] = ul_b[kk];
            roe_r[1 + kk] = ur_b[kk];
        }
        roe_l[1 + ND] = rl * SH_b;
        roe_r[1 + ND] = rr * SH_b;
#pragma unroll
        for (int s = 0; s < NC; ++s) left_row<ND>(R, s, Lrow[s]);
    }
    // every read of the staged rows is above: clear the cotangent rows
    for (int idx = lane; idx < count; idx += 64) {
#pragma unroll
        for (int r = 0; r < NV; ++r) acc[(size_t)r * cap + idx] = 0.0;
    }
    // the accumulation phase re-reads the coefficient table rather than
    // holding the read phase's values in registers
    __asm__ __volatile__("" ::: "memory");
    if (valid) {
        if (rmode == 2)
            rev_acc<ND, (1 << NC) - 1>(acc, cap, o, masks, nu, Lrow, ctab, alpha);
        else if (rmode == 1)
            rev_acc<ND, ((1 << NC) - 1) & ~2>(acc, cap, o, masks, nu, Lrow, ctab, alpha);
        else
            rev_acc<ND, 0>(acc, cap, o, masks, nu, Lrow, ctab, alpha);
        // Roe cotangents of the face's two cells
        double* cr = acc + (size_t)(2 * NC) * cap + o;
#pragma unroll
        for (int r = 0; r < ND + 2; ++r) cr[(size_t)r * cap + 2] += roe_l[r];
        __asm__ __volatile__("" ::: "memory");
#pragma unroll
        for (int r = 0; r < ND + 2; ++r) cr[(size_t)r * cap + 3] += roe_r[r];
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
        // the cell's primitives to a few ulp (reciprocal and reciprocal square
        // root refined by Newton steps; the adjoint is held to a relative bar)
        const double rho = q[0], ri = rcp_nr(rho), E = q[NC - 1];
        double u[ND], uu2 = 0.0;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            u[kk] = q[1 + kk] * ri;
            uu2 = fmad(u[kk], u[kk], uu2);
        }
        const double p = gm1 * fmad(-0.5 * rho, uu2, E);
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
            m_b[kk] = fmad(u[DIR], Fb[1 + kk], m_b[kk]);
            u_b[DIR] = fmad(q[1 + kk], Fb[1 + kk], u_b[DIR]);
        }
        p_b += Fb[1 + DIR];
        E_b = fmad(u[DIR], Fb[NC - 1], E_b);
        p_b = fmad(u[DIR], Fb[NC - 1], p_b);
        u_b[DIR] = fmad(E + p, Fb[NC - 1], u_b[DIR]);
        // H = (E + p) / rho
        const double Hr = H_b * ri;
        E_b += Hr;
        p_b += Hr;
        rho_b = fmad(-H, Hr, rho_b);
        // sqrt(rho): d sqrt(rho) / d rho = rsqrt(rho) / 2
        double y = __builtin_amdgcn_rsq(rho);
        y = y * fmad(-0.5 * rho, y * y, 1.5);
        y = y * fmad(-0.5 * rho, y * y, 1.5);
        rho_b = fmad(sr_b, 0.5 * y, rho_b);
        // p = (gamma - 1) (E - |m|^2 / (2 rho))
        E_b = fmad(gm1, p_b, E_b);
        rho_b = fmad(0.5 * gm1 * uu2, p_b, rho_b);
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) m_b[kk] = fmad(-gm1 * u[kk], p_b, m_b[kk]);
        // u_k = m_k / rho
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            m_b[kk] = fmad(u_b[kk], ri, m_b[kk]);
            rho_b = fmad(-u[kk] * ri, u_b[kk], rho_b);
        }
        gq[0] += rho_b;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) gq[1 + kk] += m_b[kk];
        gq[NC - 1] += E_b;
        if (flip) gq[1 + DIR] = -gq[1 + DIR];  // ghost image: back to the source's frame
#pragma unroll
        for (int c = 0; c < NC; ++c) A.P[adj_p_index(G, NC, k, c, idx, col)] = gq[c];
    }
}

// Pass B, once for all axes: every cell adds, axis by axis, the chunk
// partials of its images along that axis (the cell itself and the ghost cells
// it supplies), and writes the sum over the axes in the order x, y, z.
struct GatherArgs {
    const double* P[3];  // chunk partials of each axis
    double* out;
    AdjGeom G[3];        // geometry of each axis
};

template <int ND>
__global__ __launch_bounds__(256) void k_adj_gather(GatherArgs A) {
    constexpr int NC = ND + 2;
    const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (cell >= A.G[0].ncell) return;
    double tot[NC];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const AdjGeom& G = A.G[d];
        const double* P = A.P[d];
        int64_t col, b;  // column and line of the cell along d
        int i;           // its position on the line
        adj_cell_place(G, d, cell, &col, &b, &i);
        int img[7];
        const int nimg = adj_images(G.bc, G.n, i, img);
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
        for (int t = 0; t < nimg; ++t) {
            // staged cell e = image + 3 of line b is in the stencils of faces e-5 .. e
            const int e = img[t] + 3;
            int64_t ka, kz;
            adj_chunks_of(G, b, e, &ka, &kz);
            for (int64_t kk = ka; kk <= kz; ++kk) {
                const int slot = (int)adj_slot(G, b, e, kk);
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] += P[adj_p_index(G, NC, kk, c, slot, col)];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) tot[c] = (d == 0) ? acc[c] : tot[c] + acc[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) A.out[c * A.G[0].ncell + cell] = tot[c];
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
// Bytes of the chunk partials of axis d, and of all axes (each axis keeps
// its own, so that one gather sums them).
static size_t adj_P_axis_bytes(const teno_grid* g, int d) {
    const AdjGeom G = adj_geom(g->n, g->bc, d);
    return (size_t)adj_p_elems(G, g->ndim + 2) * sizeof(double);
}
static size_t adj_P_bytes(const teno_grid* g) {
    size_t sum = 0;
    for (int d = 0; d < g->ndim; ++d) sum += adj_P_axis_bytes(g, d);
    return sum;
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
    const int64_t nblk = A.G.kchunks * A.G.ncols;
    const size_t lds = (size_t)(64 + NV * A.G.cap) * sizeof(double);
    constexpr int kCapLong = 74;  // ext_cap_for(n) for every n >= 63
    const bool a5 = A.sch.scheme == TENO_SCHEME_TENO5A;
    if (A.G.cap == kCapLong) {
        if (a5)
            hipLaunchKernelGGL((k_adj_chunk<ND, DIR, true, kCapLong>), dim3((unsigned)nblk),
                               dim3(64), lds, st, A);
        else
            hipLaunchKernelGGL((k_adj_chunk<ND, DIR, false, kCapLong>), dim3((unsigned)nblk),
                               dim3(64), lds, st, A);
    } else if (a5) {
        hipLaunchKernelGGL((k_adj_chunk<ND, DIR, true, 0>), dim3((unsigned)nblk), dim3(64), lds, st, A);
    } else {
        hipLaunchKernelGGL((k_adj_chunk<ND, DIR, false, 0>), dim3((unsigned)nblk), dim3(64), lds, st, A);
    }
    return hipGetLastError();
}

static hipError_t rhs_adjoint_impl(const teno_grid* g, const double* U, const double* alpha,
                                   const double* lam, double* out, double* P, hipStream_t st) {
    GatherArgs GA;
    memset(&GA, 0, sizeof(GA));
    GA.out = out;
    char* pd = (char*)P;
    for (int d = 0; d < g->ndim; ++d) {
        AdjArgs A;
        memset(&A, 0, sizeof(A));
        A.U = U;
        A.lam = lam;
        A.alpha = alpha;
        A.P = (double*)pd;
        A.G = adj_geom(g->n, g->bc, d);
        A.dx = g->dx[d];
        GA.P[d] = A.P;
        GA.G[d] = A.G;
        pd += adj_P_axis_bytes(g, d);
        A.sch = scheme_of(g);
        A.dk = decision_consts(g, false);
        if (A.G.kchunks * A.G.ncols > (int64_t(1) << 31) - 64) return hipErrorInvalidValue;
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
    const unsigned blocks = (unsigned)((GA.G[0].ncell + 255) / 256);
    switch (g->ndim) {
        case 1: hipLaunchKernelGGL(k_adj_gather<1>, dim3(blocks), dim3(256), 0, st, GA); break;
        case 2: hipLaunchKernelGGL(k_adj_gather<2>, dim3(blocks), dim3(256), 0, st, GA); break;
        default: hipLaunchKernelGGL(k_adj_gather<3>, dim3(blocks), dim3(256), 0, st, GA); break;
    }
    return hipGetLastError();
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
