// Per-cell and per-face building blocks of the characteristic TENO5-LAD flux
// (Peng et al., arXiv:2003.09145, Sec. 2-4), shared by the grid sweep and
// the ragged-batch kernels.
//
// A stencil buffer `ext` in LDS holds, for `cap` consecutive cells of a line
// (ghost cells included), NV = 2 NC + ND + 2 structure-of-arrays rows: the
// global Lax-Friedrichs split fluxes f+ and f- in the local component order
// of the sweep axis, sqrt(rho), the velocity components and the total
// enthalpy H.
#pragma once

#include "teno_device.hpp"

namespace teno {

// Stage cell `idx` of the stencil buffer from its conserved state q (natural
// component order, ghost flip already applied): primitives (u_k = m_k / rho,
// p = (gamma - 1)(E - ke), H = (E + p) / rho), the flux along DIR (eq 4.7) and
// its split f+- = (F +- alpha U) / 2 in local order.
template <int ND, int DIR, bool MIRROR = false>
__device__ __forceinline__ void stage_cell(const double* q, double alpha, double gm1,
                                       double* __restrict__ ext, int cap, int idx) {
    constexpr int NC = ND + 2;
    using LO = LocalOrder<ND, DIR>;
    // primitives (natural order), as u_k = m_k / rho, p = (gamma-1)(E - ke)
    const double rho = q[0];
    double u[ND];
    const double rrho = rcp_nr(rho);
    // the velocity quotients and sqrt(rho) are independent: their fast
    // phases run together and share one correction branch
    double srho;
    {
        double r[ND];
        bool ok[ND];
        bool all = sqrt_fast(rho, &srho);
        const bool sok = all;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            ok[kk] = div_r_fast(q[1 + kk], rho, rrho, &u[kk], &r[kk]);
            all = all && ok[kk];
        }
        if (!all) {
            if (!sok) srho = cr_sqrt_exact(rho);
#pragma unroll
            for (int kk = 0; kk < ND; ++kk)
                if (!ok[kk]) u[kk] = div_r_fix(q[1 + kk], rho, u[kk], r[kk]);
        }
    }
    double mu = q[1] * u[0];
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) mu = mu + q[1 + kk] * u[kk];
    const double ke = 0.5 * mu;
    const double E = q[NC - 1];
    const double p = gm1 * (E - ke);
    const double H = cr_div_r(E + p, rho, rrho);
    // flux along DIR (natural order)
    double Fl[NC];
    Fl[0] = q[1 + DIR];
#pragma unroll
    for (int kk = 0; kk < ND; ++kk)
        Fl[1 + kk] = (kk == DIR) ? q[1 + kk] * u[DIR] + p : q[1 + kk] * u[DIR];
    Fl[NC - 1] = (E + p) * u[DIR];
    // global Lax-Friedrichs split in local order
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) {
        const int g = LO::nat(qq);
        ext[(size_t)qq * cap + idx] = 0.5 * __builtin_fma(alpha, q[g], Fl[g]);
        // MIRROR: the f- rows hold the cells in reverse (column cap - 1 -
        // idx), so that its mirrored stencil i+3 .. i-1 reads ascending
        // columns too
        ext[(size_t)(NC + qq) * cap + (MIRROR ? cap - 1 - idx : idx)] =
            0.5 * __builtin_fma(-alpha, q[g], Fl[g]);
    }
    ext[(size_t)(2 * NC) * cap + idx] = srho;
#pragma unroll
    for (int kk = 0; kk < ND; ++kk) ext[(size_t)(2 * NC + 1 + kk) * cap + idx] = u[kk];
    ext[(size_t)(2 * NC + 1 + ND) * cap + idx] = H;
}

// Roe average of the face between stencil cells o + 2 (i) and o + 3 (i+1)
// and the scalars of its left and right eigenvector matrices (local order:
// normal velocity un, tangential velocities ut, sound speed cs, ci = 1/cs,
// b1 = (gamma - 1)/c^2, b2 = b1 |u|^2 / 2).  Shared by the face flux and its
// adjoint so that both evaluate the same operations.
template <int ND>
struct FaceRoe {
    double rl, rr, wsum;  // sqrt(rho) of cells i, i+1 and 1 / (rl + rr)
    double ub[ND];        // averaged velocity (natural axes)
    double Hb, q2, c2, cs, ci, b1, b2, un;
    double ut[ND > 1 ? ND - 1 : 1];
    // products shared by the eigenvector entries (each rounded once, as in
    // the dense oracle matrices)
    double unci, b1un, unc, hq2;
    double b1ut[ND > 1 ? ND - 1 : 1];
};

template <int ND, int DIR>
__device__ __forceinline__ FaceRoe<ND> face_roe(const double* __restrict__ ext, int cap, int o,
                                                double gm1) {
    constexpr int NC = ND + 2;
    using LO = LocalOrder<ND, DIR>;
    const double* sr = ext + (size_t)(2 * NC) * cap;
    const double* uu = ext + (size_t)(2 * NC + 1) * cap;
    const double* hh = ext + (size_t)(2 * NC + 1 + ND) * cap;
    FaceRoe<ND> R;
    R.rl = sr[o + 2];
    R.rr = sr[o + 3];
    const double rsum = R.rl + R.rr;
    R.wsum = cr_div_r(1.0, rsum, rcp_nr(rsum));
#pragma unroll
    for (int kk = 0; kk < ND; ++kk)
        R.ub[kk] = (R.rl * uu[(size_t)kk * cap + o + 2] + R.rr * uu[(size_t)kk * cap + o + 3]) * R.wsum;
    R.Hb = (R.rl * hh[o + 2] + R.rr * hh[o + 3]) * R.wsum;
    R.q2 = R.ub[0] * R.ub[0];
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) R.q2 = R.q2 + R.ub[kk] * R.ub[kk];
    R.c2 = gm1 * (R.Hb - 0.5 * R.q2);
    {
        // c = sqrt(c2) and b1 = (gamma - 1) / c2 are independent: one
        // correction branch for both
        double r;
        const bool sok = sqrt_fast(R.c2, &R.cs);
        const bool bok = div_r_fast(gm1, R.c2, rcp_nr(R.c2), &R.b1, &r);
        if (!(sok && bok)) {
            if (!sok) R.cs = cr_sqrt_exact(R.c2);
            if (!bok) R.b1 = div_r_fix(gm1, R.c2, R.b1, r);
        }
    }
    R.ci = cr_div_r(1.0, R.cs, rcp_nr(R.cs));
    R.b2 = (0.5 * R.q2) * R.b1;
    R.un = R.ub[DIR];
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) R.ut[kk - 1] = R.ub[LO::tan_axis(kk)];
    R.unci = R.un * R.ci;
    R.b1un = R.b1 * R.un;
    R.unc = R.un * R.cs;
    R.hq2 = 0.5 * R.q2;
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) R.b1ut[kk - 1] = R.b1 * R.ut[kk - 1];
    return R;
}

// Row s of the left eigenvector matrix (local order): acoustic fields s = 0
// (u - c) and s = NC - 1 (u + c), the entropy field s = 1 and the shear
// fields s = 2 .. NC - 2, whose row is (-ut, 0, .., 1 at s, .., 0); for them
// only the first entry is set here and the unit entry is implied.
template <int ND>
__device__ __forceinline__ void left_row(const FaceRoe<ND>& R, int s, double (&Lr)[ND + 2]) {
    constexpr int NC = ND + 2;
    const bool acoustic = (s == 0 || s == NC - 1);
    const bool entropy = (s == 1);
    if (acoustic) {
        const bool minus = (s == 0);
        Lr[0] = minus ? 0.5 * (R.b2 + R.unci) : 0.5 * (R.b2 - R.unci);
        Lr[1] = minus ? 0.5 * (-R.b1un - R.ci) : 0.5 * (-R.b1un + R.ci);
#pragma unroll
        for (int kk = 1; kk < ND; ++kk) Lr[1 + kk] = 0.5 * (-R.b1ut[kk - 1]);
        Lr[NC - 1] = 0.5 * R.b1;
    } else if (entropy) {
        Lr[0] = 1.0 - R.b2;
        Lr[1] = R.b1un;
#pragma unroll
        for (int kk = 1; kk < ND; ++kk) Lr[1 + kk] = R.b1ut[kk - 1];
        Lr[NC - 1] = -R.b1;
    } else {
        double uts = R.ut[0];
#pragma unroll
        for (int kk = 2; kk < ND; ++kk) uts = (s == 1 + kk) ? R.ut[kk - 1] : uts;
#pragma unroll
        for (int qq = 0; qq < NC; ++qq) Lr[qq] = 0.0;
        Lr[0] = -uts;
    }
}

// Characteristic field s of the split flux (sg = 0: f+ on cells i-2 .. i+2;
// sg = 1: f- on the mirrored stencil i+3 .. i-1) projected on the left
// eigenvector row Lr and reconstructed at the face (eq 2.3-2.15); *code
// receives the decision code (cutoff mask in bits 5..7).
template <int ND, bool A5, bool MIRROR = false>
__device__ __forceinline__ double char_rec(const double* __restrict__ ext, int cap, int o, int s,
                                           int sg, const double (&Lr)[ND + 2],
                                           const SchemeParams& sch, const DecisionConsts& dk,
                                           const double* __restrict__ omega, uint32_t* code) {
    constexpr int NC = ND + 2;
    const bool shear = !(s == 0 || s == NC - 1) && s != 1;
    // f+ on cells o .. o+4 (point j at column o + j); f- on o+5 .. o+1: at
    // column o + 5 - j, or (MIRROR, reversed rows) at cap - 6 - o + j
    const bool asc = !sg || MIRROR;
    const double* fb = !sg ? ext + o
                           : ext + (size_t)NC * cap + (MIRROR ? cap - 6 - o : o);
    // the field-type test outside the stencil loop, so that the five points'
    // reads form one block the scheduler can issue ahead of their products
    double v[5];
    if (shear) {  // the unit entry: a plain add, as the oracle's fma by 1
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int cj = asc ? j : 5 - j;
            v[j] = Lr[0] * fb[cj] + fb[(size_t)s * cap + cj];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int cj = asc ? j : 5 - j;
            double acc = Lr[0] * fb[cj];
#pragma unroll
            for (int qq = 1; qq < NC; ++qq)
                acc = __builtin_fma(Lr[qq], fb[(size_t)qq * cap + cj], acc);
            v[j] = acc;
        }
    }
    return teno5_rec_fast<A5>(sch, dk, omega, v[0], v[1], v[2], v[3], v[4], code);
}

// Numerical flux at the face between stencil cells o + 2 and o + 3 (cells
// i-2 .. i+3 at o .. o + 5): Roe average, left/right eigenvectors, projection
// of the split fluxes, TENO5-LAD reconstruction of f+ and f- per
// characteristic field, back-projection (A5: TENO5-A cutoff, scheme 3).
// Fnat receives the flux in natural
// component order; o8 (nullable) receives the 2 NC decision codes and masks
// (nullable, initialised by the caller) the 2 NC cutoff masks, 3 bits each.
template <int ND, int DIR, bool A5, bool MIRROR = false>
__device__ __forceinline__ void face_flux(const double* __restrict__ ext, int cap, int o,
                                      double gm1, const SchemeParams& sch,
                                      const DecisionConsts& dk,
                                      const double* __restrict__ omega, uint8_t* o8,
                                      double* Fnat, uint32_t* masks = nullptr) {
    constexpr int NC = ND + 2;
    using LO = LocalOrder<ND, DIR>;
    const FaceRoe<ND> R = face_roe<ND, DIR>(ext, cap, o, gm1);

    double Fh[NC];  // local order accumulators of R * fhat
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) Fh[qq] = 0.0;

    // Characteristic fields one at a time, the loop unrolled so that each
    // field's projection, reconstruction and accumulation is specialized at
    // compile time: project the split fluxes of the stencil on the left
    // eigenvector, reconstruct f^+ and f^-, and add R[:, s] * fhat_s to the
    // face flux.
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const bool acoustic = (s == 0 || s == NC - 1);
        const bool entropy = (s == 1);
        double Lr[NC];
        left_row<ND>(R, s, Lr);
        double fh = 0.0;
#pragma unroll 1
        for (int sg = 0; sg < 2; ++sg) {
            __asm__ __volatile__("" ::: "memory");
            uint32_t code;
            const double r = char_rec<ND, A5, MIRROR>(ext, cap, o, s, sg, Lr, sch, dk, omega, &code);
            if (o8 != nullptr) o8[2 * s + sg] = (uint8_t)code;
            if (masks != nullptr) *masks |= (code >> 5) << (3 * (2 * s + sg));
            fh = sg ? fh + r : r;
        }
        // accumulate R[:, s] * fh in local order, as fused multiply-adds
        // (unit entries: plain adds; the first field's products are exact
        // additions to zero)
        if (acoustic) {
            const bool minus = (s == 0);
            Fh[0] = Fh[0] + fh;
            Fh[1] = __builtin_fma(minus ? (R.un - R.cs) : (R.un + R.cs), fh, Fh[1]);
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) Fh[1 + kk] = __builtin_fma(R.ut[kk - 1], fh, Fh[1 + kk]);
            Fh[NC - 1] = __builtin_fma(minus ? (R.Hb - R.unc) : (R.Hb + R.unc), fh, Fh[NC - 1]);
        } else if (entropy) {
            Fh[0] = Fh[0] + fh;
            Fh[1] = __builtin_fma(R.un, fh, Fh[1]);
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) Fh[1 + kk] = __builtin_fma(R.ut[kk - 1], fh, Fh[1 + kk]);
            Fh[NC - 1] = __builtin_fma(R.hq2, fh, Fh[NC - 1]);
        } else {
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) {
                if (s == 1 + kk) {
                    Fh[1 + kk] = Fh[1 + kk] + fh;
                    Fh[NC - 1] = __builtin_fma(R.ut[kk - 1], fh, Fh[NC - 1]);
                }
            }
        }
    }
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) Fnat[LO::nat(qq)] = Fh[qq];
}

}  // namespace teno
