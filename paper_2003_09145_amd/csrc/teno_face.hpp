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
template <int ND, int DIR>
__device__ __forceinline__ void stage_cell(const double* q, double alpha, double gm1,
                                       double* __restrict__ ext, int cap, int idx) {
    constexpr int NC = ND + 2;
    using LO = LocalOrder<ND, DIR>;
    // primitives (natural order), as u_k = m_k / rho, p = (gamma-1)(E - ke)
    const double rho = q[0];
    double u[ND];
    const double rrho = rcp_nr(rho);
#pragma unroll
    for (int kk = 0; kk < ND; ++kk) u[kk] = cr_div_r(q[1 + kk], rho, rrho);
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
        ext[(size_t)qq * cap + idx] = 0.5 * (Fl[g] + alpha * q[g]);
        ext[(size_t)(NC + qq) * cap + idx] = 0.5 * (Fl[g] - alpha * q[g]);
    }
    ext[(size_t)(2 * NC) * cap + idx] = cr_sqrt(rho);
#pragma unroll
    for (int kk = 0; kk < ND; ++kk) ext[(size_t)(2 * NC + 1 + kk) * cap + idx] = u[kk];
    ext[(size_t)(2 * NC + 1 + ND) * cap + idx] = H;
}

// Numerical flux at the face between stencil cells o + 2 and o + 3 (cells
// i-2 .. i+3 at o .. o + 5): Roe average, left/right eigenvectors, projection
// of the split fluxes, TENO5-LAD reconstruction of f+ and f- per
// characteristic field, back-projection (A5: TENO5-A cutoff, scheme 3).
// Fnat receives the flux in natural
// component order; o8 (nullable) receives the 2 NC decision codes and masks
// (nullable, initialised by the caller) the 2 NC cutoff masks, 3 bits each.
template <int ND, int DIR, bool A5>
__device__ __forceinline__ void face_flux(const double* __restrict__ ext, int cap, int o,
                                      double gm1, const SchemeParams& sch,
                                      const DecisionConsts& dk,
                                      const double* __restrict__ omega, uint8_t* o8,
                                      double* Fnat, uint32_t* masks = nullptr) {
    constexpr int NC = ND + 2;
    using LO = LocalOrder<ND, DIR>;
    const double* sr = ext + (size_t)(2 * NC) * cap;
    const double* uu = ext + (size_t)(2 * NC + 1) * cap;
    const double* hh = ext + (size_t)(2 * NC + 1 + ND) * cap;
    // Roe average of cells i (o+2) and i+1 (o+3)
    const double rl = sr[o + 2], rr = sr[o + 3];
    const double rsum = rl + rr;
    const double wsum = cr_div_r(1.0, rsum, rcp_nr(rsum));
    double ub[ND];
#pragma unroll
    for (int kk = 0; kk < ND; ++kk)
        ub[kk] = (rl * uu[(size_t)kk * cap + o + 2] + rr * uu[(size_t)kk * cap + o + 3]) * wsum;
    const double Hb = (rl * hh[o + 2] + rr * hh[o + 3]) * wsum;
    double q2 = ub[0] * ub[0];
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) q2 = q2 + ub[kk] * ub[kk];
    const double c2 = gm1 * (Hb - 0.5 * q2);
    const double cs = cr_sqrt(c2);
    const double ci = cr_div_r(1.0, cs, rcp_nr(cs));
    const double b1 = cr_div_r(gm1, c2, rcp_nr(c2));
    const double b2 = (0.5 * q2) * b1;
    const double un = ub[DIR];
    double ut[ND > 1 ? ND - 1 : 1];
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) ut[kk - 1] = ub[LO::tan_axis(kk)];

    double Fh[NC];  // local order accumulators of R * fhat
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) Fh[qq] = 0.0;
    // products shared by the eigenvector entries (each rounded once, as in
    // the dense oracle matrices)
    const double unci = un * ci, b1un = b1 * un, unc = un * cs, hq2 = 0.5 * q2;
    double b1ut[ND > 1 ? ND - 1 : 1];
#pragma unroll
    for (int kk = 1; kk < ND; ++kk) b1ut[kk - 1] = b1 * ut[kk - 1];

    // Characteristic fields one at a time (s is uniform across the wave, so
    // the field-type branches are scalar): project the split fluxes of the
    // stencil on the left eigenvector, reconstruct f^+ and f^-, and add
    // R[:, s] * fhat_s to the face flux.
#pragma unroll 1
    for (int s = 0; s < NC; ++s) {
        const bool acoustic = (s == 0 || s == NC - 1);
        const bool entropy = (s == 1);
        const bool shear = !acoustic && !entropy;
        double Lr[NC];
        if (acoustic) {
            const bool minus = (s == 0);
            Lr[0] = minus ? 0.5 * (b2 + unci) : 0.5 * (b2 - unci);
            Lr[1] = minus ? 0.5 * (-b1un - ci) : 0.5 * (-b1un + ci);
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) Lr[1 + kk] = 0.5 * (-b1ut[kk - 1]);
            Lr[NC - 1] = 0.5 * b1;
        } else if (entropy) {
            Lr[0] = 1.0 - b2;
            Lr[1] = b1un;
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) Lr[1 + kk] = b1ut[kk - 1];
            Lr[NC - 1] = -b1;
        } else {
            double uts = ut[0];
#pragma unroll
            for (int kk = 2; kk < ND; ++kk) uts = (s == 1 + kk) ? ut[kk - 1] : uts;
#pragma unroll
            for (int qq = 0; qq < NC; ++qq) Lr[qq] = 0.0;
            Lr[0] = -uts;
        }
        double fh = 0.0;
#pragma unroll 1
        for (int sg = 0; sg < 2; ++sg) {
            // f^+ on cells i-2..i+2, f^- on the mirrored stencil i+3..i-1
            __asm__ __volatile__("" ::: "memory");
            const double* fb = ext + (size_t)(sg ? NC : 0) * cap + o;
            double v[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const int cj = sg ? 5 - j : j;
                double acc;
                if (shear) {
                    acc = Lr[0] * fb[cj] + fb[(size_t)s * cap + cj];
                } else {
                    acc = Lr[0] * fb[cj];
#pragma unroll
                    for (int qq = 1; qq < NC; ++qq) acc = acc + Lr[qq] * fb[(size_t)qq * cap + cj];
                }
                v[j] = acc;
            }
            uint32_t code;
            const double r = teno5_rec_fast<A5>(sch, dk, omega, v[0], v[1], v[2], v[3], v[4], &code);
            if (o8 != nullptr) o8[2 * s + sg] = (uint8_t)code;
            if (masks != nullptr) *masks |= (code >> 5) << (3 * (2 * s + sg));
            fh = sg ? fh + r : r;
        }
        // accumulate R[:, s] * fh in local order
        if (acoustic) {
            const bool minus = (s == 0);
            Fh[0] = Fh[0] + fh;
            Fh[1] = Fh[1] + (minus ? (un - cs) : (un + cs)) * fh;
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) Fh[1 + kk] = Fh[1 + kk] + ut[kk - 1] * fh;
            Fh[NC - 1] = Fh[NC - 1] + (minus ? (Hb - unc) : (Hb + unc)) * fh;
        } else if (entropy) {
            Fh[0] = Fh[0] + fh;
            Fh[1] = Fh[1] + un * fh;
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) Fh[1 + kk] = Fh[1 + kk] + ut[kk - 1] * fh;
            Fh[NC - 1] = Fh[NC - 1] + hq2 * fh;
        } else {
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) {
                if (s == 1 + kk) {
                    Fh[1 + kk] = Fh[1 + kk] + fh;
                    Fh[NC - 1] = Fh[NC - 1] + ut[kk - 1] * fh;
                }
            }
        }
    }
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) Fnat[LO::nat(qq)] = Fh[qq];
}

}  // namespace teno
