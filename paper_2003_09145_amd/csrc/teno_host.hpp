// Host-side helpers shared by the HIP translation units of libteno.so:
// argument validation and the per-launch scheme / decision constants.
#pragma once

#include <cmath>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_divmagic.hpp"

namespace teno {

inline int validate(const teno_grid* g) {
    if (g == nullptr) return TENO_ERR_ARG;
    if (g->ndim < 1 || g->ndim > 3) return TENO_ERR_ARG;
    for (int k = 0; k < 3; ++k) {
        if (k < g->ndim) {
            if (g->n[k] < 3) return TENO_ERR_ARG;
            if (!(g->dx[k] > 0.0)) return TENO_ERR_ARG;
            if (g->bc[k] < 0 || g->bc[k] > 2) return TENO_ERR_ARG;
        } else if (g->n[k] != 1) {
            return TENO_ERR_ARG;
        }
    }
    if (!(g->gamma > 1.0)) return TENO_ERR_ARG;
    if (g->scheme < 0 || g->scheme > 3) return TENO_ERR_ARG;
    if (g->scheme == 0) {
        if (g->Bl < 0 || g->Bu > 20 || g->Bl > g->Bu || !(g->H > 0.0)) return TENO_ERR_ARG;
    }
    if (g->scheme == 3) {
        // floor(beta) of eq 2.16 stays in [floor(a1 - a2), floor(a1)] within the ladder
        if (!(g->a2 >= 0.0) || !(g->a1 - g->a2 >= 0.0) || !(g->a1 <= 20.0)) return TENO_ERR_ARG;
        if (!(g->cr > 0.0) || !(0.9 * g->cr < 1.0) || !(g->xi >= 0.0) || !std::isfinite(g->xi))
            return TENO_ERR_ARG;
    }
    if (!(g->eps > 0.0)) return TENO_ERR_ARG;
    if (g->flags & ~(TENO_FLAG_LITERAL_DECISIONS | TENO_FLAG_MASK_DIGEST)) return TENO_ERR_ARG;
    if (g->theta != TENO_THETA_PRINTED && g->theta != TENO_THETA_CUT) return TENO_ERR_ARG;
    return TENO_OK;
}

inline SchemeParams scheme_of(const teno_grid* g) {
    SchemeParams s;
    s.gamma = g->gamma;
    s.ct_fixed = g->ct_fixed;
    s.H = g->H;
    s.eps = g->eps;
    s.scheme = g->scheme;
    s.Bl = g->Bl;
    s.Bu = g->Bu;
    s.bu_bl = (double)(g->Bu - g->Bl);
    s.a1 = g->a1;
    s.a2 = g->a2;
    s.cr = g->cr;
    s.kA_nan = 0;
    s.theta_cut = (g->scheme == TENO_SCHEME_LAD && g->theta == TENO_THETA_CUT) ? 1 : 0;
    s.epsA = 0.0;
    if (g->scheme == 3) {
        s.kA_nan = (int)std::floor(g->a1 - g->a2);
        s.epsA = ((0.9 * g->cr) / (1.0 - 0.9 * g->cr)) * (g->xi * g->xi);  // eq 2.18
    }
    return s;
}

// The cutoff ladder of eq 3.3 on the host: kLadderHost[k] = 10^-k.
inline const double kLadderHost[21] = {1e0,   1e-1,  1e-2,  1e-3,  1e-4,  1e-5,  1e-6,
                                       1e-7,  1e-8,  1e-9,  1e-10, 1e-11, 1e-12, 1e-13,
                                       1e-14, 1e-15, 1e-16, 1e-17, 1e-18, 1e-19, 1e-20};

// Largest T with 1 / (1 + 2 (1 + T)^6) >= ct (1 + 2^-30), shrunk by 2^-30:
// stencils whose chi~_k are all <= T keep every candidate for any cutoff up
// to ct (the rounding of the literal evaluation is far inside both
// margins).  -1 when ct leaves no such T.
inline double smooth_bound(double ct) {
    if (!(ct > 0.0)) return -1.0;
    const double g = (1.0 / (ct * (1.0 + 0x1p-30)) - 1.0) / 2.0;  // bound on (1 + T)^6
    if (!(g > 1.0)) return -1.0;
    const double T = (std::pow(g, 1.0 / 6.0) - 1.0) * (1.0 - 0x1p-30);
    return T > 0.0 ? T : -1.0;
}

inline DecisionConsts decision_consts_base(const teno_grid* g, bool need_m);

// Decision constants with the host-side margin products filled in.
inline DecisionConsts decision_consts(const teno_grid* g, bool need_m) {
    DecisionConsts K = decision_consts_base(g, need_m);
    K.hi_fac = K.ct_hi * (1.0 + kDecisionMargin);
    K.lo_fac = K.ct_lo * (1.0 - kDecisionMargin);
    K.ymarg = kDecisionMargin * K.nthr_d;
    return K;
}

inline DecisionConsts decision_consts_base(const teno_grid* g, bool need_m) {
    DecisionConsts K;
    memset(&K, 0, sizeof(K));
    K.literal = (g->flags & TENO_FLAG_LITERAL_DECISIONS) ? 1 : 0;
    K.need_m = need_m ? 1 : 0;
    K.smooth_t = -1.0;
    K.h_hi = K.h_lo = NAN;
    if (g->scheme == TENO_SCHEME_FIXED_CT) {
        K.ct_hi = K.ct_lo = g->ct_fixed;
        K.smooth_t = smooth_bound(K.ct_hi);
        return K;
    }
    if (g->scheme == TENO_SCHEME_TENO5A) {
        // the cutoff is evaluated per reconstruction; its largest value bounds
        // the smooth-stencil shortcut
        const int khi = (int)std::floor(g->a1 - g->a2);
        K.ct_hi = kLadderHost[khi];
        K.ct_lo = kLadderHost[20];
        K.smooth_t = smooth_bound(K.ct_hi);
        return K;
    }
    if (g->scheme != TENO_SCHEME_LAD) return K;
    K.ct_hi = kLadderHost[g->Bl];
    K.ct_lo = kLadderHost[g->Bu];
    K.smooth_t = smooth_bound(K.ct_hi);
    K.nthr = g->Bu - g->Bl;
    K.nthr_d = (double)K.nthr;
    K.inv_h = 1.0 / g->H;
    if (g->theta == TENO_THETA_CUT) {
        // the approximate max chi~ is within a few ulp of the literal one
        K.h_hi = g->H * (1.0 + kDecisionMargin);
        K.h_lo = g->H * (1.0 - kDecisionMargin);
    }
    return K;
}


}  // namespace teno
