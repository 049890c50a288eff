// Scalar linear advection u_t + u_x = 0 on a periodic 1D grid (Sec. 4.1,
// eq 4.4) with the TENO reconstruction of the sweep kernels: global
// Lax-Friedrichs splitting with alpha = 1 gives f+ = u and f- = 0, each
// reconstructed at every face (f- on the mirrored stencil), and the flux
// difference of eq 2.2.  Used for the Table 1 convergence test on the GPU and
// for the spectral (approximate dispersion relation) analysis.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_host.hpp"

namespace teno {

struct AdvectArgs {
    const double* u;
    double* out;
    int32_t n;
    double dx;
    SchemeParams sch;
    DecisionConsts dk;
};

// Flux at face phi (between cells phi - 1 and phi) from the split values of
// cells phi - 3 .. phi + 2 (periodic).
template <bool A5>
__device__ __forceinline__ double advect_face(const AdvectArgs& A, const double* omega, int phi) {
    const int n = A.n;
    double fp[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        int c = phi - 3 + j;
        c = ((c % n) + n) % n;
        const double uj = A.u[c];
        fp[j] = 0.5 * (uj + 1.0 * uj);
    }
    uint32_t code;
    const double rp = teno5_rec_fast<A5>(A.sch, A.dk, omega, fp[0], fp[1], fp[2], fp[3], fp[4], &code);
    // f- = 0.5 (u - 1.0 u) = 0 on every cell, reconstructed on the mirrored stencil
    const double z = 0.0;
    const double rm = teno5_rec_fast<A5>(A.sch, A.dk, omega, z, z, z, z, z, &code);
    return rp + rm;
}

template <bool A5>
__global__ __launch_bounds__(256) void k_advect_rhs(AdvectArgs A) {
    __shared__ double omega[24];
    if (threadIdx.x < 24) omega[threadIdx.x] = kOmega[threadIdx.x / 3][threadIdx.x % 3];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const double fl = advect_face<A5>(A, omega, i);      // face i - 1/2
    const double fr = advect_face<A5>(A, omega, i + 1);  // face i + 1/2
    A.out[i] = 0.0 - cr_div(fr - fl, A.dx);
}

// SSP-RK3 stage updates of eq 4.1-4.3 with a given step h.
__global__ void k_advect_stage(int stage, int n, double h, const double* u, const double* u1,
                               const double* L, double* dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v;
    if (stage == 1)
        v = u[i] + h * L[i];
    else if (stage == 2)
        v = (0.75 * u[i] + 0.25 * u1[i]) + 0.25 * (h * L[i]);
    else
        v = ((1.0 / 3.0) * u[i] + (2.0 / 3.0) * u1[i]) + (2.0 / 3.0) * (h * L[i]);
    dst[i] = v;
}

static hipError_t advect_rhs_impl(const teno_grid* g, const double* u, double* out,
                                  hipStream_t st) {
    AdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.u = u;
    A.out = out;
    A.n = g->n[0];
    A.dx = g->dx[0];
    A.sch = scheme_of(g);
    A.dk = decision_consts(g, false);
    const unsigned blocks = (unsigned)((A.n + 255) / 256);
    if (g->scheme == TENO_SCHEME_TENO5A)
        hipLaunchKernelGGL((k_advect_rhs<true>), dim3(blocks), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL((k_advect_rhs<false>), dim3(blocks), dim3(256), 0, st, A);
    return hipGetLastError();
}

static int advect_validate(const teno_grid* g) {
    if (validate(g) != TENO_OK || g->ndim != 1 || g->boundary_dev != nullptr) return TENO_ERR_ARG;
    return TENO_OK;
}

}  // namespace teno

using namespace teno;

extern "C" {

size_t teno_advect_workspace_bytes(const teno_grid* g) {
    if (advect_validate(g) != TENO_OK) return 0;
    return 3 * (size_t)g->n[0] * sizeof(double);
}

int teno_advect_rhs(const teno_grid* g, const double* u, double* dudt, void* stream) {
    if (advect_validate(g) != TENO_OK || u == nullptr || dudt == nullptr || u == dudt)
        return TENO_ERR_ARG;
    return advect_rhs_impl(g, u, dudt, (hipStream_t)stream) == hipSuccess ? TENO_OK
                                                                          : TENO_ERR_DEVICE;
}

int teno_advect_step(const teno_grid* g, double* u, double h, void* ws, size_t ws_bytes,
                     void* stream) {
    if (advect_validate(g) != TENO_OK || u == nullptr || ws == nullptr ||
        ws_bytes < teno_advect_workspace_bytes(g) || !(h >= 0.0))
        return TENO_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int n = g->n[0];
    double* L = (double*)ws;
    double* u1 = L + n;
    double* u2 = u1 + n;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (advect_rhs_impl(g, u, L, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_advect_stage, dim3(blocks), dim3(256), 0, st, 1, n, h, u, u, L, u1);
    if (advect_rhs_impl(g, u1, L, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_advect_stage, dim3(blocks), dim3(256), 0, st, 2, n, h, u, u1, L, u2);
    if (advect_rhs_impl(g, u2, L, st) != hipSuccess) return TENO_ERR_DEVICE;
    hipLaunchKernelGGL(k_advect_stage, dim3(blocks), dim3(256), 0, st, 3, n, h, u, u2, L, u);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

}  // extern "C"
