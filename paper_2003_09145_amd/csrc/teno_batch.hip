// Batched form: thousands of independent 1D Euler problems of uneven length
// advanced together, each with its own global Lax-Friedrichs speed, time step
// and time (Peng et al., arXiv:2003.09145, Sec. 2-4 per problem).
//
// The tubes are concatenated into one flat sequence of faces (N_b + 1 per
// tube) and cut into chunks of 64 faces that start at multiples of 63, exactly
// like the lines of the grid sweep.  Every chunk costs the same whatever the
// tube lengths, so a persistent grid that walks the chunks round-robin is
// load-balanced by construction; one launch covers one RK stage of every
// tube.  Per-tube state lives on the device so that a whole run is a replay
// of a captured HIP graph with no host synchronisation:
//   alpha ring [3][nb]  LF speed of the stage input (slot s), of the stage
//                       output (slot s+1, reduced in the epilogue with
//                       atomicMax on the bit pattern) and a slot cleared for
//                       the stage after next;
//   status ring [3][nb] sticky non-physical flag with the same rotation, so a
//                       launch only reads flags written by earlier launches;
//   dt[nb], t[nb], nsteps[nb].
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_face.hpp"
#include "teno_host.hpp"

namespace teno {

struct BatchArgs {
    const double* Uin;          // stage input state [3][total]
    const double* Un;           // u^n
    double* Uout;               // stage output
    const int64_t* off;         // [nb + 1] first cell of each tube
    const int32_t* chunk_tube;  // [nchunks] tube of the first face of each chunk
    const double* dx;           // [nb]
    double* alpha_ring;         // [3][nb]
    int32_t* status_ring;       // [3][nb]
    double* dt;                 // [nb]
    double* t;                  // [nb]
    int64_t* nsteps;            // [nb]
    int64_t total, ftot, nchunks;
    int32_t nb, stage, bc, ext_cap;
    double cfl, t_end;
    SchemeParams sch;
    DecisionConsts dk;
};

// Per-cell LF speed |u| + c of a 1D state (the operation order of the grid
// path's reduction) and its physicality.
__device__ __forceinline__ double cell_speed(const double* q, double gamma, bool* bad) {
    const double rho = q[0];
    const double rrho = rcp_nr(rho);
    const double u = cr_div_r(q[1], rho, rrho);
    const double ke = 0.5 * (q[1] * u);
    const double p = (gamma - 1.0) * (q[2] - ke);
    const double cs = cr_sqrt(cr_div_r(gamma * p, rho, rrho));
    *bad = !(rho > 0.0) || !(p > 0.0) || !isfinite(cs);
    return fabs(u) + cs;
}

// Max of v over the lanes of the wave that share a tube id, one atomicMax per
// tube present in the wave.
__device__ __forceinline__ void tube_max(bool active, int tube, double v,
                                         unsigned long long* target) {
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int first = __ffsll((long long)pending) - 1;
        const int bt = __shfl(tube, first, 64);
        const bool in = active && tube == bt;
        double m = in ? v : 0.0;
#pragma unroll
        for (int offs = 32; offs > 0; offs >>= 1) {
            const double o = __shfl_xor(m, offs, 64);
            if (o > m) m = o;
        }
        if (lane == first && m > 0.0) atomicMax(&target[bt], (unsigned long long)__double_as_longlong(m));
        pending &= ~__ballot(in);
    }
}

template <int W, bool A5>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_stage(
    BatchArgs A) {
    constexpr int ND = 1, DIR = 0, NC = 3, NV = 2 * NC + ND + 2;
    extern __shared__ double smem[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    static_assert(NV == 9 && NC == 3, "batch_wave_lds assumes the 1D row count");
    const int cap = A.ext_cap;
    const int per_wave = batch_wave_lds(cap);
    double* omega = smem;
    double* ext = smem + 24 + (size_t)wave * per_wave;
    double* fhs = ext;  // reused after the wave's stencil reads (in-order LDS)
    if (threadIdx.x < 24) omega[threadIdx.x] = kOmega[threadIdx.x / 3][threadIdx.x % 3];

    const int nb = A.nb;
    const double* a_cur = A.alpha_ring + (size_t)A.stage * nb;
    unsigned long long* a_next =
        (unsigned long long*)(A.alpha_ring + (size_t)((A.stage + 1) % 3) * nb);
    double* a_clear = A.alpha_ring + (size_t)((A.stage + 2) % 3) * nb;
    const int32_t* st_prev = A.status_ring + (size_t)A.stage * nb;
    int32_t* st_next = A.status_ring + (size_t)((A.stage + 1) % 3) * nb;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < nb; i += blockDim.x) {
            a_clear[i] = 0.0;
            atomicMax(&st_next[i], st_prev[i]);  // sticky
        }
    }
    const double gm1 = A.sch.gamma - 1.0;
    const int64_t ngroups = (A.nchunks + W - 1) / W;

    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t chunk = g * W + wave;
        const bool wave_ok = chunk < A.nchunks;
        const BatchChunk C =
            batch_chunk(A.off, nb, A.ftot, wave_ok ? chunk : 0, wave_ok ? A.chunk_tube[chunk] : 0);
        const int count = wave_ok ? C.count : 0;
        const int64_t F = C.F0 + lane;
        const bool valid = wave_ok && F < A.ftot;
        int b = C.t0, o = 0;
        int64_t phi = 0;
        if (valid) batch_face(A.off, nb, C, F, &b, &phi, &o);
        __syncthreads();  // the previous chunk group's LDS reads are done

        for (int idx = lane; idx < count; idx += 64) {
            int bb;
            bool flip;
            const int src = batch_staged_src(A.off, nb, A.bc, C, idx, &bb, &flip);
            const int64_t base = A.off[bb];
            double q[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = A.Uin[c * A.total + base + src];
            if (flip) q[1] = -q[1];
            stage_cell<ND, DIR>(q, a_cur[bb], gm1, ext, cap, idx);
        }
        __syncthreads();

        if (valid) {
            double Fh[NC];
            face_flux<ND, DIR, A5>(ext, cap, o, gm1, A.sch, A.dk, omega, nullptr, Fh);
#pragma unroll
            for (int c = 0; c < NC; ++c) fhs[c * 64 + lane] = Fh[c];
        }
        __syncthreads();

        // A tube advances in this step when it was physical and t < t_end at
        // stage 0; stage 0 records its dt (0 when it does not advance), which
        // the later stages read.  t itself is only read at stage 0 and only
        // written at stage 2, so no launch both reads and writes it.
        bool active = valid && lane > 0 && phi > 0 && st_prev[b] == 0;
        const double dxb = active ? A.dx[b] : 1.0;
        double h = 0.0;
        if (A.stage == 0) {
            if (valid && lane > 0 && phi == 1) {
                double hh = 0.0;
                if (st_prev[b] == 0 && A.t[b] < A.t_end) {
                    const double a0 = a_cur[b];
                    hh = cr_div_r(A.cfl * dxb, a0, rcp_nr(a0));
                    if (A.t[b] + hh > A.t_end) hh = A.t_end - A.t[b];
                }
                A.dt[b] = hh;
            }
            if (active) {
                if (A.t[b] < A.t_end) {
                    const double a0 = a_cur[b];
                    h = cr_div_r(A.cfl * dxb, a0, rcp_nr(a0));
                    if (A.t[b] + h > A.t_end) h = A.t_end - A.t[b];
                } else {
                    active = false;
                }
            }
        } else if (active) {
            h = A.dt[b];
            active = h > 0.0;
        }
        double speed = 0.0;
        if (active) {
            const int64_t cell = A.off[b] + phi - 1;
            const double rdx = rcp_nr(dxb);
            double qn[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double diff = fhs[c * 64 + lane] - fhs[c * 64 + lane - 1];
                const double r = 0.0 - cr_div_r(diff, dxb, rdx);
                const size_t at = (size_t)c * A.total + cell;
                double v;
                if (A.stage == 0) {
                    v = A.Uin[at] + h * r;
                } else if (A.stage == 1) {
                    v = (0.75 * A.Un[at] + 0.25 * A.Uin[at]) + 0.25 * (h * r);
                } else {
                    v = ((1.0 / 3.0) * A.Un[at] + (2.0 / 3.0) * A.Uin[at]) + (2.0 / 3.0) * (h * r);
                }
                A.Uout[at] = v;
                qn[c] = v;
            }
            bool bad;
            speed = cell_speed(qn, A.sch.gamma, &bad);
            if (bad) atomicMax(&st_next[b], (int32_t)TENO_ERR_NONPHYSICAL);
            if (A.stage == 2 && phi == 1) {
                A.t[b] = A.t[b] + h;
                A.nsteps[b] += 1;
            }
        }
        tube_max(active, b, speed, a_next);
    }
}

// Batch set-up, part 1: clear the rings and the per-tube clocks.
__global__ void k_batch_clear(double* alpha_ring, int32_t* status_ring, double* dt, double* t,
                              int64_t* nsteps, int nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) {
        for (int s = 0; s < 3; ++s) {
            alpha_ring[(size_t)s * nb + i] = 0.0;
            status_ring[(size_t)s * nb + i] = 0;
        }
        dt[i] = 0.0;
        t[i] = 0.0;
        nsteps[i] = 0;
    }
}

// Batch set-up, part 2: LF speed of every tube of u^n into alpha slot 0 and
// its physicality into status slot 0.
__global__ void k_batch_alpha0(const double* U, const int64_t* off, int nb, int64_t total,
                               double gamma, double* alpha_ring, int32_t* status_ring) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool in = i < total;
    int b = 0;
    double v = 0.0;
    if (in) {
        int lo = 0, hi = nb - 1;  // tube containing cell i
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        b = lo;
        double q[3] = {U[i], U[total + i], U[2 * total + i]};
        bool bad;
        v = cell_speed(q, gamma, &bad);
        if (bad) atomicMax(&status_ring[b], (int32_t)TENO_ERR_NONPHYSICAL);
    }
    tube_max(in, b, v, (unsigned long long*)alpha_ring);
}

}  // namespace teno

using namespace teno;

struct teno_batch_plan {
    teno_grid g;
    int64_t nb = 0, total = 0, ftot = 0, nchunks = 0;
    int32_t min_len = 0, ext_cap = 0;
    double cfl = 0.5, t_end = INFINITY;
    int64_t* d_off = nullptr;
    int32_t* d_chunk_tube = nullptr;
    double* d_dx = nullptr;
    double* d_alpha = nullptr;
    int32_t* d_status = nullptr;
    double* d_dt = nullptr;
    double* d_t = nullptr;
    int64_t* d_nsteps = nullptr;
    double* d_U1 = nullptr;
    double* d_U2 = nullptr;
    int waves = 4;          // waves per block (1, 2 or 4)
    int blocks_per_cu = 0;  // persistent blocks per CU; 0 = one block per chunk group
    int cus = 256;
    std::string arch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double* graph_U = nullptr;
    int graph_steps = 0;
    hipStream_t cap_stream = nullptr;
};

namespace {

size_t lds_bytes(const teno_batch_plan* P, int W) {
    return (size_t)(24 + W * batch_wave_lds(P->ext_cap)) * sizeof(double);
}

int64_t grid_for(const teno_batch_plan* P, int W, int bpc) {
    const int64_t ngroups = (P->nchunks + W - 1) / W;
    if (bpc <= 0) return ngroups;
    const int64_t g = (int64_t)P->cus * bpc;
    return g < ngroups ? g : ngroups;
}

hipError_t launch_stage(teno_batch_plan* P, double* U, int stage, int W, int bpc, hipStream_t st) {
    BatchArgs A;
    memset(&A, 0, sizeof(A));
    A.Uin = stage == 0 ? U : (stage == 1 ? P->d_U1 : P->d_U2);
    A.Un = U;
    A.Uout = stage == 0 ? P->d_U1 : (stage == 1 ? P->d_U2 : U);
    A.off = P->d_off;
    A.chunk_tube = P->d_chunk_tube;
    A.dx = P->d_dx;
    A.alpha_ring = P->d_alpha;
    A.status_ring = P->d_status;
    A.dt = P->d_dt;
    A.t = P->d_t;
    A.nsteps = P->d_nsteps;
    A.total = P->total;
    A.ftot = P->ftot;
    A.nchunks = P->nchunks;
    A.nb = (int32_t)P->nb;
    A.stage = stage;
    A.bc = P->g.bc[0];
    A.ext_cap = P->ext_cap;
    A.cfl = P->cfl;
    A.t_end = P->t_end;
    A.sch = scheme_of(&P->g);
    A.dk = decision_consts(&P->g, false);
    const int64_t grid = grid_for(P, W, bpc);
    const size_t lds = lds_bytes(P, W);
    const bool a5 = P->g.scheme == TENO_SCHEME_TENO5A;
    switch (W + (a5 ? 8 : 0)) {
        case 1: hipLaunchKernelGGL((k_batch_stage<1, false>), dim3((unsigned)grid), dim3(64), lds, st, A); break;
        case 2: hipLaunchKernelGGL((k_batch_stage<2, false>), dim3((unsigned)grid), dim3(128), lds, st, A); break;
        case 4: hipLaunchKernelGGL((k_batch_stage<4, false>), dim3((unsigned)grid), dim3(256), lds, st, A); break;
        case 9: hipLaunchKernelGGL((k_batch_stage<1, true>), dim3((unsigned)grid), dim3(64), lds, st, A); break;
        case 10: hipLaunchKernelGGL((k_batch_stage<2, true>), dim3((unsigned)grid), dim3(128), lds, st, A); break;
        default: hipLaunchKernelGGL((k_batch_stage<4, true>), dim3((unsigned)grid), dim3(256), lds, st, A); break;
    }
    return hipGetLastError();
}

hipError_t enqueue_steps(teno_batch_plan* P, double* U, int64_t nsteps, hipStream_t st) {
    for (int64_t k = 0; k < nsteps; ++k)
        for (int s = 0; s < 3; ++s) {
            const hipError_t e = launch_stage(P, U, s, P->waves, P->blocks_per_cu, st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

void drop_graph(teno_batch_plan* P) {
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->gexec = nullptr;
    P->graph = nullptr;
    P->graph_U = nullptr;
    P->graph_steps = 0;
}

std::string tune_key(const teno_batch_plan* P) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s cus=%d nb=%lld total=%lld minlen=%d scheme=%d", P->arch.c_str(),
             P->cus, (long long)P->nb, (long long)P->total, P->min_len, P->g.scheme);
    return buf;
}

bool load_tuning(teno_batch_plan* P, const char* path) {
    if (path == nullptr) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    const std::string key = "\"key\": \"" + tune_key(P) + "\"";
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        if (strstr(line, key.c_str())) {
            const char* w = strstr(line, "\"waves\": ");
            const char* b = strstr(line, "\"blocks_per_cu\": ");
            if (w && b) {
                P->waves = atoi(w + 9);
                P->blocks_per_cu = atoi(b + 17);
                found = true;
            }
        }
    }
    fclose(f);
    return found;
}

void store_tuning(const teno_batch_plan* P, const char* path, double ms) {
    if (path == nullptr) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"waves\": %d, \"blocks_per_cu\": %d, \"ms_per_step\": %.6f}\n",
            tune_key(P).c_str(), P->waves, P->blocks_per_cu, ms);
    fclose(f);
}

}  // namespace

extern "C" {

int teno_batch_plan_create(const teno_grid* g, int64_t nbatch, const int64_t* lengths,
                           const double* dx, double cfl, double t_end, const char* tune_cache,
                           teno_batch_plan** out) {
    if (out == nullptr || g == nullptr || lengths == nullptr || dx == nullptr || nbatch <= 0 ||
        nbatch > 0x7fffffff || !(cfl > 0.0) || !(t_end > 0.0) || g->boundary_dev != nullptr)
        return TENO_ERR_ARG;
    teno_grid gg = *g;
    gg.ndim = 1;
    gg.n[0] = 3;
    gg.n[1] = gg.n[2] = 1;
    gg.dx[0] = 1.0;
    if (validate(&gg) != TENO_OK) return TENO_ERR_ARG;
    std::vector<int64_t> off((size_t)nbatch + 1, 0);
    int64_t mn = INT64_MAX;
    for (int64_t b = 0; b < nbatch; ++b) {
        if (lengths[b] < 3 || !(dx[b] > 0.0)) return TENO_ERR_ARG;
        off[(size_t)b + 1] = off[(size_t)b] + lengths[b];
        if (lengths[b] < mn) mn = lengths[b];
    }
    teno_batch_plan* P = new teno_batch_plan();
    P->g = gg;
    P->nb = nbatch;
    P->total = off[(size_t)nbatch];
    P->ftot = P->total + nbatch;
    P->nchunks = (P->ftot - 1 + kBatchCells - 1) / kBatchCells;
    P->min_len = (int32_t)(mn < 4096 ? mn : 4096);
    P->ext_cap = ext_cap_for(P->min_len);
    P->cfl = cfl;
    P->t_end = t_end;
    std::vector<int32_t> ct((size_t)P->nchunks);
    batch_chunk_tubes(off.data(), nbatch, P->nchunks, ct.data());
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete P;
        return TENO_ERR_DEVICE;
    }
    P->cus = prop.multiProcessorCount;
    P->arch = prop.gcnArchName;
    P->waves = (lds_bytes(P, 4) <= 64 * 1024) ? 4 : 1;
    int occ = 0;
    if (P->waves == 4 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, (g->scheme == TENO_SCHEME_TENO5A) ? k_batch_stage<4, true> : k_batch_stage<4, false>,
            256, lds_bytes(P, 4)) ==
            hipSuccess && occ > 0)
        P->blocks_per_cu = occ;
    const size_t nb = (size_t)nbatch;
    const size_t sb = 3 * (size_t)P->total * sizeof(double);
    bool ok = hipMalloc(&P->d_off, (nb + 1) * sizeof(int64_t)) == hipSuccess &&
              hipMalloc(&P->d_chunk_tube, ct.size() * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->d_dx, nb * sizeof(double)) == hipSuccess &&
              hipMalloc(&P->d_alpha, 3 * nb * sizeof(double)) == hipSuccess &&
              hipMalloc(&P->d_status, 3 * nb * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->d_dt, nb * sizeof(double)) == hipSuccess &&
              hipMalloc(&P->d_t, nb * sizeof(double)) == hipSuccess &&
              hipMalloc(&P->d_nsteps, nb * sizeof(int64_t)) == hipSuccess &&
              hipMalloc(&P->d_U1, sb) == hipSuccess && hipMalloc(&P->d_U2, sb) == hipSuccess &&
              hipMemcpy(P->d_off, off.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(P->d_chunk_tube, ct.data(), ct.size() * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(P->d_dx, dx, nb * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        teno_batch_plan_destroy(P);
        return TENO_ERR_DEVICE;
    }
    load_tuning(P, tune_cache);
    *out = P;
    return TENO_OK;
}

int teno_batch_plan_destroy(teno_batch_plan* P) {
    if (P == nullptr) return TENO_ERR_ARG;
    drop_graph(P);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    (void)hipFree(P->d_off);
    (void)hipFree(P->d_chunk_tube);
    (void)hipFree(P->d_dx);
    (void)hipFree(P->d_alpha);
    (void)hipFree(P->d_status);
    (void)hipFree(P->d_dt);
    (void)hipFree(P->d_t);
    (void)hipFree(P->d_nsteps);
    (void)hipFree(P->d_U1);
    (void)hipFree(P->d_U2);
    delete P;
    return TENO_OK;
}

int64_t teno_batch_total_cells(const teno_batch_plan* P) { return P ? P->total : -1; }

int teno_batch_init(teno_batch_plan* P, const double* U, void* stream) {
    if (P == nullptr || U == nullptr) return TENO_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)P->nb;
    hipLaunchKernelGGL(k_batch_clear, dim3((nb + 255) / 256), dim3(256), 0, st, P->d_alpha,
                       P->d_status, P->d_dt, P->d_t, P->d_nsteps, nb);
    const int64_t blocks = (P->total + 255) / 256;
    hipLaunchKernelGGL(k_batch_alpha0, dim3((unsigned)blocks), dim3(256), 0, st, U, P->d_off, nb,
                       P->total, P->g.gamma, P->d_alpha, P->d_status);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_batch_step(teno_batch_plan* P, double* U, void* stream) {
    if (P == nullptr || U == nullptr) return TENO_ERR_ARG;
    return enqueue_steps(P, U, 1, (hipStream_t)stream) == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_batch_run(teno_batch_plan* P, double* U, int64_t nsteps, void* stream) {
    if (P == nullptr || U == nullptr || nsteps < 0) return TENO_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int per_graph = 10;
    if (nsteps >= per_graph && (P->gexec == nullptr || P->graph_U != U)) {
        drop_graph(P);
        if (P->cap_stream == nullptr &&
            hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return TENO_ERR_DEVICE;
        if (hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return TENO_ERR_DEVICE;
        const hipError_t e = enqueue_steps(P, U, per_graph, P->cap_stream);
        const hipError_t e2 = hipStreamEndCapture(P->cap_stream, &P->graph);
        if (e != hipSuccess || e2 != hipSuccess) return TENO_ERR_DEVICE;
        if (hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0) != hipSuccess)
            return TENO_ERR_DEVICE;
        P->graph_U = U;
        P->graph_steps = per_graph;
    }
    int64_t done = 0;
    if (P->gexec != nullptr && P->graph_U == U) {
        for (; done + P->graph_steps <= nsteps; done += P->graph_steps)
            if (hipGraphLaunch(P->gexec, st) != hipSuccess) return TENO_ERR_DEVICE;
    }
    return enqueue_steps(P, U, nsteps - done, st) == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_batch_autotune(teno_batch_plan* P, const double* U, int32_t steps, const char* tune_cache,
                        double* best_ms) {
    if (P == nullptr || U == nullptr || steps <= 0) return TENO_ERR_ARG;
    if (load_tuning(P, tune_cache)) {
        if (best_ms) *best_ms = -1.0;
        return TENO_OK;
    }
    double* work = nullptr;
    const size_t sb = 3 * (size_t)P->total * sizeof(double);
    if (hipMalloc(&work, sb) != hipSuccess) return TENO_ERR_DEVICE;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(work);
        return TENO_ERR_DEVICE;
    }
    const int cand_w[3] = {4, 2, 1};
    const int cand_b[5] = {0, 2, 4, 8, 16};
    double best = 1e300;
    int bw = P->waves, bb = P->blocks_per_cu;
    for (int wi = 0; wi < 3; ++wi) {
        const int W = cand_w[wi];
        if (lds_bytes(P, W) > 64 * 1024) continue;
        for (int bi = 0; bi < 5; ++bi) {
            const int B = cand_b[bi];
            P->waves = W;
            P->blocks_per_cu = B;
            float ms = 0.f;
            const bool ok = hipMemcpy(work, U, sb, hipMemcpyDeviceToDevice) == hipSuccess &&
                            teno_batch_init(P, work, nullptr) == TENO_OK &&
                            enqueue_steps(P, work, 1, nullptr) == hipSuccess &&  // warm-up
                            hipEventRecord(e0, nullptr) == hipSuccess &&
                            enqueue_steps(P, work, steps, nullptr) == hipSuccess &&
                            hipEventRecord(e1, nullptr) == hipSuccess &&
                            hipEventSynchronize(e1) == hipSuccess &&
                            hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (!ok) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                (void)hipFree(work);
                return TENO_ERR_DEVICE;
            }
            const double per = ms / steps;
            if (per < best) {
                best = per;
                bw = W;
                bb = B;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(work);
    P->waves = bw;
    P->blocks_per_cu = bb;
    drop_graph(P);
    store_tuning(P, tune_cache, best);
    if (best_ms) *best_ms = best;
    return TENO_OK;
}

int teno_batch_get_config(const teno_batch_plan* P, int32_t* waves, int32_t* blocks_per_cu) {
    if (P == nullptr) return TENO_ERR_ARG;
    if (waves) *waves = P->waves;
    if (blocks_per_cu) *blocks_per_cu = P->blocks_per_cu;
    return TENO_OK;
}

int teno_batch_set_config(teno_batch_plan* P, int32_t waves, int32_t blocks_per_cu) {
    if (P == nullptr || !(waves == 1 || waves == 2 || waves == 4) || blocks_per_cu < 0 ||
        lds_bytes(P, waves) > 64 * 1024)
        return TENO_ERR_ARG;
    P->waves = waves;
    P->blocks_per_cu = blocks_per_cu;
    drop_graph(P);
    return TENO_OK;
}

int teno_batch_read(const teno_batch_plan* P, double* t, double* dt, int32_t* status,
                    int64_t* nsteps) {
    if (P == nullptr) return TENO_ERR_ARG;
    const size_t nb = (size_t)P->nb;
    if (hipDeviceSynchronize() != hipSuccess) return TENO_ERR_DEVICE;
    if (t && hipMemcpy(t, P->d_t, nb * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return TENO_ERR_DEVICE;
    if (dt && hipMemcpy(dt, P->d_dt, nb * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return TENO_ERR_DEVICE;
    if (nsteps && hipMemcpy(nsteps, P->d_nsteps, nb * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return TENO_ERR_DEVICE;
    if (status) {
        std::vector<int32_t> ring(3 * nb);
        if (hipMemcpy(ring.data(), P->d_status, 3 * nb * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            return TENO_ERR_DEVICE;
        for (size_t i = 0; i < nb; ++i) {
            int32_t s = ring[i];
            if (ring[nb + i] > s) s = ring[nb + i];
            if (ring[2 * nb + i] > s) s = ring[2 * nb + i];
            status[i] = s;
        }
    }
    return TENO_OK;
}

}  // extern "C"
