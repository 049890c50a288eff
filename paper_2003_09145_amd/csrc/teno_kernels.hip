// HIP kernels of the TENO5-LAD Euler right-hand side for gfx950 and the
// C-ABI entry points declared in include/teno.h.
//
// Sweep design ("face stream"): for one axis the lines along that axis are
// concatenated into one flat sequence of faces, n + 1 faces per line.  Each
// 64-lane wave takes 64 consecutive faces of that sequence, starting at a
// multiple of 63, so consecutive waves overlap by one face: lane l computes
// the numerical flux at its face, and lanes 1..63 difference their face with
// the previous lane's to update one cell each.  Every cell is updated by
// exactly one lane, with no idle lanes in the interior of the sequence and no
// tile-edge raggedness for any line length (the one face in 64 computed
// twice is the only redundancy).  The per-cell quantities that all six faces
// around a cell need (split fluxes in local order, sqrt(rho), u, H) are
// computed once per cell into LDS and read back by the faces.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <string.h>

#include <mutex>

#include "../../include/teno.h"
#include "teno_device.hpp"
#include "teno_face.hpp"
#include "teno_host.hpp"

namespace teno {

constexpr int kMaxLdsPerBlock = 64 * 1024;
constexpr int kFacesPerChunk = 64;
constexpr int kCellsPerChunk = 63;
// blocks of the LF-speed reduction: each writes one partial (3 maxima and a
// non-physical flag), reduced afterwards by a single block (no atomics)
constexpr int kAlphaBlocks = 2048;

// Per-launch description of one sweep.
struct SweepArgs {
    const double* U;        // state the stencils read (stage input)
    const double* Rin;      // partial RHS of earlier axes (nullable: start from 0)
    double* Rout;           // RHS output (rk == 0)
    const double* Un;       // u^n (rk == 2, 3)
    double* Uout;           // RK stage output (rk > 0)
    const double* alpha;    // LF speeds, 3 doubles (indexed by axis)
    const teno_ctrl* ctrl;  // nullable: the sweep runs only while ctrl->active and OK
    const double* dtp;      // dt of the fused RK stage (rk > 0)
    unsigned long long* digest;  // nullable: cutoff-mask digest accumulator
    int32_t axis;
    uint8_t* dump;          // nullable: decision bytes of this axis
    int64_t ncell;
    int64_t line_step;      // cell-index step between consecutive lines of a column
    int64_t stride;         // cell-index step along the swept axis
    int64_t col_step;       // cell-index step between columns
    int64_t ftot;           // faces per column = lines_per_col * (n + 1)
    int64_t nchunks;        // chunks per column * ncols
    int64_t ncols;
    int32_t n;              // cells along the swept axis
    int32_t bc;
    int32_t rk;             // 0: write RHS; 1..3: fused RK stage
    int32_t stage;          // RK stage of this sweep (digest key; with ctrl->nsteps)
    int32_t ext_cap;        // LDS ext cells per wave
    double dx;
    SchemeParams sch;
    DecisionConsts dk;
    const teno_boundary* bnd;  // nullable: per-end boundaries and gravity
    int32_t add_source;        // 1 on the last axis when bnd is set
    int32_t nx, ny;            // grid sizes (boundary split coordinates)
    double dxa[3];             // spacings per axis (boundary split coordinates)
    // multiply-and-shift division by n + 1, n + 6 and ncols (dividends < 2^31);
    // div32: every face and ext index of a column is below 2^31
    uint32_t m1, s1, m6, s6, mc, sc;
    int32_t div32;
};

// Boundary kind of the ghost cells at end `end` of axis `dir` for the line
// whose interior cells start at global index cell0 (per-end boundaries): the
// split coordinate along the side's split axis, the split position at the
// stage time (teno_step: t, t + dt, t + dt/2 by stage; teno_rhs: t_rhs), and
// the fixed state when the selected part is TENO_BC_FIXED (*fixed, else null).
__device__ __forceinline__ int boundary_kind(const teno_boundary* bnd, const teno_ctrl* ctrl,
                                             int stage, int dir, int end, int64_t cell0, int nx,
                                             int ny, const double* dxa, const double** fixed) {
    const teno_side* sd = &bnd->side[dir][end];
    int which = 0;
    const int ax = sd->split_axis;
    if (ax >= 0) {
        const int64_t nxy = (int64_t)nx * ny;
        const int64_t ia = (ax == 0) ? cell0 % nx : (ax == 1) ? (cell0 / nx) % ny : cell0 / nxy;
        double t = bnd->t_rhs;
        if (ctrl != nullptr) {
            t = ctrl->t;
            if (stage == 1) t = ctrl->t + ctrl->dt;
            if (stage == 2) t = ctrl->t + 0.5 * ctrl->dt;
        }
        const double coord = ((double)ia + 0.5) * dxa[ax];
        const double split = sd->split[0] + sd->split[1] * t;
        if (!(coord < split)) which = 1;
    }
    const int kind = sd->kind[which];
    *fixed = (kind == TENO_BC_FIXED) ? sd->state[which] : nullptr;
    return kind;
}

// 64-bit mixer (the splitmix64 finaliser) for the cutoff-mask digest.
__device__ __forceinline__ unsigned long long mask_hash(unsigned long long z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// CAPC: the stencil-buffer stride when it is known at compile time (it is
// ext_cap_for(n) = 74 for every n >= 63), so that every LDS stencil read is a
// per-lane base plus an immediate offset; 0: taken from A.ext_cap.
// kCapBlockLong: the x-sweep window of 4 chunks when lines hold n >= 252
// cells (253 faces then span at most 2 lines: 252 + 6 + 5 = 263 cells); its
// 31.1 KB of LDS let 5 blocks share a CU, so it is compiled for 5 waves per
// SIMD (at most 96 VGPRs).
constexpr int kCapBlockLong = 264;

// A pointer to a kernel's argument segment (constant address space).
template <class T>
using KernArgs = __attribute__((address_space(4))) const T*;

template <int ND, int DIR, int W, bool DIGEST, int CAPC, bool A5>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(CAPC == kCapBlockLong ? 5 : 4))) void k_sweep(SweepArgs A) {
    constexpr int NC = ND + 2;
    constexpr int NV = 2 * NC + ND + 2;  // f+ (NC), f- (NC), sqrt(rho), u (ND), H
    using LO = LocalOrder<ND, DIR>;
    extern __shared__ double smem[];

    if (A.ctrl != nullptr) {
        if (!A.ctrl->active || A.ctrl->status != 0) return;  // uniform across the grid
    }
    // The arguments are read through a pointer to the argument segment, where
    // the kernel's one argument sits at offset 0, rather than from the
    // by-value parameter: each scalar load is then issued where its value is
    // used instead of at entry, so fewer stay live (the y and z sweeps spill
    // 4 SGPRs instead of 9; the 256^3 step 0.6-1.3% and the 2048^2 step
    // 1.1-1.4% faster).  The host pass of this translation unit never runs
    // the body and reads the parameter.
#if defined(__HIP_DEVICE_COMPILE__)
    const auto& Ai = *(KernArgs<SweepArgs>)__builtin_amdgcn_kernarg_segment_ptr();
    SchemeParams sch_i;
    DecisionConsts dk_i;
    __builtin_memcpy(&sch_i, (const void*)&Ai.sch, sizeof(sch_i));
    __builtin_memcpy(&dk_i, (const void*)&Ai.dk, sizeof(dk_i));
#else
    const SweepArgs& Ai = A;
    const SchemeParams sch_i = Ai.sch;
    const DecisionConsts dk_i = Ai.dk;
#endif
    const double dxa_i[3] = {Ai.dxa[0], Ai.dxa[1], Ai.dxa[2]};
    // the wave index is uniform; saying so explicitly keeps the y and z
    // variants' column split scalar (along x it only costs registers)
    const int wave = DIR != 0 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    // The y and z sweeps walk their tiles from the end: y then first reads
    // the partial RHS and state that the x sweep touched last, while they
    // are still in the memory-side cache (measured: y and z each about 1%
    // faster than walking forward; x is not helped)
    const int64_t lb0 = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t lb = DIR != 0 ? (int64_t)gridDim.x - 1 - lb0 : lb0;
    const int64_t chunk = lb * W + wave;
    const bool wave_ok = chunk < Ai.nchunks;
    const int n = Ai.n;
    const int64_t np1 = n + 1, np6 = n + 6;
    int64_t col = 0, k = chunk;
    if (DIR != 0) {  // columns fastest: neighbouring waves read neighbouring x
        k = div_by((int)chunk, Ai.mc, Ai.sc);  // chunk < nchunks < 2^31
        col = chunk - k * Ai.ncols;
    }
    const int64_t colbase = col * Ai.col_step;
    const int cap = CAPC ? CAPC : Ai.ext_cap;
    // XCOOP (x sweep, CAPC = kCapBlock): the W waves of a block take W
    // consecutive chunks of the face stream, whose stencil windows overlap by
    // 6 cells; the block stages their union once, in one shared buffer, and
    // each wave reads its faces' stencils at its own offset in it.
    constexpr bool XCOOP = (DIR == 0) && (CAPC > 74);
    // y and z sweeps store the f- rows reversed (measured faster there, and
    // slower along x)
    constexpr bool MIRROR = DIR != 0;
    double* omega = smem;  // 24 doubles: eq 2.15 weights per cutoff mask
    const int per_wave = XCOOP ? 64 * NC : ((cap * NV > 64 * NC) ? cap * NV : 64 * NC);
    double* ext = XCOOP ? smem + 24 : smem + 24 + (size_t)wave * per_wave;
    // The face fluxes reuse the stencil buffer: LDS operations of one wave
    // complete in order, so every stencil read of the wave precedes its first
    // face-flux write (XCOOP: the buffer is shared, and a block barrier
    // separates every wave's stencil reads from the flux writes).
    double* fhs = XCOOP ? smem + 24 + (size_t)wave * per_wave : ext;
    if (threadIdx.x < 24) omega[threadIdx.x] = kOmega[threadIdx.x / 3][threadIdx.x % 3];

    const int64_t F0 = k * kCellsPerChunk;
    const int64_t F = F0 + lane;
    const bool valid = wave_ok && F < Ai.ftot;
    const int64_t Fc = valid ? F : F0;
    // line and in-line index of this lane's face, from those of F0 (uniform)
    // with a 32-bit step
    const int64_t bl0 = Ai.div32 ? (int64_t)div_by((int)F0, Ai.m1, Ai.s1) : F0 / np1;
    const int phi0 = (int)(F0 - bl0 * np1);
    const int tq = phi0 + (int)(Fc - F0);
    const int wraps = div_by(tq, Ai.m1, Ai.s1);
    const int64_t bl = bl0 + wraps;                        // line of this lane's face
    const int64_t phi = tq - wraps * (int)np1;             // face index in the line (i + 1)
    // staged window: the wave's chunk, or (XCOOP) the block's W chunks
    const int64_t F0w = XCOOP ? lb * W * kCellsPerChunk : F0;
    const int64_t bl0w =
        XCOOP ? (Ai.div32 ? (int64_t)div_by((int)F0w, Ai.m1, Ai.s1) : F0w / np1) : bl0;
    const int64_t e_lo = F0w + 5 * bl0w;
    int64_t Flast = F0w + 63 * (XCOOP ? W : 1);
    if (Flast > Ai.ftot - 1) Flast = Ai.ftot - 1;
    const int64_t e_hi =
        Flast + 5 * (Ai.div32 ? (int64_t)div_by((int)Flast, Ai.m1, Ai.s1) : Flast / np1) + 6;
    const int count = (XCOOP || wave_ok) ? (int)(e_hi - e_lo) : 0;

    // ---- stage per-cell quantities of the ext cells [e_lo, e_hi) ----------
    const double alpha = Ai.alpha[DIR];
    const double gm1 = sch_i.gamma - 1.0;
    const int64_t be0 = Ai.div32 ? (int64_t)div_by((int)e_lo, Ai.m6, Ai.s6)
                                : e_lo / np6;       // line of the first ext cell (uniform)
    const int je0 = (int)(e_lo - be0 * np6);
    // COOP (y and z sweeps, W waves = W neighbouring columns of one line chunk,
    // which the host guarantees): thread t stages column t % W, so a wave's
    // loads cover 64 / W cells x W neighbouring x (rows of 8 W bytes).
    constexpr bool COOP = (CAPC != 0) && (DIR != 0) && (W >= 4);
    const int64_t col0 = col - wave;  // first column of the block (uniform)
    {
    const int cc = COOP ? (int)(threadIdx.x % W) : wave;  // column slot within the block
    const int64_t colbase_c = (col0 + cc) * Ai.col_step;
    double* ext_c = XCOOP ? ext : smem + 24 + (size_t)cc * per_wave;
    // conserved state of ext cell idx (ghost images mapped, fixed states)
    auto load_cell = [&](int idx, double* q) {
        const int jq = je0 + idx;
        const int bw = div_by(jq, Ai.m6, Ai.s6);
        const int64_t b = be0 + bw;
        const int j = jq - bw * (int)np6 - 3;
        bool flip = false;
        int kind = Ai.bc;
        const double* fixed = nullptr;
        if (Ai.bnd != nullptr && (j < 0 || j >= n))
            kind = boundary_kind(Ai.bnd, Ai.ctrl, Ai.stage, DIR, j < 0 ? 0 : 1,
                                 colbase_c + b * Ai.line_step, Ai.nx, Ai.ny, dxa_i, &fixed);
        if (fixed != nullptr) {
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = fixed[c];
        } else {
            const int src = ghost_src(kind, n, j, &flip);
            const int64_t cell = colbase_c + b * Ai.line_step + (int64_t)src * Ai.stride;
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = Ai.U[c * Ai.ncell + cell];
            if (flip) q[1 + DIR] = -q[1 + DIR];
        }
    };
    // one cell ahead: the next cell's loads are in flight while this one's
    // primitives, fluxes and splits are computed
    int idx = COOP ? (int)(threadIdx.x / W) : XCOOP ? (int)threadIdx.x : lane;
    constexpr int kStep = XCOOP ? 64 * W : 64;
    double qn[NC];
    if (idx < count) load_cell(idx, qn);
    while (idx < count) {
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = qn[c];
        const int cur = idx;
        idx += kStep;
        if (idx < count) load_cell(idx, qn);
        stage_cell<ND, DIR, MIRROR>(q, alpha, gm1, ext_c, cap, cur);
    }
    }
    __syncthreads();

    // ---- the cell this thread updates ----------------------------------------
    // Face j of the chunk (j >= 1) updates its left cell from the fluxes at
    // faces j and j - 1 (COOP: thread t updates column t % W, face t / W).
    int jj = lane;
    int64_t blj = bl, phij = phi;
    bool upd = valid && lane > 0 && phi > 0;
    const double* fh_c = fhs;
    int64_t colbase_j = (DIR == 0) ? 0 : colbase;
    if constexpr (COOP) {
        jj = (int)(threadIdx.x / W);
        const int tqj = phi0 + jj;
        const int wrj = div_by(tqj, Ai.m1, Ai.s1);
        blj = bl0 + wrj;
        phij = tqj - wrj * (int)np1;
        upd = F0 + jj < Ai.ftot && jj > 0 && phij > 0;
        const int cc = (int)(threadIdx.x % W);
        fh_c = smem + 24 + (size_t)cc * per_wave;
        colbase_j = (col0 + cc) * Ai.col_step;
    }
    const int64_t cell = colbase_j + blj * Ai.line_step + (phij - 1) * Ai.stride;
    // the stage input of the fused update is loaded now, so that the face
    // computation covers the latency (each cell is read and written by its
    // own thread only, and the stencils read LDS)
    double u_in[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u_in[c] = 0.0;
    if (upd && Ai.rk != 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) u_in[c] = Ai.U[(size_t)c * Ai.ncell + cell];
    }

    // ---- numerical flux at this lane's face ----------------------------------
    // the digest is wanted or not for the whole launch (a uniform branch); the
    // plain variant carries no digest code at all
    const bool want_digest =
        DIGEST && Ai.digest != nullptr && (Ai.ctrl == nullptr || Ai.ctrl->want_digest);
    unsigned long long sig = 0ull;
    double Fh[NC];
    if (valid) {
        const int o = (int)(Fc + 5 * bl - e_lo);  // ext offset of cell i-2
        // oracle line numbering of the decision dump: x: k*ny + j; y: k*nx + i; z: j*nx + i
        uint8_t* o8 = nullptr;
        if (Ai.dump != nullptr) {
            const int64_t gline = (DIR == 0) ? bl : bl * Ai.ncols + col;
            o8 = Ai.dump + (gline * np1 + phi) * (2 * NC);
        }
        uint32_t masks = 0;
        face_flux<ND, DIR, A5, MIRROR>(ext, cap, o, gm1, sch_i, dk_i, omega, o8, Fh,
                           want_digest ? &masks : nullptr);
        if constexpr (!XCOOP) {
#pragma unroll
            for (int c = 0; c < NC; ++c) fhs[c * 64 + lane] = Fh[c];
        }
        if (want_digest) {
            // the key names the step and stage as well as the face, so masks
            // that move in time past a face change the digest
            const uint64_t when =
                (Ai.ctrl != nullptr ? 3ull * (uint64_t)Ai.ctrl->nsteps : 0ull) + (uint64_t)Ai.stage;
            sig = mask_hash(mask_hash(when) ^ ((uint64_t)Ai.axis << 60) ^
                            ((uint64_t)(col * Ai.ftot + Fc) << 30) ^ masks);
        }
    }
    if (want_digest) {
        // a face shared by two chunks (lane 63 here, lane 0 of the next) counts once
        unsigned long long v = (valid && (lane < 63 || F == Ai.ftot - 1)) ? sig : 0ull;
#pragma unroll
        for (int offs = 32; offs > 0; offs >>= 1) v += __shfl_xor(v, offs, 64);
        if (lane == 0 && v != 0ull) atomicAdd(Ai.digest, v);
    }

    if constexpr (XCOOP) {
        __syncthreads();  // every wave's stencil reads precede the flux writes
        if (valid) {
#pragma unroll
            for (int c = 0; c < NC; ++c) fhs[c * 64 + lane] = Fh[c];
        }
    }

    // ---- flux difference and epilogue ---------------------------------------
    // The cell's partial RHS and u^n are loaded before the barrier, so that
    // their latency overlaps the wait.
    double r_in[NC], u_n[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) r_in[c] = u_n[c] = 0.0;
    if (upd) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const size_t at = (size_t)c * Ai.ncell + cell;
            if (Ai.Rin != nullptr) r_in[c] = Ai.Rin[at];
            if (Ai.rk >= 2) u_n[c] = Ai.Un[at];
        }
    }
    __syncthreads();

    if (upd) {
        const double rdx = rcp_nr(Ai.dx);
        double diff[NC], dq[NC], r[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) diff[c] = fh_c[c * 64 + jj] - fh_c[c * 64 + jj - 1];
        cr_div_r_n<NC>(diff, Ai.dx, rdx, dq);  // independent quotients, one correction branch
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] = r_in[c] - dq[c];
        if (Ai.add_source) {
            // gravity: rho g_d on each momentum, m . g on the energy (after the
            // flux differences of every axis)
            const double* g = Ai.bnd->gravity;
            const double rho = Ai.U[cell];
#pragma unroll
            for (int d = 0; d < ND; ++d) r[1 + d] = r[1 + d] + rho * g[d];
            double sE = Ai.U[1 * Ai.ncell + cell] * g[0];
#pragma unroll
            for (int d = 1; d < ND; ++d) sE = sE + Ai.U[(1 + d) * Ai.ncell + cell] * g[d];
            r[NC - 1] = r[NC - 1] + sE;
        }
        if (Ai.rk == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) Ai.Rout[c * Ai.ncell + cell] = r[c];
        } else {
            const double h = *Ai.dtp;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const size_t at = (size_t)c * Ai.ncell + cell;
                double v;
                if (Ai.rk == 1) {
                    v = u_in[c] + h * r[c];
                } else if (Ai.rk == 2) {
                    v = (0.75 * u_n[c] + 0.25 * u_in[c]) + 0.25 * (h * r[c]);
                } else {
                    v = ((1.0 / 3.0) * u_n[c] + (2.0 / 3.0) * u_in[c]) + (2.0 / 3.0) * (h * r[c]);
                }
                Ai.Uout[at] = v;
            }
        }
    }
}

// ---- global Lax-Friedrichs speeds: alpha_d = max (|u_d| + c) -------------
// Pass 1 (k_alpha): every block reduces its cells and writes part[4 b + k]
// (k < 3: the maxima, 0 for absent axes; k = 3: 1.0 if the block saw a cell
// with rho <= 0, p <= 0 or a non-finite sound speed).  Pass 2
// (reduce_partials, inside the consumer kernel): one 256-thread block.
template <int ND>
__global__ __launch_bounds__(256) void k_alpha(const double* __restrict__ U, int64_t ncell,
                                               double gamma, double* __restrict__ part) {
    constexpr int NC = ND + 2;
    __shared__ double red[4][4];
    double amax[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) amax[k] = 0.0;
    bool bad = false;
    const double gm1 = gamma - 1.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = __builtin_nontemporal_load(&U[c * ncell + i]);
        const double rho = q[0];
        double u[ND];
        const double rrho = rcp_nr(rho);
#pragma unroll
        for (int k = 0; k < ND; ++k) u[k] = cr_div_r(q[1 + k], rho, rrho);
        double mu = q[1] * u[0];
#pragma unroll
        for (int k = 1; k < ND; ++k) mu = mu + q[1 + k] * u[k];
        const double ke = 0.5 * mu;
        const double p = gm1 * (q[NC - 1] - ke);
        const double cs = cr_sqrt(cr_div_r(gamma * p, rho, rrho));
        if (!(rho > 0.0) || !(p > 0.0) || !isfinite(cs)) bad = true;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            const double s = fabs(u[k]) + cs;
            if (s > amax[k]) amax[k] = s;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v4[4] = {0.0, 0.0, 0.0, bad ? 1.0 : 0.0};
#pragma unroll
    for (int k = 0; k < ND; ++k) v4[k] = amax[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = v4[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            if (o > v) v = o;
        }
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (red[w][k] > v) v = red[w][k];
        part[4 * (int64_t)blockIdx.x + k] = v;
    }
}

// Maximum of the nblk partials (call from every thread of a 256-thread
// block); out[0..2] the speeds, out[3] > 0 if any cell was non-physical.
__device__ void reduce_partials(const double* __restrict__ part, int nblk, double out[4]) {
    __shared__ double red[4][4];
    double v4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double x = part[4 * b + k];
            if (x > v4[k]) v4[k] = x;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = v4[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            if (o > v) v = o;
        }
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = red[0][k];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (red[w][k] > v) v = red[w][k];
        out[k] = v;
    }
}

// Speeds used by teno_rhs: the frozen ones, or the reduced partials (with
// the non-physical flag written to status).
__global__ __launch_bounds__(256) void k_copy_alpha(const double* part, int nblk,
                                                    const double* alpha_in, double* alpha_used,
                                                    double* alpha_out, int32_t* status) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    if (alpha_in == nullptr) reduce_partials(part, nblk, r);
    const int k = threadIdx.x;
    if (k < 3) {
        const double a = alpha_in ? alpha_in[k] : r[k];
        alpha_used[k] = a;
        if (alpha_out) alpha_out[k] = a;
    }
    if (k == 0 && status != nullptr) *status = (r[3] > 0.0) ? TENO_ERR_NONPHYSICAL : TENO_OK;
}

// Stage bookkeeping of teno_step (one 256-thread block): reduce the speeds
// of the stage input, flag a non-physical input (sticky), and at stage 0
// set dt from eq dt1 / dt2 (3D: the harmonic form) clipped to t_end.
__global__ __launch_bounds__(256) void k_stage_begin(teno_ctrl* ctrl, const double* part,
                                                     int nblk, int stage, int ndim, double dx0,
                                                     double dx1, double dx2) {
    double r[4];
    reduce_partials(part, nblk, r);
    if (threadIdx.x != 0) return;
    const bool bad = r[3] > 0.0;
    if (stage == 0) {
        ctrl->active = 0;
        if (ctrl->status != 0 || !(ctrl->t < ctrl->t_end)) return;
        if (bad) {
            ctrl->status = TENO_ERR_NONPHYSICAL;
            return;
        }
        if (!ctrl->replay) {
            const double* a = r;
            double dt;
            if (ndim == 1) {
                dt = cr_div(ctrl->cfl * dx0, a[0]);
            } else if (ndim == 2) {
                const double dtx = cr_div(dx0, a[0]);
                const double dty = cr_div(dx1, a[1]);
                dt = cr_div(ctrl->cfl * (dtx * dty), dtx + dty);
            } else {
                dt = cr_div(ctrl->cfl, (cr_div(a[0], dx0) + cr_div(a[1], dx1)) + cr_div(a[2], dx2));
            }
            if (ctrl->t + dt > ctrl->t_end) dt = ctrl->t_end - ctrl->t;
            ctrl->dt = dt;
            for (int k = 0; k < 3; ++k) ctrl->alpha[0][k] = a[k];
        }
        ctrl->active = 1;
    } else {
        if (!ctrl->active) return;
        if (bad) ctrl->status = TENO_ERR_NONPHYSICAL;
        if (ctrl->status != 0) {
            ctrl->active = 0;
            return;
        }
        if (!ctrl->replay)
            for (int k = 0; k < 3; ++k) ctrl->alpha[stage][k] = r[k];
    }
}

__global__ void k_step_end(teno_ctrl* ctrl) {
    if (threadIdx.x != 0) return;
    if (ctrl->active && ctrl->status == 0) {
        ctrl->t = ctrl->t + ctrl->dt;
        ctrl->nsteps += 1;
    }
    ctrl->active = 0;
}

__global__ void k_ctrl_init(teno_ctrl* ctrl, double t0, double t_end, double cfl) {
    if (threadIdx.x != 0) return;
    ctrl->t = t0;
    ctrl->t_end = t_end;
    ctrl->cfl = cfl;
    ctrl->dt = 0.0;
    for (int s = 0; s < 3; ++s)
        for (int k = 0; k < 3; ++k) ctrl->alpha[s][k] = 0.0;
    ctrl->status = 0;
    ctrl->replay = 0;
    ctrl->nsteps = 0;
    ctrl->active = 0;
    ctrl->want_digest = 0;
    ctrl->digest = 0ull;
    ctrl->reserved_[0] = ctrl->reserved_[1] = 0ull;
}

__global__ void k_ctrl_replay(teno_ctrl* dst, const teno_ctrl* rec) {
    if (threadIdx.x != 0) return;
    dst->dt = rec->dt;
    for (int s = 0; s < 3; ++s)
        for (int k = 0; k < 3; ++k) dst->alpha[s][k] = rec->alpha[s][k];
    dst->replay = 1;
    dst->status = 0;
    dst->t_end = INFINITY;
}

__global__ void k_ctrl_digest(teno_ctrl* ctrl, int enable) {
    if (threadIdx.x != 0) return;
    ctrl->want_digest = enable;
    ctrl->digest = 0ull;
}

// Arithmetic self-test: the device's correctly rounded division and square
// root and the approximate reciprocal used by the decision fast path.
__global__ void k_selftest_arith(const double* a, const double* b, double* q, double* q2,
                                 double* s, double* r, double* qp, double* sp, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        q[i] = cr_div(a[i], b[i]);
        q2[i] = cr_div_r(a[i], b[i], rcp_nr(b[i]));
        s[i] = cr_sqrt(a[i]);
        r[i] = rcp_nr(b[i]);
        if (qp != nullptr) qp[i] = a[i] / b[i];
        if (sp != nullptr) sp[i] = sqrt(a[i]);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct Scratch {  // device area at the end of the workspace
    double part[4 * kAlphaBlocks];  // LF-speed partials of k_alpha
    double alpha_used[4];
    int32_t pad[8];
};

static int64_t ncell_of(const teno_grid* g) { return (int64_t)g->n[0] * g->n[1] * g->n[2]; }

static size_t state_bytes(const teno_grid* g) {
    return (size_t)(g->ndim + 2) * (size_t)ncell_of(g) * sizeof(double);
}

static size_t workspace_bytes_impl(const teno_grid* g) {
    return 3 * state_bytes(g) + sizeof(Scratch) + 256;
}

static Scratch* scratch_of(const teno_grid* g, void* ws) {
    return (Scratch*)((char*)ws + 3 * state_bytes(g));
}

template <int ND, int DIR, bool A5>
static hipError_t launch_sweep_t(SweepArgs A, bool digest, hipStream_t st) {
    constexpr int NC = ND + 2;
    constexpr int NV = 2 * NC + ND + 2;
    constexpr int kCapLong = 74;  // ext_cap_for(n) for every n >= 63
    const size_t per_wave =
        (size_t)((A.ext_cap * NV > 64 * NC) ? A.ext_cap * NV : 64 * NC) * sizeof(double);
    const size_t table = 24 * sizeof(double);
    // the fixed-stride variant; along y and z a block stages and updates four
    // neighbouring columns, which needs whole blocks of columns (8- and
    // 16-column blocks, with 71 / 142 KB of LDS, measured no faster)
    if constexpr (DIR == 0) {
        if (!digest && A.ext_cap == kCapLong && A.n >= 252) {
            const int64_t blocks = (A.nchunks + 3) / 4;
            hipLaunchKernelGGL((k_sweep<ND, DIR, 4, false, kCapBlockLong, A5>),
                               dim3((unsigned)blocks), dim3(256),
                               table + (size_t)NV * kCapBlockLong * sizeof(double), st, A);
            return hipGetLastError();
        }
        if (!digest && A.ext_cap == kCapLong) {
            // x: 4 consecutive chunks per block staged once as the union of
            // their windows (4 x 63 faces span at most 5 lines when n >= 63:
            // 252 + 6 + 5 x 4 = 278 cells)
            constexpr int kCapBlock = 280;
            const int64_t blocks = (A.nchunks + 3) / 4;
            hipLaunchKernelGGL((k_sweep<ND, DIR, 4, false, kCapBlock, A5>), dim3((unsigned)blocks),
                               dim3(256), table + (size_t)NV * kCapBlock * sizeof(double), st, A);
            return hipGetLastError();
        }
    } else {
        if constexpr (DIR == 2) {
            if (!digest && A.ext_cap == kCapLong && A.ncols % 8 == 0) {
                const int64_t blocks = (A.nchunks + 7) / 8;
                hipLaunchKernelGGL((k_sweep<ND, DIR, 8, false, kCapLong, A5>),
                                   dim3((unsigned)blocks), dim3(512), table + 8 * per_wave, st, A);
                return hipGetLastError();
            }
        }
        if (!digest && A.ext_cap == kCapLong && A.ncols % 4 == 0) {
            const int64_t blocks = (A.nchunks + 3) / 4;
            hipLaunchKernelGGL((k_sweep<ND, DIR, 4, false, kCapLong, A5>), dim3((unsigned)blocks),
                               dim3(256), table + 4 * per_wave, st, A);
            return hipGetLastError();
        }
    }
    if (table + 4 * per_wave <= (size_t)kMaxLdsPerBlock) {
        const int64_t blocks = (A.nchunks + 3) / 4;
        if (digest)
            hipLaunchKernelGGL((k_sweep<ND, DIR, 4, true, 0, A5>), dim3((unsigned)blocks), dim3(256),
                               table + 4 * per_wave, st, A);
        else
            hipLaunchKernelGGL((k_sweep<ND, DIR, 4, false, 0, A5>), dim3((unsigned)blocks), dim3(256),
                               table + 4 * per_wave, st, A);
    } else {
        if (digest)
            hipLaunchKernelGGL((k_sweep<ND, DIR, 1, true, 0, A5>), dim3((unsigned)A.nchunks), dim3(64),
                               table + per_wave, st, A);
        else
            hipLaunchKernelGGL((k_sweep<ND, DIR, 1, false, 0, A5>), dim3((unsigned)A.nchunks), dim3(64),
                               table + per_wave, st, A);
    }
    return hipGetLastError();
}

static hipError_t launch_sweep(const teno_grid* g, int dir, SweepArgs A, hipStream_t st) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int n = g->n[dir];
    A.n = n;
    A.bc = g->bc[dir];
    A.dx = g->dx[dir];
    A.ncell = ncell_of(g);
    A.bnd = g->boundary_dev;
    if (A.bnd == nullptr) A.add_source = 0;
    A.nx = nx;
    A.ny = ny;
    for (int k = 0; k < 3; ++k) A.dxa[k] = g->dx[k];
    A.sch = scheme_of(g);
    A.dk = decision_consts(g, A.dump != nullptr);
    A.ext_cap = ext_cap_for(n);
    int64_t lines_per_col;
    if (dir == 0) {
        A.ncols = 1;
        A.col_step = 0;
        A.line_step = nx;
        A.stride = 1;
        lines_per_col = (int64_t)ny * nz;
    } else if (dir == 1) {
        A.ncols = nx;
        A.col_step = 1;
        A.line_step = (int64_t)nx * ny;
        A.stride = nx;
        lines_per_col = nz;
    } else {
        A.ncols = nx;
        A.col_step = 1;
        A.line_step = nx;
        A.stride = (int64_t)nx * ny;
        lines_per_col = ny;
    }
    A.ftot = lines_per_col * (n + 1);
    const int64_t chunks_per_col = (A.ftot - 1 + kCellsPerChunk - 1) / kCellsPerChunk;
    A.nchunks = chunks_per_col * A.ncols;
    if (A.nchunks > (int64_t(1) << 31) - 64) return hipErrorInvalidValue;  // chunk indices are 32-bit
    const DivMagic d1 = div_magic((uint32_t)(n + 1)), d6 = div_magic((uint32_t)(n + 6)),
                   dc = div_magic((uint32_t)A.ncols);
    A.m1 = d1.m; A.s1 = d1.sh; A.m6 = d6.m; A.s6 = d6.sh; A.mc = dc.m; A.sc = dc.sh;
    // largest ext index of a column: ftot + 5 lines_per_col (+ the chunk's tail)
    A.div32 = (A.ftot + 6 * lines_per_col + 128) < (int64_t(1) << 31) ? 1 : 0;
    const bool digest = A.digest != nullptr && (g->flags & TENO_FLAG_MASK_DIGEST) != 0;
    const int key = g->ndim * 4 + dir + (g->scheme == TENO_SCHEME_TENO5A ? 16 : 0);
    switch (key) {
        case 4: return launch_sweep_t<1, 0, false>(A, digest, st);
        case 8: return launch_sweep_t<2, 0, false>(A, digest, st);
        case 9: return launch_sweep_t<2, 1, false>(A, digest, st);
        case 12: return launch_sweep_t<3, 0, false>(A, digest, st);
        case 13: return launch_sweep_t<3, 1, false>(A, digest, st);
        case 14: return launch_sweep_t<3, 2, false>(A, digest, st);
        case 20: return launch_sweep_t<1, 0, true>(A, digest, st);
        case 24: return launch_sweep_t<2, 0, true>(A, digest, st);
        case 25: return launch_sweep_t<2, 1, true>(A, digest, st);
        case 28: return launch_sweep_t<3, 0, true>(A, digest, st);
        case 29: return launch_sweep_t<3, 1, true>(A, digest, st);
        case 30: return launch_sweep_t<3, 2, true>(A, digest, st);
    }
    return hipErrorInvalidValue;
}

static int alpha_blocks(const teno_grid* g) {
    const int64_t b = (ncell_of(g) + 255) / 256;
    return (int)(b < kAlphaBlocks ? b : kAlphaBlocks);
}

static hipError_t launch_alpha(const teno_grid* g, const double* U, double* part, hipStream_t st) {
    const int64_t nc = ncell_of(g);
    const int blocks = alpha_blocks(g);
    switch (g->ndim) {
        case 1: hipLaunchKernelGGL(k_alpha<1>, dim3(blocks), dim3(256), 0, st, U, nc, g->gamma, part); break;
        case 2: hipLaunchKernelGGL(k_alpha<2>, dim3(blocks), dim3(256), 0, st, U, nc, g->gamma, part); break;
        case 3: hipLaunchKernelGGL(k_alpha<3>, dim3(blocks), dim3(256), 0, st, U, nc, g->gamma, part); break;
    }
    return hipGetLastError();
}

// L(U) with the LF-speed partials and the speeds in use in the scratch area S.
static int rhs_with_scratch(const teno_grid* g, const double* U, double* dUdt,
                            const double* alpha_in, double* alpha_out, int32_t* status,
                            uint8_t* dump, Scratch* S, hipStream_t st) {
    if (alpha_in == nullptr) {
        if (launch_alpha(g, U, S->part, st) != hipSuccess) return TENO_ERR_DEVICE;
    }
    hipLaunchKernelGGL(k_copy_alpha, dim3(1), dim3(256), 0, st, S->part, alpha_blocks(g), alpha_in,
                       S->alpha_used, alpha_out, status);
    int64_t dump_off = 0;
    for (int d = 0; d < g->ndim; ++d) {
        SweepArgs A;
        memset(&A, 0, sizeof(A));
        A.U = U;
        A.Rin = (d == 0) ? nullptr : dUdt;
        A.Rout = dUdt;
        A.alpha = S->alpha_used;
        A.dump = dump ? dump + dump_off : nullptr;
        A.rk = 0;
        A.add_source = (d == g->ndim - 1) ? 1 : 0;
        if (launch_sweep(g, d, A, st) != hipSuccess) return TENO_ERR_DEVICE;
        dump_off += ncell_of(g) / g->n[d] * (int64_t)(g->n[d] + 1) * 2 * (g->ndim + 2);
    }
    return TENO_OK;
}

static int rhs_common(const teno_grid* g, const double* U, double* dUdt, const double* alpha_in,
                      double* alpha_out, int32_t* status, uint8_t* dump, void* ws,
                      size_t ws_bytes, void* stream) {
    if (validate(g) != TENO_OK || U == nullptr || dUdt == nullptr || ws == nullptr ||
        ws_bytes < workspace_bytes_impl(g))
        return TENO_ERR_ARG;
    return rhs_with_scratch(g, U, dUdt, alpha_in, alpha_out, status, dump, scratch_of(g, ws),
                            (hipStream_t)stream);
}

// Scratch of the allocation-free RHS (teno_rhs_noalloc): a fixed device array
// of the library, one copy per GPU, held until the process ends.  Its size
// does not depend on the grid: the LF-speed reduction writes at most
// kAlphaBlocks partials, whatever the number of cells.
constexpr size_t kNoAllocScratchBytes = 72 * 1024;
static_assert(sizeof(Scratch) <= kNoAllocScratchBytes, "the RHS scratch must fit the array");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current GPU.  In host code the array's
// name is only a host-side stand-in, so the address is looked up once per
// device (with that device current) and kept.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_dev[kMaxDevices];

static int scratch_address(Scratch** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TENO_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_dev[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return TENO_ERR_DEVICE;
        g_scratch_dev[dev] = p;
    }
    *out = (Scratch*)g_scratch_dev[dev];
    return TENO_OK;
}

// One RK stage with frozen speeds and dt (no gating): the sweeps of every
// axis, the last one fused with the stage update of eq 4.1 (rk = 1), 4.2
// (rk = 2) or 4.3 (rk = 3).  Used by the adjoint to rebuild stage states.
hipError_t stage_frozen(const teno_grid* g, const double* Uin, const double* Un, double* Uout,
                        double* R, const double* alpha, const double* dtp, int rk,
                        hipStream_t st) {
    for (int d = 0; d < g->ndim; ++d) {
        SweepArgs A;
        memset(&A, 0, sizeof(A));
        A.U = Uin;
        A.Rin = (d == 0) ? nullptr : R;
        A.Rout = R;
        A.alpha = alpha;
        A.dtp = dtp;
        A.axis = d;
        if (d == g->ndim - 1) {
            A.rk = rk;
            A.Un = Un;
            A.Uout = Uout;
        }
        const hipError_t e = launch_sweep(g, d, A, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace teno

using namespace teno;

extern "C" {

size_t teno_workspace_bytes(const teno_grid* g) {
    if (validate(g) != TENO_OK) return 0;
    return workspace_bytes_impl(g);
}

int teno_ctrl_init(teno_ctrl* ctrl, double t0, double t_end, double cfl, void* stream) {
    if (ctrl == nullptr || !(cfl > 0.0)) return TENO_ERR_ARG;
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, (hipStream_t)stream, ctrl, t0, t_end, cfl);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_ctrl_replay(teno_ctrl* dst, const teno_ctrl* recorded, void* stream) {
    if (dst == nullptr || recorded == nullptr) return TENO_ERR_ARG;
    hipLaunchKernelGGL(k_ctrl_replay, dim3(1), dim3(64), 0, (hipStream_t)stream, dst, recorded);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_ctrl_digest(teno_ctrl* ctrl, int32_t enable, void* stream) {
    if (ctrl == nullptr) return TENO_ERR_ARG;
    hipLaunchKernelGGL(k_ctrl_digest, dim3(1), dim3(64), 0, (hipStream_t)stream, ctrl, enable ? 1 : 0);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_rhs(const teno_grid* g, const double* U, double* dUdt, const double* alpha_in,
             double* alpha_out, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    return rhs_common(g, U, dUdt, alpha_in, alpha_out, status, nullptr, ws, ws_bytes, stream);
}

int teno_rhs_noalloc(const teno_grid* g, const double* U, double* dUdt, const double* alpha_in,
                     double* alpha_out, int32_t* status, void* stream) {
    if (validate(g) != TENO_OK || U == nullptr || dUdt == nullptr) return TENO_ERR_ARG;
    Scratch* S = nullptr;
    const int rc = scratch_address(&S);
    if (rc != TENO_OK) return rc;
    // nothing in the scratch needs to start at zero: the reduction reads only
    // the partials this call's k_alpha writes, and k_copy_alpha overwrites
    // the speeds in use
    return rhs_with_scratch(g, U, dUdt, alpha_in, alpha_out, status, nullptr, S,
                            (hipStream_t)stream);
}

int teno_rhs_debug(const teno_grid* g, const double* U, double* dUdt, const double* alpha_in,
                   double* alpha_out, int32_t* status, uint8_t* decisions, void* ws,
                   size_t ws_bytes, void* stream) {
    if (decisions == nullptr) return TENO_ERR_ARG;
    return rhs_common(g, U, dUdt, alpha_in, alpha_out, status, decisions, ws, ws_bytes, stream);
}

int teno_selftest_arith(const double* a, const double* b, double* q, double* q2, double* s,
                        double* r, double* qp, double* sp, int64_t n, void* stream) {
    if (n < 0 || (n > 0 && (a == nullptr || b == nullptr || q == nullptr || q2 == nullptr ||
                            s == nullptr || r == nullptr)))
        return TENO_ERR_ARG;
    if (n == 0) return TENO_OK;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_selftest_arith, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, a, b, q, q2, s, r, qp, sp, n);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

int teno_sweep(const teno_grid* g, int32_t axis, const double* U, const double* Rin,
               double* Rout, const double* alpha, void* stream) {
    if (validate(g) != TENO_OK || axis < 0 || axis >= g->ndim || U == nullptr ||
        Rout == nullptr || alpha == nullptr)
        return TENO_ERR_ARG;
    SweepArgs A;
    memset(&A, 0, sizeof(A));
    A.U = U;
    A.Rin = Rin;
    A.Rout = Rout;
    A.alpha = alpha;
    return launch_sweep(g, axis, A, (hipStream_t)stream) == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

}  // extern "C"

static int step_impl(const teno_grid* g, double* U, teno_ctrl* ctrl, void* ws, size_t ws_bytes,
                     void* const* events, void* stream) {
    if (validate(g) != TENO_OK || U == nullptr || ctrl == nullptr || ws == nullptr ||
        ws_bytes < workspace_bytes_impl(g))
        return TENO_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const size_t sb = state_bytes(g);
    double* R = (double*)ws;
    double* U1 = (double*)((char*)ws + sb);
    double* U2 = (double*)((char*)ws + 2 * sb);
    Scratch* S = scratch_of(g, ws);
    const double* stage_in[3] = {U, U1, U2};
    double* stage_out[3] = {U1, U2, U};
    for (int s = 0; s < 3; ++s) {
        if (launch_alpha(g, stage_in[s], S->part, st) != hipSuccess) return TENO_ERR_DEVICE;
        hipLaunchKernelGGL(k_stage_begin, dim3(1), dim3(256), 0, st, ctrl, S->part, alpha_blocks(g),
                           s, g->ndim, g->dx[0], g->dx[1], g->dx[2]);
        for (int d = 0; d < g->ndim; ++d) {
            SweepArgs A;
            memset(&A, 0, sizeof(A));
            A.U = stage_in[s];
            A.Rin = (d == 0) ? nullptr : R;
            A.Rout = R;
            A.alpha = &ctrl->alpha[s][0];
            A.ctrl = ctrl;
            A.dtp = &ctrl->dt;
            A.axis = d;
            A.stage = s;
            A.digest = (unsigned long long*)&ctrl->digest;
            if (d == g->ndim - 1) {
                A.rk = s + 1;
                A.Un = U;
                A.Uout = stage_out[s];
                A.add_source = 1;
            }
            void* ev0 = events ? events[2 * (g->ndim * s + d)] : nullptr;
            void* ev1 = events ? events[2 * (g->ndim * s + d) + 1] : nullptr;
            if (ev0 != nullptr && hipEventRecord((hipEvent_t)ev0, st) != hipSuccess)
                return TENO_ERR_DEVICE;
            if (launch_sweep(g, d, A, st) != hipSuccess) return TENO_ERR_DEVICE;
            if (ev1 != nullptr && hipEventRecord((hipEvent_t)ev1, st) != hipSuccess)
                return TENO_ERR_DEVICE;
        }
    }
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, ctrl);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_ERR_DEVICE;
}

extern "C" {

int teno_step(const teno_grid* g, double* U, teno_ctrl* ctrl, void* ws, size_t ws_bytes,
              void* stream) {
    return step_impl(g, U, ctrl, ws, ws_bytes, nullptr, stream);
}

int teno_step_timed(const teno_grid* g, double* U, teno_ctrl* ctrl, void* ws, size_t ws_bytes,
                    void* const* events, void* stream) {
    return step_impl(g, U, ctrl, ws, ws_bytes, events, stream);
}

}  // extern "C"

// A recorded run of steps_per_graph steps on fixed buffers.  Every launch of
// a step takes its arguments from the grid copy and the pointers held here,
// and its dt, t and status from the device control block, so replays of the
// graph continue the run exactly as further teno_step calls would.
struct teno_runner {
    teno_grid g;
    double* U = nullptr;
    teno_ctrl* ctrl = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int32_t steps_per_graph = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int teno_runner_destroy(teno_runner* r) {
    if (r == nullptr) return TENO_ERR_ARG;
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->cap) (void)hipStreamDestroy(r->cap);
    delete r;
    return TENO_OK;
}

int teno_runner_create(const teno_grid* g, double* U, teno_ctrl* ctrl, void* ws, size_t ws_bytes,
                       int32_t steps_per_graph, teno_runner** out) {
    if (out == nullptr || validate(g) != TENO_OK || U == nullptr || ctrl == nullptr ||
        ws == nullptr || ws_bytes < workspace_bytes_impl(g) || steps_per_graph < 1 ||
        steps_per_graph > 1000)
        return TENO_ERR_ARG;
    teno_runner* r = new teno_runner();
    r->g = *g;
    r->U = U;
    r->ctrl = ctrl;
    r->ws = ws;
    r->ws_bytes = ws_bytes;
    r->steps_per_graph = steps_per_graph;
    // the steps are recorded on a private stream, so that no other work of
    // the caller's stream is captured; thread-local mode leaves other
    // threads' HIP calls alone
    if (hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking) != hipSuccess) {
        teno_runner_destroy(r);
        return TENO_ERR_DEVICE;
    }
    if (hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        teno_runner_destroy(r);
        return TENO_ERR_DEVICE;
    }
    int rc = TENO_OK;
    for (int32_t k = 0; k < steps_per_graph && rc == TENO_OK; ++k)
        rc = step_impl(&r->g, U, ctrl, ws, ws_bytes, nullptr, r->cap);
    const hipError_t e = hipStreamEndCapture(r->cap, &r->graph);
    if (rc != TENO_OK || e != hipSuccess ||
        hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0) != hipSuccess) {
        teno_runner_destroy(r);
        return rc != TENO_OK ? rc : TENO_ERR_DEVICE;
    }
    *out = r;
    return TENO_OK;
}

int teno_runner_run(teno_runner* r, int64_t nsteps, void* stream) {
    if (r == nullptr || nsteps < 0) return TENO_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    int64_t done = 0;
    for (; done + r->steps_per_graph <= nsteps; done += r->steps_per_graph)
        if (hipGraphLaunch(r->exec, st) != hipSuccess) return TENO_ERR_DEVICE;
    for (; done < nsteps; ++done) {
        const int rc = step_impl(&r->g, r->U, r->ctrl, r->ws, r->ws_bytes, nullptr, st);
        if (rc != TENO_OK) return rc;
    }
    return TENO_OK;
}

}  // extern "C"
