// Index maps of the line-based kernels: ghost cells, the multiply-and-shift
// division, the XCD-aware block order, and the chunk, staging and gather
// maps of the batched-tube kernel and of the adjoint's chunked passes.
//
// Plain integer arithmetic with no HIP dependency: under hipcc every function
// is compiled for host and device, under a host compiler for the host only,
// so the CPU tests run the very index code the kernels run and check every
// global and LDS index it produces.
#pragma once

#include <stdint.h>

#include "teno_divmagic.hpp"

#ifdef __HIPCC__
#define TENO_HD __host__ __device__ __forceinline__
#else
#define TENO_HD inline
#endif

namespace teno {

// Ghost-cell source along a swept axis: periodic wrap, zero-gradient copy or
// reflecting mirror (normal momentum negated), three cells per side.
TENO_HD int ghost_src(int bc, int n, int j, bool* flip) {
    *flip = false;
    if (j >= 0 && j < n) return j;
    if (bc == 0) return j < 0 ? j + n : j - n;  // |j| <= 3 <= n
    if (bc == 1) return j < 0 ? 0 : n - 1;
    *flip = true;
    return j < 0 ? -1 - j : 2 * n - 1 - j;
}

// floor(x / d) for 0 <= x < 2^31 from the host's DivMagic constants of d.
TENO_HD int div_by(int x, uint32_t m, uint32_t sh) {
    return (int)(((uint64_t)(uint32_t)x * m) >> sh);
}

// Map the hardware block index to a logical index such that blocks that run
// on the same XCD (hardware assigns block b to XCD b % 8) get consecutive
// logical indices, so neighbouring tiles share that XCD's L2.
TENO_HD int64_t xcd_logical_block(int64_t b, int64_t G) {
    const int64_t q = G / 8, r = G % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Cells a 64-face chunk stages (its faces' stencils, ghost cells included)
// when every line has at least n cells: 63 faces plus 6 stencil cells, plus
// the 5 extra ghost cells of each line boundary the chunk crosses.
TENO_HD int ext_cap_for(int n) { return 69 + 5 * (63 / (n + 1) + 1); }

// ---------------------------------------------------------------------------
// Batched tubes.  Tube b holds cells off[b] .. off[b+1]-1 of the packed state
// and faces off[b] + b .. off[b+1] + b of the concatenated face stream (N_b + 1
// faces, face phi between tube cells phi-1 and phi); its ghost-extended cells
// are off[b] + 6 b .. off[b+1] + 6 b + 5 (cell j at off[b] + 6 b + j + 3).
// Chunk k holds the 64 faces 63 k .. 63 k + 63; lane 0 only supplies the left
// flux of lane 1, so each face > 0 updates its left cell exactly once.
// ---------------------------------------------------------------------------
constexpr int kBatchCells = 63;

// Largest tube b' >= b whose first face (off[b'] + b') is <= F.
TENO_HD int batch_tube_of_face(const int64_t* off, int nb, int b, int64_t F) {
    while (b + 1 < nb && off[b + 1] + (b + 1) <= F) ++b;
    return b;
}
// Largest tube b' >= b whose first ghost-extended cell (off[b'] + 6 b') is <= e.
TENO_HD int batch_tube_of_ext(const int64_t* off, int nb, int b, int64_t e) {
    while (b + 1 < nb && off[b + 1] + 6 * (int64_t)(b + 1) <= e) ++b;
    return b;
}

struct BatchChunk {
    int64_t F0;     // first face
    int64_t Flast;  // last face (clipped to the stream)
    int64_t e_lo;   // first staged cell (the stencil start of face F0)
    int t0;         // tube of F0
    int b_last;     // tube of Flast
    int count;      // staged cells
};

// Geometry of chunk k, whose first face lies in tube t0 (host table).
TENO_HD BatchChunk batch_chunk(const int64_t* off, int nb, int64_t ftot, int64_t k, int t0) {
    BatchChunk C;
    C.F0 = k * kBatchCells;
    C.t0 = t0;
    C.e_lo = C.F0 + 5 * (int64_t)t0;
    C.Flast = C.F0 + 63;
    if (C.Flast > ftot - 1) C.Flast = ftot - 1;
    C.b_last = batch_tube_of_face(off, nb, t0, C.Flast);
    C.count = (int)(C.Flast + 5 * (int64_t)C.b_last + 6 - C.e_lo);
    return C;
}

// Staged cell idx of chunk C: its tube, the tube-local cell it copies and
// whether the copy negates the momentum (reflecting ghost).
TENO_HD int batch_staged_src(const int64_t* off, int nb, int bc, const BatchChunk& C, int idx,
                             int* tube, bool* flip) {
    const int64_t e = C.e_lo + idx;
    const int bb = batch_tube_of_ext(off, nb, C.t0, e);
    const int n = (int)(off[bb + 1] - off[bb]);
    const int j = (int)(e - (off[bb] + 6 * (int64_t)bb)) - 3;
    *tube = bb;
    return ghost_src(bc, n, j, flip);
}

// Face F of chunk C: its tube, its index phi in the tube and the staged
// offset o of its first stencil cell (cells o .. o + 5).
TENO_HD void batch_face(const int64_t* off, int nb, const BatchChunk& C, int64_t F, int* tube,
                        int64_t* phi, int* o) {
    const int b = batch_tube_of_face(off, nb, C.t0, F);
    *tube = b;
    *phi = F - (off[b] + b);
    *o = (int)(F + 5 * (int64_t)b - C.e_lo);
}

// Tube of the first face of every chunk (the host table the kernel reads).
inline void batch_chunk_tubes(const int64_t* off, int64_t nb, int64_t nchunks, int32_t* out) {
    int64_t b = 0;
    for (int64_t k = 0; k < nchunks; ++k) {
        const int64_t F0 = k * kBatchCells;
        while (b + 1 < nb && off[b + 1] + (b + 1) <= F0) ++b;
        out[k] = (int32_t)b;
    }
}

// LDS doubles of one wave of the batched kernel: the staged rows (NV = 9 for
// 1D) or, reused after the face computation, 64 face fluxes per component.
TENO_HD int batch_wave_lds(int cap) { return (cap * 9 > 64 * 3) ? cap * 9 : 64 * 3; }

// ---------------------------------------------------------------------------
// Adjoint chunks.  The lines of one column (all lines of the grid for the x
// axis; the lines of one x column for y and z) are concatenated into a face
// stream of `ftot` faces (n + 1 per line); chunk k holds faces 64 k ..
// 64 k + 63, and stages the ghost-extended cells of its lines (n + 6 per
// line) that its faces' stencils touch.
// ---------------------------------------------------------------------------
constexpr int kAdjChunk = 64;

struct AdjGeom {
    int64_t ncell, line_step, stride, col_step, ftot, ncols, kchunks;
    int32_t n, bc, cap, nb;  // nb: lines of a DIR-2 column (ny)
    // multiply-and-shift division by n + 1, n + 6, ncols, n and nb; div32:
    // every cell, face and staged index is below 2^31
    uint32_t m1, s1, m6, s6, mc, sc, mn, sn, mb, sb;
    int32_t div32;
};

// Geometry of axis d of an nx x ny x nz grid (host side).  x: one column
// holding every line; y: nx columns of nz lines; z: nx columns of ny lines.
inline AdjGeom adj_geom(const int32_t n[3], const int32_t bc[3], int d) {
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    AdjGeom G;
    int64_t lines;
    if (d == 0) {
        G.ncols = 1; G.col_step = 0; G.line_step = nx; G.stride = 1; lines = ny * nz;
    } else if (d == 1) {
        G.ncols = nx; G.col_step = 1; G.line_step = nx * ny; G.stride = nx; lines = nz;
    } else {
        G.ncols = nx; G.col_step = 1; G.line_step = nx; G.stride = nx * ny; lines = ny;
    }
    G.ncell = nx * ny * nz;
    G.n = n[d];
    G.bc = bc[d];
    G.ftot = lines * (G.n + 1);
    G.kchunks = (G.ftot + kAdjChunk - 1) / kAdjChunk;
    G.cap = ext_cap_for(G.n);
    G.nb = (int32_t)((d == 2) ? G.stride / G.ncols : 1);
    const DivMagic d1 = div_magic((uint32_t)(G.n + 1)), d6 = div_magic((uint32_t)(G.n + 6)),
                   dc = div_magic((uint32_t)G.ncols), dn = div_magic((uint32_t)G.n),
                   db = div_magic((uint32_t)G.nb);
    G.m1 = d1.m; G.s1 = d1.sh; G.m6 = d6.m; G.s6 = d6.sh; G.mc = dc.m; G.sc = dc.sh;
    G.mn = dn.m; G.sn = dn.sh; G.mb = db.m; G.sb = db.sh;
    // the largest index: a cell, or a staged index ftot + 5 lines (+ a chunk's tail)
    G.div32 = (G.ncell < (int64_t(1) << 31) && G.ftot + 6 * lines + 128 < (int64_t(1) << 31)) ? 1 : 0;
    return G;
}

struct AdjChunk {
    int64_t k, col, colbase;  // chunk within its column, column, first cell of the column
    int64_t F0, bl0, e_lo, be0;
    int phi0, je0, count;
};

// Chunk of logical block index `chunk` (columns fastest for DIR != 0).
TENO_HD AdjChunk adj_chunk(const AdjGeom& G, int dir, int64_t chunk) {
    AdjChunk C;
    C.col = 0;
    C.k = chunk;
    if (dir != 0) {
        C.k = div_by((int)chunk, G.mc, G.sc);  // chunk < kchunks ncols < 2^31
        C.col = chunk - C.k * G.ncols;
    }
    C.colbase = C.col * G.col_step;
    const int64_t np1 = G.n + 1, np6 = G.n + 6;
    C.F0 = C.k * kAdjChunk;
    C.bl0 = G.div32 ? (int64_t)div_by((int)C.F0, G.m1, G.s1) : C.F0 / np1;
    C.phi0 = (int)(C.F0 - C.bl0 * np1);
    C.e_lo = C.F0 + 5 * C.bl0;
    int64_t Flast = C.F0 + kAdjChunk - 1;
    if (Flast > G.ftot - 1) Flast = G.ftot - 1;
    C.count = (int)(Flast + 5 * (G.div32 ? (int64_t)div_by((int)Flast, G.m1, G.s1) : Flast / np1) +
                    6 - C.e_lo);
    C.be0 = G.div32 ? (int64_t)div_by((int)C.e_lo, G.m6, G.s6) : C.e_lo / np6;
    C.je0 = (int)(C.e_lo - C.be0 * np6);
    return C;
}

// Face of lane `lane` (F = F0 + lane < ftot): its line, its index phi in the
// line and the staged offset o of its first stencil cell.
TENO_HD void adj_lane_face(const AdjGeom& G, const AdjChunk& C, int lane, int64_t* bl, int* phi,
                           int* o) {
    const int np1 = G.n + 1;
    const int tq = C.phi0 + lane;
    const int wraps = div_by(tq, G.m1, G.s1);
    *bl = C.bl0 + wraps;
    *phi = tq - wraps * np1;
    *o = (int)(C.F0 + lane + 5 * *bl - C.e_lo);
}

// Flat cell that staged cell idx of chunk C copies, and whether the copy
// negates the normal momentum.
TENO_HD int64_t adj_staged_cell(const AdjGeom& G, const AdjChunk& C, int idx, bool* flip) {
    const int np6 = G.n + 6;
    const int jq = C.je0 + idx;
    const int bw = div_by(jq, G.m6, G.s6);
    const int j = jq - bw * np6 - 3;
    const int src = ghost_src(G.bc, G.n, j, flip);
    return C.colbase + (C.be0 + bw) * G.line_step + (int64_t)src * G.stride;
}

// Chunk partials P[k][c][idx][col] (NC components): index of one entry.
TENO_HD int64_t adj_p_index(const AdjGeom& G, int nc, int64_t k, int c, int idx, int64_t col) {
    return ((k * nc + c) * G.cap + idx) * G.ncols + col;
}

// Doubles of the partial buffer of one axis.
TENO_HD int64_t adj_p_elems(const AdjGeom& G, int nc) {
    return G.kchunks * nc * (int64_t)G.cap * G.ncols;
}

// (column, line, position along the axis) of flat cell `cell`.
TENO_HD void adj_cell_place(const AdjGeom& G, int dir, int64_t cell, int64_t* col, int64_t* b,
                            int* i) {
    if (G.div32) {
        if (dir == 0) {
            *col = 0;
            *b = div_by((int)cell, G.mn, G.sn);
            *i = (int)(cell - *b * G.n);
        } else {
            const int64_t rest = div_by((int)cell, G.mc, G.sc);  // (z, y) for DIR 1: y fastest
            *col = cell - rest * G.ncols;
            const int64_t hi = div_by((int)rest, dir == 1 ? G.mn : G.mb, dir == 1 ? G.sn : G.sb);
            const int64_t lo = rest - hi * (dir == 1 ? G.n : G.nb);
            if (dir == 1) {
                *i = (int)lo;
                *b = hi;
            } else {  // DIR 2: rest = z ny + y, lines ordered by y
                *b = lo;
                *i = (int)hi;
            }
        }
    } else if (dir == 0) {
        *col = 0;
        *b = cell / G.n;
        *i = (int)(cell - *b * G.n);
    } else {
        *col = cell % G.ncols;
        const int64_t rest = cell / G.ncols;
        if (dir == 1) {
            *i = (int)(rest % G.n);
            *b = rest / G.n;
        } else {
            const int64_t ny = G.stride / G.ncols;
            *b = rest % ny;
            *i = (int)(rest / ny);
        }
    }
}

// Positions on its line of the images of cell i: the cell itself and the
// ghost cells it supplies.  Returns their number (at most 4 for n >= 3).
TENO_HD int adj_images(int bc, int n, int i, int img[7]) {
    int m = 0;
    img[m++] = i;
    if (bc == 0) {
        if (i >= n - 3) img[m++] = i - n;
        if (i <= 2) img[m++] = i + n;
    } else if (bc == 1) {
        if (i == 0) { img[m++] = -1; img[m++] = -2; img[m++] = -3; }
        if (i == n - 1) { img[m++] = n; img[m++] = n + 1; img[m++] = n + 2; }
    } else {
        if (i <= 2) img[m++] = -1 - i;
        if (i >= n - 3) img[m++] = 2 * n - 1 - i;
    }
    return m;
}

// Chunks whose faces have the staged cell at position e (ext numbering,
// e = image + 3) of line b in their stencils: faces e-5 .. e of the line.
TENO_HD void adj_chunks_of(const AdjGeom& G, int64_t b, int e, int64_t* ka, int64_t* kz) {
    const int64_t np1 = G.n + 1;
    const int64_t Fa = b * np1 + (e - 5 > 0 ? e - 5 : 0);
    const int64_t Fz = b * np1 + (e < G.n ? e : G.n);
    *ka = Fa / kAdjChunk;
    *kz = Fz / kAdjChunk;
}

// Staged index of the cell at position e of line b in chunk kk.
TENO_HD int64_t adj_slot(const AdjGeom& G, int64_t b, int e, int64_t kk) {
    const int64_t np1 = G.n + 1;
    const int64_t E = b * (G.n + 6) + e;
    const int64_t F0 = kk * kAdjChunk;
    return E - (F0 + 5 * (G.div32 ? (int64_t)div_by((int)F0, G.m1, G.s1) : F0 / np1));
}

}  // namespace teno
