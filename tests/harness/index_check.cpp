// CPU check of the index maps of the batched-tube kernel and of the
// adjoint's chunked passes (teno_index.hpp, the functions the kernels call).
// For every chunk and lane it runs the kernels' own index computations and
// checks every global index against its buffer, every LDS index against the
// launch's LDS size, and the coverage the kernels rely on: each tube cell is
// updated by exactly one lane per stage, each tube's time step is written by
// exactly one lane, and every partial the adjoint gather reads was written by
// the chunk pass.
//
// usage: index_check batch <bc> <lengths file (int64 binary)>
//        index_check adj <nx> <ny> <nz> <ndim> <bc_x> <bc_y> <bc_z>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "teno_index.hpp"

using namespace teno;

static long long g_fail = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            if (g_fail < 20) {                             \
                fprintf(stderr, "FAIL %s: ", #cond);       \
                fprintf(stderr, __VA_ARGS__);              \
                fprintf(stderr, "\n");                     \
            }                                              \
            ++g_fail;                                      \
        }                                                  \
    } while (0)

static int check_batch(const std::vector<int64_t>& len, int bc) {
    const int64_t nb = (int64_t)len.size();
    std::vector<int64_t> off(nb + 1, 0);
    int64_t mn = INT64_MAX;
    for (int64_t b = 0; b < nb; ++b) {
        off[b + 1] = off[b] + len[b];
        if (len[b] < mn) mn = len[b];
    }
    const int64_t total = off[nb], ftot = total + nb;
    const int64_t nchunks = (ftot - 1 + kBatchCells - 1) / kBatchCells;
    const int cap = ext_cap_for((int)(mn < 4096 ? mn : 4096));
    const int per_wave = batch_wave_lds(cap);
    std::vector<int32_t> ct(nchunks);
    batch_chunk_tubes(off.data(), nb, nchunks, ct.data());
    std::vector<int> upd(total, 0), dtw(nb, 0);
    int maxcount = 0;
    for (int64_t k = 0; k < nchunks; ++k) {
        CHECK(ct[k] >= 0 && ct[k] < nb, "chunk %lld tube %d", (long long)k, ct[k]);
        const BatchChunk C = batch_chunk(off.data(), (int)nb, ftot, k, ct[k]);
        CHECK(C.count >= 6 && C.count <= cap, "chunk %lld count %d cap %d", (long long)k, C.count, cap);
        if (C.count > maxcount) maxcount = C.count;
        // staged rows: 9 rows of cap doubles in the wave's LDS region
        CHECK(9 * cap <= per_wave, "rows");
        for (int idx = 0; idx < C.count; ++idx) {
            int bb;
            bool flip;
            const int src = batch_staged_src(off.data(), (int)nb, bc, C, idx, &bb, &flip);
            CHECK(bb >= C.t0 && bb <= C.b_last, "chunk %lld idx %d tube %d", (long long)k, idx, bb);
            CHECK(src >= 0 && src < len[bb], "chunk %lld idx %d src %d n %lld", (long long)k, idx, src,
                  (long long)len[bb]);
            CHECK(off[bb] + src < total, "global");
        }
        for (int lane = 0; lane < 64; ++lane) {
            const int64_t F = C.F0 + lane;
            if (F >= ftot) continue;
            int b, o;
            int64_t phi;
            batch_face(off.data(), (int)nb, C, F, &b, &phi, &o);
            CHECK(b >= C.t0 && b <= C.b_last && b < nb, "face tube");
            CHECK(phi >= 0 && phi <= len[b], "phi %lld", (long long)phi);
            CHECK(o >= 0 && o + 5 < C.count, "chunk %lld lane %d o %d count %d", (long long)k, lane, o,
                  C.count);
            CHECK(2 * 64 + lane < per_wave, "face flux slots");
            if (lane > 0 && phi > 0) {
                // the left flux is lane - 1's face: the same tube, one face back
                int b1, o1;
                int64_t phi1;
                batch_face(off.data(), (int)nb, C, F - 1, &b1, &phi1, &o1);
                CHECK(b1 == b && phi1 == phi - 1, "left face");
                const int64_t cell = off[b] + phi - 1;
                CHECK(cell >= off[b] && cell < off[b + 1], "cell");
                upd[cell] += 1;
                if (phi == 1) dtw[b] += 1;
            }
        }
    }
    for (int64_t i = 0; i < total; ++i) CHECK(upd[i] == 1, "cell %lld updated %d times", (long long)i, upd[i]);
    for (int64_t b = 0; b < nb; ++b) CHECK(dtw[b] == 1, "tube %lld dt written %d times", (long long)b, dtw[b]);
    for (int W = 1; W <= 4; W *= 2)
        CHECK((24 + (int64_t)W * per_wave) * 8 <= 160 * 1024, "lds of %d waves", W);
    printf("batch: %lld tubes, %lld cells, %lld chunks, cap %d, max staged %d, failures %lld\n",
           (long long)nb, (long long)total, (long long)nchunks, cap, maxcount, g_fail);
    return g_fail ? 1 : 0;
}

static int check_adj(const int32_t n[3], const int32_t bc[3], int nd) {
    const int nc = nd + 2;
    for (int d = 0; d < nd; ++d) {
        const AdjGeom G = adj_geom(n, bc, d);
        const int64_t pel = adj_p_elems(G, nc);
        const int64_t lines = G.ftot / (G.n + 1);
        const int64_t nblk = G.kchunks * G.ncols;
        std::vector<char> written((size_t)(pel / nc), 0), seen((size_t)nblk, 0);
        int maxcount = 0;
        for (int64_t blk = 0; blk < nblk; ++blk) {
            const int64_t lb = xcd_logical_block(blk, nblk);
            CHECK(lb >= 0 && lb < nblk && !seen[lb], "block order");
            seen[lb] = 1;
            const AdjChunk C = adj_chunk(G, d, lb);
            CHECK(C.k >= 0 && C.k < G.kchunks && C.col >= 0 && C.col < G.ncols, "chunk place");
            CHECK(C.count >= 6 && C.count <= G.cap, "axis %d chunk %lld count %d cap %d", d,
                  (long long)C.k, C.count, G.cap);
            if (C.count > maxcount) maxcount = C.count;
            for (int idx = 0; idx < C.count; ++idx) {
                bool flip;
                const int64_t cell = adj_staged_cell(G, C, idx, &flip);
                CHECK(cell >= 0 && cell < G.ncell, "staged cell");
                for (int c = 0; c < nc; ++c) {
                    const int64_t p = adj_p_index(G, nc, C.k, c, idx, C.col);
                    CHECK(p >= 0 && p < pel, "partial index");
                }
                written[(size_t)((C.k * G.cap + idx) * G.ncols + C.col)] = 1;
            }
            for (int lane = 0; lane < 64; ++lane) {
                if (C.F0 + lane >= G.ftot) continue;
                int64_t bl;
                int phi, o;
                adj_lane_face(G, C, lane, &bl, &phi, &o);
                CHECK(bl >= 0 && bl < lines && phi >= 0 && phi <= G.n, "lane face");
                CHECK(o >= 0 && o + 5 < C.count, "axis %d chunk %lld lane %d o %d", d, (long long)C.k,
                      lane, o);
                const int64_t lbase = C.colbase + bl * G.line_step;
                if (phi <= G.n - 1) CHECK(lbase + (int64_t)phi * G.stride < G.ncell, "lam right");
                if (phi >= 1) CHECK(lbase + (int64_t)(phi - 1) * G.stride >= 0, "lam left");
            }
        }
        for (int64_t cell = 0; cell < G.ncell; ++cell) {
            int64_t col, b;
            int i;
            adj_cell_place(G, d, cell, &col, &b, &i);
            CHECK(col * G.col_step + b * G.line_step + (int64_t)i * G.stride == cell, "cell place");
            int img[7];
            const int m = adj_images(G.bc, G.n, i, img);
            CHECK(m >= 1 && m <= 4, "images");
            for (int t = 0; t < m; ++t) {
                const int e = img[t] + 3;
                CHECK(e >= 0 && e < G.n + 6, "image position");
                int64_t ka, kz;
                adj_chunks_of(G, b, e, &ka, &kz);
                CHECK(ka <= kz && kz - ka <= 1 && kz < G.kchunks, "gather chunks");
                for (int64_t kk = ka; kk <= kz; ++kk) {
                    const int64_t slot = adj_slot(G, b, e, kk);
                    CHECK(slot >= 0 && slot < G.cap, "slot %lld", (long long)slot);
                    if (slot >= 0 && slot < G.cap)
                        CHECK(written[(size_t)((kk * G.cap + slot) * G.ncols + col)],
                              "axis %d cell %lld reads an unwritten partial", d, (long long)cell);
                }
            }
        }
        printf("adjoint axis %d of %dx%dx%d: %lld chunks, cap %d, max staged %d, partials %lld, "
               "failures %lld\n", d, n[0], n[1], n[2], (long long)nblk, G.cap, maxcount,
               (long long)pel, g_fail);
    }
    return g_fail ? 1 : 0;
}

int main(int argc, char** argv) {
    if (argc >= 4 && argv[1][0] == 'b') {
        FILE* f = fopen(argv[3], "rb");
        if (!f) return 2;
        std::vector<int64_t> len;
        int64_t v;
        while (fread(&v, sizeof(v), 1, f) == 1) len.push_back(v);
        fclose(f);
        return check_batch(len, atoi(argv[2]));
    }
    if (argc >= 9 && argv[1][0] == 'a') {
        const int32_t n[3] = {atoi(argv[2]), atoi(argv[3]), atoi(argv[4])};
        const int32_t bc[3] = {atoi(argv[6]), atoi(argv[7]), atoi(argv[8])};
        return check_adj(n, bc, atoi(argv[5]));
    }
    return 2;
}
