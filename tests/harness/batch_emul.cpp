// The batched-tube kernels of teno_batch.hip run on the host through the HIP
// emulation in hip_emu/ (test infrastructure): the very kernel and host code
// of the library, with device buffers on the heap, so that AddressSanitizer
// checks every global and LDS access, and the emulated wave operations check
// that every live lane of a wave reaches them.
//
// BATCH_SRC names a copy of teno_batch.hip whose dynamic-LDS declaration was
// rewritten to the emulation's per-block buffer (the only change).
//
// usage: batch_emul <dir> <steps> <waves> <blocks_per_cu> <scheme> <t_end> <cus> <occ>
//   <dir>/lengths.bin (int64 per tube), dx.bin (double per tube), U.bin
//   (3 x total doubles) in; U_out.bin, t.bin, status.bin, nsteps.bin out.
//   waves 0 keeps the plan's default configuration.
#include BATCH_SRC

#include <string>
#include <vector>

static std::vector<char> slurp(const std::string& path) {
    std::vector<char> v;
    FILE* f = fopen(path.c_str(), "rb");
    if (!f) {
        fprintf(stderr, "cannot read %s\n", path.c_str());
        exit(2);
    }
    char buf[1 << 16];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) v.insert(v.end(), buf, buf + n);
    fclose(f);
    return v;
}

static void spill(const std::string& path, const void* p, size_t n) {
    FILE* f = fopen(path.c_str(), "wb");
    if (!f || fwrite(p, 1, n, f) != n) {
        fprintf(stderr, "cannot write %s\n", path.c_str());
        exit(2);
    }
    fclose(f);
}

int main(int argc, char** argv) {
    if (argc < 9) return 2;
    const std::string dir = argv[1];
    const int steps = atoi(argv[2]), waves = atoi(argv[3]), bpc = atoi(argv[4]);
    const int scheme = atoi(argv[5]);
    const double t_end = atof(argv[6]);
    emu::g_cus = atoi(argv[7]);
    emu::g_occ = atoi(argv[8]);

    const std::vector<char> lb = slurp(dir + "/lengths.bin"), db = slurp(dir + "/dx.bin"),
                            ub = slurp(dir + "/U.bin");
    const int64_t nb = (int64_t)(lb.size() / sizeof(int64_t));
    teno_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = 1;
    g.n[0] = 3;
    g.n[1] = g.n[2] = 1;
    g.dx[0] = g.dx[1] = g.dx[2] = 1.0;
    g.bc[0] = TENO_BC_TRANSMISSIVE;
    g.scheme = scheme;
    g.gamma = 1.4;
    g.ct_fixed = 1e-7;
    g.H = 10.0;
    g.Bl = 4;
    g.Bu = 10;
    g.eps = 1e-6;
    g.a1 = 10.5;
    g.a2 = 3.5;
    g.cr = 0.25;
    g.xi = 1e-3;
    teno_batch_plan* P = nullptr;
    int rc = teno_batch_plan_create(&g, nb, (const int64_t*)lb.data(), (const double*)db.data(),
                                    0.5, t_end, nullptr, &P);
    if (rc != TENO_OK) {
        fprintf(stderr, "plan_create %d\n", rc);
        return 3;
    }
    if (waves > 0 && teno_batch_set_config(P, waves, bpc) != TENO_OK) return 4;
    int32_t w = 0, b = 0;
    teno_batch_get_config(P, &w, &b);
    const int64_t total = teno_batch_total_cells(P);
    if ((int64_t)ub.size() != 3 * total * (int64_t)sizeof(double)) return 5;
    double* U = nullptr;
    if (hipMalloc(&U, ub.size()) != hipSuccess) return 6;
    memcpy(U, ub.data(), ub.size());
    if (teno_batch_init(P, U, nullptr) != TENO_OK) return 7;
    for (int s = 0; s < steps; ++s)
        if (teno_batch_step(P, U, nullptr) != TENO_OK) return 8;
    std::vector<double> t((size_t)nb), dt((size_t)nb);
    std::vector<int32_t> st((size_t)nb);
    std::vector<int64_t> ns((size_t)nb);
    if (teno_batch_read(P, t.data(), dt.data(), st.data(), ns.data()) != TENO_OK) return 9;
    spill(dir + "/U_out.bin", U, ub.size());
    spill(dir + "/t.bin", t.data(), t.size() * sizeof(double));
    spill(dir + "/status.bin", st.data(), st.size() * sizeof(int32_t));
    spill(dir + "/nsteps.bin", ns.data(), ns.size() * sizeof(int64_t));
    printf("emulated %lld tubes, %lld cells, %d steps, %d waves per block, %d blocks per CU of %d\n",
           (long long)nb, (long long)total, steps, w, b, emu::g_cus);
    hipFree(U);
    teno_batch_plan_destroy(P);
    return 0;
}
