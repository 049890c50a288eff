"""Host-side logic checked on the CPU: the multiply-and-shift constants that
replace per-lane divisions by the line length (n + 1, n + 6) and the column
count in the sweep kernels, the exactness of the fused power-of-two products,
the map from a flipped decision to the cells the GPU parity tests leave out,
and the kernel names under which bench.py looks up the sweeps' counters."""
import os
import subprocess

import numpy as np
import pytest

from paper_2003_09145_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2003_09145_amd", "csrc")

HARNESS = r'''
#include <stdio.h>
#include "teno_divmagic.hpp"
int main() {
    unsigned long long seed = 7, checks = 0;
    for (unsigned d = 1; d <= 20000; ++d) {
        const teno::DivMagic q = teno::div_magic(d);
        for (unsigned x = 0; x < 4096; ++x) {
            if ((unsigned)(((unsigned long long)x * q.m) >> q.sh) != x / d) { printf("FAIL %u %u\n", d, x); return 1; }
        }
        for (int t = 0; t < 400; ++t) {
            seed = seed * 6364136223846793005ull + 1442695040888963407ull;
            const unsigned xs[3] = {(unsigned)(seed >> 33), 0x7fffffffu - (unsigned)t,
                                    (0x7fffffffu / d) * d - (unsigned)(t % 2)};
            for (unsigned x : xs)
                if ((unsigned)(((unsigned long long)x * q.m) >> q.sh) != x / d) { printf("FAIL %u %u\n", d, x); return 1; }
        }
        checks += 4096 + 1200;
    }
    for (unsigned long long d = 20001; d < 0x80000000ull; d = d * 5 / 4 + 3) {
        const teno::DivMagic q = teno::div_magic((unsigned)d);
        if (q.sh > 63) { printf("FAIL shift %llu\n", d); return 1; }
        for (int t = 0; t < 20000; ++t) {
            seed = seed * 6364136223846793005ull + 1442695040888963407ull;
            const unsigned x = (unsigned)(seed >> 33);
            if ((unsigned)(((unsigned long long)x * q.m) >> q.sh) != x / (unsigned)d) { printf("FAIL %llu %u\n", d, x); return 1; }
        }
    }
    printf("ok %llu\n", checks);
    return 0;
}
'''


def test_div_magic_matches_integer_division(tmp_path):
    src = tmp_path / "divmagic.cpp"
    exe = tmp_path / "divmagic"
    src.write_text(HARNESS)
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout


FUSE_HARNESS = r'''
#include <initializer_list>
#include <math.h>
#include <stdio.h>
#include <string.h>
// The kernels fuse a - 2 b and a - 4 b into fma(-2, b, a) and fma(-4, b, a)
// where the oracle forms the product first; with |b| below 2^1021 the
// product is exact, so both round once to the same double.
static double bits(unsigned long long u) { double d; memcpy(&d, &u, 8); return d; }
int main() {
    unsigned long long s = 12345, n = 0;
    for (int t = 0; t < 4000000; ++t) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        unsigned long long ua = s;
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        unsigned long long ub = s;
        // exponents spread over the whole range below 2^1021, subnormals included
        const double a = bits(ua & ~(0x7ffull << 52) | ((ua >> 52) % 2045ull) << 52);
        const double b = bits(ub & ~(0x7ffull << 52) | ((ub >> 52) % 2044ull) << 52);
        const double near_b = (t & 1) ? b : a * 0.5 * (1.0 + ldexp((double)(t % 64), -52));
        for (double k : {2.0, 4.0}) {
            const double x = near_b;
            const double p = a - k * x, f = fma(-k, x, a);
            if (memcmp(&p, &f, 8) != 0 && !(isnan(p) && isnan(f))) {
                printf("FAIL %a %a %g\n", a, x, k);
                return 1;
            }
            ++n;
        }
    }
    printf("ok %llu\n", n);
    return 0;
}
'''


def test_power_of_two_products_fuse_exactly(tmp_path):
    src = tmp_path / "fuse.cpp"
    exe = tmp_path / "fuse"
    src.write_text(FUSE_HARNESS)
    subprocess.run(["g++", "-O2", "-std=c++17", "-mfma", "-ffp-contract=off", "-o", str(exe),
                    str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout


def test_bench_sweep_names_resolve_in_counter_summary():
    """The kernel name bench.py derives for each axis's 3D sweep picks out
    exactly one kernel of the committed counter summary (else its traffic
    figure would silently read as missing)."""
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    names = [line[len("kernel "):].split(":", 1)[0].strip()
             for line in open(bench.TRAFFIC_FILE) if line.startswith("kernel ")]
    assert len(names) == 3
    for d in range(3):
        kname = f"k_sweep<3,{d},{bench.SWEEP_WAVES[d]},false>"
        assert len(bench.match_kernel(names, kname)) == 1, (kname, names)


def test_cells_next_to_flips_mapping(orc):
    # The GPU tests leave out the cells next to a face whose decision differs
    # between two dumps.  Plant one differing byte at a known face of each
    # axis of an oracle dump and check that exactly the face's two cells (one
    # at a boundary face) are marked, located independently from the face's
    # line and position.
    from test_gpu_parity import cells_next_to_flips
    prob = W.uniform_problem(3, [7, 5, 4], [0.0] * 3, [1.0] * 3, "periodic")
    U = W.random_field(prob, seed=2)
    _, dc = orc.rhs(prob, U, dump=True)
    nx, ny, nz = prob.n
    nc = prob.nc
    off = 0
    for d, (line, phi) in enumerate([(13, 3), (9, 0), (30, 4)]):
        n = prob.n[d]
        dg = dc.copy()
        dg[off + (line * (n + 1) + phi) * 2 * nc + 2 * nc - 1] ^= 1
        bad = cells_next_to_flips(prob, dg, dc)
        # the sweep's line numbering: x lines by (z, y), y lines by (z, x),
        # z lines by (y, x)
        a, b = [(line % ny, line // ny), (line % nx, line // nx), (line % nx, line // nx)][d]
        want = np.zeros((nz, ny, nx), dtype=bool)
        for i in (phi - 1, phi):
            if 0 <= i < n:
                pos = {0: (b, a, i), 1: (b, i, a), 2: (i, b, a)}[d]
                want[pos] = True
        assert np.array_equal(bad, want), d
        off += (prob.ncell // n) * (n + 1) * 2 * nc


# --------------------------------------------------------------------------
# Index maps of the batched-tube kernel and the adjoint's chunked passes
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def index_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("idx") / "index_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "harness", "index_check.cpp")], check=True)
    return exe


def _small_batch_lengths(seed, count):
    # the tube lengths of the batched GPU tests (3 .. 200 cells, several tubes
    # sharing one 64-face chunk)
    rng = np.random.default_rng(seed)
    return np.concatenate([[3, 4, 5, 6, 7, 64, 63, 65], rng.integers(3, 200, count - 8)])


@pytest.mark.parametrize("name", ["small_7_37", "small_3_30", "small_9_10", "full_4096",
                                  "all_length_3", "lengths_3_to_5", "one_long_tube"])
def test_batch_index_maps(index_check, tmp_path, name):
    # Every chunk and lane of the batched stage kernel, through the same
    # index functions the kernel calls: staged sources inside their tubes,
    # stencils inside the staged window (<= the LDS rows), each cell updated
    # by exactly one lane and each tube's dt written by exactly one lane.
    lengths = {
        "small_7_37": lambda: _small_batch_lengths(7, 37),
        "small_3_30": lambda: _small_batch_lengths(3, 30),
        "small_9_10": lambda: _small_batch_lengths(9, 10),
        "full_4096": lambda: W.batched_tubes().lengths,
        "all_length_3": lambda: np.full(700, 3),
        "lengths_3_to_5": lambda: np.random.default_rng(1).integers(3, 6, 3000),
        "one_long_tube": lambda: np.array([5, 100000, 3, 4]),
    }[name]()
    f = tmp_path / "lengths.bin"
    np.asarray(lengths, dtype=np.int64).tofile(f)
    for bc in (1, 0, 2):
        r = subprocess.run([index_check, "batch", str(bc), str(f)], capture_output=True, text=True)
        print(r.stdout.strip())
        assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("shape,nd,bc", [
    ((256, 256, 256), 3, (0, 0, 0)), ((128, 128, 128), 3, (0, 1, 2)),
    ((20, 1, 1), 1, (0, 0, 0)), ((17, 1, 1), 1, (2, 0, 0)), ((2048, 1, 1), 1, (1, 0, 0)),
    ((8, 7, 1), 2, (2, 0, 0)), ((63, 66, 1), 2, (2, 0, 0)), ((130, 67, 1), 2, (1, 0, 0)),
    ((5, 5, 4), 3, (1, 0, 2)), ((70, 66, 9), 3, (0, 2, 1)), ((9, 5, 131), 3, (2, 1, 0)),
    ((3, 3, 3), 3, (2, 2, 2)), ((64, 65, 70), 3, (0, 2, 1))])
def test_adjoint_index_maps(index_check, shape, nd, bc):
    # Every chunk of the adjoint's pass A and every cell of its gather, through
    # the kernels' index functions: staged cells, partial-buffer writes within
    # the workspace's partial area, lane faces inside the staged window, and
    # every partial the gather reads written by its chunk.
    r = subprocess.run([index_check, "adj", *map(str, shape), str(nd), *map(str, bc)],
                       capture_output=True, text=True)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stderr
