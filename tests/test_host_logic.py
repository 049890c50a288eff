"""Host-side integer logic of the kernels, checked on the CPU: the
multiply-and-shift constants that replace per-lane divisions by the line
length (n + 1, n + 6) and the column count in the sweep kernels."""
import os
import subprocess

import pytest

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
