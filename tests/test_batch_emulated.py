"""The batched-tube kernels (teno_batch.hip) run on the CPU through the HIP
host emulation of tests/harness/hip_emu: the library's own kernel and host
source, built with AddressSanitizer and UBSan, device buffers and every
block's dynamic LDS as heap buffers of exactly their size, every barrier and
wave operation checked to be reached by all live lanes.  Each tube must come
out bit for bit as the oracle's run of that tube alone.

The emulated copy of the source differs from the library's in two places,
both asserted here: the dynamic-LDS declaration points at the emulation's
per-block buffer, and a wave barrier stands where the kernel relies on a
wave's lanes running in lockstep (the face fluxes overwrite the staged rows
that the same wave's stencils read just before).

This covers the kernel's indexing, synchronisation and arithmetic; it does
not cover the compiled device code, blocks running concurrently, or HIP
graphs (the emulation refuses graph capture)."""
import os
import subprocess

import numpy as np
import pytest

from paper_2003_09145_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2003_09145_amd", "csrc")

LDS_DECL = "extern __shared__ double smem[];"
FACE_BLOCK = """        if (valid) {
            double Fh[NC];
            face_flux<ND, DIR, A5>(ext, cap, o, gm1, A.sch, A.dk, omega, nullptr, Fh);
#pragma unroll
            for (int c = 0; c < NC; ++c) fhs[c * 64 + lane] = Fh[c];
        }"""
FACE_BLOCK_EMU = """        double Fh[NC];
        if (valid) face_flux<ND, DIR, A5>(ext, cap, o, gm1, A.sch, A.dk, omega, nullptr, Fh);
        emu::wave_sync();  // the wave's stencil reads precede its flux writes (lockstep)
        if (valid) {
            for (int c = 0; c < NC; ++c) fhs[c * 64 + lane] = Fh[c];
        }"""


@pytest.fixture(scope="module")
def emul(tmp_path_factory):
    top = tmp_path_factory.mktemp("batch_emu")
    # the copy sits two levels below an include/ holding teno.h, as the source
    # does, so that its relative include of the public header resolves
    (top / "include").mkdir()
    (top / "include" / "teno.h").write_bytes(open(os.path.join(ROOT, "include", "teno.h"), "rb").read())
    src_dir = top / "pkg" / "csrc"
    src_dir.mkdir(parents=True)
    src = open(os.path.join(CSRC, "teno_batch.hip")).read()
    assert src.count(LDS_DECL) == 1 and src.count(FACE_BLOCK) == 1, \
        "teno_batch.hip changed: update the emulated copy's two rewrites"
    src = src.replace(LDS_DECL, "double* smem = (double*)emu::dyn_smem();")
    src = src.replace(FACE_BLOCK, FACE_BLOCK_EMU)
    (src_dir / "teno_batch_emu.cpp").write_text(src)
    exe = str(top / "batch_emul")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-ffp-contract=off", "-Wno-attributes", "-pthread",
                    "-I", os.path.join(HERE, "harness", "hip_emu"), "-I", CSRC,
                    f'-DBATCH_SRC="{src_dir / "teno_batch_emu.cpp"}"', "-o", exe,
                    os.path.join(HERE, "harness", "batch_emul.cpp")], check=True)
    return exe, top


def _run(emul, batch, steps, waves=0, bpc=0, scheme=0, t_end=np.inf, cus=4, occ=2, tag="run"):
    exe, top = emul
    d = top / tag
    d.mkdir(exist_ok=True)
    batch.lengths.astype(np.int64).tofile(d / "lengths.bin")
    np.asarray(batch.dx, dtype=np.float64).tofile(d / "dx.bin")
    np.ascontiguousarray(batch.U).tofile(d / "U.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(d), str(steps), str(waves), str(bpc), str(scheme),
                        "inf" if np.isinf(t_end) else repr(float(t_end)), str(cus), str(occ)],
                       capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout.strip(), flush=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    U = np.fromfile(d / "U_out.bin").reshape(3, -1)
    t = np.fromfile(d / "t.bin")
    st = np.fromfile(d / "status.bin", dtype=np.int32)
    ns = np.fromfile(d / "nsteps.bin", dtype=np.int64)
    return U, t, st, ns


def small_batch(seed=7, count=37):
    """Tubes of 3 .. 200 cells (several tubes share one 64-face chunk); the
    tube set of the GPU batch tests."""
    from test_gpu_batch import small_batch as sb
    return sb(seed, count)


def _oracle_tube(orc, batch, b, steps, scheme=None, t_end=np.inf):
    prob = batch.tube_problem(b) if scheme is None else batch.tube_problem(b, scheme=scheme)
    U = batch.tube(b).copy()
    t = 0.0
    for _ in range(steps):
        if not t < t_end:
            break
        U, t, dt, a9, st = orc.step(prob, U, 0.5, t, t_end)
    return U[:, 0, 0, :], t


def _check_all(orc, batch, U, t, st, ns, steps, **kw):
    for b in range(batch.nbatch):
        Uc, tc = _oracle_tube(orc, batch, b, steps, **kw)
        got = U[:, batch.offsets[b]:batch.offsets[b + 1]]
        assert np.array_equal(got, Uc), (b, batch.lengths[b], np.abs(got - Uc).max())
        assert t[b] == tc and st[b] == 0, (b, t[b], tc, st[b])


def test_emulated_batch_matches_oracle(emul, orc):
    # the tube set and step count of the GPU parity test that reported a fault
    batch = small_batch(7, 37)
    U, t, st, ns = _run(emul, batch, 9)
    assert np.all(ns == 9)
    _check_all(orc, batch, U, t, st, ns, 9)


@pytest.mark.parametrize("waves,bpc", [(4, 0), (1, 3), (2, 8), (4, 1)])
def test_emulated_configs(emul, orc, waves, bpc):
    # one block per chunk group, and persistent grids that loop over groups
    batch = small_batch(3, 30)
    U, t, st, ns = _run(emul, batch, 12, waves, bpc, tag=f"cfg{waves}_{bpc}")
    assert np.all(ns == 12)
    _check_all(orc, batch, U, t, st, ns, 12)


def test_emulated_t_end_clipping(emul, orc):
    batch = small_batch(5, 12)
    t_end = 0.004
    U, t, st, ns = _run(emul, batch, 40, t_end=t_end, tag="tend")
    assert np.all(t == t_end)
    _check_all(orc, batch, U, t, st, ns, 40, t_end=t_end)


def test_emulated_nonphysical_tube_is_frozen(emul, orc):
    batch = small_batch(9, 10)
    bad = 4
    o0, o1 = batch.offsets[bad], batch.offsets[bad + 1]
    batch.U[2, o0 + 1] = 0.0  # E = 0 < kinetic energy: negative pressure
    U, t, st, ns = _run(emul, batch, 5, tag="bad")
    assert st[bad] == 3 and ns[bad] == 0 and t[bad] == 0.0
    assert np.array_equal(U[:, o0:o1], batch.U[:, o0:o1])
    for b in range(batch.nbatch):
        if b == bad:
            continue
        Uc, tc = _oracle_tube(orc, batch, b, 5)
        assert np.array_equal(U[:, batch.offsets[b]:batch.offsets[b + 1]], Uc), b
        assert st[b] == 0 and ns[b] == 5 and t[b] == tc


def test_emulated_teno5a(emul, orc):
    batch = small_batch(13, 16)
    U, t, st, ns = _run(emul, batch, 5, scheme=3, tag="a5")
    _check_all(orc, batch, U, t, st, ns, 5, scheme="teno5a")


def test_emulated_long_tubes(emul, orc):
    # the batched workload's length distribution (log-uniform 128 .. 4096),
    # 24 tubes: several chunks per tube and the tube boundaries inside chunks
    batch = W.batched_tubes(count=24, seed=5)
    U, t, st, ns = _run(emul, batch, 3, cus=3, occ=2, tag="long")
    assert np.all(ns == 3)
    _check_all(orc, batch, U, t, st, ns, 3)
