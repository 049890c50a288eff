"""Batched ragged-1D form (teno_batch_*) against the oracle and the plain
solver: every tube must evolve exactly as the same tube run alone."""
import numpy as np
import pytest

from paper_2003_09145_amd import workloads as W

# A GPU fault was reported while test_batch_matches_oracle_per_tube ran, in a
# build whose batch kernel performs the same operations as the one that had
# passed it (a shared-header refactor changed only its register allocation).
# No cause has been found by reading the kernel or by checking its indices on
# the CPU, so the batched kernels stay off the GPU until one is shown.
BATCH_HELD = ("held off the GPU: an unexplained GPU fault was reported during "
              "test_batch_matches_oracle_per_tube; no cause found yet")
pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason=BATCH_HELD)]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def B():
    from paper_2003_09145_amd import binding
    binding.lib()
    return binding


def small_batch(seed=7, count=37):
    """Tubes of 3 .. 200 cells (several tubes share one 64-face chunk)."""
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([[3, 4, 5, 6, 7, 64, 63, 65], rng.integers(3, 200, count - 8)])
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lengths)
    U = np.empty((3, off[-1]))
    for k, N in enumerate(lengths):
        x = (np.arange(N) + 0.5) / N
        rl, rr = rng.uniform(0.1, 1.0, 2)
        ul, ur = rng.uniform(-1.0, 1.0, 2)
        pl, pr = rng.uniform(0.1, 1.0, 2)
        left = x <= 0.5
        U[:, off[k]:off[k + 1]] = W.conserved(np.where(left, rl, rr), [np.where(left, ul, ur)],
                                              np.where(left, pl, pr), 1.4)
    return W.Batch(lengths=lengths.astype(np.int64), offsets=off, dx=1.0 / lengths, U=U)


def _tube_oracle(orc, batch, b, steps, cfl=0.5, t_end=np.inf):
    prob = batch.tube_problem(b)
    U = batch.tube(b).copy()
    t = 0.0
    for _ in range(steps):
        if not t < t_end:
            break
        U, t, dt, a9, st = orc.step(prob, U, cfl, t, t_end)
    return U[:, 0, 0, :], t


def _plan_run(torch, B, batch, steps, **kw):
    P = B.BatchPlan(batch.lengths, batch.dx, **kw)
    Ud = torch.from_numpy(batch.U.copy()).cuda()
    P.init(Ud)
    for _ in range(steps):
        P.step(Ud)
    torch.cuda.synchronize()
    return P, Ud


def test_batch_matches_oracle_per_tube(torch, B, orc):
    batch = small_batch()
    steps = 9
    P, Ud = _plan_run(torch, B, batch, steps)
    Ug = Ud.cpu().numpy()
    t, dt, st, ns = P.read()
    assert np.all(st == 0) and np.all(ns == steps)
    for b in range(batch.nbatch):
        Uc, tc = _tube_oracle(orc, batch, b, steps)
        got = Ug[:, batch.offsets[b]:batch.offsets[b + 1]]
        assert np.array_equal(got, Uc), (b, batch.lengths[b], np.abs(got - Uc).max())
        assert t[b] == tc
    print(f"[batch] {batch.nbatch} tubes x {steps} steps bitwise equal to the oracle", flush=True)


def test_batch_matches_plain_solver(torch, B):
    batch = small_batch(seed=11, count=20)
    steps = 6
    _, Ud = _plan_run(torch, B, batch, steps)
    Ug = Ud.cpu().numpy()
    for b in range(batch.nbatch):
        S = B.Solver(batch.tube_problem(b))
        S.init(0.0, float("inf"), 0.5)
        u = torch.from_numpy(batch.tube(b).copy()).cuda()
        for _ in range(steps):
            S.step(u)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy()[:, 0, 0, :], Ug[:, batch.offsets[b]:batch.offsets[b + 1]])


def test_batch_graph_and_configs_identical(torch, B, tmp_path):
    batch = small_batch(seed=3, count=30)
    _, ref = _plan_run(torch, B, batch, 23)
    P = B.BatchPlan(batch.lengths, batch.dx)
    for waves, bpc in [(4, 0), (1, 3), (2, 8), (4, 1)]:
        P.set_config(waves, bpc)
        Ud = torch.from_numpy(batch.U.copy()).cuda()
        P.init(Ud)
        P.run(Ud, 23)  # two graph replays of 10 steps + 3 direct steps
        torch.cuda.synchronize()
        assert torch.equal(Ud, ref), (waves, bpc)
    cache = tmp_path / "tune.jsonl"
    P2 = B.BatchPlan(batch.lengths, batch.dx, tune_cache=cache)
    Ud = torch.from_numpy(batch.U.copy()).cuda()
    ms = P2.autotune(Ud, steps=2)
    assert ms > 0 and cache.exists()
    cfg = P2.config()
    P3 = B.BatchPlan(batch.lengths, batch.dx, tune_cache=cache)
    assert P3.config() == cfg
    P3.init(Ud)
    P3.run(Ud, 23)
    torch.cuda.synchronize()
    assert torch.equal(Ud, ref)


def test_batch_t_end_clipping(torch, B, orc):
    batch = small_batch(seed=5, count=12)
    t_end = 0.004
    P, Ud = _plan_run(torch, B, batch, 40, t_end=t_end)
    t, dt, st, ns = P.read()
    assert np.all(t == t_end)
    Ug = Ud.cpu().numpy()
    for b in range(batch.nbatch):
        Uc, tc = _tube_oracle(orc, batch, b, 40, t_end=t_end)
        assert tc == t_end
        assert np.array_equal(Ug[:, batch.offsets[b]:batch.offsets[b + 1]], Uc)


def test_batch_nonphysical_tube_is_frozen(torch, B, orc):
    batch = small_batch(seed=9, count=10)
    bad = 4
    o0 = batch.offsets[bad]
    batch.U[2, o0 + 1] = 0.0  # E = 0 < kinetic energy: negative pressure (forced on the host)
    P, Ud = _plan_run(torch, B, batch, 5)
    t, dt, st, ns = P.read()
    assert st[bad] == 3 and ns[bad] == 0 and t[bad] == 0.0
    Ug = Ud.cpu().numpy()
    assert np.array_equal(Ug[:, o0:batch.offsets[bad + 1]], batch.U[:, o0:batch.offsets[bad + 1]])
    for b in range(batch.nbatch):
        if b != bad:
            assert st[b] == 0 and ns[b] == 5
            Uc, _ = _tube_oracle(orc, batch, b, 5)
            assert np.array_equal(Ug[:, batch.offsets[b]:batch.offsets[b + 1]], Uc)


def test_batch_full_config_sampled(torch, B, orc):
    # the 4096-tube workload (N log-uniform in [128, 4096]) a few steps, with
    # 12 seeded tubes checked against the oracle
    batch = W.batched_tubes()
    steps = 4
    P, Ud = _plan_run(torch, B, batch, steps)
    t, dt, st, ns = P.read()
    assert np.all(st == 0) and np.all(ns == steps)
    Ug = Ud.cpu().numpy()
    rng = np.random.default_rng(12)
    for b in rng.choice(batch.nbatch, 12, replace=False):
        Uc, tc = _tube_oracle(orc, batch, b, steps)
        assert np.array_equal(Ug[:, batch.offsets[b]:batch.offsets[b + 1]], Uc), b
        assert t[b] == tc


def test_batch_teno5a_matches_oracle(torch, B, orc):
    # the TENO5-A cutoff (eq 2.16-2.18) through the batched kernel
    batch = small_batch(seed=13, count=16)
    steps = 5
    P = B.BatchPlan(batch.lengths, batch.dx, prob={"scheme": "teno5a"})
    Ud = torch.from_numpy(batch.U.copy()).cuda()
    P.init(Ud)
    for _ in range(steps):
        P.step(Ud)
    torch.cuda.synchronize()
    Ug = Ud.cpu().numpy()
    for b in range(batch.nbatch):
        prob = batch.tube_problem(b, scheme="teno5a")
        U = batch.tube(b).copy()
        t = 0.0
        for _ in range(steps):
            U, t, dt, a9, st = orc.step(prob, U, 0.5, t, np.inf)
        assert np.array_equal(Ug[:, batch.offsets[b]:batch.offsets[b + 1]], U[:, 0, 0, :]), b
