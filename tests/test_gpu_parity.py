"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Bar (per RHS evaluation): every cutoff decision identical (flips counted and
required to be zero) and, per component, max |RHS_gpu - RHS_oracle| /
max |RHS_oracle| <= 1e-12.  The library is built without FMA contraction and
evaluates the oracle's operation order, so the RHS is in fact expected to be
bit-identical; that is asserted separately.
"""
import ctypes

import numpy as np
import pytest

from paper_2003_09145_amd import workloads as W

pytestmark = pytest.mark.gpu
REL = 1e-12


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


def _gpu_rhs(torch, B, prob, U, alpha=None):
    S = B.Solver(prob)
    Ud = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    a = None if alpha is None else torch.from_numpy(np.asarray(alpha, dtype=np.float64)).cuda()
    out, dec = S.rhs(Ud, alpha_in=a, decisions=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), dec.cpu().numpy(), S.alpha.cpu().numpy(), int(S.status.cpu()[0])


def compare(Rg, Rc, dg, dc, label=""):
    flips = int(np.count_nonzero(dg != dc))
    mflips = int(np.count_nonzero((dg & 31) != (dc & 31)))
    kflips = int(np.count_nonzero((dg >> 5) != (dc >> 5)))
    nc = Rc.shape[0]
    scale = np.abs(Rc).reshape(nc, -1).max(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    rel = (np.abs(Rg - Rc).reshape(nc, -1).max(axis=1) / scale).max()
    bitwise = bool(np.array_equal(Rg, Rc))
    print(f"[parity] {label}: flips={flips} (m {mflips}, mask {kflips}) max_rel={rel:.3e} "
          f"bitwise={bitwise}", flush=True)
    return flips, rel, bitwise


def cells_next_to_flips(prob, dg, dc):
    """Boolean field (nz, ny, nx): cells with a face whose decision bytes
    differ between two dumps (layout: per axis, per line, per face 2 nc
    bytes; lines ordered as the sweeps take them)."""
    n = list(prob.n) + [1] * (3 - prob.ndim)
    nx, ny, nz = n
    nc = prob.nc
    bad = np.zeros((nz, ny, nx), dtype=bool)
    off = 0
    for d in range(prob.ndim):
        nd = n[d]
        lines = prob.ncell // nd
        seg = slice(off, off + lines * (nd + 1) * 2 * nc)
        face = np.any((dg[seg] != dc[seg]).reshape(lines, nd + 1, 2 * nc), axis=2)
        cell = face[:, :-1] | face[:, 1:]              # faces i-1/2 and i+1/2 of cell i
        if d == 0:
            bad |= cell.reshape(nz, ny, nx)
        elif d == 1:
            bad |= cell.reshape(nz, nx, ny).transpose(0, 2, 1)
        else:
            bad |= cell.reshape(ny, nx, nz).transpose(2, 0, 1)
        off += lines * (nd + 1) * 2 * nc
    return bad


def compare_literal(prob, Rg, Rl, dg, dl, fmax, label=""):
    """The kernel against the FMA-free oracle: decisions that differ are
    counted (a tie between two roundings of the same formula is not an
    error), the cells next to faces whose kept set differs are left out, and
    on every other cell the error is measured normwise per component, against
    the larger of the
    component's largest RHS and its largest back-projection term
    sum_s |R_cs f^_s| / dx (fmax, from the oracle): a component whose RHS
    vanishes in exact arithmetic -- the density of a fluid at rest with
    uniform density -- is the rounding noise of cancelling characteristic
    terms in both evaluations.

    A face's flux depends on its decisions only through the kept set (the
    eq 2.15 weights), so a ladder index that differs under the same kept set
    leaves the flux unchanged; such flips are counted but exclude no cell.
    They occur where tau = |beta_2 - beta_0| vanishes in exact arithmetic (a
    stencil symmetric about its centre): its computed value is rounding
    noise of either order, and theta = 1 / (1 + x / H) lands on 1 or just
    below it."""
    flips = int(np.count_nonzero(dg != dl))
    kflips = int(np.count_nonzero((dg >> 5) != (dl >> 5)))
    bad = cells_next_to_flips(prob, dg >> 5, dl >> 5)
    nc = Rl.shape[0]
    keep = ~bad.reshape(-1)
    A = Rg.reshape(nc, -1)[:, keep]
    C = Rl.reshape(nc, -1)[:, keep]
    scale = np.abs(C).max(axis=1) if C.size else np.ones(nc)
    scale = np.maximum(scale, np.asarray(fmax)[:nc])
    scale = np.where(scale > 0, scale, 1.0)
    rel = float((np.abs(A - C).max(axis=1) / scale).max()) if C.size else 0.0
    print(f"[parity vs literal oracle] {label}: decision flips={flips} (kept set {kflips}, "
          f"ladder index only {flips - kflips}) cells excluded={int(bad.sum())} of {bad.size} "
          f"max_rel={rel:.3e}", flush=True)
    return flips, rel, int(bad.sum())


CASES = {
    "1d_sod200": lambda: W.sod(200),
    "1d_shu_osher400": lambda: W.shu_osher(400),
    "1d_blast400_reflective": lambda: W.blast_waves(400),
    "1d_random131_reflective": lambda: (lambda p: (p, W.random_field(p, seed=4)))(
        W.uniform_problem(1, [131], [0.0], [1.0], "reflective")),
    "1d_random3_periodic": lambda: (lambda p: (p, W.random_field(p, seed=5)))(
        W.uniform_problem(1, [3], [0.0], [1.0], "periodic")),
    "2d_random67x45_mixed": lambda: (lambda p: (p, W.random_field(p, seed=6)))(
        W.uniform_problem(2, [67, 45], [0.0, 0.0], [1.0, 1.0], ["periodic", "transmissive"])),
    "2d_riemann3_96x80": lambda: W.riemann_2d(96, ny=80),
    "2d_random5x7_reflective": lambda: (lambda p: (p, W.random_field(p, seed=7)))(
        W.uniform_problem(2, [5, 7], [0.0, 0.0], [1.0, 1.0], "reflective")),
    "3d_random21x18x13_mixed": lambda: (lambda p: (p, W.random_field(p, seed=8)))(
        W.uniform_problem(3, [21, 18, 13], [0.0] * 3, [1.0] * 3,
                          ["periodic", "transmissive", "reflective"])),
    "3d_turbulence24": lambda: W.turbulence_3d(24),
    "3d_random9x8x7_periodic": lambda: (lambda p: (p, W.random_field(p, seed=9)))(
        W.uniform_problem(3, [9, 8, 7], [0.0] * 3, [1.0] * 3, "periodic")),
    # every axis >= 63 cells (the fixed-stride sweeps; y and z with four
    # columns per block since nx % 4 == 0), ragged chunk tails on each axis
    "3d_random64x65x70_mixed": lambda: (lambda p: (p, W.random_field(p, seed=10)))(
        W.uniform_problem(3, [64, 65, 70], [0.0] * 3, [1.0] * 3,
                          ["periodic", "reflective", "transmissive"])),
    # nx % 4 != 0: the y sweep falls back to one column per wave
    "2d_random98x70_mixed": lambda: (lambda p: (p, W.random_field(p, seed=11)))(
        W.uniform_problem(2, [98, 70], [0.0, 0.0], [1.0, 1.0], ["transmissive", "periodic"])),
    # the shortest lines of the fixed-stride sweeps (n = 63: 64 faces per
    # line, so a 4-chunk x block spans 5 lines), x blocks with a partial last
    # block, and eight-column z blocks (nx % 8 == 0)
    "2d_random63x66_mixed": lambda: (lambda p: (p, W.random_field(p, seed=12)))(
        W.uniform_problem(2, [63, 66], [0.0, 0.0], [1.0, 1.0], ["reflective", "periodic"])),
    "3d_random72x63x64_mixed": lambda: (lambda p: (p, W.random_field(p, seed=13)))(
        W.uniform_problem(3, [72, 63, 64], [0.0] * 3, [1.0] * 3,
                          ["transmissive", "periodic", "reflective"])),
    # an oblique contact: the acoustic and shear fields carry rounding noise
    # only, and only the entropy field is cut
    "3d_contact64x64x64": lambda: W.contact(3, [64, 64, 64]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_parity(torch, B, orc, name):
    prob, U = CASES[name]()
    Rg, dg, ag, stg = _gpu_rhs(torch, B, prob, U)
    ac, stc = orc.alpha(prob, U)
    assert np.array_equal(ag, ac), (ag, ac)
    assert stg == stc
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, name)
    assert flips == 0
    assert rel <= REL
    assert bitwise


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_parity_literal_oracle(torch, B, orc, name):
    # the same kernel result against the FMA-free oracle (every formula as
    # its plain product-then-sum): the spec bar of 1e-12 per RHS,
    # normwise per component, with flipped decisions counted
    prob, U = CASES[name]()
    Rg, dg, _, _ = _gpu_rhs(torch, B, prob, U)
    Rl, dl = orc.rhs(prob, U, dump=True, literal=True)
    _, _, fmax = orc.rhs_flux_abs(prob, U, literal=True, with_max=True)
    flips, rel, nbad = compare_literal(prob, Rg, Rl, dg, dl, fmax, name)
    assert rel <= REL
    assert nbad <= max(8, 1e-3 * prob.ncell)


@pytest.mark.parametrize("name", ["1d_blast400_reflective", "2d_riemann3_96x80",
                                  "3d_random21x18x13_mixed"])
def test_rhs_parity_literal_decisions(torch, B, orc, name):
    # every decision through the literal formula: same bits as the fast path
    prob, U = CASES[name]()
    Rf, df, _, _ = _gpu_rhs(torch, B, prob, U)
    lit = prob.replace()
    lit.literal_decisions = True
    Rl, dl, _, _ = _gpu_rhs(torch, B, lit, U)
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rl, Rc, dl, dc, name + " literal")
    assert flips == 0 and bitwise
    assert np.array_equal(Rf, Rl) and np.array_equal(df, dl)


@pytest.mark.parametrize("scheme", ["fixed_ct", "linear5", "teno5a"])
def test_rhs_parity_other_schemes(torch, B, orc, scheme):
    prob = W.uniform_problem(2, [40, 33], [0.0, 0.0], [1.0, 1.0], "transmissive",
                             scheme=scheme, ct_fixed=1e-6)
    U = W.random_field(prob, seed=12)
    Rg, dg, _, _ = _gpu_rhs(torch, B, prob, U)
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, scheme)
    assert flips == 0 and rel <= REL and bitwise


# The cut form of the LAD sensor (theta = 0 where max chi-tilde > H, Sec. 3's
# description of H): every decision (ladder index and mask) through the fast
# path and through the literal formula, and steps without decision dumps.
# (inputs with stencils whose max chi-tilde lies in (H, 5 H], where the two
# forms give different ladder indices)
@pytest.mark.parametrize("name,steps", [("1d_random131_reflective", 4),
                                        ("2d_random67x45_mixed", 3),
                                        ("3d_random21x18x13_mixed", 2),
                                        ("3d_random64x65x70_mixed", 1)])
def test_lad_cut_form_parity(torch, B, orc, name, steps):
    prob, U = CASES[name]()
    prob = prob.replace(theta="cut")
    Rg, dg, _, _ = _gpu_rhs(torch, B, prob, U)
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, name + " cut")
    assert flips == 0 and bitwise
    # the printed form differs on this input (some stencil has max chi~ > H)
    _, dp, _, _ = _gpu_rhs(torch, B, prob.replace(theta="printed"), U)
    m_cut, m_printed = dg & 31, dp & 31
    print(f"[cut form] {name}: ladder indices that differ from the printed form: "
          f"{int(np.count_nonzero(m_cut != m_printed))} of {dg.size}", flush=True)
    assert np.count_nonzero(m_cut != m_printed) > 0
    lit = prob.replace()
    lit.literal_decisions = True
    Rl, dl, _, _ = _gpu_rhs(torch, B, lit, U)
    assert np.array_equal(Rl, Rg) and np.array_equal(dl, dg)
    # against the FMA-free oracle under the same form, flips counted
    Ro, do = orc.rhs(prob, U, dump=True, literal=True)
    _, _, fmax = orc.rhs_flux_abs(prob, U, literal=True, with_max=True)
    _, lrel, nbad = compare_literal(prob, Rg, Ro, dg, do, fmax, name + " cut")
    assert lrel <= REL and nbad <= max(8, 1e-3 * prob.ncell)
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, 1e9, steps)
    Uc = U.copy()
    t = 0.0
    for _ in range(steps):
        Uc, t, dt, a9, st = orc.step(prob, Uc, 0.5, t, 1e9)
    assert c.status == st and c.t == t
    assert np.array_equal(Ug, Uc)


# TENO5-A (eq 2.16-2.18): RHS with every decision (cutoff exponent and
# mask), the literal-decision mode, and steps (no decision dump, so the
# smooth-stencil shortcut is on), with the default and the Rayleigh-Taylor
# parameter sets.
@pytest.mark.parametrize("name,kw,steps", [
    ("1d_shu_osher400", {}, 6), ("2d_riemann3_96x80", {}, 3),
    ("3d_random21x18x13_mixed", {}, 2), ("1d_blast400_reflective", {"a2": 5.5, "cr": 0.3}, 4),
    ("3d_turbulence24", {"a2": 5.5, "cr": 0.3}, 2)])
def test_teno5a_parity(torch, B, orc, name, kw, steps):
    prob, U = CASES[name]()
    prob = prob.replace(scheme="teno5a", **kw)
    Rg, dg, _, _ = _gpu_rhs(torch, B, prob, U)
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, name + " teno5a")
    assert flips == 0 and bitwise
    assert set(np.unique(dc & 31)) <= set(range(int(np.floor(prob.a1 - prob.a2)), 11))
    lit = prob.replace()
    lit.literal_decisions = True
    Rl, dl, _, _ = _gpu_rhs(torch, B, lit, U)
    assert np.array_equal(Rl, Rg) and np.array_equal(dl, dg)
    # against the FMA-free oracle under the same form, flips counted
    Ro, do = orc.rhs(prob, U, dump=True, literal=True)
    _, _, fmax = orc.rhs_flux_abs(prob, U, literal=True, with_max=True)
    _, lrel, nbad = compare_literal(prob, Rg, Ro, dg, do, fmax, name + " cut")
    assert lrel <= REL and nbad <= max(8, 1e-3 * prob.ncell)
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, 1e9, steps)
    Uc = U.copy()
    t = 0.0
    for _ in range(steps):
        Uc, t, dt, a9, st = orc.step(prob, Uc, 0.5, t, 1e9)
    assert c.status == st
    assert np.array_equal(Ug, Uc)


def test_rhs_frozen_alpha(torch, B, orc):
    prob, U = W.shu_osher(256)
    alpha = np.array([7.5, 0.0, 0.0])
    Rg, dg, ag, _ = _gpu_rhs(torch, B, prob, U, alpha=alpha)
    assert np.array_equal(ag, alpha)
    Rc, dc = orc.rhs(prob, U, alpha, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, "frozen alpha")
    assert flips == 0 and bitwise


def test_rhs_deterministic(torch, B):
    prob, U = W.turbulence_3d(32)
    R1, d1, _, _ = _gpu_rhs(torch, B, prob, U)
    R2, d2, _, _ = _gpu_rhs(torch, B, prob, U)
    assert np.array_equal(R1, R2) and np.array_equal(d1, d2)


def test_free_stream_gpu(torch, B):
    prob = W.uniform_problem(3, [17, 9, 11], [0.0] * 3, [1.0] * 3, "periodic")
    U = W.conserved(np.full(prob.shape[1:], 1.1), [0.2, -0.1, 0.3], 0.9, 1.4)
    Rg, _, _, _ = _gpu_rhs(torch, B, prob, U)
    assert np.all(Rg == 0.0)


# --------------------------------------------------------------------------
# SSP-RK3 steps
# --------------------------------------------------------------------------
def _gpu_steps(torch, B, prob, U, cfl, t_end, nsteps):
    S = B.Solver(prob)
    S.init(0.0, t_end, cfl)
    Ud = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    for _ in range(nsteps):
        S.step(Ud)
    torch.cuda.synchronize()
    return Ud.cpu().numpy(), S.read_ctrl()


@pytest.mark.parametrize("name,steps", [("1d_sod200", 12), ("2d_riemann3_96x80", 4),
                                        ("3d_random21x18x13_mixed", 3), ("3d_turbulence24", 3),
                                        ("3d_random64x65x70_mixed", 2),
                                        ("3d_random72x63x64_mixed", 2),
                                        ("2d_random63x66_mixed", 3)])
def test_step_parity(torch, B, orc, name, steps):
    prob, U = CASES[name]()
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, 1e9, steps)
    Uc = U.copy()
    t = 0.0
    for _ in range(steps):
        Uc, t, dt, a9, st = orc.step(prob, Uc, 0.5, t, 1e9)
    assert c.nsteps == steps and c.status == 0
    assert c.t == t and c.dt == dt
    assert np.array_equal(np.array(c.alpha), a9)
    print(f"[step parity] {name}: bitwise={np.array_equal(Ug, Uc)} "
          f"max_abs={np.abs(Ug - Uc).max():.3e}", flush=True)
    assert np.array_equal(Ug, Uc)


@pytest.mark.parametrize("name", ["1d_sod200", "2d_riemann3_96x80", "3d_random21x18x13_mixed"])
def test_step_timed_matches_step(torch, B, name):
    # teno_step_timed: 2 * 3 * ndim events, pair (ndim * s + d) around the
    # sweep of axis d in stage s; the state equals teno_step's bit for bit
    prob, U = CASES[name]()
    nd = prob.ndim
    plain = B.Solver(prob)
    timed = B.Solver(prob)
    plain.init(0.0, 1e9, 0.5)
    timed.init(0.0, 1e9, 0.5)
    u0 = torch.from_numpy(U.copy()).cuda()
    u1 = torch.from_numpy(U.copy()).cuda()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 3 * nd)]
    for e in evs:
        e.record(stream)
    for _ in range(2):
        plain.step(u0)
        timed.step(u1, events=evs)
    torch.cuda.synchronize()
    assert torch.equal(u0, u1)
    for s in range(3):
        for d in range(nd):
            assert evs[2 * (nd * s + d)].elapsed_time(evs[2 * (nd * s + d) + 1]) >= 0.0


def test_sod_run_to_t_end(torch, B, orc):
    from oracle import riemann
    prob, U = W.sod(200)
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, 0.2, 400)
    assert c.t == 0.2
    Uc, t, k = orc.run(prob, U, 0.5, t_end=0.2)
    assert c.nsteps == k
    assert np.array_equal(Ug, Uc)
    r, _, _ = riemann.solution(W.SOD_LEFT, W.SOD_RIGHT, prob.centres(0), 0.2, x0=0.5)
    assert np.mean(np.abs(Ug[0, 0, 0] - r)) < 1e-2


def test_replay_step(torch, B, orc):
    prob, U = W.adjoint_case(512)
    S = B.Solver(prob)
    S.init(0.0, 1e9, 0.5)
    c = S.read_ctrl()
    c.replay = 1
    c.dt = 1.3e-4
    a9 = np.array([[9.0, 0, 0], [9.5, 0, 0], [10.0, 0, 0]])
    for s in range(3):
        for k in range(3):
            c.alpha[s][k] = a9[s, k]
    S.write_ctrl(c)
    Ud = torch.from_numpy(U.copy()).cuda()
    S.step(Ud)
    torch.cuda.synchronize()
    Uc, t, dt, a9c, st = orc.step(prob, U, 0.5, 0.0, 1e9, replay=(1.3e-4, a9))
    assert np.array_equal(Ud.cpu().numpy(), Uc)
    c2 = S.read_ctrl()
    assert c2.t == 1.3e-4 and c2.nsteps == 1


def test_nonphysical_status_and_rollback(torch, B, orc):
    prob, U = W.blast_waves(400)
    S = B.Solver(prob)
    S.init(0.0, 0.038, 0.5)
    Ud = torch.from_numpy(U.copy()).cuda()
    Uc = U.copy()
    t = 0.0
    for k in range(40):
        before = Ud.clone()
        S.step(Ud)
        Uc2, t, dt, a9, st = orc.step(prob, Uc, 0.5, t, 0.038)
        c = S.read_ctrl()
        if st:
            assert c.status == 3
            assert torch.equal(Ud, before)  # the failed step left U unchanged
            assert c.nsteps == k
            S.step(Ud)  # sticky: later steps are no-ops
            assert torch.equal(Ud, before)
            return
        assert c.status == 0
        assert np.array_equal(Ud.cpu().numpy(), Uc2)
        Uc = Uc2
    pytest.fail("oracle never flagged the blast-wave state")


# --------------------------------------------------------------------------
# Full-size shapes: every cell against the oracle
# --------------------------------------------------------------------------
def _full_field(torch, B, orc, prob, U):
    """GPU RHS and decisions of the whole field against both oracle builds:
    the fused-order one (bit for bit, no flipped decision) and the FMA-free
    literal one (within REL on cells next to no flipped decision)."""
    S = B.Solver(prob)
    Ud = torch.from_numpy(U).cuda()
    out, dec = S.rhs(Ud, decisions=True)
    torch.cuda.synchronize()
    a = S.alpha.cpu().numpy()
    ac, _ = orc.alpha(prob, U)
    assert np.array_equal(a, ac)
    Rg, dg = out.cpu().numpy(), dec.cpu().numpy()
    del out, dec, Ud, S
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, f"full field {prob.n}")
    del Rc, dc
    Rl, dl = orc.rhs(prob, U, dump=True, literal=True)
    _, _, fmax = orc.rhs_flux_abs(prob, U, literal=True, with_max=True)
    lflips, lrel, nbad = compare_literal(prob, Rg, Rl, dg, dl, fmax, f"full field {prob.n}")
    return flips, rel, bitwise, lflips, lrel, Rg


def test_full_field_3d_256(torch, B, orc):
    prob, U = W.turbulence_3d(256)
    flips, rel, bitwise, lflips, lrel, Rg = _full_field(torch, B, orc, prob, U)
    assert flips == 0 and rel <= REL and bitwise
    assert lrel <= REL
    # Periodic: the RHS sums to zero up to rounding (eq 2.2 telescopes: each
    # face flux enters its two cells with opposite signs).  Per cell and axis
    # the kernel rounds the difference a - b of its two face fluxes
    # (<= u (|a| + |b|), u = 2^-53), the quotient by dx (<= u |a - b| / dx)
    # and the accumulation over the axes (<= u (1 + u) sum_d |a_d - b_d| /
    # dx_d), i.e. <= 4u (1 + u)^2 sum_d (|a_d| + |b_d|) / dx_d per cell, and
    # every face enters two cells: |sum RHS| <= 8u (1 + u)^2 S with S = sum
    # over axes and faces of |F^| / dx (from the oracle, whose face fluxes
    # are the kernel's bit for bit).  The host sum is taken in 80-bit
    # precision, whose own error (< 2^-63 log2(N) sum |RHS|) is added.
    _, Sabs = orc.rhs_flux_abs(prob, U)
    nc = prob.nc
    tot = Rg.reshape(nc, -1).sum(axis=1, dtype=np.longdouble)
    u = 2.0 ** -53
    bound = 8.0 * u * (1 + u) ** 2 * Sabs + 2.0 ** -63 * 25 * np.abs(Rg).reshape(nc, -1).sum(1)
    print(f"[full field] RHS sums {tot.astype(np.float64)} vs rounding bound {bound}", flush=True)
    assert np.all(np.abs(tot.astype(np.float64)) <= bound)


def test_full_field_2d_2048(torch, B, orc):
    prob, U = W.riemann_2d(2048)
    flips, rel, bitwise, lflips, lrel, _ = _full_field(torch, B, orc, prob, U)
    assert flips == 0 and rel <= REL and bitwise
    assert lrel <= REL


# --------------------------------------------------------------------------
# Per-end boundaries, moving splits and gravity (Sec. 4.3 workloads)
# --------------------------------------------------------------------------
def _mixed3d():
    prob = W.uniform_problem(3, [64, 16, 64], [0.0] * 3, [1.0, 0.5, 1.0], "transmissive")
    U = W.random_field(prob, seed=14)
    a = W.conserved(1.2, [0.1, -0.2, 0.05], 0.9, prob.gamma).tolist()
    b = W.conserved(0.6, [0.0, 0.3, -0.1], 0.4, prob.gamma).tolist()
    bnd = W.Boundary(sides=[
        [W.Side("fixed", state_a=a), W.Side("transmissive")],
        [W.Side("fixed", "reflective", split_axis=0, split0=0.3, split_rate=2.0, state_a=b),
         W.Side("periodic")],
        [W.Side("reflective"), W.Side("transmissive", "fixed", split_axis=1, split0=0.2,
                                      split_rate=-1.0, state_b=a)]],
        gravity=(0.1, -0.2, 0.3), time=0.05)
    return prob.replace(boundary=bnd), U


BOUNDARY_CASES = {
    "2d_rayleigh_taylor16x64": lambda: W.rayleigh_taylor(16, 64),
    "2d_double_mach64x16": lambda: W.double_mach(64, 16),
    "3d_mixed_ends64x16x64": _mixed3d,
}


@pytest.mark.parametrize("name,steps", [("2d_rayleigh_taylor16x64", 5),
                                        ("2d_double_mach64x16", 5),
                                        ("3d_mixed_ends64x16x64", 2)])
def test_boundary_parity(torch, B, orc, name, steps):
    prob, U = BOUNDARY_CASES[name]()
    Rg, dg, ag, _ = _gpu_rhs(torch, B, prob, U)
    Rc, dc = orc.rhs(prob, U, dump=True)
    flips, rel, bitwise = compare(Rg, Rc, dg, dc, name)
    assert flips == 0 and bitwise
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, 1e9, steps)
    Uc = U.copy()
    t = 0.0
    for _ in range(steps):
        Uc, t, dt, a9, st = orc.step(prob, Uc, 0.5, t, 1e9)
    assert c.status == st == 0 and c.t == t
    print(f"[boundary parity] {name}: steps bitwise={np.array_equal(Ug, Uc)}", flush=True)
    assert np.array_equal(Ug, Uc)


# Whole runs of the Table 2 problems (Sec. 4.3) at reduced size to their
# final times: adaptive dt (eq dt2) every step, the gravity source and the
# fixed, split and moving boundaries, and every cutoff decision along the way.
FULL_RUNS = {
    "riemann_case1_128x128_t0.3": (lambda: W.riemann_2d_table2(1, 128), 0.3),
    "riemann_case2_128x128_t0.25": (lambda: W.riemann_2d_table2(2, 128), 0.25),
    # the comparison schemes of Table 2 on case 1: TENO5 with the default
    # C_T = 1e-7, TENO5-A with the adjusted alpha_2 = 5.5, C_r = 0.3
    "riemann_case1_teno5_128x128_t0.3":
        (lambda: W.riemann_2d_table2(1, 128, scheme="fixed_ct", ct_fixed=1e-7), 0.3),
    "riemann_case1_teno5a_128x128_t0.3":
        (lambda: W.riemann_2d_table2(1, 128, scheme="teno5a", a2=5.5, cr=0.3), 0.3),
    "rayleigh_taylor_32x128_t1.95": (lambda: W.rayleigh_taylor(32, 128), 1.95),
    # the double Mach reflection with H = 1: with the printed H = 10 the
    # method goes non-physical in a wall cell ahead of the shock foot
    "double_mach_H1_128x32_t0.2":
        (lambda: (lambda p, u: (p.replace(H=1.0), u))(*W.double_mach(128, 32)), 0.2),
    # ... and with H = 10 under the cut form of the sensor (theta = 0 where
    # max chi-tilde > H)
    "double_mach_cut_128x32_t0.2": (lambda: W.double_mach(128, 32, theta="cut"), 0.2),
}


@pytest.mark.parametrize("name,prob_u,nsteps", [
    # the Shu-Osher problem of Sec. 4.2 to its final time
    ("shu_osher400_t1.8", lambda: W.shu_osher(400), None),
    # 3D periodic turbulence through 200 adaptive steps (t = 2.79)
    ("turbulence_3d_24_200steps", lambda: W.turbulence_3d(24), 200),
])
def test_long_run(torch, B, orc, name, prob_u, nsteps):
    prob, U = prob_u()
    t_end = 1.8 if nsteps is None else np.inf
    Uc, t, k = orc.run(prob, U, 0.5, t_end=t_end, nsteps=nsteps)
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, 1e9 if nsteps else t_end, k if nsteps else k + 5)
    print(f"[long run] {name}: {k} steps to t = {t}, device {c.nsteps} steps to t = {c.t}, "
          f"bitwise {np.array_equal(Ug, Uc)}", flush=True)
    assert c.status == 0 and c.nsteps == k and c.t == t
    assert np.array_equal(Ug, Uc)


@pytest.mark.parametrize("name", list(FULL_RUNS))
def test_full_run_to_final_time(torch, B, orc, name):
    mk, t_end = FULL_RUNS[name]
    prob, U = mk()
    Uc, t, k = orc.run(prob, U, 0.5, t_end=t_end)
    # steps after t_end are no-ops on the device
    Ug, c = _gpu_steps(torch, B, prob, U, 0.5, t_end, k + 5)
    print(f"[full run] {name}: {k} steps to t = {t}, device {c.nsteps} steps to t = {c.t}, "
          f"bitwise {np.array_equal(Ug, Uc)}", flush=True)
    assert c.status == 0 and c.nsteps == k and c.t == t == t_end
    assert np.array_equal(Ug, Uc)


def test_double_mach_full_size_cut_form(torch, B):
    # Sec. 4.3.3 at the Table 2 grid 1024 x 256 with H = 10 to t = 0.2: the
    # printed sensor goes non-physical within the first steps, the cut form
    # runs to the final time
    t_end = 0.2
    out = {}
    for theta in ("printed", "cut"):
        prob, U = W.double_mach(1024, 256, theta=theta)
        Ug, c = _gpu_steps(torch, B, prob, U, 0.5, t_end, 5000)
        out[theta] = (int(c.status), float(c.t), int(c.nsteps), float(Ug[0].min()))
        print(f"[double Mach 1024x256 H=10] theta {theta}: status {c.status} t {c.t} "
              f"steps {c.nsteps} rho_min {Ug[0].min():.4f}", flush=True)
    assert out["printed"][0] == 3 and out["printed"][1] < 0.01
    assert out["cut"][0] == 0 and out["cut"][1] == t_end and out["cut"][3] > 0.0


def test_boundary_rejected_by_adjoint_and_batch(torch, B):
    prob, U = W.double_mach(64, 16)
    g = B.grid(prob)
    L = B.lib()
    d = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert L.teno_rhs_adjoint(ctypes.byref(g), d, d, d, d, d, 1 << 40, None) == B.ERR_ARG
    with pytest.raises(B.TenoError):
        B.BatchPlan([8, 9], [0.1, 0.1], prob={"boundary": prob.boundary})


# --------------------------------------------------------------------------
# A grid whose component offsets pass 2^31 and 2^32 (64-bit indexing)
# --------------------------------------------------------------------------
HASH_SALT = [(73856093, 19349663, 83492791), (2654435761, 40503, 97), (31, 1000003, 7919),
             (2246822519, 3266489917, 668265263), (374761393, 16777619, 1299709)]


def _hash_field_np(ii, jj, kk):
    """Conserved state from an integer hash of the cell indices: every value
    is a dyadic rational, so host and device build identical bits.
    rho = 1 + h/1024, m_d = (h - 512)/4096, E = 2.5 + h/1024."""
    out = []
    for c, (a, b, cc) in enumerate(HASH_SALT):
        h = ((ii * a) ^ (jj * b) ^ (kk * cc)) & 1023
        h = h.astype(np.float64)
        out.append(1.0 + h / 1024.0 if c == 0 else 2.5 + h / 1024.0 if c == 4 else (h - 512.0) / 4096.0)
    return np.stack(out)


def test_huge_grid_64bit_offsets(torch, B, orc):
    nx, ny, nz = 1024, 1024, 832
    ncell = nx * ny * nz
    assert 4 * ncell + ncell > 2 ** 32
    prob = W.uniform_problem(3, [nx, ny, nz], [0.0] * 3, [1.0, 1.0, 0.8], "periodic")
    g = B.grid(prob)
    U = torch.empty((5, nz, ny, nx), dtype=torch.float64, device="cuda")
    i = torch.arange(nx, device="cuda", dtype=torch.int64).view(1, 1, nx)
    j = torch.arange(ny, device="cuda", dtype=torch.int64).view(1, ny, 1)
    for c, (a, b, cc) in enumerate(HASH_SALT):
        for k0 in range(0, nz, 64):
            k = torch.arange(k0, min(nz, k0 + 64), device="cuda", dtype=torch.int64).view(-1, 1, 1)
            h = (((i * a) ^ (j * b) ^ (k * cc)) & 1023).to(torch.float64)
            U[c, k0:k0 + k.shape[0]] = (1.0 + h / 1024.0 if c == 0 else 2.5 + h / 1024.0 if c == 4
                                        else (h - 512.0) / 4096.0)
    alpha = torch.tensor([2.0, 2.5, 3.0], dtype=torch.float64, device="cuda")
    R = torch.empty_like(U)
    for axis in range(3):
        B.teno_sweep(g, axis, U, R, alpha, Rin=(R if axis else None))
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    cells = [tuple(int(v) for v in (rng.integers(nx), rng.integers(ny), rng.integers(nz)))
             for _ in range(40)]
    cells += [(nx - 1, ny - 1, nz - 1), (0, ny - 1, nz - 1), (nx - 2, 3, nz - 1), (5, 0, 0)]
    # the RHS of a cell needs its 7^3 neighbourhood only (3 cells per side)
    box = W.Problem(ndim=3, n=[7, 7, 7], dx=list(prob.dx), bc=["periodic"] * 3)
    off = np.arange(-3, 4)
    idx = torch.tensor([[k, jy, ix] for ix, jy, k in cells], device="cuda")
    got = R[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T
    for s, (ix, jy, k) in enumerate(cells):
        kk, jj, ii = np.meshgrid((k + off) % nz, (jy + off) % ny, (ix + off) % nx, indexing="ij")
        Ubox = np.ascontiguousarray(_hash_field_np(ii, jj, kk))
        ref = orc.rhs_cells(box, Ubox, alpha.cpu().numpy(), np.array([3 * 49 + 3 * 7 + 3]))
        assert np.array_equal(got[s], ref[0]), (ix, jy, k, got[s], ref[0])


# --------------------------------------------------------------------------
# Graph-replayed steps (teno_runner): bit-identical to teno_step calls
# --------------------------------------------------------------------------
def test_runner_replays_match_steps(torch, B):
    # Every replay is checked against eager steps on a copy, with eager steps
    # of the runner's own buffers and host synchronizations in between
    # (replays after the first must continue the run exactly), and the run
    # crosses t_end inside a replay (the remaining steps are no-ops).
    prob, U = W.sod(200)
    t_end = 0.05
    S_ref = B.Solver(prob)
    S = B.Solver(prob)
    u_ref = torch.from_numpy(U.copy()).cuda()
    u = torch.from_numpy(U.copy()).cuda()
    S_ref.init(0.0, t_end, 0.5)
    S.init(0.0, t_end, 0.5)
    R = B.Runner(S.g, u, S.ctrl, S.ws, steps_per_graph=7)
    plan = [("graph", 7), ("eager", 2), ("graph", 14), ("graph", 3), ("eager", 1), ("graph", 21),
            ("graph", 7)]
    for kind, n in plan:
        if kind == "graph":
            R.run(n)
        else:
            for _ in range(n):
                S.step(u)
        for _ in range(n):
            S_ref.step(u_ref)
        torch.cuda.synchronize()
        c, cr = S.read_ctrl(), S_ref.read_ctrl()
        assert torch.equal(u, u_ref), (kind, n, c.nsteps)
        assert (c.t, c.dt, c.nsteps, c.status) == (cr.t, cr.dt, cr.nsteps, cr.status)
    print(f"[runner] sod200: {c.nsteps} steps to t = {c.t} (t_end {t_end}) bitwise equal "
          f"to teno_step over {len(plan)} segments", flush=True)
    assert c.t == t_end and c.nsteps < sum(n for _, n in plan)
    R.close()


@pytest.mark.parametrize("name,steps", [("2d_riemann3_96x80", 23), ("3d_random21x18x13_mixed", 12)])
def test_runner_matches_oracle(torch, B, orc, name, steps):
    prob, U = CASES[name]()
    S = B.Solver(prob)
    u = torch.from_numpy(U.copy()).cuda()
    S.init(0.0, 1e9, 0.5)
    S.run(u, steps, steps_per_graph=5)
    torch.cuda.synchronize()
    Uc = U.copy()
    t = 0.0
    for _ in range(steps):
        Uc, t, dt, a9, st = orc.step(prob, Uc, 0.5, t, 1e9)
    c = S.read_ctrl()
    assert c.status == st == 0 and c.t == t and c.nsteps == steps
    assert np.array_equal(u.cpu().numpy(), Uc)


def test_runner_rejects_bad_arguments(torch, B):
    prob, U = W.sod(50)
    S = B.Solver(prob)
    u = torch.from_numpy(U.copy()).cuda()
    L = B.lib()
    h = ctypes.c_void_p()
    nb = S.ws.numel()
    args = lambda spg, ws_bytes: (ctypes.byref(S.g), B._ptr(u), B._ptr(S.ctrl), B._ptr(S.ws),
                                  ws_bytes, spg, ctypes.byref(h))
    assert L.teno_runner_create(*args(0, nb)) == B.ERR_ARG
    assert L.teno_runner_create(*args(1001, nb)) == B.ERR_ARG
    assert L.teno_runner_create(*args(4, nb - 1)) == B.ERR_ARG
    assert L.teno_runner_run(None, 3, None) == B.ERR_ARG
    assert L.teno_runner_destroy(None) == B.ERR_ARG
