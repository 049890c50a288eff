"""Discrete adjoint (teno_rhs_adjoint, teno_step_adjoint, the checkpointed
trajectory gradient) against the oracle's forward-mode dual numbers (the
same frozen cutoff flags and speeds) and against finite differences."""
import numpy as np
import pytest

from paper_2003_09145_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _adj_rows(torch, B, prob, U, alpha, lams):
    g = B.grid(prob)
    ws = torch.empty(B.adjoint_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    Ud = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    ad = torch.from_numpy(np.asarray(alpha, dtype=np.float64)).cuda()
    out = []
    for lam in lams:
        ld = torch.from_numpy(np.ascontiguousarray(lam)).cuda()
        gd = torch.empty_like(Ud)
        B.teno_rhs_adjoint(g, Ud, ad, ld, gd, ws)
        out.append(gd)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


SMALL = {
    "1d_periodic": lambda: (lambda p: (p, W.random_field(p, seed=21)))(
        W.uniform_problem(1, [20], [0.0], [1.0], "periodic")),
    "1d_transmissive": lambda: W.shu_osher(24),
    "1d_reflective": lambda: (lambda p: (p, W.random_field(p, seed=22)))(
        W.uniform_problem(1, [17], [0.0], [1.0], "reflective")),
    "2d_mixed": lambda: (lambda p: (p, W.random_field(p, seed=23)))(
        W.uniform_problem(2, [8, 7], [0.0, 0.0], [1.0, 1.0], ["reflective", "periodic"])),
    "3d_mixed": lambda: (lambda p: (p, W.random_field(p, seed=24)))(
        W.uniform_problem(3, [5, 5, 4], [0.0] * 3, [1.0] * 3,
                          ["transmissive", "periodic", "reflective"])),
    "2d_teno5a": lambda: (lambda p: (p, W.random_field(p, seed=25)))(
        W.uniform_problem(2, [7, 6], [0.0, 0.0], [1.0, 1.0], ["periodic", "transmissive"],
                          scheme="teno5a")),
    # contacts: only the entropy field is cut, so every chunk runs either the
    # all-linear or the all-but-entropy-linear reverse
    "1d_contact": lambda: W.contact(1, [20]),
    "2d_contact": lambda: W.contact(2, [9, 8]),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_rhs_adjoint_full_jacobian(torch, B, orc, name):
    prob, U = SMALL[name]()
    a, _ = orc.alpha(prob, U)
    n = U.size
    eye = np.eye(n)
    Jo = np.stack([orc.rhs_jvp(prob, U, eye[j].reshape(U.shape), a)[1].ravel()
                   for j in range(n)], axis=1)          # columns J e_j
    Jg = np.stack([r.ravel() for r in _adj_rows(torch, B, prob, U, a,
                                                 [eye[k].reshape(U.shape) for k in range(n)])])
    err = np.abs(Jg - Jo).max() / np.abs(Jo).max()
    print(f"[adjoint] {name}: full Jacobian {n}x{n}, max rel err {err:.2e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("name,mk", [
    ("1d_shu_osher512", lambda: W.shu_osher(512)),
    ("2d_random40x33", lambda: (lambda p: (p, W.random_field(p, seed=31)))(
        W.uniform_problem(2, [40, 33], [0.0, 0.0], [1.0, 1.0], ["transmissive", "reflective"]))),
    ("3d_turbulence12", lambda: W.turbulence_3d(12)),
    # lines longer than one 64-face chunk and chunks that wrap between lines
    # on every axis, each boundary kind on each axis
    ("3d_random70x66x9_mixed", lambda: (lambda p: (p, W.random_field(p, seed=32)))(
        W.uniform_problem(3, [70, 66, 9], [0.0] * 3, [1.0] * 3,
                          ["periodic", "reflective", "transmissive"]))),
    ("3d_random9x5x131_mixed", lambda: (lambda p: (p, W.random_field(p, seed=33)))(
        W.uniform_problem(3, [9, 5, 131], [0.0] * 3, [1.0] * 3,
                          ["reflective", "transmissive", "periodic"]))),
    ("1d_contact300", lambda: W.contact(1, [300])),
    ("3d_contact40x36x33", lambda: W.contact(3, [40, 36, 33])),
    ("2d_teno5a_130x67", lambda: (lambda p: (p, W.random_field(p, seed=34)))(
        W.uniform_problem(2, [130, 67], [0.0, 0.0], [1.0, 1.0], ["transmissive", "periodic"],
                          scheme="teno5a"))),
    # the cut form of the LAD sensor (theta = 0 where max chi-tilde > H): the
    # frozen ladder indices and masks are the cut form's
    ("3d_random70x66x9_cut", lambda: (lambda p: (p, W.random_field(p, seed=32)))(
        W.uniform_problem(3, [70, 66, 9], [0.0] * 3, [1.0] * 3,
                          ["periodic", "reflective", "transmissive"], theta="cut"))),
])
def test_rhs_adjoint_dot_product(torch, B, orc, name, mk):
    prob, U = mk()
    a, _ = orc.alpha(prob, U)
    rng = np.random.default_rng(5)
    for trial in range(3):
        lam = rng.normal(size=U.shape)
        v = rng.normal(size=U.shape) * np.abs(U)
        _, jv = orc.rhs_jvp(prob, U, v, a)
        (jtl,) = _adj_rows(torch, B, prob, U, a, [lam])
        lhs = float(np.sum(lam * jv))
        rhs = float(np.sum(jtl * v))
        scale = float(np.sum(np.abs(lam * jv)))
        rel = abs(lhs - rhs) / scale
        print(f"[adjoint] {name}: <l, Jv> = {lhs:.12e}, <J^T l, v> = {rhs:.12e}, rel {rel:.1e}",
              flush=True)
        assert rel <= 1e-12


def _recorder(B, prob):
    from paper_2003_09145_amd.adjoint import Recorder
    return Recorder(prob)


def _log_host(B, log):
    recs = [B.TenoCtrl.from_buffer_copy(bytes(log[k].cpu().numpy())) for k in range(log.shape[0])]
    dts = np.array([r.dt for r in recs])
    alphas = np.array([np.array(r.alpha) for r in recs])
    return dts, alphas


def test_step_adjoint_dot_product(torch, B, orc):
    prob, U = W.shu_osher(300)
    rec = _recorder(B, prob)
    Ud = torch.from_numpy(U.copy()).cuda()
    UK, log, ckpt = rec.forward(Ud, 1, 0.5)
    dts, alphas = _log_host(B, log)
    rng = np.random.default_rng(8)
    lam = rng.normal(size=U.shape)
    v = rng.normal(size=U.shape) * np.abs(U)
    UT, VT = orc.run_jvp(prob, U, v, dts, alphas)
    assert np.array_equal(UT, UK.cpu().numpy())
    g = rec.backward(torch.from_numpy(lam).cuda(), log, ckpt).cpu().numpy()
    lhs, rhs = float(np.sum(lam * VT)), float(np.sum(g * v))
    rel = abs(lhs - rhs) / float(np.sum(np.abs(lam * VT)))
    print(f"[adjoint] one RK3 step: rel {rel:.1e}", flush=True)
    assert rel <= 1e-12


def _loss_setup(N, noise=0.01):
    prob, U0 = W.adjoint_case(N, noise=noise)
    _, Ut = W.adjoint_case(N, noise=0.0)
    return prob, U0, Ut


def test_trajectory_gradient_and_checkpoint_invariance(torch, B, orc):
    N, steps = 512, 60
    prob, U0, Utarget = _loss_setup(N)
    dx = prob.dx[0]
    rec = _recorder(B, prob)
    Ud = torch.from_numpy(U0.copy()).cuda()
    # target: final density of the noise-free run
    tgt, _, _ = rec.forward(torch.from_numpy(Utarget.copy()).cuda(), steps, 0.5)
    rho_star = tgt[0].clone()
    grads = {}
    for seg in (20, 1, 60):
        UK, log, ckpt = rec.forward(Ud, steps, 0.5, seg=seg)
        lamT = torch.zeros_like(UK)
        lamT[0] = dx * (UK[0] - rho_star)
        grads[seg] = rec.backward(lamT, log, ckpt, seg=seg)
    torch.cuda.synchronize()
    assert torch.equal(grads[20], grads[1]) and torch.equal(grads[20], grads[60])
    g = grads[20].cpu().numpy()
    dts, alphas = _log_host(B, log)
    lam = lamT.cpu().numpy()
    rng = np.random.default_rng(9)
    for trial in range(3):
        v = rng.normal(size=U0.shape) * np.abs(U0) * 1e-3
        _, VT = orc.run_jvp(prob, U0, v, dts, alphas)
        lhs, rhs = float(np.sum(lam * VT)), float(np.sum(g * v))
        rel = abs(lhs - rhs) / max(abs(lhs), 1e-300)
        print(f"[adjoint] {steps}-step gradient vs forward mode: rel {rel:.1e}", flush=True)
        assert rel <= 1e-10


def test_gradient_400_steps_against_forward_mode(torch, B, orc):
    # The adjoint workload at full size: N = 2048, 400 RK3 steps, the
    # gradient of J = dx/2 sum (rho(T) - rho*)^2 with respect to the initial
    # density (u0, p0 fixed) at 64 seeded cells ahead of the shock, each
    # against the oracle's forward-mode derivative along that cell through
    # the same recorded steps (replayed dt and speeds, decisions on real
    # parts).  Bar: 1e-10 relative, with a floor of 1e-10 of the largest
    # derivative for cells whose own derivative is tiny.
    N, steps = 2048, 400
    prob, U0, Utarget = _loss_setup(N)
    dx = prob.dx[0]
    rec = _recorder(B, prob)
    tgt, _, _ = rec.forward(torch.from_numpy(Utarget.copy()).cuda(), steps, 0.5)
    rho_star = tgt[0].clone()
    Ud = torch.from_numpy(U0.copy()).cuda()
    UK, log, ckpt = rec.forward(Ud, steps, 0.5)
    lamT = torch.zeros_like(UK)
    lamT[0] = dx * (UK[0] - rho_star)
    lam0 = rec.backward(lamT, log, ckpt).cpu().numpy()
    dts, alphas = _log_host(B, log)
    u0 = U0[1] / U0[0]
    grad_rho = lam0[0] + u0 * lam0[1] + 0.5 * u0 * u0 * lam0[2]
    rng = np.random.default_rng(3)
    x = prob.centres(0)
    cells = rng.choice(np.nonzero(x >= -4.0)[0], 64, replace=False)
    V = np.zeros((len(cells),) + U0.shape)
    for k, i in enumerate(cells):
        V[k, 0, 0, 0, i] = 1.0
        V[k, 1, 0, 0, i] = u0[0, 0, i]
        V[k, 2, 0, 0, i] = 0.5 * u0[0, 0, i] ** 2
    UT, _ = orc.run_jvp(prob, U0, np.zeros_like(U0), dts, alphas)
    assert np.array_equal(UT, UK.cpu().numpy())   # the oracle replays the same trajectory
    VT = orc.run_jvp_batch(prob, U0, V, dts, alphas)
    lam = lamT.cpu().numpy()
    fwd = np.einsum("kcabi,cabi->k", VT, lam)
    ad = grad_rho[0, 0, cells]
    err = np.abs(ad - fwd)
    floor = 1e-10 * float(np.abs(fwd).max())
    worst = float((err / np.maximum(np.abs(fwd), 1e-300)).max())
    print(f"[adjoint] {steps}-step gradient at {len(cells)} cells vs forward mode: max "
          f"|ad - fwd| {err.max():.2e}, max relative {worst:.2e}, largest |dJ| "
          f"{np.abs(fwd).max():.2e}", flush=True)
    assert np.all(err <= 1e-10 * np.abs(fwd) + floor)


def test_gradient_finite_differences_with_digest(torch, B):
    # The adjoint workload at full size (N = 2048, 400 steps): d J / d rho0
    # (u0, p0 fixed) against central differences h = 1e-6 with replayed dt
    # and speeds, at 64 cells whose cutoff masks do not change anywhere in
    # the trajectory (seeded cells ahead of the shock are drawn until 64 such
    # cells are found).  Bar: 1e-6 relative where the gradient is at least
    # 10% of its largest value, else 1e-7 of that value (the difference
    # quotient's rounding floor grows as 1/h and sits near 2e-8 of it here).
    N, steps, ncheck = 2048, 400, 64
    prob, U0, Utarget = _loss_setup(N)
    dx = prob.dx[0]
    rec = _recorder(B, prob)
    tgt, _, _ = rec.forward(torch.from_numpy(Utarget.copy()).cuda(), steps, 0.5)
    rho_star = tgt[0].clone()
    Ud = torch.from_numpy(U0.copy()).cuda()
    UK, log, ckpt = rec.forward(Ud, steps, 0.5, digest=True)
    base_digest = rec.digest()
    lamT = torch.zeros_like(UK)
    lamT[0] = dx * (UK[0] - rho_star)
    lam0 = rec.backward(lamT, log, ckpt).cpu().numpy()
    u0 = U0[1] / U0[0]
    grad_rho = lam0[0] + u0 * lam0[1] + 0.5 * u0 * u0 * lam0[2]

    def J(Uin):
        UT = rec.replay(torch.from_numpy(Uin).cuda(), log, digest=True)
        return 0.5 * dx * float(((UT[0] - rho_star) ** 2).sum()), rec.digest()

    def J_free(Uin):
        # the same steps with dt and the speeds recomputed from the perturbed
        # states (the map the adjoint does not differentiate)
        UT, _, _ = rec.forward(torch.from_numpy(Uin).cuda(), steps, 0.5)
        return 0.5 * dx * float(((UT[0] - rho_star) ** 2).sum())

    Jb, db = J(U0)
    assert db == base_digest
    rng = np.random.default_rng(3)
    x = prob.centres(0)
    order = rng.permutation(np.nonzero(x >= -4.0)[0])
    h = 1e-6
    gmax = float(np.abs(grad_rho).max())
    checked = skipped = 0
    worst = 0.0
    gaps = []
    for i in order:
        if checked == ncheck:
            break
        dU = np.zeros_like(U0)
        dU[0, 0, 0, i] = 1.0
        dU[1, 0, 0, i] = u0[0, 0, i]
        dU[2, 0, 0, i] = 0.5 * u0[0, 0, i] ** 2
        Jp, dp = J(U0 + h * dU)
        Jm, dm = J(U0 - h * dU)
        if dp != base_digest or dm != base_digest:
            skipped += 1
            continue
        fd = (Jp - Jm) / (2 * h)
        ad = grad_rho[0, 0, i]
        bar = 1e-6 * max(abs(ad), 0.1 * gmax)
        assert abs(fd - ad) <= bar, (i, fd, ad, gmax)
        worst = max(worst, abs(fd - ad) / bar)
        if len(gaps) < 4:
            fd_free = (J_free(U0 + h * dU) - J_free(U0 - h * dU)) / (2 * h)
            gaps.append(abs(fd_free - ad) / max(abs(ad), 0.1 * gmax))
        checked += 1
    print(f"[adjoint] FD check, {steps} steps: {checked} cells within the bar (worst "
          f"{worst:.2f} of it), {skipped} skipped (mask change); without replayed dt and "
          f"speeds the difference quotient differs from the fixed-step gradient by "
          f"{', '.join(f'{g:.1e}' for g in gaps)} (relative)", flush=True)
    assert checked == ncheck


def test_digest_variant_identical_and_flag_required(torch, B):
    prob, U = W.shu_osher(300)
    rec = _recorder(B, prob)
    Ud = torch.from_numpy(U.copy()).cuda()
    U1, log1, _ = rec.forward(Ud, 5, 0.5, digest=True)
    d1 = rec.digest()
    U2, log2, _ = rec.forward(Ud, 5, 0.5, digest=False)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)
    assert np.array_equal(_log_host(B, log1)[0], _log_host(B, log2)[0])
    assert np.array_equal(_log_host(B, log1)[1], _log_host(B, log2)[1])
    assert d1 != 0
    # a grid without TENO_FLAG_MASK_DIGEST never touches the digest
    S = B.Solver(prob)
    S.init(0.0, float("inf"), 0.5)
    B.ctrl_digest(S.ctrl, True)
    u = Ud.clone()
    S.step(u)
    torch.cuda.synchronize()
    assert S.read_ctrl().digest == 0 and torch.equal(u, _first_step(rec, Ud))


def _first_step(rec, Ud):
    U1, _, _ = rec.forward(Ud, 1, 0.5)
    return U1
