"""Reverse-mode differentiation of SSP-RK3 trajectories through the discrete
adjoint of libteno.so.

The cutoff flags of every face are frozen at their forward values (they are
piecewise constant in the state), and so are the time steps and the
per-stage Lax-Friedrichs speeds: the map being differentiated is
u^0 -> u^K for the recorded (dt_n, alpha_{n,s}), which is also what a
finite-difference check must replay.  The forward pass keeps one state
every `seg` steps; the backward pass recomputes each segment from its
checkpoint (replaying the recorded steps) and walks it backwards with
teno_step_adjoint.  Every arithmetic step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import binding as B


class Recorder:
    """A solver plus the adjoint workspace of one grid."""

    def __init__(self, prob, device="cuda"):
        self.S = B.Solver(prob, device=device)
        self.g = self.S.g
        # the same grid with the mask digest compiled in (finite-difference checks)
        self.g_digest = B.grid(prob)
        self.g_digest.flags |= B.FLAG_MASK_DIGEST
        self.device = self.S.device
        self.ws_adj = torch.empty(B.adjoint_workspace_bytes(self.g), dtype=torch.uint8,
                                  device=self.device)

    def forward(self, U0, nsteps, cfl, t_end=float("inf"), seg=20, digest=False):
        """Run nsteps recorded steps from U0.  Returns (U_K, log, checkpoints)
        with log[k] the control block after step k."""
        S = self.S
        U = U0.clone()
        S.init(0.0, t_end, cfl)
        if digest:
            B.ctrl_digest(S.ctrl, True)
        log = torch.empty((nsteps, B.CTRL_BYTES), dtype=torch.uint8, device=self.device)
        ckpt = {0: U0.clone()}
        g = self.g_digest if digest else self.g
        for k in range(nsteps):
            B.teno_step(g, U, S.ctrl, S.ws)
            log[k].copy_(S.ctrl)
            if (k + 1) % seg == 0 and k + 1 < nsteps:
                ckpt[k + 1] = U.clone()
        return U, log, ckpt

    def replay(self, U0, log, digest=False):
        """Re-run the recorded steps (frozen dt and speeds) from U0."""
        S = self.S
        U = U0.clone()
        S.init(0.0, float("inf"), 1.0)
        if digest:
            B.ctrl_digest(S.ctrl, True)
        g = self.g_digest if digest else self.g
        for k in range(log.shape[0]):
            B.ctrl_replay(S.ctrl, log[k])
            B.teno_step(g, U, S.ctrl, S.ws)
        return U

    def backward(self, lam_T, log, ckpt, seg=20):
        """Cotangent of u^0 from the cotangent lam_T of u^K."""
        S = self.S
        lam = lam_T.clone().contiguous()
        nsteps = log.shape[0]
        for start in reversed(range(0, nsteps, seg)):
            end = min(start + seg, nsteps)
            states = [ckpt[start].clone()]
            U = states[0].clone()
            S.init(0.0, float("inf"), 1.0)
            for k in range(start, end - 1):
                B.ctrl_replay(S.ctrl, log[k])
                S.step(U)
                states.append(U.clone())
            for k in reversed(range(start, end)):
                B.teno_step_adjoint(self.g, states[k - start], log[k], lam, self.ws_adj)
        return lam

    def digest(self) -> int:
        return int(self.S.read_ctrl().digest)


class TenoRK3(torch.autograd.Function):
    """u^K = RK3^K(u^0) with gradients through the discrete adjoint.

    Usage: TenoRK3.apply(U0, recorder, nsteps, cfl, seg)."""

    @staticmethod
    def forward(ctx, U0, rec: Recorder, nsteps: int, cfl: float, seg: int = 20):
        UK, log, ckpt = rec.forward(U0.detach(), nsteps, cfl, seg=seg)
        ctx.rec, ctx.log, ctx.ckpt, ctx.seg = rec, log, ckpt, seg
        return UK

    @staticmethod
    def backward(ctx, gU):
        lam = ctx.rec.backward(gU, ctx.log, ctx.ckpt, ctx.seg)
        return lam, None, None, None, None
