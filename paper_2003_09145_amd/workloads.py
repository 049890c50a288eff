"""Seeded synthetic inputs: problem descriptions and initial conditions.

This module holds no part of the numerical method.  It only builds problem
descriptions and conserved-variable fields (component order rho, rho*u_x,
[rho*u_y], [rho*u_z], E; array shape (ndim + 2, nz, ny, nx)) from the initial
conditions of Peng et al. (arXiv:2003.09145, Sec. 4) and the synthetic
workloads derived from them.  Both the GPU path and its CPU checker consume
these arrays.

Cell centres are x_i = x0 + (i + 1/2) dx; a point exactly on an initial
discontinuity takes the left / lower state (the "x <= 0" convention of
eq 4.8).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Side:
    """One end of an axis.  Ghost cells take kind_a where the split coordinate
    (the cell centre (i + 1/2) dx along split_axis, measured from the grid's
    low corner, on the boundary line) lies below split0 + split_rate * t, and
    kind_b elsewhere; split_axis = -1 means kind_a everywhere.  Kinds:
    "periodic", "transmissive", "reflective", "fixed" (the conserved state
    state_a / state_b)."""
    kind_a: str
    kind_b: Optional[str] = None
    split_axis: int = -1
    split0: float = 0.0
    split_rate: float = 0.0
    state_a: Optional[Sequence[float]] = None
    state_b: Optional[Sequence[float]] = None


@dataclasses.dataclass
class Boundary:
    """Per-end boundaries sides[axis][0 low / 1 high], a gravity source
    (momentum += rho g, energy += m . g) and the time of RHS evaluations."""
    sides: list
    gravity: Sequence[float] = (0.0, 0.0, 0.0)
    time: float = 0.0


@dataclasses.dataclass
class Problem:
    """Grid, gas and scheme parameters of one Euler problem."""
    ndim: int
    n: List[int]
    dx: List[float]
    bc: List[str]
    gamma: float = 1.4
    scheme: str = "lad"          # "lad", "fixed_ct", "linear5", "teno5a"
    ct_fixed: float = 1e-7       # C_T of the fixed-cutoff TENO5 (Sec. 4 default)
    H: float = 10.0              # LAD parameters (Sec. 4)
    Bl: int = 4
    Bu: int = 10
    theta: str = "printed"       # LAD sensor of eq 3.2: "printed", or "cut" (0 above H)
    eps: float = 1e-6            # epsilon of eq 2.8 (Sec. 2)
    a1: float = 10.5             # TENO5-A parameters (eq 2.16-2.18, Sec. 4 defaults)
    a2: float = 3.5
    cr: float = 0.25
    xi: float = 1e-3
    x0: List[float] = dataclasses.field(default_factory=lambda: [0.0, 0.0, 0.0])
    boundary: Optional[Boundary] = None   # per-end boundaries and gravity (Sec. 4.3)

    @property
    def nc(self) -> int:
        return self.ndim + 2

    @property
    def shape(self):
        n = list(self.n) + [1, 1, 1]
        return (self.nc, n[2] if self.ndim > 2 else 1, n[1] if self.ndim > 1 else 1, n[0])

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n[: self.ndim]))

    def centres(self, axis: int) -> np.ndarray:
        return self.x0[axis] + (np.arange(self.n[axis]) + 0.5) * self.dx[axis]

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def uniform_problem(ndim, n, lo, hi, bc, **kw) -> Problem:
    n = list(n)
    dx = [(hi[k] - lo[k]) / n[k] for k in range(ndim)]
    if isinstance(bc, str):
        bc = [bc] * ndim
    return Problem(ndim=ndim, n=n, dx=dx, bc=list(bc), x0=list(lo) + [0.0] * (3 - ndim), **kw)


def conserved(rho, vel: Sequence, p, gamma: float) -> np.ndarray:
    """Stack (rho, rho*u_k..., E) with E = p/(gamma-1) + rho |u|^2 / 2 (eq 4.7)."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    ke = sum(v * v for v in vel)
    E = p / (gamma - 1.0) + 0.5 * rho * ke
    return np.stack([rho] + [rho * v for v in vel] + [E])


def _as_field(prob: Problem, U: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(U.reshape(prob.shape), dtype=np.float64)


# --------------------------------------------------------------------------
# 1D Riemann problems of Sec. 4.2
# --------------------------------------------------------------------------
def riemann_1d(prob: Problem, left, right, x_split: float) -> np.ndarray:
    x = prob.centres(0)
    isl = x <= x_split
    rho = np.where(isl, left[0], right[0])
    u = np.where(isl, left[1], right[1])
    p = np.where(isl, left[2], right[2])
    return _as_field(prob, conserved(rho, [u], p, prob.gamma))


SOD_LEFT = (1.0, 0.0, 1.0)          # eq 4.8
SOD_RIGHT = (0.125, 0.0, 0.1)
LAX_LEFT = (0.445, 0.698, 3.528)    # eq 4.9
LAX_RIGHT = (0.5, 0.0, 0.571)


def sod(N: int = 200, **kw):
    """Sod tube on [0, 1], split at 0.5, zero-gradient ends."""
    prob = uniform_problem(1, [N], [0.0], [1.0], "transmissive", **kw)
    return prob, riemann_1d(prob, SOD_LEFT, SOD_RIGHT, 0.5)


def sod_paper(N: int = 400, **kw):
    """Sod tube as printed in Sec. 4.2: [-0.5, 0.5], split at 0."""
    prob = uniform_problem(1, [N], [-0.5], [0.5], "transmissive", **kw)
    return prob, riemann_1d(prob, SOD_LEFT, SOD_RIGHT, 0.0)


def lax(N: int = 400, **kw):
    prob = uniform_problem(1, [N], [-5.0], [5.0], "transmissive", **kw)
    return prob, riemann_1d(prob, LAX_LEFT, LAX_RIGHT, 0.0)


SHU_OSHER_POST = (27.0 / 7.0, 4.0 * math.sqrt(35.0) / 9.0, 31.0 / 3.0)  # eq 4.10


def shu_osher(N: int = 400, noise: float = 0.0, seed: int = 2, **kw):
    """Mach-3 shock at x = -4 meeting rho = 1 + 0.2 sin 5x (eq 4.10);
    optional seeded Gaussian density noise ahead of the shock."""
    prob = uniform_problem(1, [N], [-5.0], [5.0], "transmissive", **kw)
    x = prob.centres(0)
    pre = x >= -4.0
    rho = np.where(pre, 1.0 + 0.2 * np.sin(5.0 * x), SHU_OSHER_POST[0])
    if noise:
        rng = np.random.default_rng(seed)
        rho = rho + np.where(pre, noise * rng.standard_normal(N), 0.0)
    u = np.where(pre, 0.0, SHU_OSHER_POST[1])
    p = np.where(pre, 1.0, SHU_OSHER_POST[2])
    return prob, _as_field(prob, conserved(rho, [u], p, prob.gamma))


def blast_waves(N: int = 400, **kw):
    """Two interacting blast waves (eq 4.11, middle interval read as
    0.1 <= x < 0.9), reflecting walls."""
    prob = uniform_problem(1, [N], [0.0], [1.0], "reflective", **kw)
    x = prob.centres(0)
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    return prob, _as_field(prob, conserved(np.ones(N), [np.zeros(N)], p, prob.gamma))


def adjoint_case(N: int = 2048, noise: float = 0.01, seed: int = 2, **kw):
    """Shu-Osher initial state with seeded density noise (sigma = noise)."""
    return shu_osher(N, noise=noise, seed=seed, **kw)


# --------------------------------------------------------------------------
# 2D four-quadrant Riemann problems (Sec. 4.3)
# --------------------------------------------------------------------------
RIEMANN2D_CONFIG3 = {  # eq 4.14: (rho, u, v, p) for NE, NW, SW, SE
    "NE": (1.5, 0.0, 0.0, 1.5), "NW": (0.5323, 1.206, 0.0, 0.3),
    "SW": (0.138, 1.206, 1.206, 0.029), "SE": (0.5323, 0.0, 1.206, 0.3)}
RIEMANN2D_CONFIG12 = {  # eq 4.13
    "NE": (0.5313, 0.0, 0.0, 0.4), "NW": (1.0, 0.7276, 0.0, 1.0),
    "SW": (0.8, 0.0, 0.0, 1.0), "SE": (1.0, 0.0, 0.7276, 1.0)}


def riemann_2d(n: int = 2048, states=RIEMANN2D_CONFIG3, split=(0.8, 0.8), ny=None, **kw):
    ny = n if ny is None else ny
    prob = uniform_problem(2, [n, ny], [0.0, 0.0], [1.0, 1.0], "transmissive", **kw)
    x = prob.centres(0)[None, :]
    y = prob.centres(1)[:, None]
    east = x > split[0]
    north = y > split[1]
    out = np.empty((4, ny, n))
    for q, (e, nn) in {"NE": (True, True), "NW": (False, True),
                       "SW": (False, False), "SE": (True, False)}.items():
        m = (east == e) & (north == nn)
        for c in range(4):
            out[c][m] = states[q][c]
    U = conserved(out[0], [out[1], out[2]], out[3], prob.gamma)
    return prob, _as_field(prob, U)


def riemann_2d_table2(case: int, n: int = 1024, **kw):
    """The 2D Riemann problems timed in Table 2: case 1 = eq 4.14
    (configuration 3), case 2 = eq 4.13 (configuration 12), quadrants split
    at (0.5, 0.5) on [0, 1]^2, transmissive."""
    states = RIEMANN2D_CONFIG3 if case == 1 else RIEMANN2D_CONFIG12
    return riemann_2d(n, states=states, split=(0.5, 0.5), **kw)


# --------------------------------------------------------------------------
# Rayleigh-Taylor instability (Sec. 4.3, eq 4.12) and double Mach reflection
# --------------------------------------------------------------------------
def rayleigh_taylor(nx: int = 128, ny: int = 512, gamma: float = 5.0 / 3.0, **kw):
    """[0, 0.25] x [0, 1], heavy fluid below y = 1/2, v perturbed by
    -0.025 c cos(8 pi x) (c the sound speed), gravity source (0, 1) on
    (rho v, E) as (rho, rho v); reflective left / right, fixed states
    (rho, u, v, p) = (2, 0, 0, 1) below and (1, 0, 0, 2.5) above."""
    prob = uniform_problem(2, [nx, ny], [0.0, 0.0], [0.25, 1.0], "reflective", gamma=gamma, **kw)
    x = prob.centres(0)[None, :]
    y = prob.centres(1)[:, None]
    low = y < 0.5
    rho = np.where(low, 2.0, 1.0) + 0.0 * x
    p = np.where(low, 2.0 * y + 1.0, y + 1.5) + 0.0 * x
    c = np.sqrt(gamma * p / rho)
    v = -0.025 * c * np.cos(8.0 * math.pi * x)
    U = conserved(rho, [np.zeros_like(rho), v], p, gamma)
    bottom = conserved(2.0, [0.0, 0.0], 1.0, gamma).tolist()
    top = conserved(1.0, [0.0, 0.0], 2.5, gamma).tolist()
    bnd = Boundary(sides=[[Side("reflective"), Side("reflective")],
                          [Side("fixed", state_a=bottom), Side("fixed", state_a=top)],
                          [Side("periodic"), Side("periodic")]],
                   gravity=(0.0, 1.0, 0.0))
    prob = prob.replace(boundary=bnd)
    return prob, _as_field(prob, U)


DMR_PRE = (1.4, 0.0, 0.0, 1.0)   # (rho, u, v, p) ahead of the Mach-10 shock
DMR_POST = (8.0, 8.25 * math.cos(math.pi / 6.0), -8.25 * math.sin(math.pi / 6.0), 116.5)


def double_mach(nx: int = 1024, ny: int = 256, **kw):
    """[0, 4] x [0, 1]: a Mach-10 shock inclined at 60 degrees through
    (1/6, 0) moving right; reflecting wall from x = 1/6 on the bottom (fixed
    post-shock state before it), post-shock inflow on the left, zero-gradient
    outflow on the right, and a top boundary that follows the exact shock
    position x = 1/6 + (1 + 20 t) / sqrt(3)."""
    prob = uniform_problem(2, [nx, ny], [0.0, 0.0], [4.0, 1.0], "transmissive", **kw)
    g = prob.gamma
    x = prob.centres(0)[None, :]
    y = prob.centres(1)[:, None]
    post = x < 1.0 / 6.0 + y / math.sqrt(3.0)
    prim = [np.where(post, DMR_POST[k], DMR_PRE[k]) for k in range(4)]
    U = conserved(prim[0], [prim[1], prim[2]], prim[3], g)
    s_post = conserved(DMR_POST[0], [DMR_POST[1], DMR_POST[2]], DMR_POST[3], g).tolist()
    s_pre = conserved(DMR_PRE[0], [DMR_PRE[1], DMR_PRE[2]], DMR_PRE[3], g).tolist()
    r3 = math.sqrt(3.0)
    bnd = Boundary(sides=[
        [Side("fixed", state_a=s_post), Side("transmissive")],
        [Side("fixed", "reflective", split_axis=0, split0=1.0 / 6.0, state_a=s_post),
         Side("fixed", "fixed", split_axis=0, split0=1.0 / 6.0 + 1.0 / r3, split_rate=20.0 / r3,
              state_a=s_post, state_b=s_pre)],
        [Side("periodic"), Side("periodic")]])
    prob = prob.replace(boundary=bnd)
    return prob, _as_field(prob, U)


# --------------------------------------------------------------------------
# 3D periodic compressible turbulence (throughput workload)
# --------------------------------------------------------------------------
def turbulence_3d(n: int = 256, seed: int = 0, k0: float = 4.0, mach_t: float = 0.6,
                  u_rms: float = 1.0, **kw):
    """Periodic box [0, 2 pi]^3: rho = 1, p = 1 / (gamma Mt^2), solenoidal
    random-phase velocity with E(k) ~ k^4 exp(-2 k^2 / k0^2), scaled so that
    sqrt(<u.u>) = u_rms."""
    L = 2.0 * math.pi
    prob = uniform_problem(3, [n, n, n], [0.0] * 3, [L] * 3, "periodic", **kw)
    rng = np.random.default_rng(seed)
    k1 = np.fft.fftfreq(n, d=1.0 / n).astype(np.float64)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    kmag = np.sqrt(k2)
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.sqrt(kmag ** 4 * np.exp(-2.0 * k2 / (k0 * k0)) / (4.0 * math.pi * k2))
    amp[0, 0, 0] = 0.0
    comps = []
    for _ in range(3):
        comps.append(rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n)))
    inv_k2 = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    kdot = (kx * comps[0] + ky * comps[1] + kz * comps[2]) * inv_k2
    vel = []
    for c, kc in zip(comps, (kx, ky, kz)):
        hat = (c - kc * kdot) * amp
        vel.append(np.real(np.fft.ifftn(hat)))
        del hat
    del comps, kdot
    scale = u_rms / math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vel = [v * scale for v in vel]
    p = 1.0 / (prob.gamma * mach_t * mach_t)
    U = conserved(np.ones((n, n, n)), vel, np.full((n, n, n), p), prob.gamma)
    return prob, _as_field(prob, U)


# --------------------------------------------------------------------------
# Batched ragged 1D shock tubes
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Batch:
    """Packed ragged batch: U[c, offsets[b] + i] for tube b, cell i."""
    lengths: np.ndarray   # int64 [nb]
    offsets: np.ndarray   # int64 [nb + 1]
    dx: np.ndarray        # float64 [nb]
    U: np.ndarray         # float64 [3, total]
    gamma: float = 1.4

    @property
    def nbatch(self) -> int:
        return len(self.lengths)

    def tube(self, b: int) -> np.ndarray:
        o0, o1 = self.offsets[b], self.offsets[b + 1]
        return self.U[:, o0:o1].reshape(3, 1, 1, o1 - o0)

    def tube_problem(self, b: int, **kw) -> Problem:
        N = int(self.lengths[b])
        return Problem(ndim=1, n=[N], dx=[float(self.dx[b])], bc=["transmissive"],
                       gamma=self.gamma, **kw)


def batched_tubes(count: int = 4096, nmin: int = 128, nmax: int = 4096, seed: int = 1,
                  gamma: float = 1.4) -> Batch:
    """Sod-type tubes on [0, 1] with N log-uniform in [nmin, nmax] and seeded
    random left/right states rho in [0.1, 1], u in [-1, 1], p in [0.1, 1],
    interface at 0.5."""
    rng = np.random.default_rng(seed)
    lengths = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(np.int64)
    states = np.stack([rng.uniform(0.1, 1.0, (count, 2)), rng.uniform(-1.0, 1.0, (count, 2)),
                       rng.uniform(0.1, 1.0, (count, 2))], axis=-1)  # [b, side, (rho,u,p)]
    offsets = np.zeros(count + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    U = np.empty((3, int(offsets[-1])))
    dx = 1.0 / lengths.astype(np.float64)
    for b in range(count):
        N = int(lengths[b])
        x = (np.arange(N) + 0.5) * dx[b]
        left = x <= 0.5
        rho = np.where(left, states[b, 0, 0], states[b, 1, 0])
        u = np.where(left, states[b, 0, 1], states[b, 1, 1])
        p = np.where(left, states[b, 0, 2], states[b, 1, 2])
        U[:, offsets[b]:offsets[b + 1]] = conserved(rho, [u], p, gamma)
    return Batch(lengths=lengths, offsets=offsets, dx=dx, U=U, gamma=gamma)


# --------------------------------------------------------------------------
# Smooth test fields and random parity inputs
# --------------------------------------------------------------------------
def entropy_wave(ndim: int, n: int, t: float = 0.0, amp: float = 0.2, **kw):
    """rho = 1 + amp sin(2 pi (s - ndim t)) with s the sum of the coordinates,
    velocity 1 along every axis, p = 1, periodic unit box (exact solution:
    translation along the diagonal)."""
    prob = uniform_problem(ndim, [n] * ndim, [0.0] * ndim, [1.0] * ndim, "periodic", **kw)
    grids = np.meshgrid(*[prob.centres(k) for k in reversed(range(ndim))], indexing="ij")
    coords = list(reversed(grids))  # x, y, z
    s = sum(coords)
    rho = 1.0 + amp * np.sin(2.0 * math.pi * (s - ndim * t))
    vel = [np.ones_like(rho) for _ in range(ndim)]
    U = conserved(rho, vel, np.ones_like(rho), prob.gamma)
    return prob, _as_field(prob, U)


def contact(ndim: int, n: Sequence, rho=(1.0, 0.3), vel=(0.4, -0.3, 0.2), p: float = 1.0,
            bc="periodic", **kw):
    """Oblique contact discontinuity in the unit box: density rho[0] where the
    sum of the cell-centre coordinates is below ndim / 2, rho[1] elsewhere;
    uniform velocity (the first ndim entries of vel) and pressure.  The jump
    in U and in each directional flux is a multiple of the entropy
    eigenvector (1, u, v, w, |u|^2 / 2), which is the same in every direction,
    so only the entropy field sees it."""
    prob = uniform_problem(ndim, list(n), [0.0] * ndim, [1.0] * ndim, bc, **kw)
    grids = np.meshgrid(*[prob.centres(k) for k in reversed(range(ndim))], indexing="ij")
    s = sum(reversed(grids))
    r = np.where(s < 0.5 * ndim, rho[0], rho[1])
    U = conserved(r, [np.full_like(r, vel[k]) for k in range(ndim)], np.full_like(r, p),
                  prob.gamma)
    return prob, _as_field(prob, U)


def random_field(prob: Problem, seed: int = 4, jumps: int = 3, modes: int = 4,
                 amp: float = 0.3) -> np.ndarray:
    """Positive-density, positive-pressure field: a few random Fourier modes
    plus random planar jumps.  Deterministic in (shape, seed)."""
    rng = np.random.default_rng(seed)
    nd = prob.ndim
    axes = [np.linspace(0.0, 1.0, prob.n[k], endpoint=False) for k in range(nd)]
    grids = np.meshgrid(*list(reversed(axes)), indexing="ij")
    coords = list(reversed(grids))
    shape = grids[0].shape

    def smooth(base, a):
        f = np.full(shape, base)
        for _ in range(modes):
            kv = rng.integers(1, 4, nd)
            ph = rng.uniform(0, 2 * math.pi)
            f = f + a * rng.uniform(-1, 1) * np.sin(2 * math.pi * sum(k * c for k, c in zip(kv, coords)) + ph)
        return f

    rho = smooth(1.0, amp / modes)
    p = smooth(1.0, amp / modes)
    vel = [smooth(0.0, 0.5 / modes) for _ in range(nd)]
    for _ in range(jumps):
        normal = rng.normal(size=nd)
        off = rng.uniform(0.2, 0.8) * float(np.sum(np.abs(normal)))
        side = sum(nv * c for nv, c in zip(normal, coords)) > off - 0.5 * float(np.sum(normal))
        rho = np.where(side, rho * rng.uniform(0.2, 2.0), rho)
        p = np.where(side, p * rng.uniform(0.2, 2.0), p)
        for k in range(nd):
            vel[k] = np.where(side, vel[k] + rng.uniform(-0.5, 0.5), vel[k])
    U = conserved(rho, vel, p, prob.gamma)
    return _as_field(prob, U)
