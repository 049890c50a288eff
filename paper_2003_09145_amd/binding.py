"""Thin ctypes binding of libteno.so (include/teno.h).

Argument marshalling only: every step of the numerical path runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors) and the
stream.  Loading fails loudly when the library has not been built; there is
no CPU fallback.

Fields are float64 CUDA tensors of shape (ndim + 2, nz, ny, nx) (unused axes
of size 1), component order rho, rho*u_x, [rho*u_y], [rho*u_z], E.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libteno.so")

OK, ERR_ARG, ERR_DEVICE, ERR_NONPHYSICAL = 0, 1, 2, 3
BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
BC_FIXED = 3
SCHEME = {"lad": 0, "fixed_ct": 1, "linear5": 2, "teno5a": 3}
# teno_grid.theta: the LAD sensor of eq 3.2 as printed, or cut to 0 above H
THETA = {"printed": 0, "cut": 1}


class TenoSide(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32 * 2),
        ("split_axis", ctypes.c_int32),
        ("reserved_", ctypes.c_int32),
        ("split", ctypes.c_double * 2),
        ("state", ctypes.c_double * 10),
    ]


class TenoBoundary(ctypes.Structure):
    _fields_ = [
        ("side", TenoSide * 6),   # [axis][end]
        ("gravity", ctypes.c_double * 3),
        ("t_rhs", ctypes.c_double),
    ]


class TenoGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("bc", ctypes.c_int32 * 3),
        ("scheme", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("ct_fixed", ctypes.c_double),
        ("H", ctypes.c_double),
        ("Bl", ctypes.c_int32),
        ("Bu", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("flags", ctypes.c_int32),
        ("theta", ctypes.c_int32),
        ("a1", ctypes.c_double),
        ("a2", ctypes.c_double),
        ("cr", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("boundary_dev", ctypes.c_void_p),
    ]


FLAG_LITERAL_DECISIONS = 1
FLAG_MASK_DIGEST = 2


class TenoCtrl(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("t_end", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("alpha", (ctypes.c_double * 3) * 3),
        ("status", ctypes.c_int32),
        ("replay", ctypes.c_int32),
        ("nsteps", ctypes.c_int64),
        ("active", ctypes.c_int32),
        ("want_digest", ctypes.c_int32),
        ("digest", ctypes.c_uint64),
        ("reserved_", ctypes.c_uint64 * 2),
    ]


CTRL_BYTES = ctypes.sizeof(TenoCtrl)
assert CTRL_BYTES == 152

# Every symbol declared in include/teno.h (checked by the ABI tests).
SYMBOLS = ["teno_workspace_bytes", "teno_ctrl_init", "teno_ctrl_replay", "teno_ctrl_digest",
           "teno_rhs", "teno_rhs_noalloc", "teno_rhs_debug", "teno_sweep",
           "teno_selftest_arith", "teno_step", "teno_step_timed",
           "teno_runner_create", "teno_runner_run", "teno_runner_destroy",
           "teno_adjoint_workspace_bytes", "teno_rhs_adjoint", "teno_step_adjoint",
           "teno_advect_workspace_bytes", "teno_advect_rhs", "teno_advect_step",
           "teno_batch_plan_create", "teno_batch_plan_destroy", "teno_batch_total_cells",
           "teno_batch_init", "teno_batch_step", "teno_batch_run", "teno_batch_autotune",
           "teno_batch_get_config", "teno_batch_set_config", "teno_batch_read"]

_lib = None


class TenoError(RuntimeError):
    pass


def lib():
    """Load libteno.so (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TenoError(f"{LIB_PATH} is missing: build it with "
                            "`python paper_2003_09145_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        G = ctypes.POINTER(TenoGrid)
        L.teno_workspace_bytes.argtypes = [G]
        L.teno_workspace_bytes.restype = ctypes.c_size_t
        L.teno_ctrl_init.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]
        L.teno_ctrl_init.restype = ctypes.c_int
        L.teno_ctrl_replay.argtypes = [vp, vp, vp]
        L.teno_ctrl_replay.restype = ctypes.c_int
        L.teno_ctrl_digest.argtypes = [vp, ctypes.c_int32, vp]
        L.teno_ctrl_digest.restype = ctypes.c_int
        L.teno_rhs.argtypes = [G, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.teno_rhs.restype = ctypes.c_int
        L.teno_rhs_noalloc.argtypes = [G, vp, vp, vp, vp, vp, vp]
        L.teno_rhs_noalloc.restype = ctypes.c_int
        L.teno_rhs_debug.argtypes = [G, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.teno_rhs_debug.restype = ctypes.c_int
        L.teno_sweep.argtypes = [G, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.teno_sweep.restype = ctypes.c_int
        L.teno_selftest_arith.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp]
        L.teno_selftest_arith.restype = ctypes.c_int
        L.teno_step.argtypes = [G, vp, vp, vp, ctypes.c_size_t, vp]
        L.teno_step.restype = ctypes.c_int
        L.teno_step_timed.argtypes = [G, vp, vp, vp, ctypes.c_size_t, vp, vp]
        L.teno_step_timed.restype = ctypes.c_int
        L.teno_runner_create.argtypes = [G, vp, vp, vp, ctypes.c_size_t, ctypes.c_int32,
                                         ctypes.POINTER(vp)]
        L.teno_runner_create.restype = ctypes.c_int
        L.teno_runner_run.argtypes = [vp, ctypes.c_int64, vp]
        L.teno_runner_run.restype = ctypes.c_int
        L.teno_runner_destroy.argtypes = [vp]
        L.teno_runner_destroy.restype = ctypes.c_int
        L.teno_adjoint_workspace_bytes.argtypes = [G]
        L.teno_adjoint_workspace_bytes.restype = ctypes.c_size_t
        L.teno_rhs_adjoint.argtypes = [G, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.teno_rhs_adjoint.restype = ctypes.c_int
        L.teno_step_adjoint.argtypes = [G, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.teno_step_adjoint.restype = ctypes.c_int
        L.teno_advect_workspace_bytes.argtypes = [G]
        L.teno_advect_workspace_bytes.restype = ctypes.c_size_t
        L.teno_advect_rhs.argtypes = [G, vp, vp, vp]
        L.teno_advect_rhs.restype = ctypes.c_int
        L.teno_advect_step.argtypes = [G, vp, ctypes.c_double, vp, ctypes.c_size_t, vp]
        L.teno_advect_step.restype = ctypes.c_int
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        P = ctypes.c_void_p
        L.teno_batch_plan_create.argtypes = [G, i64, ctypes.POINTER(i64), ctypes.POINTER(dbl), dbl,
                                             dbl, ctypes.c_char_p, ctypes.POINTER(P)]
        L.teno_batch_plan_create.restype = ctypes.c_int
        L.teno_batch_plan_destroy.argtypes = [P]
        L.teno_batch_plan_destroy.restype = ctypes.c_int
        L.teno_batch_total_cells.argtypes = [P]
        L.teno_batch_total_cells.restype = i64
        L.teno_batch_init.argtypes = [P, vp, vp]
        L.teno_batch_init.restype = ctypes.c_int
        L.teno_batch_step.argtypes = [P, vp, vp]
        L.teno_batch_step.restype = ctypes.c_int
        L.teno_batch_run.argtypes = [P, vp, i64, vp]
        L.teno_batch_run.restype = ctypes.c_int
        L.teno_batch_autotune.argtypes = [P, vp, i32, ctypes.c_char_p, ctypes.POINTER(dbl)]
        L.teno_batch_autotune.restype = ctypes.c_int
        L.teno_batch_get_config.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.teno_batch_get_config.restype = ctypes.c_int
        L.teno_batch_set_config.argtypes = [P, i32, i32]
        L.teno_batch_set_config.restype = ctypes.c_int
        L.teno_batch_read.argtypes = [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                      ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.teno_batch_read.restype = ctypes.c_int
        _lib = L
    return _lib


def _get(prob, key, default=None):
    if isinstance(prob, dict):
        return prob.get(key, default)
    return getattr(prob, key, default)


def grid(prob) -> TenoGrid:
    """teno_grid from a problem description (attributes or dict keys ndim, n,
    dx, bc, gamma, scheme, ct_fixed, H, Bl, Bu, eps, a1, a2, cr, xi)."""
    g = TenoGrid()
    nd = int(_get(prob, "ndim"))
    n = list(_get(prob, "n"))
    dx = list(_get(prob, "dx"))
    bc = _get(prob, "bc")
    if isinstance(bc, (str, int)):
        bc = [bc] * nd
    g.ndim = nd
    for k in range(3):
        g.n[k] = int(n[k]) if k < nd else 1
        g.dx[k] = float(dx[k]) if k < nd else 1.0
        b = bc[k] if k < nd else 0
        g.bc[k] = BC[b] if isinstance(b, str) else int(b)
    sch = _get(prob, "scheme", "lad")
    g.scheme = SCHEME[sch] if isinstance(sch, str) else int(sch)
    g.gamma = float(_get(prob, "gamma", 1.4))
    g.ct_fixed = float(_get(prob, "ct_fixed", 1e-7))
    g.H = float(_get(prob, "H", 10.0))
    g.Bl = int(_get(prob, "Bl", 4))
    g.Bu = int(_get(prob, "Bu", 10))
    g.eps = float(_get(prob, "eps", 1e-6))
    g.a1 = float(_get(prob, "a1", 10.5))
    g.a2 = float(_get(prob, "a2", 3.5))
    g.cr = float(_get(prob, "cr", 0.25))
    g.xi = float(_get(prob, "xi", 1e-3))
    th = _get(prob, "theta", "printed")
    g.theta = THETA[th] if isinstance(th, str) else int(th)
    g.flags = ((FLAG_LITERAL_DECISIONS if _get(prob, "literal_decisions", False) else 0) |
               (FLAG_MASK_DIGEST if _get(prob, "mask_digest", False) else 0))
    bnd = _get(prob, "boundary", None)
    if bnd is not None:
        g.boundary_buf = boundary_device(bnd)   # keeps the device copy alive
        g.boundary_dev = g.boundary_buf.data_ptr()
    return g


def boundary_struct(bnd) -> TenoBoundary:
    """teno_boundary from a workloads.Boundary description."""
    kinds = dict(BC, fixed=BC_FIXED)
    b = TenoBoundary()
    for d in range(3):
        for e in range(2):
            sd = bnd.sides[d][e]
            o = b.side[d * 2 + e]
            o.kind[0] = kinds[sd.kind_a]
            o.kind[1] = kinds[sd.kind_b] if sd.kind_b is not None else o.kind[0]
            o.split_axis = int(sd.split_axis)
            o.split[0] = float(sd.split0)
            o.split[1] = float(sd.split_rate)
            for w, st in enumerate((sd.state_a, sd.state_b)):
                if st is not None:
                    for q, v in enumerate(st):
                        o.state[w * 5 + q] = float(v)
    for k in range(3):
        b.gravity[k] = float(bnd.gravity[k])
    b.t_rhs = float(bnd.time)
    return b


def boundary_device(bnd, device="cuda"):
    """The teno_boundary of a description in a device uint8 tensor."""
    import torch
    host = bytes(boundary_struct(bnd))
    return torch.frombuffer(bytearray(host), dtype=torch.uint8).to(device)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, what):
    if rc != OK:
        raise TenoError(f"{what} failed with status {rc}")


def workspace_bytes(g: TenoGrid) -> int:
    return int(lib().teno_workspace_bytes(ctypes.byref(g)))


def ctrl_init(ctrl, t0, t_end, cfl, stream=None):
    _check(lib().teno_ctrl_init(_ptr(ctrl), float(t0), float(t_end), float(cfl), _stream(stream)),
           "teno_ctrl_init")


def ctrl_replay(ctrl, recorded, stream=None):
    _check(lib().teno_ctrl_replay(_ptr(ctrl), _ptr(recorded), _stream(stream)), "teno_ctrl_replay")


def ctrl_digest(ctrl, enable=True, stream=None):
    _check(lib().teno_ctrl_digest(_ptr(ctrl), 1 if enable else 0, _stream(stream)),
           "teno_ctrl_digest")


def teno_rhs(g, U, dUdt, ws, alpha_in=None, alpha_out=None, status=None, stream=None):
    _check(lib().teno_rhs(ctypes.byref(g), _ptr(U), _ptr(dUdt), _ptr(alpha_in), _ptr(alpha_out),
                          _ptr(status), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "teno_rhs")


def teno_rhs_noalloc(g, U, dUdt, alpha_in=None, alpha_out=None, status=None, stream=None):
    _check(lib().teno_rhs_noalloc(ctypes.byref(g), _ptr(U), _ptr(dUdt), _ptr(alpha_in),
                                  _ptr(alpha_out), _ptr(status), _stream(stream)),
           "teno_rhs_noalloc")


def teno_rhs_debug(g, U, dUdt, decisions, ws, alpha_in=None, alpha_out=None, status=None,
                   stream=None):
    _check(lib().teno_rhs_debug(ctypes.byref(g), _ptr(U), _ptr(dUdt), _ptr(alpha_in),
                                _ptr(alpha_out), _ptr(status), _ptr(decisions), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)),
           "teno_rhs_debug")


def teno_sweep(g, axis, U, Rout, alpha, Rin=None, stream=None):
    _check(lib().teno_sweep(ctypes.byref(g), int(axis), _ptr(U), _ptr(Rin), _ptr(Rout),
                            _ptr(alpha), _stream(stream)), "teno_sweep")


def selftest_arith(a, b, stream=None, plain=False):
    """(a / b, a / b via the reciprocal route, sqrt(a), approximate 1 / b)
    computed by the device; with plain=True also the compiler's uncorrected
    a / b and sqrt(a)."""
    import torch
    q, q2, s, r = (torch.empty_like(a) for _ in range(4))
    qp, sp = (torch.empty_like(a), torch.empty_like(a)) if plain else (None, None)
    _check(lib().teno_selftest_arith(_ptr(a), _ptr(b), _ptr(q), _ptr(q2), _ptr(s), _ptr(r),
                                     _ptr(qp), _ptr(sp), a.numel(), _stream(stream)),
           "teno_selftest_arith")
    return (q, q2, s, r, qp, sp) if plain else (q, q2, s, r)


def teno_step(g, U, ctrl, ws, stream=None):
    _check(lib().teno_step(ctypes.byref(g), _ptr(U), _ptr(ctrl), _ptr(ws),
                           ws.numel() * ws.element_size(), _stream(stream)), "teno_step")


def teno_step_timed(g, U, ctrl, ws, events, stream=None):
    """teno_step recording events[2 * (ndim * s + d)] / [... + 1] (torch.cuda.Event
    objects, already recorded once so that they exist) around the sweep of
    axis d in stage s."""
    n = 2 * 3 * g.ndim
    if len(events) != n:
        raise TenoError(f"teno_step_timed needs {n} events")
    arr = (ctypes.c_void_p * n)(*[e.cuda_event for e in events])
    _check(lib().teno_step_timed(ctypes.byref(g), _ptr(U), _ptr(ctrl), _ptr(ws),
                                 ws.numel() * ws.element_size(), arr, _stream(stream)),
           "teno_step_timed")


def adjoint_workspace_bytes(g: TenoGrid) -> int:
    return int(lib().teno_adjoint_workspace_bytes(ctypes.byref(g)))


def teno_rhs_adjoint(g, U, alpha, lam, gradU, ws, stream=None):
    _check(lib().teno_rhs_adjoint(ctypes.byref(g), _ptr(U), _ptr(alpha), _ptr(lam), _ptr(gradU),
                                  _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "teno_rhs_adjoint")


def teno_step_adjoint(g, Un, ctrl, lam, ws, stream=None):
    _check(lib().teno_step_adjoint(ctypes.byref(g), _ptr(Un), _ptr(ctrl), _ptr(lam), _ptr(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)),
           "teno_step_adjoint")


def advect_grid(n: int, dx: float, scheme="lad", **kw) -> TenoGrid:
    """Grid of the periodic scalar advection problem (Sec. 4.1)."""
    return grid(dict(ndim=1, n=[n], dx=[dx], bc="periodic", scheme=scheme, **kw))


def teno_advect_rhs(g, u, out, stream=None):
    _check(lib().teno_advect_rhs(ctypes.byref(g), _ptr(u), _ptr(out), _stream(stream)),
           "teno_advect_rhs")


def teno_advect_step(g, u, h, ws, stream=None):
    _check(lib().teno_advect_step(ctypes.byref(g), _ptr(u), float(h), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)),
           "teno_advect_step")


def advect_run(g, u, dt, t_end, stream=None):
    """Fixed steps dt until t_end, the last one shortened to end at t_end;
    returns the number of steps."""
    import torch
    ws = torch.empty(int(lib().teno_advect_workspace_bytes(ctypes.byref(g))), dtype=torch.uint8,
                     device=u.device)
    t = 0.0
    steps = 0
    while t < t_end:
        h = dt
        if t + h > t_end:
            h = t_end - t
        teno_advect_step(g, u, h, ws, stream)
        t = t + h
        steps += 1
    return steps


def decisions_bytes(g: TenoGrid) -> int:
    nc = g.ndim + 2
    ncell = g.n[0] * g.n[1] * g.n[2]
    return sum(ncell // g.n[d] * (g.n[d] + 1) * 2 * nc for d in range(g.ndim))


class Solver:
    """Owns the device workspace and control block of one grid."""

    def __init__(self, prob, device="cuda"):
        import torch
        self.g = grid(prob)
        nb = workspace_bytes(self.g)
        if nb == 0:
            raise TenoError("invalid grid")
        self.device = torch.device(device)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.ctrl = torch.zeros(CTRL_BYTES, dtype=torch.uint8, device=self.device)
        self.alpha = torch.zeros(3, dtype=torch.float64, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)

    def rhs(self, U, alpha_in=None, out=None, decisions=False):
        import torch
        out = torch.empty_like(U) if out is None else out
        if decisions:
            dec = torch.empty(decisions_bytes(self.g), dtype=torch.uint8, device=self.device)
            teno_rhs_debug(self.g, U, out, dec, self.ws, alpha_in, self.alpha, self.status)
            return out, dec
        teno_rhs(self.g, U, out, self.ws, alpha_in, self.alpha, self.status)
        return out

    def init(self, t0=0.0, t_end=float("inf"), cfl=0.5):
        ctrl_init(self.ctrl, t0, t_end, cfl)

    def step(self, U, events=None):
        if events is None:
            teno_step(self.g, U, self.ctrl, self.ws)
        else:
            teno_step_timed(self.g, U, self.ctrl, self.ws, events)

    def run(self, U, nsteps, steps_per_graph=10):
        """nsteps teno_step calls on U, replayed from a HIP graph of
        steps_per_graph steps (teno_runner; recorded on first use for this U)."""
        r = self._runners.get((U.data_ptr(), steps_per_graph)) if hasattr(self, "_runners") else None
        if r is None:
            self._runners = getattr(self, "_runners", {})
            r = Runner(self.g, U, self.ctrl, self.ws, steps_per_graph)
            self._runners[(U.data_ptr(), steps_per_graph)] = r
        r.run(nsteps)

    def read_ctrl(self) -> TenoCtrl:
        host = self.ctrl.cpu().numpy().tobytes()
        return TenoCtrl.from_buffer_copy(host)

    def write_ctrl(self, c: TenoCtrl):
        import torch
        buf = torch.frombuffer(bytearray(bytes(c)), dtype=torch.uint8)
        self.ctrl.copy_(buf.to(self.device))


class Runner:
    """A recorded run of steps_per_graph teno_step calls on fixed buffers
    (teno_runner); keeps references to the tensors it was recorded on."""

    def __init__(self, g, U, ctrl, ws, steps_per_graph=10):
        self.g, self.U, self.ctrl, self.ws = g, U, ctrl, ws
        h = ctypes.c_void_p()
        _check(lib().teno_runner_create(ctypes.byref(g), _ptr(U), _ptr(ctrl), _ptr(ws),
                                        ws.numel() * ws.element_size(), int(steps_per_graph),
                                        ctypes.byref(h)),
               "teno_runner_create")
        self.h = h

    def run(self, nsteps, stream=None):
        _check(lib().teno_runner_run(self.h, int(nsteps), _stream(stream)), "teno_runner_run")

    def close(self):
        if getattr(self, "h", None):
            lib().teno_runner_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """A batched ragged-1D plan (teno_batch_plan) over packed fields
    U[c, off_b + i] (float64 CUDA tensor of shape (3, total))."""

    def __init__(self, lengths, dx, prob=None, cfl=0.5, t_end=float("inf"), tune_cache=None):
        import numpy as np
        base = dict(ndim=1, n=[3], dx=[1.0], bc="transmissive")
        if prob is not None:
            base.update({k: v for k, v in (prob.items() if isinstance(prob, dict) else
                                            vars(prob).items()) if k not in ("ndim", "n", "dx")})
        self.g = grid(base)
        self.lengths = np.ascontiguousarray(lengths, dtype=np.int64)
        self.dx = np.ascontiguousarray(dx, dtype=np.float64)
        self.nb = len(self.lengths)
        self.tune_cache = None if tune_cache is None else str(tune_cache).encode()
        h = ctypes.c_void_p()
        _check(lib().teno_batch_plan_create(
            ctypes.byref(self.g), self.nb,
            self.lengths.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            self.dx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(cfl), float(t_end),
            self.tune_cache, ctypes.byref(h)), "teno_batch_plan_create")
        self.h = h
        self.total = int(lib().teno_batch_total_cells(h))

    def close(self):
        if getattr(self, "h", None):
            lib().teno_batch_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, U, stream=None):
        _check(lib().teno_batch_init(self.h, _ptr(U), _stream(stream)), "teno_batch_init")

    def step(self, U, stream=None):
        _check(lib().teno_batch_step(self.h, _ptr(U), _stream(stream)), "teno_batch_step")

    def run(self, U, nsteps, stream=None):
        _check(lib().teno_batch_run(self.h, _ptr(U), int(nsteps), _stream(stream)), "teno_batch_run")

    def autotune(self, U, steps=3):
        ms = ctypes.c_double()
        _check(lib().teno_batch_autotune(self.h, _ptr(U), int(steps), self.tune_cache,
                                         ctypes.byref(ms)), "teno_batch_autotune")
        return ms.value

    def config(self):
        w, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().teno_batch_get_config(self.h, ctypes.byref(w), ctypes.byref(b)),
               "teno_batch_get_config")
        return w.value, b.value

    def set_config(self, waves, blocks_per_cu):
        _check(lib().teno_batch_set_config(self.h, int(waves), int(blocks_per_cu)),
               "teno_batch_set_config")

    def read(self):
        import numpy as np
        t = np.zeros(self.nb)
        dt = np.zeros(self.nb)
        st = np.zeros(self.nb, dtype=np.int32)
        ns = np.zeros(self.nb, dtype=np.int64)
        _check(lib().teno_batch_read(self.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     dt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               "teno_batch_read")
        return t, dt, st, ns
