"""TENO5-LAD reference oracle (test infrastructure only).

A plain FP64 CPU implementation of the semi-discrete Euler right-hand side with
characteristic-wise TENO5-LAD reconstruction (Peng et al., arXiv:2003.09145,
Sec. 2-4), written from the paper and sharing no code with the GPU path.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the product path never does.

The arithmetic lives in ``teno_oracle.cpp`` (built with ``-O2
-ffp-contract=off``); this module only marshals numpy arrays.  The exact
Riemann solver used to pin the Sod result is in ``riemann.py``.

Problems are described by any object (or dict) with the attributes ``ndim,
n, dx, bc, gamma`` and optionally ``scheme, ct_fixed, H, Bl, Bu, eps``.
Fields are numpy float64 arrays of shape ``(ndim + 2, nz, ny, nx)`` (unused
axes of size 1), component order rho, rho*u_x, [rho*u_y], [rho*u_z], E.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "teno_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with -DORACLE_LITERAL: every formula as its plain
# product-then-sum, no fused multiply-add (see the file header)
_LIB_LITERAL = os.path.join(_HERE, "liboracle_literal.so")

BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
SCHEME = {"lad": 0, "fixed_ct": 1, "linear5": 2, "teno5a": 3}
# LAD theta of eq 3.2: as printed, or also 0 where max chi-tilde > H (Sec. 3's
# description of H)
THETA = {"printed": 0, "cut": 1}


class OrParams(ctypes.Structure):
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
        ("a1", ctypes.c_double),
        ("a2", ctypes.c_double),
        ("cr", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("has_ext", ctypes.c_int32),
        ("side_kind", ctypes.c_int32 * 12),
        ("side_axis", ctypes.c_int32 * 6),
        ("side_split", ctypes.c_double * 12),
        ("side_state", ctypes.c_double * 60),
        ("gravity", ctypes.c_double * 3),
        ("time", ctypes.c_double),
        ("theta_form", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile both oracle libraries with g++: no fast-math and no FMA
    contraction; the explicit fused multiply-adds of the default build use the
    hardware instruction (-mfma), the literal build has none."""
    for out, extra in ((_LIB, []), (_LIB_LITERAL, ["-DORACLE_LITERAL"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-mfma", "-fopenmp",
                   "-fPIC", "-shared", "-std=c++17", *extra, "-o", out + ".tmp", _SRC]
            subprocess.run(cmd, check=True)
            os.replace(out + ".tmp", out)
    return _LIB


_libs = {}


def lib(literal: bool = False):
    """The oracle library; literal=True loads the FMA-free build."""
    key = bool(literal)
    if key not in _libs:
        build()
        L = ctypes.CDLL(_LIB_LITERAL if key else _LIB)
        P = ctypes.POINTER(OrParams)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.or_rec.argtypes = [P, dp, i32p, i32p, dp]
        L.or_rec.restype = ctypes.c_double
        L.or_eigen.argtypes = [P, ctypes.c_int, dp, dp, dp, dp]
        L.or_eigen.restype = None
        L.or_alpha.argtypes = [P, dp, dp]
        L.or_alpha.restype = ctypes.c_int
        L.or_rhs.argtypes = [P, dp, dp, dp, u8p]
        L.or_rhs.restype = ctypes.c_int
        L.or_rhs_cells.argtypes = [P, dp, dp, ctypes.c_int64, i64p, dp, u8p]
        L.or_rhs_cells.restype = ctypes.c_int
        L.or_rhs_jvp.argtypes = [P, dp, dp, dp, dp, dp]
        L.or_rhs_jvp.restype = ctypes.c_int
        L.or_step.argtypes = [P, dp, ctypes.c_double, dp, ctypes.c_double,
                              ctypes.c_int, dp, dp]
        L.or_step.restype = ctypes.c_int
        L.or_run_jvp.argtypes = [P, dp, dp, ctypes.c_int64, dp, dp]
        L.or_run_jvp.restype = ctypes.c_int
        L.or_advect_rhs.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp]
        L.or_advect_rhs.restype = None
        L.or_advect_run.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, dp]
        L.or_advect_run.restype = ctypes.c_int64
        L.or_run_jvp_batch.argtypes = [P, dp, dp, ctypes.c_int64, ctypes.c_int64, dp, dp]
        L.or_run_jvp_batch.restype = ctypes.c_int
        L.or_rhs_fluxabs.argtypes = [P, dp, dp, dp, dp]
        L.or_rhs_fluxabs.restype = ctypes.c_int
        L.or_literal.argtypes = []
        L.or_literal.restype = ctypes.c_int
        assert L.or_literal() == int(key)
        _libs[key] = L
    return _libs[key]


def _get(prob, key, default=None):
    if isinstance(prob, dict):
        return prob.get(key, default)
    return getattr(prob, key, default)


def params(prob) -> OrParams:
    """Build the C parameter block from a problem description."""
    p = OrParams()
    ndim = int(_get(prob, "ndim"))
    n = list(_get(prob, "n")) + [1, 1, 1]
    dx = list(_get(prob, "dx")) + [1.0, 1.0, 1.0]
    bc = _get(prob, "bc")
    if isinstance(bc, (str, int)):
        bc = [bc] * 3
    bc = [BC[b] if isinstance(b, str) else int(b) for b in list(bc) + [0, 0, 0]]
    scheme = _get(prob, "scheme", "lad")
    p.ndim = ndim
    for k in range(3):
        p.n[k] = int(n[k]) if k < ndim else 1
        p.dx[k] = float(dx[k]) if k < ndim else 1.0
        p.bc[k] = bc[k] if k < ndim else 0
    p.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    p.gamma = float(_get(prob, "gamma", 1.4))
    p.ct_fixed = float(_get(prob, "ct_fixed", 1e-7))
    p.H = float(_get(prob, "H", 10.0))
    p.Bl = int(_get(prob, "Bl", 4))
    p.Bu = int(_get(prob, "Bu", 10))
    p.eps = float(_get(prob, "eps", 1e-6))
    p.a1 = float(_get(prob, "a1", 10.5))   # TENO5-A parameters (Sec. 2, Sec. 4)
    p.a2 = float(_get(prob, "a2", 3.5))
    p.cr = float(_get(prob, "cr", 0.25))
    p.xi = float(_get(prob, "xi", 1e-3))
    tf = _get(prob, "theta", "printed")
    p.theta_form = THETA[tf] if isinstance(tf, str) else int(tf)
    bnd = _get(prob, "boundary", None)
    if bnd is not None:
        kinds = dict(BC, fixed=3)
        p.has_ext = 1
        for d in range(3):
            for e in range(2):
                sd = bnd.sides[d][e]
                ka = kinds[sd.kind_a]
                kb = kinds[sd.kind_b] if sd.kind_b is not None else ka
                p.side_kind[(d * 2 + e) * 2 + 0] = ka
                p.side_kind[(d * 2 + e) * 2 + 1] = kb
                p.side_axis[d * 2 + e] = int(sd.split_axis)
                p.side_split[(d * 2 + e) * 2 + 0] = float(sd.split0)
                p.side_split[(d * 2 + e) * 2 + 1] = float(sd.split_rate)
                for w, st in enumerate((sd.state_a, sd.state_b)):
                    if st is not None:
                        for q, v in enumerate(st):
                            p.side_state[((d * 2 + e) * 2 + w) * 5 + q] = float(v)
        for k in range(3):
            p.gravity[k] = float(bnd.gravity[k])
        p.time = float(bnd.time)
    return p


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape(p: OrParams):
    return (p.ndim + 2, p.n[2], p.n[1], p.n[0])


def rec(v, prob=None, trace: bool = False, literal=False):
    """One scalar TENO reconstruction of (f_{i-2}, ..., f_{i+2}).

    Returns (fhat, m, mask) or, with trace=True, also a dict of the
    intermediate values (beta, tau, t = chi-tilde, gamma, chi, x, theta, ct)."""
    p = params(prob or {"ndim": 1, "n": [8], "dx": [1.0], "bc": "periodic"})
    v = _f64(v)
    m = ctypes.c_int32()
    mask = ctypes.c_int32()
    tr = np.zeros(17)
    f = lib(literal).or_rec(ctypes.byref(p), _dp(v), ctypes.byref(m), ctypes.byref(mask), _dp(tr))
    if not trace:
        return f, m.value, mask.value
    d = {"beta": tr[0:3].copy(), "tau": tr[3], "t": tr[4:7].copy(), "gamma": tr[7:10].copy(),
         "chi": tr[10:13].copy(), "x": tr[13], "theta": tr[14], "ct": tr[15]}
    return f, m.value, mask.value, d


def eigen(prob, UL, UR, d: int):
    """Left/right eigenvector matrices at the Roe state (local order)."""
    p = params(prob)
    nc = p.ndim + 2
    L = np.zeros(25)
    R = np.zeros(25)
    lib().or_eigen(ctypes.byref(p), d, _dp(_f64(UL)), _dp(_f64(UR)), _dp(L), _dp(R))
    return L.reshape(5, 5)[:nc, :nc].copy(), R.reshape(5, 5)[:nc, :nc].copy()


def alpha(prob, U):
    """Global LF speeds alpha_d = max(|u_d| + c); returns (alpha[3], status)."""
    p = params(prob)
    U = _f64(U)
    a = np.zeros(3)
    st = lib().or_alpha(ctypes.byref(p), _dp(U), _dp(a))
    return a, st


def dump_size(prob) -> int:
    p = params(prob)
    nc = p.ndim + 2
    ncell = p.n[0] * p.n[1] * p.n[2]
    return sum((ncell // p.n[d]) * (p.n[d] + 1) * 2 * nc for d in range(p.ndim))


def rhs(prob, U, alpha3=None, dump: bool = False, literal=False):
    """dU/dt = L(U) (eq 2.2 per direction).  alpha3 freezes the LF speeds.

    Returns dUdt, or (dUdt, decisions) with dump=True."""
    p = params(prob)
    U = _f64(U)
    assert U.shape == _shape(p), (U.shape, _shape(p))
    out = np.zeros_like(U)
    a = None if alpha3 is None else _f64(alpha3)
    dmp = np.zeros(dump_size(prob), dtype=np.uint8) if dump else None
    lib(literal).or_rhs(ctypes.byref(p), _dp(U), None if a is None else _dp(a), _dp(out),
                 None if dmp is None else dmp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return (out, dmp) if dump else out


def rhs_flux_abs(prob, U, literal=False, with_max=False):
    """(dUdt, S[, M]): S[q] the sum over axes d and faces f of |F^_{f,q}| /
    dx_d (the face-flux terms whose differences form the RHS), M[q] the max
    over them of sum_s |R_qs f^_s| / dx_d (the terms the back-projection adds
    into F^_q); magnitudes for rounding bounds."""
    p = params(prob)
    U = _f64(U)
    out = np.zeros_like(U)
    S = np.zeros(5)
    M = np.zeros(5)
    lib(literal).or_rhs_fluxabs(ctypes.byref(p), _dp(U), _dp(out), _dp(S), _dp(M))
    nc = p.ndim + 2
    return (out, S[:nc].copy(), M[:nc].copy()) if with_max else (out, S[:nc].copy())


def rhs_cells(prob, U, alpha3, cells, dump: bool = False, literal=False):
    """RHS at selected flat cell indices; returns (ncell, nc) [and decisions
    of shape (ncell, ndim, 2 faces, 2*nc), faces i-1/2 then i+1/2]."""
    p = params(prob)
    nc = p.ndim + 2
    U = _f64(U)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), nc))
    dmp = np.zeros((len(cells), p.ndim, 2, 2 * nc), dtype=np.uint8) if dump else None
    lib(literal).or_rhs_cells(ctypes.byref(p), _dp(U), _dp(_f64(alpha3)), len(cells),
                       cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out),
                       None if dmp is None else dmp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return (out, dmp) if dump else out


def rhs_jvp(prob, U, V, alpha3, literal=False):
    """(L(U), dL/dU . V) with alpha and the cutoff decisions frozen."""
    p = params(prob)
    U = _f64(U)
    V = _f64(V)
    out = np.zeros_like(U)
    jv = np.zeros_like(U)
    lib(literal).or_rhs_jvp(ctypes.byref(p), _dp(U), _dp(V), _dp(_f64(alpha3)), _dp(out), _dp(jv))
    return out, jv


def step(prob, U, cfl, t, t_end, replay=None, literal=False):
    """One SSP-RK3 step (eq 4.1-4.3) on a copy of U.

    replay = (dt, alpha9) freezes dt and the per-stage LF speeds.
    Returns (U_new, t_new, dt, alpha9 (3x3), status)."""
    p = params(prob)
    U = _f64(U).copy()
    tt = ctypes.c_double(t)
    if replay is None:
        dt = ctypes.c_double(0.0)
        a9 = np.zeros(9)
        rp = 0
    else:
        dt = ctypes.c_double(float(replay[0]))
        a9 = _f64(replay[1]).reshape(9).copy()
        rp = 1
    st = lib(literal).or_step(ctypes.byref(p), _dp(U), float(cfl), ctypes.byref(tt), float(t_end),
                       rp, ctypes.byref(dt), _dp(a9))
    return U, tt.value, dt.value, a9.reshape(3, 3), st


def run(prob, U, cfl, t_end=np.inf, nsteps=None, record=False, literal=False):
    """Advance with RK3 until t_end or nsteps.  Returns (U, t, steps[, dts, alphas])."""
    t = 0.0
    k = 0
    dts, als = [], []
    while t < t_end and (nsteps is None or k < nsteps):
        U, t, dt, a9, st = step(prob, U, cfl, t, t_end, literal=literal)
        if st != 0:
            raise FloatingPointError(f"non-physical state at step {k}")
        dts.append(dt)
        als.append(a9)
        k += 1
    if record:
        return U, t, k, np.array(dts), np.array(als)
    return U, t, k


def run_jvp(prob, U, V, dts, alphas, literal=False):
    """Forward-mode derivative through replayed RK3 steps."""
    p = params(prob)
    U = _f64(U).copy()
    V = _f64(V).copy()
    dts = _f64(dts)
    alphas = _f64(alphas).reshape(-1)
    lib(literal).or_run_jvp(ctypes.byref(p), _dp(U), _dp(V), len(dts), _dp(dts), _dp(alphas))
    return U, V


def run_jvp_batch(prob, U, Vs, dts, alphas, literal=False):
    """Forward-mode derivatives of the same replayed run along several
    tangents Vs (shape (k,) + U.shape), in parallel; returns the k final
    tangents."""
    p = params(prob)
    U = _f64(U)
    Vs = _f64(Vs).copy()
    dts = _f64(dts)
    alphas = _f64(alphas).reshape(-1)
    lib(literal).or_run_jvp_batch(ctypes.byref(p), _dp(U), _dp(Vs), Vs.shape[0], len(dts),
                                  _dp(dts), _dp(alphas))
    return Vs


def advect_rhs(u, dx, scheme="lad", literal=False, **kw):
    prob = dict(ndim=1, n=[len(u)], dx=[dx], bc="periodic", scheme=scheme, **kw)
    p = params(prob)
    u = _f64(u)
    out = np.zeros_like(u)
    lib(literal).or_advect_rhs(ctypes.byref(p), len(u), float(dx), _dp(u), _dp(out))
    return out


def advect_run(u, dx, dt, t_end, scheme="lad", literal=False, **kw):
    """Linear advection u_t + u_x = 0 (Sec. 4.1), periodic, RK3 with fixed dt."""
    prob = dict(ndim=1, n=[len(u)], dx=[dx], bc="periodic", scheme=scheme, **kw)
    p = params(prob)
    u = _f64(u).copy()
    steps = lib(literal).or_advect_run(ctypes.byref(p), len(u), float(dx), float(dt), float(t_end), _dp(u))
    return u, steps
