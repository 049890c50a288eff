"""Exact solution of the 1D Euler Riemann problem for an ideal gas
(test infrastructure only).

Used to pin the Sod shock tube (Sec. 4.2, eq 4.8) of the oracle.  The star
pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0, with f_K the shock
(Rankine-Hugoniot) branch for p > p_K and the isentropic rarefaction branch
otherwise; the solution is self-similar in x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    """Velocity change across the left/right wave and its derivative in p."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk  # rarefaction
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * ck / (g - 1.0) * (r ** e - 1.0), (1.0 / (rho * ck)) * r ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, gamma=1.4, tol=1e-15, maxit=200):
    """Star-region pressure and velocity (p*, u*) for states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    du = ur - ul
    if 2.0 * (cl + cr) / (gamma - 1.0) <= du:
        raise ValueError("vacuum is generated")
    p = max(0.5 * (pl + pr), 1e-12)
    for _ in range(maxit):
        fl, dfl = _fk(p, rl, pl, cl, gamma)
        fr, dfr = _fk(p, rr, pr, cr, gamma)
        pn = p - (fl + fr + du) / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, gamma)
    fr, _ = _fk(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, xi, gamma=1.4):
    """Primitive state (rho, u, p) at similarity coordinate xi = (x - x0) / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    ps, us = star_state(left, right, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    if xi <= us:  # left of the contact
        if ps > pl:  # left shock
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if xi <= sl:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
        # left rarefaction
        csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if xi <= ul - cl:
            return rl, ul, pl
        if xi >= us - csl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        u = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + xi)
        c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - xi))
        rho = rl * (c / cl) ** (2.0 / (g - 1.0))
        return rho, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    # right of the contact
    if ps > pr:  # right shock
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if xi >= sr:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
    csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if xi >= ur + cr:
        return rr, ur, pr
    if xi <= us + csr:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    u = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + xi)
    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - xi))
    rho = rr * (c / cr) ** (2.0 / (g - 1.0))
    return rho, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def solution(left, right, x, t, x0=0.0, gamma=1.4):
    """Arrays (rho, u, p) of the exact solution at points x and time t > 0."""
    out = np.array([sample(left, right, (xi - x0) / t, gamma) for xi in np.asarray(x, float)])
    return out[:, 0], out[:, 1], out[:, 2]
