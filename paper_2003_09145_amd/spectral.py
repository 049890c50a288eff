"""Approximate dispersion relation of the scalar TENO schemes (Sec. 3, Fig. 1).

For a periodic grid of N cells and each wavenumber phi_k = 2 pi k / N
(k = 1 .. N/2), the scheme's semi-discrete operator L (u_t + u_x = 0,
teno_advect_rhs in libteno.so) is applied to the single mode
u_j = A cos(phi_k j); the modified wavenumber is the response at that mode,

    Phi(phi_k) = i dx Lhat_k / uhat_k,

with hat the discrete Fourier coefficient.  The exact operator gives
Phi = phi; Re Phi measures dispersion and Im Phi dissipation (negative:
damping).  For a non-linear scheme the result depends on the amplitude A
through the smoothness indicators and the absolute epsilon of eq 2.8.

The operator runs on the GPU; this module only builds the inputs and takes
the Fourier coefficients of inputs and outputs.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B


def linear5_symbol(phi):
    """Phi of the fifth-order upwind scheme (every stencil kept): the face
    value (2, -13, 47, 27, -3)/60 . u_{i-2..i+2} and the flux difference give
    Phi = -i C(phi) (1 - e^{-i phi}) with C(phi) = sum_m c_m e^{i m phi}."""
    phi = np.asarray(phi, dtype=np.float64)
    c = np.array([2.0, -13.0, 47.0, 27.0, -3.0]) / 60.0
    C = sum(c[m + 2] * np.exp(1j * m * phi) for m in range(-2, 3))
    return -1j * C * (1.0 - np.exp(-1j * phi))


def adr(scheme: str = "lad", n: int = 128, amplitude: float = 1.0, device="cuda", **kw):
    """(phi, Phi) for k = 1 .. n/2 on an n-cell periodic grid with dx = 1.
    scheme and kw as for teno_grid ("lad", "fixed_ct" with ct_fixed,
    "linear5", "teno5a" with a1, a2, cr, xi)."""
    import torch
    g = B.advect_grid(n, 1.0, scheme=scheme, **kw)
    j = np.arange(n)
    ks = np.arange(1, n // 2 + 1)
    phis = 2.0 * math.pi * ks / n
    U = torch.empty((len(ks), n), dtype=torch.float64, device=device)
    for r, k in enumerate(ks):
        U[r] = torch.from_numpy(amplitude * np.cos(2.0 * math.pi * k * j / n))
    L = torch.empty_like(U)
    for r in range(len(ks)):
        B.teno_advect_rhs(g, U[r], L[r])
    torch.cuda.synchronize()
    u = U.cpu().numpy()
    lv = L.cpu().numpy()
    out = np.empty(len(ks), dtype=np.complex128)
    for r, k in enumerate(ks):
        e = np.exp(-2j * math.pi * k * j / n)
        out[r] = 1j * np.sum(lv[r] * e) / np.sum(u[r] * e)
    return phis, out
