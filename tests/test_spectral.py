"""The closed-form modified wavenumber of the linear scheme (CPU): it must
reproduce the exact derivative to fifth order at small phi and the known
limits, and agree with the oracle's linear operator (an independent
implementation of eq 2.3 and eq 2.2)."""
import math

import numpy as np

from paper_2003_09145_amd.spectral import linear5_symbol


def test_linear5_symbol_limits():
    # fifth-order upwind: the leading error is dissipative, the truncation
    # term dx^5/60 u^(6), i.e. Im(Phi - phi) = -phi^6/60 + O(phi^8), with
    # dispersion one order higher
    phi = np.array([0.01, 0.1])
    err = linear5_symbol(phi) - phi
    assert abs(err[1].imag / (-(0.1 ** 6) / 60.0) - 1.0) < 0.01
    assert 0.9e6 < abs(err[1]) / abs(err[0]) < 1.1e6
    assert abs(err[1].real) < 0.1 * abs(err[1].imag)
    # at phi = pi (odd-even mode) the scheme is purely dissipative:
    # C(pi) = (2 + 13 + 47 - 27 - 3)/60 = 32/60, Phi = -2 i C(pi)
    assert abs(linear5_symbol(math.pi) - (-2j * 32.0 / 60.0)) < 1e-14


def test_linear5_symbol_matches_oracle_operator(orc):
    n = 64
    j = np.arange(n)
    for k in (1, 5, 17, 32):
        u = np.cos(2 * math.pi * k * j / n)
        L = orc.advect_rhs(u, 1.0, scheme="linear5")
        e = np.exp(-2j * math.pi * k * j / n)
        phi = 2 * math.pi * k / n
        assert abs(1j * np.sum(L * e) / np.sum(u * e) - linear5_symbol(phi)) < 1e-13
