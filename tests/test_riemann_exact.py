"""Self-checks of the exact Riemann solver that pins the Sod result."""
import math

import numpy as np

from oracle import riemann
from paper_2003_09145_amd import workloads as W


def test_sod_star_state_textbook():
    # Textbook star values of the Sod problem (gamma = 1.4): p* = 0.30313,
    # u* = 0.92745.
    p, u = riemann.star_state(W.SOD_LEFT, W.SOD_RIGHT)
    assert abs(p - 0.30313) < 5e-6 and abs(u - 0.92745) < 5e-6


def test_rankine_hugoniot_and_isentrope():
    g = 1.4
    for left, right in [(W.SOD_LEFT, W.SOD_RIGHT), (W.LAX_LEFT, W.LAX_RIGHT),
                        ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01))]:
        ps, us = riemann.star_state(left, right, g)
        # right-going shock: mass and momentum flux continuous in the shock frame
        rr, ur, pr = right
        rs, _, _ = riemann.sample(left, right, us + 1e-9, g)
        S = (rs * us - rr * ur) / (rs - rr)
        assert math.isclose(rs * (us - S), rr * (ur - S), rel_tol=1e-9)
        assert math.isclose(rs * (us - S) ** 2 + ps, rr * (ur - S) ** 2 + pr, rel_tol=1e-9)
        # left rarefaction: p / rho^gamma constant; p and u continuous at the contact
        rl, ul, pl = left
        rsl, usl, psl = riemann.sample(left, right, us - 1e-9, g)
        assert math.isclose(psl / rsl ** g, pl / rl ** g, rel_tol=1e-9)
        assert math.isclose(psl, ps, rel_tol=1e-12) and math.isclose(usl, us, rel_tol=1e-12)
        xs = np.linspace(-1, 1, 201)
        r, u, p = riemann.solution(left, right, xs, 0.1)
        inside = (xs / 0.1 < us) & (p < pl)  # fan and left star region
        assert np.allclose(p[inside] / r[inside] ** g, pl / rl ** g, rtol=1e-9)
