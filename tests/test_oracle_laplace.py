"""Bubble-test pin of the oracle's fluid-fluid interaction (Sec. 3.3, Table 1).

The paper prints the interfacial tension gamma = dp * R of a 2-D bubble
(D2Q9, fully periodic) for G_inter,12 = 1.50, 1.75, 2.00 as 0.051, 0.078, 0.104
(and the asymptote 0.077 at 1.75).  These numbers fix the normalisation of the
interaction stencil of Eq. (SC_F_inter): with the lattice weights w_i as
printed (g_scale = 1) the oracle lands within a few per cent of them, while
the alternative normalisation sum_i W_i c_i c_i = I (g_scale = 3) gives an
interfacial tension several times larger.

Measurement (the paper does not state its own; this is the reading taken):
R from the area of component 1, A = (M_1 - rho_1,out N) / (rho_1,in - rho_1,out),
R = sqrt(A / pi); p_in = mean pressure (Eq. SC_pressure) within R/2 of the
centre, p_out = mean pressure farther than R + 6 (minimum image).
Initial state: Table 1 densities 0.99 / 0.01, a tanh interface of width 2.5.
Because the two fluids are symmetric the interaction term of Eq. (SC_pressure)
is the same in both bulk phases and dp depends on the total density only.
"""
import functools
import os

import numpy as np
import pytest

from oracle.ref import Oracle, Setup

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@functools.lru_cache(maxsize=None)
def bubble_gamma(G, g_scale=1.0, H=100, R0=25.0, steps=8000, ns_val=0.0):
    y, x = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")
    c = (H - 1) / 2
    d = np.sqrt((x - c) ** 2 + (y - c) ** 2)
    s = 0.5 * (1 - np.tanh((d - R0) / 2.5))
    rho = np.empty((2, 1, H, H))
    rho[0, 0] = 0.01 + 0.98 * s
    rho[1, 0] = 0.99 - 0.98 * s
    ns = np.full((1, 1, H, H), ns_val, np.float32)
    o = Oracle(Setup((H, H, 1), ncomp=2, tau=(1.0, 1.0), G=G, g_scale=g_scale, lattice=9), ns)
    f = o.run(o.init(rho), steps)
    m = o.moments(f)
    r1, p = m["rho"][0, 0], m["p"][0]
    dx = np.minimum(np.abs(x - c), H - np.abs(x - c))
    dy = np.minimum(np.abs(y - c), H - np.abs(y - c))
    dmin = np.sqrt(dx * dx + dy * dy)
    rin, rout = r1[d <= R0 / 2].mean(), r1[dmin >= R0 + 8].mean()
    R = np.sqrt((r1.sum() - rout * H * H) / (rin - rout) / np.pi)
    dp = p[d <= R / 2].mean() - p[dmin >= R + 6].mean()
    return dp * R, R, np.abs(m["u"]).max()


def _printed():
    return np.loadtxt(os.path.join(GOLD, "interfacial_tension.txt"), comments="#")


@pytest.mark.parametrize("row", [0, 1, 2])
def test_interfacial_tension_matches_printed_values(row):
    G, gamma_paper = _printed()[row]
    gamma, R, umax = bubble_gamma(G)
    assert 20 < R < 27
    assert abs(gamma / gamma_paper - 1) < 0.06, (G, gamma, gamma_paper)


def test_alternative_stencil_normalisation_is_rejected_by_the_printed_value():
    gamma, _, _ = bubble_gamma(1.5, g_scale=3.0, H=64, R0=16.0, steps=3000)
    assert gamma > 3 * 0.051


def test_laplace_law_pressure_jump_scales_as_inverse_radius():
    """Laplace's law in 2-D, dp = gamma / R: bubbles of radius about 16, 24
    and 31 at G_inter,12 = 1.75 give the same gamma = dp R within 3 %."""
    g = [bubble_gamma(1.75, R0=18.0)[:2], bubble_gamma(1.75)[:2], bubble_gamma(1.75, H=110, R0=32.0)[:2]]
    radii = [r for _, r in g]
    assert radii[0] < 18 < radii[1] < 26 < radii[2]
    gam = np.array([x for x, _ in g])
    assert gam.max() / gam.min() - 1 < 0.03, g
