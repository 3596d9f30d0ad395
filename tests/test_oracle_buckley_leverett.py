"""Buckley-Leverett waterflooding on the oracle (Supporting Information,
Eqs. BuckleyLeverettEq, FractionalFlowFunction, BuckleyLeverettPerm,
BuckleyLeverettVel).

Set-up (inputs.buckley_leverett_channel): H = 100, L = 5, 2-D (the oracle's
D2Q9 mode), uniform n_s = 0.1 for both components, no adhesion, G_inter =
1.75, tau = 1, a body force 1e-4 from the inlet (x = 0) to the outlet (x = H).
The Supporting Information calls the force G and its direction +y, but puts
the inlet and outlet at x = 0 and x = H; the force runs along the flow here.

Readings:
* The reservoirs and the initial phases hold the coexistence densities of the
  two fluids (found on a flat periodic interface with the oracle: 0.98739 and
  0.03548), not Table 1's 0.99 / 0.01.  Those are out of equilibrium with the
  bulk phases and feed fluid 1 into the medium by diffusion even without a
  force (on the oracle, at n_s = 0.9 the front then runs 13.6 lu in 2e5 steps
  where q t is 1.1 lu, and about as far at F = 0), which the theory's
  injection at constant composition rules out.
* Porosity phi = 1: in the homogenized model every cell holds the full
  density of both components, so the Darcy flux q itself carries the
  saturation.
* S_1 per column = (rho_1 - rho_dis) / (rho_main - rho_dis).

Pins (between t = 2e4 and 5e4, q measured between the reservoirs):
* the front (S_1 = 1/2) advances by q dt times a factor between the shock
  speeds f(S_f)/S_f of a = 1.01 (1.003) and a = 1.3 (1.076), with 5 %
  allowance for the diffuse front;
* behind the front the profile lies between the a = 1.3 solution and the
  a = 1.01 one (which is 1 there to 1e-3), 5e-3 allowance.
A velocity that leaves out the (1 - n_s) weight of Eq. (HMCSC_u_macro)
overstates q by 1/(1 - n_s) and fails the first pin (mutant harness).
"""
import numpy as np
import pytest

from oracle.ref import Oracle, Reservoir, Setup
from paper_2206_11524_amd import inputs

import _bl

RES = 4


def coexistence(G=1.75, n=64, steps=40000):
    ns = np.zeros((1, 1, 1, n))
    rho = np.empty((2, 1, 1, n))
    rho[0], rho[1] = 0.01, 0.99
    rho[0, ..., n // 4:3 * n // 4], rho[1, ..., n // 4:3 * n // 4] = 0.99, 0.01
    o = Oracle(Setup((n, 1, 1), ncomp=2, tau=(1.0, 1.0), G=G, g_scale=1.0, lattice=9, nthreads=1), ns)
    m = o.moments(o.run(o.init(rho), steps))
    r = m["rho"].reshape(2, n)
    p = m["p"].reshape(n)
    return r, p


def _oracle(w):
    st = Setup(w.shape, ncomp=2, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext, g_scale=w.g_scale, lattice=9,
               reservoirs=[Reservoir(a, lo, hi, r) for a, lo, hi, r in w.reservoirs], nthreads=1)
    return Oracle(st, w.ns.astype(np.float64))


def test_coexistence_is_symmetric():
    """The two bulk phases of the flat interface mirror each other and share
    one pressure (Eq. SC_pressure)."""
    r, p = coexistence()
    n = r.shape[1]
    assert abs(r[0, n // 2] - r[1, 0]) < 1e-12 and abs(r[1, n // 2] - r[0, 0]) < 1e-12
    assert abs(p[n // 2] - p[0]) < 1e-12
    assert 0.98 < r[0, n // 2] < 0.995 and 0.02 < r[1, n // 2] < 0.05


@pytest.fixture(scope="module")
def flood():
    r, _ = coexistence()
    rm, rd = float(r[0, 32]), float(r[1, 32])
    w = inputs.buckley_leverett_channel(0.1, rm, rd)
    o = _oracle(w)
    f = o.run(o.init(w.rho), 20000)
    m1 = o.moments(f)
    f = o.run(f, 30000)
    m2 = o.moments(f)
    return rm, rd, m1, m2


def test_front_moves_with_the_buckley_leverett_shock(flood):
    rm, rd, m1, m2 = flood
    H = m1["rho"].shape[-1]
    q = 0.5 * (_bl.flux(m1["rho"], m1["u"], RES, H - RES) + _bl.flux(m2["rho"], m2["u"], RES, H - RES))
    x1 = _bl.front(_bl.saturation(m1["rho"], rm, rd))
    x2 = _bl.front(_bl.saturation(m2["rho"], rm, rd))
    ratio = (x2 - x1) / (q * 30000)
    lo, hi = _bl.welge(1.01)[1], _bl.welge(1.3)[1]
    print(f"q {q:.4e}, front {x1:.2f} -> {x2:.2f}, advance / (q dt) {ratio:.4f}, shock factors {lo:.4f} .. {hi:.4f}")
    assert 0.95 * lo <= ratio <= 1.05 * hi, (ratio, lo, hi)


def test_profile_lies_between_the_analytic_bounds(flood):
    rm, rd, _, m2 = flood
    H = m2["rho"].shape[-1]
    q = _bl.flux(m2["rho"], m2["u"], RES, H - RES)
    S = _bl.saturation(m2["rho"], rm, rd)
    travel = q * 50000
    xs = np.arange(RES, int(RES + _bl.welge(1.01)[1] * travel) - 4)
    lower = _bl.profile(1.3, xs, RES, travel)
    upper = _bl.profile(1.01, xs, RES, travel)
    print("S", np.round(S[xs][::4], 4), "a=1.3", np.round(lower[::4], 4))
    assert (upper > 1 - 1e-3).all()
    assert (S[xs] >= lower - 5e-3).all() and (S[xs] <= upper + 5e-3).all()
