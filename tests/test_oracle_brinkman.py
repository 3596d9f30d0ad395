"""Darcy-Brinkman pins of the oracle (Sec. 3.2 and Appendix C).

* Homogeneous gray channel between bounce-back walls, closed form of
  Eq. (DarcyBrinkmanPoiseuille) with k from Eq. (GS_perm), r = sqrt(2 n_s / nu).
  Reading of the wall position: the no-slip plane sits half-way between the
  wall cell (n_s = 1) and the first fluid cell.
* Two stratified gray layers, periodic (paragraph "Open boundary flow"): the
  maximum velocity printed in Table C.1, and the piece-wise closed form of
  Eq. (DarcyBrinkmanOpenBoundary) with the parameters of Table 2, both for the
  paper's own D2Q9 lattice and for D3Q19 (the flow is one-dimensional, the
  profile does not depend on the velocity set beyond discretisation error).

The problems are one-dimensional, so the transverse extent is one periodic cell.
"""
import os

import numpy as np
import pytest

from oracle.ref import Oracle, Setup

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0


def _f32(v):
    return float(np.float32(v))


def poiseuille_closed_form(x, H, n, nu, F):
    k = (1 - n) * nu / (2 * n)
    r = np.sqrt(2 * n / nu)
    return F * k / nu * (1 - np.cosh(r * (x - H / 2)) / np.cosh(r * H / 2))


def open_boundary_closed_form(x, H, nl, nr, nu, F):
    kl, kr = (1 - nl) * nu / (2 * nl), (1 - nr) * nu / (2 * nr)
    U0l, U0r = kl * F / nu, kr * F / nu
    pl, pr = kr / kl, kl / kr
    ql, qr = np.sqrt(nl / nr), np.sqrt(nr / nl)
    rl, rr = np.sqrt(2 * nl / nu), np.sqrt(2 * nr / nu)
    coth = lambda v: 1 / np.tanh(v)  # noqa: E731
    ul = U0l * (1 - (1 - pl) * np.cosh(rl * (x - H / 4)) /
                (np.sinh(rl * H / 4) * (ql * coth(rr * H / 4) + coth(rl * H / 4))))
    ur = U0r * (1 + (pr - 1) * np.cosh(rr * (3 * H / 4 - x)) /
                (np.sinh(rr * H / 4) * (qr * coth(rl * H / 4) + coth(rr * H / 4))))
    return np.where(x <= H / 2, ul, ur)


@pytest.mark.parametrize("n", [0.001, 0.01, 0.1, 0.5, 0.9])
def test_gray_poiseuille_profile(n):
    H, F, tau = 50, 1e-5, 1.0
    nu = CS2 * (tau - 0.5)
    ny = H + 2
    ns = np.full((1, 1, ny, 1), n, np.float32)
    ns[0, 0, 0, 0] = ns[0, 0, -1, 0] = 1.0
    o = Oracle(Setup((1, ny, 1), ncomp=1, tau=(tau,), F_ext=(F, 0, 0)), ns)
    f = o.run(o.init(np.ones((1, 1, ny, 1))), 12000)
    u = o.moments(f)["u"][0, 0, 1:-1, 0]
    x = np.arange(1, ny - 1) - 0.5
    ua = poiseuille_closed_form(x, H, _f32(n), nu, F)
    umax = ua.max()
    # the centre is Darcy/Brinkman-exact; the first cells resolve the boundary
    # layer of width 1/r only when r is small
    assert abs(u[H // 2] / ua[H // 2] - 1) < 2e-4
    tol = 0.01 if n <= 0.1 else 0.1
    assert np.abs(u - ua).max() / umax < tol


def _table_c1():
    return np.loadtxt(os.path.join(GOLD, "table_c1_open_boundary_umax.txt"), comments="#")


@pytest.mark.parametrize("lattice", [9, 19])
@pytest.mark.parametrize("row", [1, 2, 3, 4])
def test_open_boundary_two_layer_flow(lattice, row):
    """u_max of Table C.1 (rows n_s,right = 0.01 ... 0.8) to the four printed
    digits, and the closed-form profile away from the two layer interfaces.
    The n_s,right = 0.001 row matches neither the closed form nor the oracle
    (its printed value exceeds the closed-form maximum); it is not used."""
    nr, umax_paper = _table_c1()[row]
    nl, H, F, tau = 0.9, 100, 1e-6, 1.0
    nu = CS2 * (tau - 0.5)
    ns = np.zeros((1, 1, 1, H), np.float32)
    ns[0, 0, 0, : H // 2] = nl
    ns[0, 0, 0, H // 2:] = nr
    o = Oracle(Setup((H, 1, 1), ncomp=1, tau=(tau,), F_ext=(0, F, 0), lattice=lattice), ns)
    f = o.run(o.init(np.ones((1, 1, 1, H))), 8000)
    u = o.moments(f)["u"][1, 0, 0, :]
    assert abs(u.max() / umax_paper - 1) < 2e-4
    x = np.arange(H) + 0.5
    ua = open_boundary_closed_form(x, H, _f32(nl), _f32(nr), nu, F)
    d = np.minimum(np.abs(x - H / 2), np.minimum(x, H - x))
    far = d >= 3
    assert np.abs(u - ua)[far].max() / ua.max() < 0.03


def three_layer_closed_form(eta, n, nu, F, half_w, half_s):
    """Gray Brinkman channel of the single-phase benchmark: free fluid between
    no-slip walls at |eta| = half_w and a gray slab |eta| < half_s of bounce-back
    fraction n in the middle.  Free layers: nu u'' = -F; slab: the Brinkman
    equation behind Eq. (DarcyBrinkmanPoiseuille), nu u'' - 2 n u + (1 - n) F =
    0 (r = sqrt(2 n / nu), k of Eq. GS_perm, nu_B = nu); u and du/deta
    continuous at |eta| = half_s.  With u_f = F/(2 nu) (half_w^2 - eta^2) +
    C (half_w - |eta|) and u_g = u_inf + D cosh(r eta), u_inf = (1 - n) F / (2 n),
    the two matching conditions give D and C below."""
    r = np.sqrt(2 * n / nu)
    uinf = (1 - n) * F / (2 * n)
    a = half_w - half_s
    D = (F / nu * ((half_w ** 2 - half_s ** 2) / 2 - a * half_s) - uinf) / (np.cosh(r * half_s) +
                                                                            a * r * np.sinh(r * half_s))
    C = -half_s * F / nu - D * r * np.sinh(r * half_s)
    e = np.abs(eta)
    return np.where(e < half_s, uinf + D * np.cosh(r * e), F / (2 * nu) * (half_w ** 2 - e ** 2) + C * (half_w - e))


def three_layer_oracle(refine, n, steps, tau=0.8, F=1e-6):
    """The channel of the gray Brinkman benchmark (walls at y = 0 and ny - 1,
    slab of 16 cells in the middle, force along z, tau = 0.8) at `refine`
    times its resolution, as a one-cell-wide periodic column (the flow is
    one-dimensional).  Returns (u_z at the fluid cells, k = nu <rho u_z> / F,
    cell-centre coordinates from the channel centre)."""
    ny = 62 * refine + 2
    lo = 23 * refine + 1
    ns = np.zeros((1, 1, ny, 1), np.float32)
    ns[0, 0, 0, 0] = ns[0, 0, -1, 0] = 1.0
    ns[0, 0, lo:lo + 16 * refine, 0] = n
    nu = CS2 * (tau - 0.5)
    o = Oracle(Setup((1, ny, 1), ncomp=1, tau=(tau,), F_ext=(0, 0, F)), ns)
    m = o.moments(o.run(o.init(np.ones((1, 1, ny, 1))), steps))
    u = m["u"][2, 0, 1:-1, 0]
    k = nu * (m["rho"][0, 0, 1:-1, 0] * u).mean() / F
    return u, k, np.arange(1, ny - 1) - (ny - 1) / 2


@pytest.mark.parametrize("n", [0.05, 0.1, 0.2, 0.4, 0.8])
def test_three_layer_gray_channel_closed_form(n):
    """The single-phase gray channel (Sec. 3.2 set-up, 64 cells across, slab
    of 16 cells, tau = 0.8): the channel permeability k = nu <rho u_z> / F
    against the three-layer closed form.  The closed form is the continuum
    limit; the slab's Brinkman layer 1/r = sqrt(nu / 2n) is 0.25 to 1 cell at
    this resolution, so the lattice lies 0.8 % (n = 0.05) to 2.8 % (n = 0.8)
    below it.  At twice the resolution (same r times slab width: n / 4 on a
    126-cell channel with a 32-cell slab) the difference drops about
    fourfold (asserted: threefold) and is within 1 % for every n, profile
    included: the lattice converges to the closed form at second order."""
    nu = CS2 * 0.3
    u1, k1, e1 = three_layer_oracle(1, n, 20000)
    kc1 = nu * three_layer_closed_form(e1, _f32(n), nu, 1e-6, 31.0, 8.0).mean() / 1e-6
    u2, k2, e2 = three_layer_oracle(2, n / 4, 60000)
    uc2 = three_layer_closed_form(e2, _f32(n / 4), nu, 1e-6, 62.0, 16.0)
    kc2 = nu * uc2.mean() / 1e-6
    err1, err2 = k1 / kc1 - 1, k2 / kc2 - 1
    print(f"n={n}: k={k1:.4f} closed {kc1:.4f} ({err1:+.2e}); refined k={k2:.4f} closed {kc2:.4f} ({err2:+.2e})")
    assert abs(err1) < 0.03 and (n > 0.05 or abs(err1) < 0.01)
    assert abs(err2) < 0.01 and abs(err2) < abs(err1) / 3
    assert np.abs(u2 - uc2).max() / uc2.max() < 0.012
