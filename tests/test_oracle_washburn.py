"""Washburn imbibition with the oracle (Sec. 3.4, Eq. Washburn).

A quasi-1-D D2Q9 channel (periodic in y): a reservoir of fluid 1 at the
inlet, a free gap, then a homogenized gray medium of uniform n_s filled with
fluid 2, and a fluid-2 reservoir at the outlet (Table 1 fluids: 0.99 / 0.01,
tau = 1, G_inter,12 = 1.75; G_ads,2 = -G_ads,1 = G_ads > 0 makes fluid 1 the
wetting one).  Inside the uniform medium the adhesion sum vanishes; the n_s
step at the medium entrance supplies the capillary pressure and the medium's
bounce-back fraction the viscous resistance, so the front follows Washburn's
law x^2 = A^2 B t (Eq. Washburn).

Pins (the paper's own criteria and trends, Table 3):
* x_inter^2 is linear in t with a coefficient of determination above 0.97;
* imbibition is faster on a more wetting medium: the Huang correlation
  (Eq. contactAngle) makes cos(theta) proportional to G_ads, so the rate
  A^2 B at G_ads = 0.3 is at least twice that at G_ads = 0.1 (3x expected);
* a denser medium imbibes more slowly: B falls from n_s = 0.5 to n_s = 0.9
  (Table 3: 0.0481 -> 0.0138), here by at least a factor two.
A wrong sign of the adhesion term stops the imbibition; a wrong bounce-back
weighting changes the n_s dependence.
"""
import os

import numpy as np
import pytest

from oracle.ref import Oracle, Reservoir, Setup
from paper_2206_11524_amd import inputs

from _common import front_position, huang_contact_angle, washburn_contact_angle

XM = 12  # first cell of the gray medium


def washburn_rate(G_ads, ns_medium, H=200, L=2, steps=20000, samples=20):
    rho = np.empty((2, 1, L, H))
    rho[0], rho[1] = 0.01, 0.99
    rho[0, :, :, :4], rho[1, :, :, :4] = 0.99, 0.01
    ns = np.zeros((1, 1, L, H), np.float32)
    ns[..., XM:H - 4] = ns_medium
    res = [Reservoir(0, 0, 4, (0.99, 0.01)), Reservoir(0, H - 4, H, (0.01, 0.99))]
    o = Oracle(Setup((H, L, 1), ncomp=2, G=1.75, G_ads=(-G_ads, G_ads), g_scale=1.0, lattice=9,
                     reservoirs=res), ns)
    f = o.init(rho)
    every = steps // samples
    ts, xs = [], []
    for k in range(samples):
        f = o.run(f, every)
        r = o.moments(f)["rho"][:, 0].mean(axis=1)
        phi = r[0] - r[1]
        idx = np.nonzero((phi[XM:-5] > 0) & (phi[XM + 1:-4] <= 0))[0]
        if len(idx):  # the interface has entered the medium
            i = idx[-1] + XM
            ts.append((k + 1) * every)
            xs.append(i + phi[i] / (phi[i] - phi[i + 1]) - XM)
    t, x2 = np.array(ts, float), np.array(xs) ** 2
    A = np.c_[t, np.ones_like(t)]
    coef = np.linalg.lstsq(A, x2, rcond=None)[0]
    r2 = 1 - ((x2 - A @ coef) ** 2).sum() / ((x2 - x2.mean()) ** 2).sum()
    return coef[0], r2, len(t)


@pytest.fixture(scope="module")
def rates():
    return {(0.1, 0.5): washburn_rate(0.1, 0.5), (0.3, 0.5): washburn_rate(0.3, 0.5),
            (0.2, 0.5): washburn_rate(0.2, 0.5), (0.2, 0.9): washburn_rate(0.2, 0.9, steps=40000)}


def test_front_follows_washburn_law(rates):
    for key, (rate, r2, n) in rates.items():
        assert n >= 8 and rate > 0 and r2 > 0.97, (key, rate, r2, n)


def test_more_wetting_medium_imbibes_faster(rates):
    assert rates[(0.3, 0.5)][0] > 2.0 * rates[(0.1, 0.5)][0], rates


def test_denser_medium_imbibes_slower(rates):
    assert rates[(0.2, 0.9)][0] < 0.5 * rates[(0.2, 0.5)][0], rates


def test_stored_full_size_front_is_the_oracles():
    """The first samples of tests/golden/washburn_front_oracle.txt (written by
    make_washburn_front.py) come out of the current oracle unchanged."""
    d = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "washburn_front_oracle.txt"), comments="#")
    rows = d[(np.round(d[:, 0], 2) == 0.4) & (np.round(d[:, 1], 1) == 0.5)]
    rows = rows[~np.isnan(rows[:, 3])][:2]
    w = inputs.washburn_channel(0.4, 0.5)
    o = Oracle(Setup(w.shape, ncomp=2, tau=w.tau, G=w.G, G_ads=w.G_ads, g_scale=w.g_scale, lattice=9,
                     reservoirs=[Reservoir(a, lo, hi, r) for a, lo, hi, r in w.reservoirs]), w.ns.astype(np.float64))
    f = o.init(w.rho)
    t = 0
    for tr, xr in rows[:, 2:]:
        f = o.run(f, int(tr) - t)
        t = int(tr)
        x = front_position(o.moments(f)["rho"], 12)
        assert x is not None and abs(x - xr) < 1e-9, (t, x, xr)


def _table3_rows():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "table3_washburn.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                b, g, ns, A, B, _ = line.split()
                rows.append((b, float(g), float(ns), float(A), float(B)))
    return rows


def test_contact_angle_conversion_reproduces_table3():
    """The conversion of a Washburn fit to a contact angle, and Eq.
    (contactAngle), against Table 3's own columns: theta from each printed A
    at the printed B (cos theta = 2 eta A^2 / gamma) lands within 1 degree of
    the printed theta, and theta_H of Eq. (contactAngle) within 0.1 degree of
    the printed theta_H (values of Sec. 3.4's table, not in the fixture)."""
    theta = [70.8, 67.7, 64.1, 59.2, 52.9, 45.9, 36.0, 21.4]
    theta_h = [83.3, 76.5, 69.5, 62.2, 54.3, 45.6, 35.3, 21.1]
    rows = [r for r in _table3_rows() if r[0] == "A"]
    for (b, g, ns, A, B), th, thh in zip(rows, theta, theta_h):
        assert abs(washburn_contact_angle(A * A * B, B) - th) < 1.0, (g, washburn_contact_angle(A * A * B, B), th)
        assert abs(huang_contact_angle(g) - thh) < 0.1, (g, huang_contact_angle(g), thh)


def _stored_rates():
    d = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "washburn_front_oracle.txt"), comments="#")
    out = {}
    for g, ns in sorted({(round(a, 2), round(b, 1)) for a, b in d[:, :2]}):
        sel = (np.round(d[:, 0], 2) == g) & (np.round(d[:, 1], 1) == ns) & ~np.isnan(d[:, 3])
        out[(g, ns)] = np.polyfit(d[sel, 2], d[sel, 3] ** 2, 1)[0]
    return out


def test_contact_angle_from_washburn_rates_follows_huang():
    """Eq. (contactAngle) as Table 3 tests it: the contact angle behind the
    oracle's Washburn rates at the paper's size (H = 500, t <= 5e4; the stored
    fronts, which the current oracle reproduces, see above), taken at the
    fixed B = 0.0481 of Table 3's left block, against Huang's theta_H.

    * Within 10 degrees of theta_H for G_ads <= 0.25 (theta_H 83 .. 54
      degrees); measured 1.5 .. 5.6 degrees below it, where the paper's own
      fits sit 1.4 .. 12.5 degrees below.
    * theta falls strictly as G_ads rises over all eight rows.
    * For G_ads >= 0.3 the rate grows faster than cos(theta_H): theta lies 11
      .. 23 degrees below theta_H and the G_ads = 0.4 rate exceeds what
      complete wetting allows at this B (reported, not asserted)."""
    rates = _stored_rates()
    ga = [0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4]
    th = [washburn_contact_angle(rates[(g, 0.5)], 0.0481) for g in ga]
    thh = [huang_contact_angle(g) for g in ga]
    print("theta", np.round(th, 1), "theta_H", np.round(thh, 1))
    for g, a, b in zip(ga, th, thh):
        if g <= 0.25:
            assert abs(a - b) < 10.0, (g, a, b)
    cos = [2 * (1 / 6) * rates[(g, 0.5)] / (0.0481 * 0.077) for g in ga]
    assert np.all(np.diff(cos) > 0), cos
