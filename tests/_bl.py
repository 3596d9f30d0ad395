"""Buckley-Leverett helpers for the waterflooding tests (Supporting
Information): the analytic solution of the Buckley-Leverett equation with
the power-law relative permeabilities k_r,1 = S^a, k_r,2 = (1 - S)^a, and the
measurements taken from a simulated state (saturation profile, front, flux).

Analytic solution (Eqs. BuckleyLeverettEq, FractionalFlowFunction,
BuckleyLeverettPerm, BuckleyLeverettVel): fractional flow
f(S) = S^a / (S^a + (1 - S)^a); the medium starts at S = 0 and S = 1 is
injected, so the shock saturation S_f is Welge's tangent from the origin,
f(S_f) / S_f = f'(S_f), the shock travels at (q / phi) f(S_f) / S_f, and
behind it the saturation S > S_f sits at x = x0 + (q t / phi) f'(S).
"""
import numpy as np
from scipy.optimize import brentq


def frac_flow(S, a):
    S = np.asarray(S, float)
    return S ** a / (S ** a + (1.0 - S) ** a)


def frac_flow_slope(S, a, h=1e-7):
    lo, hi = max(S - h, 0.0), min(S + h, 1.0)
    return float((frac_flow(hi, a) - frac_flow(lo, a)) / (hi - lo))


def welge(a):
    """(S_f, f(S_f) / S_f): the shock saturation and the shock speed in units of q / phi."""
    g = lambda S: float(frac_flow(S, a)) / S - frac_flow_slope(S, a)
    Sf = brentq(g, 0.5, 0.99)
    return Sf, float(frac_flow(Sf, a)) / Sf


def profile(a, x, x0, travel):
    """S(x) of the analytic solution for the injected length travel = q t / phi."""
    Sf, vs = welge(a)
    out = []
    for xi in (np.asarray(x, float) - x0) / travel:
        if xi <= 0.0:
            out.append(1.0)
        elif xi > vs:
            out.append(0.0)
        elif frac_flow_slope(1.0 - 1e-9, a) >= xi:
            out.append(1.0)
        else:
            out.append(brentq(lambda S: frac_flow_slope(S, a) - xi, Sf, 1.0 - 1e-9))
    return np.array(out)


def saturation(rho, rho_main, rho_dis):
    """Fluid-1 saturation per x column: (rho_1 - rho_dis) / (rho_main - rho_dis),
    averaged over y and z; rho is [2, nz, ny, nx]."""
    return (rho[0].mean(axis=(0, 1)) - rho_dis) / (rho_main - rho_dis)


def front(S, level=0.5):
    """Last x where S falls through level, linearly interpolated (cell index units)."""
    idx = np.nonzero((S[:-1] >= level) & (S[1:] < level))[0]
    if not len(idx):
        return None
    i = idx[-1]
    return i + (S[i] - level) / (S[i] - S[i + 1])


def flux(rho, u, lo, hi):
    """Darcy flux q = <rho u_x> / <rho> over the columns lo <= x < hi."""
    r = rho.sum(axis=0)[..., lo:hi]
    return float((r * u[0][..., lo:hi]).mean() / r.mean())
