"""Laplace's law for a static 3-D droplet on the GPU (Sec. 3.3): the pressure jump
across the interface is dp = 2 gamma / R, so dp R / 2 is the same interfacial
tension for every radius; and gamma hardly depends on the bounce-back fraction
of a uniform gray medium (the paper reports it independent of n_s).

Droplets of initial radius 8 .. 14 in a periodic 64^3 box, G = 0.9 (stencil
weights sum_i W_i c_i c_i = I), FP32, 20 000 steps (the droplets swell from
the initial 1.0 / 0.03 densities towards coexistence while the test runs; the
law holds at every state).  R from the volume of component A, dp from the
pressure of Eq. (SC_pressure) inside R/2 and beyond R + 4, measured on the
device by lbm_droplet_get.  Measured spread of dp R / 2 over the radii: 0.6 % (n_s = 0);
gamma at n_s = 0.1 and 0.5 within 0.3 % and 3.2 % of n_s = 0 (a gray medium
relaxes more slowly).
"""
import numpy as np
import pytest

from paper_2206_11524_amd import inputs, lbm

pytestmark = pytest.mark.gpu

N, STEPS = 64, 20000


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _gamma(r0, ns_value):
    sim = lbm.from_workload(inputs.droplet(n=N, radius=r0, ns_value=ns_value), storage="f32")
    sim.step(STEPS)
    c = (N - 1) / 2
    d = sim.droplet((c, c, c), r_core=3.0, r_far=N / 2 - 1, margin=4.0, comp=0)
    sim.close()
    assert abs(d["gamma"] - d["dp"] * d["R"] / 2) <= 1e-15
    return d["R"], d["dp"]


def test_pressure_jump_scales_as_inverse_radius():
    res = [_gamma(r0, 0.0) for r0 in (8, 10, 12, 14)]
    radii = np.array([r for r, _ in res])
    dps = np.array([d for _, d in res])
    print("R", radii, "dp", dps, "gamma", dps * radii / 2)
    assert np.all(np.diff(radii) > 0) and np.all(np.diff(dps) < 0)
    gam = dps * radii / 2
    assert gam.max() / gam.min() - 1 < 0.02, gam
    # dp against 1/R: a line through the origin (the radii span only 12 .. 16
    # after swelling, so the fitted intercept extrapolates far and amplifies
    # the 0.6 % drift of gamma: measured -2.5 % of the smallest dp)
    a, b = np.polyfit(1 / radii, dps, 1)
    assert abs(b) < 0.05 * dps.min(), (a, b)


def test_interfacial_tension_hardly_depends_on_n_s():
    g0 = np.prod(_gamma(12, 0.0)) / 2
    g1 = np.prod(_gamma(12, 0.1)) / 2
    g5 = np.prod(_gamma(12, 0.5)) / 2
    print("gamma", g0, g1, g5)
    assert abs(g1 / g0 - 1) < 0.01
    assert abs(g5 / g0 - 1) < 0.05
