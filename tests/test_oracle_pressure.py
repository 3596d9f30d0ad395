"""Eq. (SC_pressure) against mechanical equilibrium (Sec. 2; Appendix on
multi-phase quantities).

Across a flat interface at rest the normal momentum flux is the same
everywhere, so the pressure of the two bulk phases on either side must be
equal; in a uniform phase that flux is p = c_s^2 (rho + g_scale G rho_1
rho_2), the interaction term carrying the same stencil factor as the force
(the stencil-normalisation reading).  A periodic quasi-1-D channel (D2Q9,
64 cells, two flat interfaces) settles to two phases whose total densities
differ by about 0.1 % because the components are not present in equal
amounts; their pressures must still agree.  Dropping the interaction term,
or its g_scale factor, leaves a relative pressure gap of order 1e-3 there.
"""
import numpy as np
import pytest

from oracle.ref import Oracle, Setup


@pytest.mark.parametrize("g_scale,G", [(3.0, 0.9), (1.0, 2.5)])
def test_flat_interface_bulk_pressures_equal(g_scale, G):
    nx = 64
    x = np.arange(nx)
    s_b = 0.5 * (np.tanh((x - 16) / 3.0) - np.tanh((x - 48) / 3.0))  # phase B in the middle half
    rho = np.empty((2, 1, 1, nx))
    rho[0, 0, 0] = 0.06 + (1.0 - 0.06) * (1 - s_b)
    rho[1, 0, 0] = 0.04 + (1.4 - 0.04) * s_b
    o = Oracle(Setup((nx, 1, 1), ncomp=2, G=G, g_scale=g_scale, lattice=9), np.zeros((1, 1, 1, nx)))
    m = o.moments(o.run(o.init(rho), 20000))
    assert np.abs(m["u"]).max() < 1e-10  # settled
    a = list(range(0, 6)) + list(range(58, 64))
    b = list(range(26, 38))
    p = m["p"][0, 0]
    r = m["rho"][:, 0, 0].sum(axis=0)
    ra, rb = r[a].mean(), r[b].mean()
    pa, pb = p[a].mean(), p[b].mean()
    assert abs(ra - rb) / ra > 5e-4  # the phases differ, so the check has teeth
    assert abs(pa - pb) / pa < 1e-7, (pa, pb)
