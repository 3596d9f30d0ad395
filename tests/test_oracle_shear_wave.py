"""Viscosity pin of the oracle: with n_s = 0 and no forces Eq. (LGS) is the
LBGK equation of Appendix A, whose shear waves decay at the rate nu k^2 with
nu = c_s^2 (tau - 1/2).  The rate is a property of the scheme, not of how the
initial state was built, so the initial populations are simply the
second-order equilibrium of a sinusoidal shear flow.
"""
import numpy as np
import pytest

import oracle
from oracle.ref import Oracle, Setup

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("tau,L", [(0.8, 64), (1.0, 48), (1.7, 64)])
def test_shear_wave_decay_rate(tau, L):
    c, w, _ = oracle.lattice(19)
    y = np.arange(L)
    U = 1e-4
    ux = U * np.sin(2 * np.pi * y / L)
    cu = c[:, 0][:, None] * ux[None, :]
    feq = w[:, None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * ux[None, :] ** 2)
    f = feq.reshape(1, 19, 1, L, 1).copy()
    o = Oracle(Setup((1, L, 1), ncomp=1, tau=(tau,)), np.zeros((1, 1, L, 1), np.float32))

    def amp(state):
        u = o.moments(state)["u"][0, 0, :, 0]
        return 2.0 / L * np.sum(u * np.sin(2 * np.pi * y / L))

    f = o.run(f, 50)
    a1 = amp(f)
    f = o.run(f, 400)
    a2 = amp(f)
    nu = CS2 * (tau - 0.5)
    k = 2 * np.pi / L
    rate = np.log(a1 / a2) / 400
    assert abs(rate / (nu * k * k) - 1) < 5e-3
