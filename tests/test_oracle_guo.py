"""Pins of the oracle's GS-WBS with Guo forcing (Appendix, Guo vs. Shan-Chen
forcing, Eq. GS-WBS): the scheme the paper contrasts the HMCSC with.

The paper does not print the forcing term; the oracle takes the one of Guo,
Zheng and Shi (2002).  Pins, none of which re-evaluates that expression:
  * the moments every second-order forcing term must have (Guo et al. 2002):
    zeroth 0, first (1 - 1/(2 tau)) F, second (1 - 1/(2 tau)) (u F + F u),
    read off one collision of a single periodic cell through the moments of
    the BGK equilibrium (rho, rho u, rho c_s^2 I + rho u u);
  * the momentum of a uniform gray medium follows the affine map obtained by
    taking the first moment of Eq. (GS-WBS) (bounce-back reverses j);
  * n_s = 1 everywhere is pure bounce-back: the state repeats after two steps;
  * two components with equal tau conserve the total momentum (the cohesion
    forces cancel in pairs over a periodic domain; this needs u_macro to carry
    both components' half forces);
  * Poiseuille flow between n_s = 1 walls: with BGK and bounce-back the
    steady profile is the parabola with walls half-way plus a uniform slip
    F/(2 nu) (16 Lambda - 3)/12, Lambda = (tau - 1/2)^2 (Ginzburg and
    d'Humieres 2003; exact at tau = 1/2 + sqrt(3)/4);
  * without forces and with n_s = 0 the scheme is the plain LBGK of the HMCSC.
"""
import numpy as np
import pytest

from oracle import ref

CS2 = 1.0 / 3.0


def _lat():
    c, w, opp = ref.lattice(19)
    return np.asarray(c, float), np.asarray(w), np.asarray(opp)


def _oracle(shape, ns, forcing="guo", **kw):
    s = ref.Setup(shape=shape, g_scale=3.0, forcing=forcing, **kw)
    return ref.Oracle(s, ns)


def test_guo_term_moments_single_cell():
    c, w, _ = _lat()
    rng = np.random.default_rng(7)
    tau = 0.8
    F = np.array([1e-3, -2e-3, 5e-4])
    f = (w * 1.3 * (1 + 0.2 * rng.uniform(-1, 1, 19)))[None, :, None, None, None]
    o = _oracle((1, 1, 1), np.zeros((1, 1, 1, 1)), ncomp=1, tau=(tau,), F_ext=tuple(F))
    g = o.step(f)
    f0, f1 = f[0, :, 0, 0, 0], g[0, :, 0, 0, 0]
    rho, j = f0.sum(), f0 @ c
    u = (j + F / 2) / rho
    Pi = np.einsum("i,ia,ib->ab", f0, c, c)
    Pi_eq = rho * CS2 * np.eye(3) + rho * np.outer(u, u)
    k = 1 - 1 / (2 * tau)
    assert abs(f1.sum() - rho) < 1e-15
    np.testing.assert_allclose(f1 @ c, j - (j - rho * u) / tau + k * F, rtol=0, atol=1e-15)
    Pi1 = np.einsum("i,ia,ib->ab", f1, c, c)
    np.testing.assert_allclose(Pi1, Pi - (Pi - Pi_eq) / tau + k * (np.outer(u, F) + np.outer(F, u)),
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("ns,tau", [(0.0, 0.7), (0.3, 1.3), (0.9, 0.7), (0.05, 1.0)])
def test_gswbs_uniform_medium_momentum_map(ns, tau):
    c, w, _ = _lat()
    F = np.array([2e-5, 0.0, -1e-5])
    rho = 1.2
    o = _oracle((2, 2, 2), np.full((1, 2, 2, 2), ns), ncomp=1, tau=(tau,), F_ext=tuple(F))
    f = o.init(np.full((1, 2, 2, 2), rho))
    j = np.zeros(3)
    k = 1 - 1 / (2 * tau)
    for _ in range(40):
        f = o.step(f)
        rho_u = (1 - ns) * (j + F / 2)
        j = (1 - ns) * j - (1 - ns) / tau * (j - rho_u) - ns * j + (1 - ns) * k * F
        jg = np.einsum("izyx,ia->a", f[0], c) / 8
        np.testing.assert_allclose(jg, j, rtol=1e-12, atol=1e-15)
    assert abs(f[0].sum() / 8 - rho) < 1e-14


@pytest.mark.parametrize("ns", [0.0, 0.3])
def test_gswbs_two_component_momentum_map(ns):
    """The same map per component, two components with unequal tau and
    density: each relaxes towards rho_s u with its own tau_s and receives its
    own share F_s = rho_s / rho F of the force through its own prefactor
    1 - 1/(2 tau_s); u = sum_s (1 - n)(j_s + F_s/2) / rho is common."""
    c, w, _ = _lat()
    F = np.array([2e-5, -1e-5, 3e-5])
    tau = (0.7, 1.4)
    rho_s = np.array([0.9, 0.3])
    rho = rho_s.sum()
    o = _oracle((2, 2, 2), np.full((1, 2, 2, 2), ns), ncomp=2, tau=tau, G=0.9, F_ext=tuple(F))
    f = o.init(np.stack([np.full((1, 2, 2, 2), r) for r in rho_s]).reshape(2, 2, 2, 2))
    j = np.zeros((2, 3))
    Fs = [rho_s[s] / rho * F for s in range(2)]
    for _ in range(40):
        f = o.step(f)
        u = sum((1 - ns) * (j[s] + Fs[s] / 2) for s in range(2)) / rho
        j = np.array([(1 - ns) * j[s] - (1 - ns) / tau[s] * (j[s] - rho_s[s] * u) - ns * j[s]
                      + (1 - ns) * (1 - 1 / (2 * tau[s])) * Fs[s] for s in range(2)])
        for s in range(2):
            jg = np.einsum("izyx,ia->a", f[s], c) / 8
            np.testing.assert_allclose(jg, j[s], rtol=1e-11, atol=1e-16)


def test_gswbs_full_bounce_back_has_period_two():
    rng = np.random.default_rng(3)
    shape = (5, 4, 3)
    o = _oracle(shape, np.ones((1, 3, 4, 5)), ncomp=2, tau=(0.9, 1.2), G=0.9, G_ads=(-0.1, 0.1),
                F_ext=(1e-4, 0, 0))
    f = rng.uniform(0.01, 0.1, (2, 19, 3, 4, 5))
    assert np.array_equal(o.step(o.step(f)), f)


def test_gswbs_two_components_conserve_momentum():
    c, w, _ = _lat()
    n = 10
    rng = np.random.default_rng(11)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    inside = (x - 4.5) ** 2 + (y - 4.5) ** 2 + (z - 4.5) ** 2 <= 9
    rho = np.stack([np.where(inside, 0.97, 0.06), np.where(inside, 0.06, 0.97)])
    u = 1e-3 * rng.uniform(-1, 1, (3, n, n, n))
    cu = np.einsum("ia,azyx->izyx", c, u)
    uu = (u ** 2).sum(0)
    feq = w[None, :, None, None, None] * rho[:, None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu)[None]
    o = _oracle((n, n, n), np.zeros((1, n, n, n)), ncomp=2, tau=(1.0, 1.0), G=0.9)
    J0 = np.einsum("sizyx,ia->a", feq, c)
    f = o.run(feq, 20)
    J1 = np.einsum("sizyx,ia->a", f, c)
    assert np.abs(J0).max() > 1e-3
    np.testing.assert_allclose(J1, J0, rtol=0, atol=1e-14 * np.abs(f).sum())
    # and the forces are not trivially zero: the droplet keeps its cohesion
    ft = o.moments(f)["ftot"]
    assert np.abs(ft).max() > 1e-3


@pytest.mark.parametrize("tau", [0.8, 0.5 + np.sqrt(3) / 4, 1.0, 1.5])
def test_gswbs_poiseuille_profile(tau):
    H, F = 8, 1e-5
    ns = np.zeros((1, 1, H + 2, 1))
    ns[0, 0, 0, 0] = ns[0, 0, H + 1, 0] = 1.0
    o = _oracle((1, H + 2, 1), ns, ncomp=1, tau=(tau,), F_ext=(F, 0, 0))
    f = o.run(o.init(np.ones((1, 1, H + 2, 1))), 20000)
    u = o.moments(f)["u"][0, 0, 1:H + 1, 0]
    nu = (tau - 0.5) / 3
    lam = (tau - 0.5) ** 2
    y = np.arange(1, H + 1)
    ua = F / (2 * nu) * ((y - 0.5) * (H + 0.5 - y) + (16 * lam - 3) / 12)
    np.testing.assert_allclose(u, ua, rtol=1e-9)


def test_gswbs_without_forces_is_the_plain_lbgk():
    rng = np.random.default_rng(5)
    shape = (6, 5, 4)
    f = rng.uniform(0.02, 0.08, (1, 19, 4, 5, 6))
    ns = np.zeros((1, 4, 5, 6))
    a = _oracle(shape, ns, forcing="guo", ncomp=1, tau=(0.9,)).run(f, 5)
    b = _oracle(shape, ns, forcing="shan-chen", ncomp=1, tau=(0.9,)).run(f, 5)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_invalid_forcing_is_rejected():
    s = ref.Setup(shape=(2, 2, 2), ncomp=1, tau=(1.0,))
    p = ref.params_struct(s)
    p.forcing = 7
    o = ref.Oracle(s, np.zeros((1, 2, 2, 2)))
    o.p = p
    with pytest.raises(ValueError):
        o.init(np.ones((1, 2, 2, 2)))
