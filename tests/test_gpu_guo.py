"""The GS-WBS with Guo forcing (Eq. GS-WBS) on the GPU against the FP64 oracle's
GS-WBS (pinned in test_oracle_guo.py), element by element: FP64 within 1e-10,
FP32 within 1e-4 on the fields, the 16-bit formats within their storage
rounding; and the bounce-back Poiseuille closed form on the device."""
import numpy as np
import pytest

from paper_2206_11524_amd import inputs, lbm

from _common import oracle_for, rel_max_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _both(w, steps, storage="f64", **kw):
    o = oracle_for(w, forcing="guo")
    fo = o.run(o.init(w.rho), steps)
    mo = o.moments(fo)
    sim = lbm.from_workload(w, storage=storage, forcing="guo", **kw)
    sim.step(steps)
    mg, fg = sim.moments(), sim.populations()
    sim.close()
    return fo, mo, fg, mg


def _errs(fo, mo, fg, mg, ncomp):
    e = {f"rho{s}": rel_max_err(mg["rho"][s], mo["rho"][s]) for s in range(ncomp)}
    for a in range(3):
        if np.abs(mo["u"][a]).max() > 1e-14:
            e[f"u{a}"] = rel_max_err(mg["u"][a], mo["u"][a])
    e["f"] = rel_max_err(fg, fo)
    return e


@pytest.mark.parametrize("shape,seed,c_ns", [((70, 13, 11), 201, 2), ((65, 9, 17), 202, 1),
                                               ((1, 20, 2), 203, 1)])
def test_gswbs_ragged_domains_all_terms_fp64(shape, seed, c_ns):
    """Ragged tiles, every force term, exact 0 / 1 bounce-back fractions,
    per-component n_s, two reservoirs."""
    w = inputs.random_state(shape, seed, c_ns=c_ns, ns_choices=[0.0, 0.05, 0.4, 0.9, 1.0],
                            rho_range=(0.3, 0.7))
    w.tau = (0.8, 1.3)
    w.G, w.G_ads, w.F_ext = 0.7, (0.2, -0.15), (2e-4, -1e-4, 3e-4)
    nz = shape[2]
    if nz >= 4:
        w.reservoirs = [(2, 0, 1, (0.6, 0.4)), (2, nz - 1, nz, (0.4, 0.6))]
    e = _errs(*_both(w, 25), 2)
    assert max(e.values()) <= 1e-10, e


def test_gswbs_droplet_fp64_and_reduced():
    """Droplet in a gray medium: with an external force, 300 steps in FP64;
    without it (as the HMCSC's FP32 droplet check), 200 steps in the reduced
    formats."""
    w = inputs.droplet(n=24, radius=6)
    w.F_ext = (1e-5, 0.0, -2e-5)
    e = _errs(*_both(w, 300), 2)
    assert max(e.values()) <= 1e-10, e
    w.F_ext = (0.0, 0.0, 0.0)
    fo, mo, fg, mg = _both(w, 200, storage="f32")
    e32 = _errs(fo, mo, fg, mg, 2)
    e32.pop("f")
    print("f32", e32)
    assert max(e32.values()) <= 1e-4, e32
    for storage, tol in (("f16s", 2e-3), ("bf16s", 2e-2)):
        fo, mo, fg, mg = _both(w, 200, storage=storage)
        e16 = {k: v for k, v in _errs(fo, mo, fg, mg, 2).items() if k.startswith("rho")}
        print(storage, e16)
        assert max(e16.values()) <= tol, (storage, e16)


@pytest.mark.parametrize("tau", [0.5 + np.sqrt(3) / 4, 1.0])
def test_gswbs_poiseuille_closed_form_on_device(tau):
    """Body-force channel between n_s = 1 walls, FP64 on the device: the BGK
    bounce-back closed form (parabola with walls half-way plus the slip
    F/(2 nu)(16 Lambda - 3)/12), here with a ragged 5-wide, 3-deep domain."""
    H, F = 12, 1e-5
    ns = np.zeros((1, 3, H + 2, 5), np.float32)
    ns[:, :, 0, :] = ns[:, :, H + 1, :] = 1.0
    w = inputs.Workload((5, H + 2, 3), ns, np.ones((1, 3, H + 2, 5)), ncomp=1, tau=(tau,), G=0.0,
                        G_ads=(0.0,), F_ext=(F, 0.0, 0.0), g_scale=3.0, name="poiseuille")
    sim = lbm.from_workload(w, storage="f64", forcing="guo")
    sim.step(20000)
    u = sim.moments()["u"][0]
    sim.close()
    nu, lam = (tau - 0.5) / 3, (tau - 0.5) ** 2
    y = np.arange(1, H + 1)
    ua = F / (2 * nu) * ((y - 0.5) * (H + 0.5 - y) + (16 * lam - 3) / 12)
    np.testing.assert_allclose(u[:, 1:H + 1, :], np.broadcast_to(ua[None, :, None], (3, H, 5)), rtol=1e-9)


def test_gswbs_is_refused_by_the_batched_path():
    w = inputs.droplet(n=16, radius=4)
    a = lbm.from_workload(w, storage="f32", forcing="guo")
    with pytest.raises(Exception):
        lbm.Group([a])
    a.close()
