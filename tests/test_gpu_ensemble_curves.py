"""Outputs of the batched ensemble (Sec. 3.1's quantities over many media):
64 random-sphere porous domains of edge 32 .. 128 (porosity U[0.35, 0.65],
smoothed gray n_s in [0, 0.9], component A in the pore space of the lowest
quarter, body force 1e-5 along z, as the ensemble benchmark draws them), FP16
storage, all domains advanced by one batched launch per step for 10,000 steps.
Every 500 steps each domain reports

* its permeability k = nu <rho u_z> / F (Eq. Permeability) and component A's
  share of it, from lbm_permeability_get, and
* the saturation S_A of its pore space (Eq. Saturation, rho_A >= 0.5, pore
  cells weighted by 1 - n_s), from lbm_fill_state_get.

Within these 10,000 steps the domains are still rearranging their phases
(component A starts as a slab in the lowest quarter): capillary flows carry
mean momenta of order 1e-5, larger than the Darcy flow the force drives
(k F / nu ~ 6e-6 for these media), so the apparent k of Eq. (Permeability)
still changes and takes either sign in many domains (printed; the curves
are what the workload asks for, not a converged permeability).

Checks: every output finite; S_A in [0, 1]; the component shares add up to
k; each component's mass conserved (the domains are periodic) to the FP16
storage drift (measured 2.4e-4); the curves at 10,000 steps equal those of
the same domains advanced one by one (spot check of four domains, bitwise,
since group and single launches compute the same sums).  The per-domain
curves are printed.
"""
import numpy as np
import pytest

from paper_2206_11524_amd import inputs, lbm

pytestmark = pytest.mark.gpu

NDOM, STEPS, EVERY, SEED = 64, 10000, 500, 3000


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _domains():
    g = np.random.Generator(np.random.PCG64(SEED))
    edges = g.choice([32, 48, 64, 96, 128], size=NDOM)
    return [inputs.porous_domain(int(e), SEED + 1 + k) for k, e in enumerate(edges)]


def _outputs(sim, edge):
    k = sim.permeability(2)
    st = sim.fill_state(2, (0, 1), (edge - 1, edge), (0, edge), comp=0, threshold=0.5)
    assert abs(k["k_comp"][0] + k["k_comp"][1] - k["k"]) <= 1e-12 * max(abs(k["k_comp"][0]), abs(k["k_comp"][1]))
    return k["k"], k["k_comp"][0], st["saturation"]


@pytest.mark.timeout(900)
def test_ensemble_permeability_and_saturation_curves():
    ws = _domains()
    sims = [lbm.from_workload(w, storage="f16s") for w in ws]
    m0 = np.array([s.totals()["mass"] for s in sims])
    grp = lbm.Group(sims)
    curves = np.zeros((NDOM, STEPS // EVERY, 3))
    for j in range(STEPS // EVERY):
        grp.step(EVERY)
        for d, (sim, w) in enumerate(zip(sims, ws)):
            curves[d, j] = _outputs(sim, w.shape[0])
    grp.close()
    m1 = np.array([s.totals()["mass"] for s in sims])
    last = curves[:, -1].copy()
    for sim in sims:
        sim.close()
    print("domain edge porosity | k(t) every 2000 steps | S_A(t) every 2000 steps")
    for d, w in enumerate(ws):
        por = float((w.ns[0] < 1).mean())
        print(f"{d:2d} {w.shape[0]:3d} {por:.3f} | " + " ".join(f"{v:.3e}" for v in curves[d, 3::4, 0]) +
              " | " + " ".join(f"{v:.3f}" for v in curves[d, 3::4, 2]))
    assert np.isfinite(curves).all()
    assert (curves[:, :, 2] >= 0).all() and (curves[:, :, 2] <= 1).all()
    drift = np.abs(m1 / m0 - 1).max()
    print("max relative mass drift", drift)
    assert drift < 1e-3
    # (k_comp[1] is not kept; the library's own shares add up to k, checked on the last sample)
    print("median |k| over the domains at 10,000 steps", float(np.median(np.abs(curves[:, -1, 0]))))
    # the same domains one by one
    for d in (0, 17, 40, 63):
        sim = lbm.from_workload(ws[d], storage="f16s")
        sim.step(STEPS)
        assert _outputs(sim, ws[d].shape[0]) == tuple(last[d]), d
        sim.close()
