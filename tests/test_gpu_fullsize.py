"""Full-size parity on the benchmark workload (256^3 synthetic electrode, two
components, reservoirs, solid spheres and gray binder) in the launch
configuration the benchmark times.

The oracle cannot run this domain for many steps, so one GPU step is checked
cell by cell: from the GPU state at t (read back exactly, as FP64), the oracle
computes the state at t+1 at sampled cells (every sampled cell needs the
collisions of its 19 source cells and their neighbourhoods), and the GPU's own
state at t+1 must agree within the storage rounding of the result plus FP32
arithmetic: |f_gpu - f_ref| <= k u |h_ref| + 2e-6 max|f| (k = 1 for rounding
to nearest, 2 for the stochastic rounding the 16-bit formats use by default).

Samples: random cells plus the planes and lines where the decomposition
changes hands (tile borders in x and y, z-chunk borders, the periodic wrap),
the reservoir slabs and their neighbours, and solid/fluid/binder interfaces.
"""
import numpy as np
import pytest

from paper_2206_11524_amd import inputs, lbm

from _common import oracle_for

pytestmark = pytest.mark.gpu

_U = {"f32": 2.0 ** -24, "f16s": 2.0 ** -11, "bf16s": 2.0 ** -8}


@pytest.fixture(scope="module")
def electrode():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return inputs.electrode(256)


def _sample_cells(w, seed=5):
    nx, ny, nz = w.shape
    g = np.random.Generator(np.random.PCG64(seed))
    pts = [g.integers(0, [nx, ny, nz], size=(1500, 3))]
    special_x = [0, 1, 31, 32, 63, 64, 65, 127, 128, 191, 192, 254, 255]
    special_y = [0, 1, 7, 8, 9, 15, 16, 127, 128, 247, 248, 255]
    special_z = [0, 1, 15, 16, 17, 31, 32, 63, 64, 65, 127, 128, 223, 239, 240, 241, 254, 255]
    for _ in range(800):
        pts.append(np.array([[g.choice(special_x), g.choice(special_y), g.choice(special_z)]]))
        pts.append(np.array([[g.integers(nx), g.choice(special_y), g.choice(special_z)]]))
        pts.append(np.array([[g.choice(special_x), g.integers(ny), g.integers(nz)]]))
    # interface cells: solid next to fluid, binder next to free pore
    ns = w.ns[0]
    solid = ns == 1.0
    iface = solid & ~np.roll(solid, 1, axis=2)
    zi, yi, xi = np.nonzero(iface)
    k = g.choice(len(zi), size=min(400, len(zi)), replace=False)
    pts.append(np.stack([xi[k], yi[k], zi[k]], axis=1))
    gray = (ns > 0) & (ns < 1)
    zi, yi, xi = np.nonzero(gray)
    k = g.choice(len(zi), size=min(400, len(zi)), replace=False)
    pts.append(np.stack([xi[k], yi[k], zi[k]], axis=1))
    p = np.concatenate(pts)
    cells = (p[:, 2].astype(np.int64) * ny + p[:, 1]) * nx + p[:, 0]
    return np.unique(cells)


@pytest.mark.parametrize("storage,forcing", [("f32", "shan-chen"), ("f16s", "shan-chen"), ("f32", "guo")])
def test_one_step_at_full_size(electrode, storage, forcing):
    """(forcing = "guo": the GS-WBS kernel against the oracle's GS-WBS)"""
    import oracle
    _, w19, _ = oracle.lattice(19)
    w = electrode
    sim = lbm.from_workload(w, storage=storage, forcing=forcing)
    sim.step(3)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    rho0 = np.array(lbm.default_shift(storage, 2, w.rho))[:2]
    sim.close()
    cells = _sample_cells(w)
    o = oracle_for(w, forcing=forcing)
    ref = o.cell_update(f_t, cells)                       # [k, s, i]
    got = f_t1.reshape(2, 19, -1)[:, :, cells].transpose(2, 0, 1)
    h_ref = ref - w19[None, None, :] * rho0[None, :, None]
    k = 2.0 if lbm.default_rounding(storage) == "stochastic" else 1.0  # one unit / half a unit in the last place
    bound = k * _U[storage] * np.abs(h_ref) + 2e-6 * np.abs(ref).max()
    excess = np.abs(got - ref) - bound
    worst = np.unravel_index(np.argmax(excess), excess.shape)
    assert excess.max() <= 0.0, (storage, len(cells), float(excess.max()), int(cells[worst[0]]), worst)
    assert np.isfinite(f_t1).all()


def test_one_step_beyond_two_gib_per_component():
    """320^3 in FP32: the 19 direction arrays of one component span 2.49 GB,
    beyond 2^31 bytes, so the kernel's 32-bit buffer offsets go past the sign
    bit (and the offset that parks lanes without a ring cell may land inside
    the buffer: a wasted load there, never a wrong value).  One step, sampled
    cells, against the oracle, to the same bound as above."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    _, w19, _ = oracle.lattice(19)
    w = inputs.electrode(320)
    assert 19 * w.ncells * 4 > 2 ** 31
    sim = lbm.from_workload(w, storage="f32")
    sim.step(2)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    rho0 = np.array(lbm.default_shift("f32", 2, w.rho))[:2]
    sim.close()
    nx, ny, nz = w.shape
    g = np.random.Generator(np.random.PCG64(11))
    p = np.concatenate([g.integers(0, [nx, ny, nz], size=(800, 3)),
                        np.stack([g.integers(0, nx, 400), g.integers(0, ny, 400), g.choice([nz - 1, nz - 2, 0, 1], 400)], 1)])
    cells = np.unique((p[:, 2].astype(np.int64) * ny + p[:, 1]) * nx + p[:, 0])
    ref = oracle_for(w).cell_update(f_t, cells)
    got = f_t1.reshape(2, 19, -1)[:, :, cells].transpose(2, 0, 1)
    h_ref = ref - w19[None, None, :] * rho0[None, :, None]
    bound = _U["f32"] * np.abs(h_ref) + 2e-6 * np.abs(ref).max()
    assert (np.abs(got - ref) - bound).max() <= 0.0
    assert np.isfinite(f_t1).all()
