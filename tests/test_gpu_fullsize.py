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
    special_y = [0, 1, 7, 8, 9, 15, 16, 17, 18, 26, 27, 127, 128, 247, 248, 251, 252, 255]
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


@pytest.mark.parametrize("storage,forcing", [("f32", "shan-chen"), ("f16s", "shan-chen"), ("bf16s", "shan-chen"),
                                             ("f32", "guo")])
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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n,storage", [(320, "f32"), (512, "f16s")])
def test_one_step_on_domains_beyond_4_gib(n, storage):
    """Domains whose population buffers exceed 4 GiB: 320^3 in FP32 (the 19
    direction arrays of one component span 2.49 GB, 4.98 GB per buffer) and
    512^3 in FP16 (10.2 GB per buffer, two components in the paired layout).
    Every plane block is addressed through its own buffer descriptor and the
    cell index is 64-bit, so no 32-bit offset spans more than one plane.  One
    step, sampled cells (random ones plus the first and last planes), against
    the oracle, to the bound of the 256^3 test.  The host copies of the state
    are freed as soon as they are used (the 512^3 state is 41 GB in FP64)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    _, w19, _ = oracle.lattice(19)
    w = inputs.electrode(n)
    nx, ny, nz = w.shape
    assert 2 * 19 * w.ncells * lbm.STORE_BYTES[storage] > 2 ** 32
    g = np.random.Generator(np.random.PCG64(11))
    p = np.concatenate([g.integers(0, [nx, ny, nz], size=(800, 3)),
                        np.stack([g.integers(0, nx, 400), g.integers(0, ny, 400), g.choice([nz - 1, nz - 2, 0, 1], 400)], 1)])
    cells = np.unique((p[:, 2].astype(np.int64) * ny + p[:, 1]) * nx + p[:, 0])
    sim = lbm.from_workload(w, storage=storage)
    sim.step(2)
    f_t = sim.populations()
    ref = oracle_for(w).cell_update(f_t, cells)
    del f_t
    sim.step(1)
    f_t1 = sim.populations()
    rho0 = np.array(lbm.default_shift(storage, 2, w.rho))[:2]
    sim.close()
    got = f_t1.reshape(2, 19, -1)[:, :, cells].transpose(2, 0, 1)
    finite = bool(np.isfinite(f_t1).all())
    del f_t1
    h_ref = ref - w19[None, None, :] * rho0[None, :, None]
    k = 2.0 if lbm.default_rounding(storage) == "stochastic" else 1.0
    bound = k * _U[storage] * np.abs(h_ref) + 2e-6 * np.abs(ref).max()
    excess = np.abs(got - ref) - bound
    assert excess.max() <= 0.0, (n, storage, float(excess.max()))
    assert finite
