"""Seeded synthetic inputs for the HMCSC workloads.

Each generator returns host arrays only: the bounce-back-fraction field(s)
``ns[k, z, y, x]`` (float32) and initial component densities ``rho[s, z, y, x]``
(float64).  Nothing here computes any part of the lattice Boltzmann method; both
the GPU library and the CPU checker consume these arrays unchanged.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.

Interaction strengths: the droplet, electrode and porous-domain workloads quote
G_inter = 0.9 and G_ads = +-0.1 / +-0.3 in the normalisation where the
interaction stencil weights sum to sum_i W_i c_i c_i = I (W_i = 3 w_i), common for
multi-component Shan-Chen set-ups; they therefore carry ``g_scale = 3``.  With
the paper's literal stencil (g_scale = 1) G_inter = 0.9 at these densities lies
below the demixing threshold and a droplet dissolves.

Workloads (the paper's own 3-D microstructure and separator images are not
available, these synthetic stand-ins have the same structure):

* ``droplet``        static droplet in a uniform gray medium (bubble test, Sec. 3.3)
* ``gray_channel``   walls plus a gray slab between free fluid (Sec. 3.2, Brinkman flow)
* ``electrode``      random overlapping spheres + smoothed gray binder + reservoirs
                     (electrolyte filling, Sec. 4)
* ``porous_domain``  random-sphere packing with a smoothed gray field (ensembles)
* ``washburn_channel`` imbibition into a uniform gray medium (Sec. 3.4)
* ``obstacle_channel`` two-phase flow past porous obstacles (Sec. 3.5)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Workload:
    """Arrays and parameters of one problem (x fastest in every array)."""
    shape: tuple                      # (nx, ny, nz)
    ns: np.ndarray                    # float32 [c_ns, nz, ny, nx]
    rho: np.ndarray                   # float64 [ncomp, nz, ny, nx]
    ncomp: int = 2
    tau: tuple = (1.0, 1.0)
    G: float = 0.0
    G_ads: tuple = (0.0, 0.0)
    F_ext: tuple = (0.0, 0.0, 0.0)
    g_scale: float = 1.0
    reservoirs: list = field(default_factory=list)  # [(axis, lo, hi, (rho_1, rho_2))]
    name: str = ""

    @property
    def c_ns(self) -> int:
        return int(self.ns.shape[0])

    @property
    def ncells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


def uniform(shape, ns_value=0.0, rho=(1.0, 0.0), ncomp=2) -> Workload:
    nx, ny, nz = shape
    ns = np.full((1, nz, ny, nx), ns_value, np.float32)
    r = np.empty((ncomp, nz, ny, nx))
    for s in range(ncomp):
        r[s] = rho[s]
    return Workload(shape, ns, r, ncomp=ncomp, name="uniform")


def random_state(shape, seed, ncomp=2, c_ns=1, ns_choices=None, rho_range=(0.05, 1.0)) -> Workload:
    """Random densities and a random bounce-back field (values drawn from
    ``ns_choices`` when given, e.g. to include exact 0 and 1, else U[0,1))."""
    nx, ny, nz = shape
    g = rng(seed)
    if ns_choices is None:
        ns = g.uniform(0.0, 1.0, size=(c_ns, nz, ny, nx)).astype(np.float32)
    else:
        ns = g.choice(np.asarray(ns_choices, np.float32), size=(c_ns, nz, ny, nx))
    r = g.uniform(rho_range[0], rho_range[1], size=(ncomp, nz, ny, nx))
    return Workload(shape, ns.astype(np.float32), r, ncomp=ncomp, name=f"random{seed}")


def droplet(n=32, radius=8.0, ns_value=0.1, rho_in=1.0, rho_out=0.03, noise=1e-3, seed=0,
            G=0.9, tau=1.0) -> Workload:
    """Sphere of component A (densities rho_in / rho_out inside, swapped outside),
    centred at ((n-1)/2)^3, inside when |x - c|^2 <= R^2, plus U(-noise, noise) per
    component and cell drawn component-major then z, y, x."""
    c = (n - 1) / 2.0
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    inside = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= radius * radius
    r = np.empty((2, n, n, n))
    r[0] = np.where(inside, rho_in, rho_out)
    r[1] = np.where(inside, rho_out, rho_in)
    if noise:
        r += rng(seed).uniform(-noise, noise, size=r.shape)
    ns = np.full((1, n, n, n), ns_value, np.float32)
    return Workload((n, n, n), ns, r, ncomp=2, tau=(tau, tau), G=G, g_scale=3.0, name=f"droplet{n}")


def gray_channel(nx=64, ny=64, nz=128, slab=(24, 40), ns_slab=0.1, force=1e-6, tau=0.8) -> Workload:
    """Single component between walls (n_s = 1 at y = 0 and y = ny-1) with a gray
    slab ``slab[0] <= y < slab[1]`` of bounce-back fraction ``ns_slab``, free fluid
    elsewhere, body force along z."""
    ns = np.zeros((1, nz, ny, nx), np.float32)
    ns[0, :, slab[0]:slab[1], :] = ns_slab
    ns[0, :, 0, :] = 1.0
    ns[0, :, ny - 1, :] = 1.0
    r = np.ones((1, nz, ny, nx))
    return Workload((nx, ny, nz), ns, r, ncomp=1, tau=(tau, tau), F_ext=(0.0, 0.0, force),
                    name=f"channel_ns{ns_slab}")


def _gaussian_smooth(a: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(a, sigma=sigma, mode="wrap")


def _sphere_pack(shape, g, target_solid, rmin, rmax, zlo=0, zhi=None, batch=64):
    """Overlapping spheres (centres U[0,n)^3, radius U[rmin,rmax]) painted with
    periodic minimum image in x and y until the solid fraction inside
    ``zlo <= z < zhi`` reaches ``target_solid``.  Returns a bool [nz, ny, nx]."""
    nx, ny, nz = shape
    zhi = nz if zhi is None else zhi
    solid = np.zeros((nz, ny, nx), bool)
    vol = (zhi - zlo) * ny * nx
    count = 0
    while solid[zlo:zhi].sum() < target_solid * vol:
        for _ in range(batch):
            cx, cy, cz = g.uniform(0, nx), g.uniform(0, ny), g.uniform(0, nz)
            R = g.uniform(rmin, rmax)
            r0 = int(np.ceil(R))
            xs = np.arange(int(np.floor(cx)) - r0, int(np.floor(cx)) + r0 + 2)
            ys = np.arange(int(np.floor(cy)) - r0, int(np.floor(cy)) + r0 + 2)
            zs = np.arange(max(int(np.floor(cz)) - r0, zlo), min(int(np.floor(cz)) + r0 + 2, zhi))
            if len(zs) == 0:
                continue
            dz = (zs - cz)[:, None, None]
            dy = (ys - cy)[None, :, None]
            dx = (xs - cx)[None, None, :]
            m = dx * dx + dy * dy + dz * dz <= R * R
            zi, yi, xi = np.nonzero(m)
            solid[zs[zi], ys[yi] % ny, xs[xi] % nx] = True
            count += 1
        if count > 10_000_000:
            raise RuntimeError("sphere packing did not reach the target")
    return solid


def electrode(n=256, seed=2000, res_layers=16, solid_fraction=0.5, rmin=6.0, rmax=12.0,
              binder_frac=0.2, G=0.9, G_ads=(-0.3, 0.3), rho_main=1.0, rho_dis=0.03,
              tau=1.0, membrane=0) -> Workload:
    """Synthetic electrode for the electrolyte-filling workload.

    * spheres (n_s = 1) of radius U[rmin, rmax] fill ``res_layers <= z < n-res_layers``
      to the solid fraction ``solid_fraction`` (periodic in x, y; none in the reservoirs)
    * binder: white noise, Gaussian-smoothed (sigma 3), thresholded at its
      (1-binder_frac) quantile over the pore cells; binder n_s =
      clip(0.5 + 0.15 * zscore, 0.2, 0.8)
    * component A (wetting, index 0) fills the inlet reservoir z < res_layers,
      component B fills everything else; reservoirs hold (rho_main, rho_dis) at the
      inlet and (rho_dis, rho_main) at the outlet.
    * membrane > 0: Sec. 4's semi-permeable membranes of that many layers next
      to each reservoir, with one bounce-back field per component (c_ns = 2):
      the inlet membrane blocks B (n_s,B = 1), the outlet membrane blocks A;
      the structure then lies between the membranes.
    """
    g = rng(seed)
    shape = (n, n, n)
    zlo, zhi = res_layers + membrane, n - res_layers - membrane
    solid = _sphere_pack(shape, g, solid_fraction, rmin, rmax, zlo, zhi)
    noise = _gaussian_smooth(g.standard_normal((n, n, n)), 3.0)
    pore = ~solid
    pore[:zlo] = False
    pore[zhi:] = False
    vals = noise[pore]
    thr = np.quantile(vals, 1.0 - binder_frac)
    binder = pore & (noise >= thr)
    zscore = (noise - vals.mean()) / vals.std()
    ns = np.zeros((2 if membrane else 1, n, n, n), np.float32)
    for c in range(ns.shape[0]):
        ns[c][binder] = np.clip(0.5 + 0.15 * zscore[binder], 0.2, 0.8)
        ns[c][solid] = 1.0
    if membrane:
        ns[1, res_layers:zlo] = 1.0      # inlet membrane: A only
        ns[0, zhi:n - res_layers] = 1.0  # outlet membrane: B only
    r = np.empty((2, n, n, n))
    r[0] = rho_dis
    r[1] = rho_main
    r[0, :zlo] = rho_main
    r[1, :zlo] = rho_dis
    res = [(2, 0, res_layers, (rho_main, rho_dis)), (2, n - res_layers, n, (rho_dis, rho_main))]
    return Workload(shape, ns, r, ncomp=2, tau=(tau, tau), G=G, G_ads=tuple(G_ads), g_scale=3.0,
                    reservoirs=res, name=f"electrode{n}" + (f"_m{membrane}" if membrane else ""))


def filling_cell(nxy=48, nz=64, seed=2100, res_layers=4, membrane=2, solid_fraction=0.45, rmin=4.0, rmax=7.0,
                 binder_frac=0.2, G=0.9, G_ads=(-0.04, 0.04), rho_main=1.0, rho_dis=0.03, tau=1.0) -> Workload:
    """Electrolyte-filling set-up of Sec. 4 along z, two bounce-back fields
    (c_ns = 2): reservoirs of ``res_layers`` at both ends (electrolyte, index
    0, at the inlet; gas, index 1, at the outlet), then a semi-permeable
    membrane of ``membrane`` layers on each side (the inlet one blocks the gas,
    n_s,gas = 1; the outlet one blocks the electrolyte), and between them a
    sphere packing (n_s = 1 for both) with a gray binder (same n_s for both)
    initially filled with gas.  The default G_ads is weakly wetting for the
    electrolyte (cos theta ~ 0.2 by Eq. contactAngle with G = 0.9)."""
    g = rng(seed)
    shape = (nxy, nxy, nz)
    z0, z1 = res_layers + membrane, nz - res_layers - membrane
    solid = _sphere_pack(shape, g, solid_fraction, rmin, rmax, z0, z1)
    noise = _gaussian_smooth(g.standard_normal((nz, nxy, nxy)), 2.0)
    pore = ~solid
    pore[:z0] = False
    pore[z1:] = False
    vals = noise[pore]
    thr = np.quantile(vals, 1.0 - binder_frac)
    binder = pore & (noise >= thr)
    zscore = (noise - vals.mean()) / vals.std()
    ns = np.zeros((2, nz, nxy, nxy), np.float32)
    for c in range(2):
        ns[c][binder] = np.clip(0.5 + 0.15 * zscore[binder], 0.2, 0.8)
        ns[c][solid] = 1.0
    ns[1, res_layers:z0] = 1.0   # inlet membrane: electrolyte only
    ns[0, z1:nz - res_layers] = 1.0  # outlet membrane: gas only
    r = np.empty((2, nz, nxy, nxy))
    r[0], r[1] = rho_dis, rho_main
    r[0, :z0], r[1, :z0] = rho_main, rho_dis
    res = [(2, 0, res_layers, (rho_main, rho_dis)), (2, nz - res_layers, nz, (rho_dis, rho_main))]
    return Workload(shape, ns, r, ncomp=2, tau=(tau, tau), G=G, G_ads=tuple(G_ads), g_scale=3.0,
                    reservoirs=res, name=f"filling{nxy}x{nz}")


def porous_domain(edge, seed, porosity=None, ns_max=0.9, G=0.9, G_ads=(0.1, -0.1),
                  force=1e-5, rho_main=1.0, rho_dis=0.03, tau=1.0) -> Workload:
    """Cubic random-sphere packing (porosity U[0.35, 0.65] unless given) with a
    gray field n_s = ns_max * minmax(smoothed noise) in the pores; component A in
    the pore space of z < edge/4, B elsewhere; body force along z."""
    g = rng(seed)
    if porosity is None:
        porosity = g.uniform(0.35, 0.65)
    n = int(edge)
    solid = _sphere_pack((n, n, n), g, 1.0 - porosity, max(2.0, n / 24), max(3.0, n / 12), batch=16)
    noise = _gaussian_smooth(g.standard_normal((n, n, n)), 3.0)
    lo, hi = noise.min(), noise.max()
    gray = ns_max * (noise - lo) / (hi - lo if hi > lo else 1.0)
    ns = np.where(solid, 1.0, gray).astype(np.float32)[None]
    r = np.empty((2, n, n, n))
    r[0] = rho_dis
    r[1] = rho_main
    quarter = max(1, n // 4)
    r[0, :quarter][~solid[:quarter]] = rho_main
    r[1, :quarter][~solid[:quarter]] = rho_dis
    return Workload((n, n, n), ns, r, ncomp=2, tau=(tau, tau), G=G, G_ads=tuple(G_ads), g_scale=3.0,
                    F_ext=(0.0, 0.0, force), name=f"porous{n}_{seed}")


def washburn_channel(G_ads, ns_medium, H=500, L=2, res_width=4, gap=8, rho_main=0.99, rho_dis=0.01) -> Workload:
    """Imbibition channel of Sec. 3.4, one cell deep in z (the paper's 2-D
    set-up; periodic in y, where the state stays uniform, so L only sets the
    tile shape): a fluid-1 reservoir at x < res_width, a free gap of `gap`
    cells, then a homogenized medium of uniform n_s up to the fluid-2
    reservoir at x >= H - res_width; fluid 2 fills the rest at the start.
    Table 1 fluids (0.99 / 0.01, tau = 1), G_inter,12 = 1.75 and
    G_ads,2 = -G_ads,1 = G_ads: fluid 1 wets the medium for G_ads > 0.  The
    paper does not state how its inlet meets the medium; the n_s step at the
    end of the gap is what drives the front here."""
    x0 = res_width + gap
    ns = np.zeros((1, 1, L, H), np.float32)
    ns[..., x0:H - res_width] = ns_medium
    r = np.empty((2, 1, L, H))
    r[0], r[1] = rho_dis, rho_main
    r[0, ..., :res_width], r[1, ..., :res_width] = rho_main, rho_dis
    res = [(0, 0, res_width, (rho_main, rho_dis)), (0, H - res_width, H, (rho_dis, rho_main))]
    return Workload((H, L, 1), ns, r, ncomp=2, tau=(1.0, 1.0), G=1.75, G_ads=(-G_ads, G_ads), g_scale=1.0,
                    reservoirs=res, name=f"washburn{H}_{G_ads}_{ns_medium}")


def buckley_leverett_channel(ns_medium, rho_main, rho_dis, H=100, L=5, res_width=4, force=1e-4,
                             G=1.75) -> Workload:
    """Waterflooding set-up of the Supporting Information (Buckley-Leverett),
    one cell deep in z (the paper's 2-D set-up): a homogenized medium of
    uniform n_s (both components) between a fluid-1 reservoir at
    x < res_width and a fluid-2 reservoir at x >= H - res_width, fluid 2
    everywhere else at the start, no adhesion, G_inter = G, tau = 1, a body
    force along +x (inlet to outlet).  The reservoirs and the initial phases
    hold (rho_main, rho_dis) and (rho_dis, rho_main): the caller chooses them
    (the two fluids' coexistence densities keep the reservoirs in equilibrium
    with the bulk phases)."""
    ns = np.full((1, 1, L, H), ns_medium, np.float32)
    r = np.empty((2, 1, L, H))
    r[0], r[1] = rho_dis, rho_main
    r[0, ..., :res_width], r[1, ..., :res_width] = rho_main, rho_dis
    res = [(0, 0, res_width, (rho_main, rho_dis)), (0, H - res_width, H, (rho_dis, rho_main))]
    return Workload((H, L, 1), ns, r, ncomp=2, tau=(1.0, 1.0), G=G, G_ads=(0.0, 0.0), g_scale=1.0,
                    F_ext=(force, 0.0, 0.0), reservoirs=res, name=f"buckley_leverett_{ns_medium}")


def obstacle_channel(ns1, L=300, H=50, radius=16.5, spacing=60, first=30.0, res_width=4, force=5e-5,
                     rho_main=0.99, rho_dis=0.01) -> Workload:
    """Porous-obstacle channel of Sec. 3.5, one cell deep in z: five discs of
    radius 16.5 on the channel axis y = (H - 1)/2, centres `spacing` apart
    from x = `first` (the paper gives diameter and spacing, not the offset),
    periodic in y.  Two n_s fields: n_s,1 = ns1 inside the discs and 0
    elsewhere, n_s,2 = 0 everywhere.  Fluid-1 reservoir at x < res_width,
    fluid-2 reservoir at x >= L - res_width, fluid 2 elsewhere at the start;
    body force `force` along +x on both fluids; Table 1 fluids, G_inter =
    1.75, no adhesion (the paper states no contact angle here)."""
    y, x = np.meshgrid(np.arange(H), np.arange(L), indexing="ij")
    inside = np.zeros((H, L), bool)
    for k in range(5):
        inside |= (x - (first + spacing * k)) ** 2 + (y - (H - 1) / 2) ** 2 <= radius * radius
    ns = np.zeros((2, 1, H, L), np.float32)
    ns[0, 0][inside] = ns1
    r = np.empty((2, 1, H, L))
    r[0], r[1] = rho_dis, rho_main
    r[0, ..., :res_width], r[1, ..., :res_width] = rho_main, rho_dis
    res = [(0, 0, res_width, (rho_main, rho_dis)), (0, L - res_width, L, (rho_dis, rho_main))]
    return Workload((L, H, 1), ns, r, ncomp=2, tau=(1.0, 1.0), G=1.75, G_ads=(0.0, 0.0), F_ext=(force, 0.0, 0.0),
                    g_scale=1.0, reservoirs=res, name=f"obstacles{L}x{H}_{ns1}")
