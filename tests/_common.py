"""Shared test helpers: build the oracle and the GPU simulation of one workload
from the same host arrays (only the seeded input generators are shared)."""
import numpy as np

from oracle.ref import Oracle, Reservoir, Setup


def oracle_for(w, nthreads=0, forcing="shan-chen"):
    res = [Reservoir(a, lo, hi, tuple(r)) for (a, lo, hi, r) in w.reservoirs]
    st = Setup(w.shape, ncomp=w.ncomp, c_ns=w.c_ns, tau=tuple(w.tau) + (1.0,) * (2 - len(w.tau)),
               G=w.G, G_ads=w.G_ads, F_ext=w.F_ext, g_scale=w.g_scale, reservoirs=res,
               nthreads=nthreads, forcing=forcing)
    return Oracle(st, w.ns.astype(np.float64))


def rel_max_err(a, b):
    """max |a - b| / max |b| (field max-norm relative error)."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def front_position(rho, x0, tail=5):
    """Washburn front (Sec. 3.4): the last x >= x0 where rho_1 - rho_2,
    averaged over y and z, changes sign from positive to negative, refined by
    linear interpolation, measured from x0; None before the front reaches x0.
    rho is [2, nz, ny, nx]; the last `tail` cells (outlet reservoir) are left out."""
    r = rho.mean(axis=(1, 2))
    phi = r[0] - r[1]
    idx = np.nonzero((phi[x0:-tail] > 0) & (phi[x0 + 1:-tail + 1] <= 0))[0]
    if not len(idx):
        return None
    i = idx[-1] + x0
    return i + phi[i] / (phi[i] - phi[i + 1]) - x0


def washburn_contact_angle(rate, B, gamma=0.077, eta=1.0 / 6.0):
    """Contact angle (degrees) behind a Washburn rate (Eq. Washburn): the fit
    x_inter^2 = rate * t gives A^2 = rate / B at a given B, and A^2 = gamma
    cos(theta) / (2 eta), so cos(theta) = 2 eta rate / (B gamma).  gamma is
    the interfacial tension of the Table 1 fluids at G_inter = 1.75 (the
    large-domain value of Sec. 3.3), eta = rho nu with tau = 1 and the
    nominal density 1 (the pair that turns Table 3's A column into its theta
    column, gamma / (2 eta) = 0.231).  Returns 0
    where the rate exceeds what complete wetting allows (cos > 1)."""
    c = 2.0 * eta * rate / (B * gamma)
    return float(np.degrees(np.arccos(min(c, 1.0))))


def huang_contact_angle(G_ads, G_inter=1.75, rho_1=0.99, rho_dis=0.01):
    """theta_H of Eq. (contactAngle), degrees: cos = 4 G_ads / (G_inter (rho_1 - rho_dis))."""
    return float(np.degrees(np.arccos(4.0 * G_ads / (G_inter * (rho_1 - rho_dis)))))


def build_c_driver(out):
    """Compile tests/c_driver/abi_driver.c against include/lbm.h and link it to
    the built library (gcc only; no Python or PyTorch in the program)."""
    import os
    import subprocess

    from paper_2206_11524_amd import lbm

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.dirname(lbm.LIB_PATH)
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(root, "include"),
           os.path.join(root, "tests", "c_driver", "abi_driver.c"), "-L", pkg, "-lhmcsc", f"-Wl,-rpath,{pkg}",
           "-Wl,-rpath-link,/opt/rocm/lib", "-lm", "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out

