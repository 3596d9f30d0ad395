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

