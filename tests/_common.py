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
