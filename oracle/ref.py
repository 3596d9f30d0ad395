"""ctypes binding of the plain FP64 CPU oracle (``hmcsc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it to check the GPU library.

All arrays are numpy float64, C-contiguous, in the layouts of ``hmcsc_oracle.h``:
populations ``f[s, i, z, y, x]``, bounce-back fractions ``ns[k, z, y, x]``,
densities ``rho[s, z, y, x]``, velocity ``u[a, z, y, x]``, pressure ``p[z, y, x]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hmcsc_oracle.c")
LIB = os.path.join(HERE, "libhmcsc_oracle.so")
# A compiled copy elsewhere (the tests' mutation check loads deliberately
# broken copies this way); never rebuilt here.
LIB_OVERRIDE = os.environ.get("HMCSC_ORACLE_LIB")
MAX_RES = 4
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def compile_to(src: str, out: str, verbose: bool = False) -> str:
    """Compile an oracle source with gcc (plain -O2, no fast-math, no FMA contraction)."""
    cmd = ["gcc", *CFLAGS, "-I", HERE, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return compile_to(SRC, LIB, verbose)


class _Res(C.Structure):
    _fields_ = [("axis", C.c_int32), ("lo", C.c_int32), ("hi", C.c_int32), ("pad", C.c_int32),
                ("rho", C.c_double * 2)]


class _Params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("ncomp", C.c_int32), ("c_ns", C.c_int32), ("n_res", C.c_int32),
                ("nthreads", C.c_int32), ("tau", C.c_double * 2), ("G", C.c_double),
                ("G_ads", C.c_double * 2), ("F_ext", C.c_double * 3), ("g_scale", C.c_double),
                ("res", _Res * MAX_RES), ("forcing", C.c_int32), ("pad", C.c_int32)]


FORCING = {"shan-chen": 0, "guo": 1}


@dataclass
class Reservoir:
    """Slab ``lo <= coord[axis] < hi`` held at the rest equilibrium of ``rho``."""
    axis: int
    lo: int
    hi: int
    rho: Sequence[float]


@dataclass
class Setup:
    shape: tuple  # (nx, ny, nz)
    ncomp: int = 2
    c_ns: int = 1
    tau: Sequence[float] = (1.0, 1.0)
    G: float = 0.0
    G_ads: Sequence[float] = (0.0, 0.0)
    F_ext: Sequence[float] = (0.0, 0.0, 0.0)
    g_scale: float = 1.0
    lattice: int = 19
    reservoirs: list = field(default_factory=list)
    nthreads: int = 0
    forcing: str = "shan-chen"  # "guo": the GS-WBS with Guo forcing, Eq. (GS-WBS)


def params_struct(s: Setup) -> _Params:
    p = _Params()
    p.lattice = s.lattice
    p.nx, p.ny, p.nz = (int(v) for v in s.shape)
    p.ncomp, p.c_ns, p.nthreads = s.ncomp, s.c_ns, s.nthreads
    p.n_res = len(s.reservoirs)
    if p.n_res > MAX_RES:
        raise ValueError("too many reservoirs")
    t = list(s.tau) + [1.0] * (2 - len(s.tau))
    p.tau[0], p.tau[1] = t[0], t[1]
    p.G = s.G
    ga = list(s.G_ads) + [0.0] * (2 - len(s.G_ads))
    p.G_ads[0], p.G_ads[1] = ga[0], ga[1]
    for a in range(3):
        p.F_ext[a] = s.F_ext[a]
    p.g_scale = s.g_scale
    p.forcing = FORCING[s.forcing]
    for k, r in enumerate(s.reservoirs):
        p.res[k].axis, p.res[k].lo, p.res[k].hi = r.axis, r.lo, r.hi
        rr = list(r.rho) + [0.0] * (2 - len(r.rho))
        p.res[k].rho[0], p.res[k].rho[1] = rr[0], rr[1]
    return p


_lib = None


def _load():
    global _lib
    if _lib is None:
        if LIB_OVERRIDE:
            lib = C.CDLL(LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            lib = C.CDLL(LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        pp = C.POINTER(_Params)
        lib.href_lattice.argtypes = [C.c_int32, C.POINTER(C.c_int32),
                                     np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"), dp,
                                     np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")]
        lib.href_init.argtypes = [pp, dp, dp]
        lib.href_step.argtypes = [pp, dp, dp, dp]
        lib.href_run.argtypes = [pp, dp, dp, dp, C.c_int64]
        lib.href_moments.argtypes = [pp, dp, dp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.href_cell_update.argtypes = [pp, dp, dp, C.c_int64,
                                         np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"), dp]
        for fn in ("href_lattice", "href_init", "href_step", "href_run", "href_moments",
                   "href_cell_update"):
            getattr(lib, fn).restype = C.c_int
        _lib = lib
    return _lib


def lattice(which: int = 19):
    """Velocity set of the oracle: (c[q,3] int, w[q], opp[q])."""
    lib = _load()
    q = C.c_int32()
    c = np.zeros(3 * 19, np.int32)
    w = np.zeros(19, np.float64)
    opp = np.zeros(19, np.int32)
    if lib.href_lattice(which, C.byref(q), c, w, opp):
        raise ValueError("unknown lattice")
    n = q.value
    return c[: 3 * n].reshape(n, 3).copy(), w[:n].copy(), opp[:n].copy()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One configured problem of the oracle; state arrays are passed explicitly."""

    def __init__(self, setup: Setup, ns: np.ndarray):
        self.setup = setup
        self.p = params_struct(setup)
        self.lib = _load()
        nx, ny, nz = setup.shape
        self.q = 19 if setup.lattice == 19 else 9
        self.N = nx * ny * nz
        ns = np.ascontiguousarray(ns, dtype=np.float64).reshape(setup.c_ns, nz, ny, nx)
        self.ns = ns

    def pop_shape(self):
        nx, ny, nz = self.setup.shape
        return (self.setup.ncomp, self.q, nz, ny, nx)

    def init(self, rho_init: np.ndarray) -> np.ndarray:
        nx, ny, nz = self.setup.shape
        r = np.ascontiguousarray(rho_init, dtype=np.float64).reshape(self.setup.ncomp, nz, ny, nx)
        f = np.empty(self.pop_shape(), np.float64)
        if self.lib.href_init(C.byref(self.p), r, f):
            raise ValueError("href_init rejected the parameters")
        return f

    def step(self, f: np.ndarray) -> np.ndarray:
        out = np.empty_like(f)
        if self.lib.href_step(C.byref(self.p), self.ns, np.ascontiguousarray(f), out):
            raise ValueError("href_step failed")
        return out

    def run(self, f: np.ndarray, nsteps: int) -> np.ndarray:
        a = np.array(f, dtype=np.float64, order="C", copy=True)
        work = np.empty_like(a)
        if self.lib.href_run(C.byref(self.p), self.ns, a, work, int(nsteps)):
            raise ValueError("href_run failed")
        return a

    def moments(self, f: np.ndarray):
        """Returns dict(rho[s,z,y,x], u[a,z,y,x], p[z,y,x], ftot[s,a,z,y,x])."""
        nx, ny, nz = self.setup.shape
        C_ = self.setup.ncomp
        rho = np.empty((C_, nz, ny, nx))
        u = np.empty((3, nz, ny, nx))
        p = np.empty((nz, ny, nx))
        ft = np.empty((C_, 3, nz, ny, nx))
        if self.lib.href_moments(C.byref(self.p), self.ns, np.ascontiguousarray(f), _ptr(rho),
                                 _ptr(u), _ptr(p), _ptr(ft)):
            raise ValueError("href_moments failed")
        return {"rho": rho, "u": u, "p": p, "ftot": ft}

    def cell_update(self, f: np.ndarray, cells: np.ndarray) -> np.ndarray:
        """State at t+1 at the given flat cell indices: out[k, s, i]."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((len(cells), self.setup.ncomp, self.q))
        if self.lib.href_cell_update(C.byref(self.p), self.ns, np.ascontiguousarray(f),
                                     len(cells), cells, out):
            raise ValueError("href_cell_update failed")
        return out
