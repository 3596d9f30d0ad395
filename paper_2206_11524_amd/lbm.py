"""ctypes binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

PyTorch provides the device memory (one uint8 tensor per buffer, sized by
``lbm_required_bytes``) and the HIP stream (the current torch stream); every
step of the method runs in the HIP library ``libhmcsc.so``.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(PKG, "libhmcsc.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ENOTFOUND, LBM_EAGAIN = 0, -1, -2, -3, -4, -5, -6
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
MAX_RES = 4
Q = 19


class LbmError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_lib().lbm_strerror(code).decode()} ({code})")


class Domain(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class Reservoir(C.Structure):
    _fields_ = [("axis", C.c_int32), ("lo", C.c_int32), ("hi", C.c_int32), ("pad", C.c_int32),
                ("rho", C.c_double * 2)]


class Params(C.Structure):
    _fields_ = [("ncomp", C.c_int32), ("c_ns", C.c_int32), ("tau", C.c_double * 2),
                ("G_inter", C.c_double), ("G_ads", C.c_double * 2), ("F_ext", C.c_double * 3),
                ("g_scale", C.c_double), ("rho_shift", C.c_double * 2), ("storage", C.c_int32),
                ("store_scale_log2", C.c_int32), ("n_res", C.c_int32), ("check_every", C.c_int32),
                ("res", Reservoir * MAX_RES)]


class Sizes(C.Structure):
    _fields_ = [("pop_bytes", C.c_uint64), ("ns_bytes", C.c_uint64), ("scratch_bytes", C.c_uint64)]


class DeviceBuffers(C.Structure):
    _fields_ = [("f_a", C.c_void_p), ("f_b", C.c_void_p), ("n_s", C.c_void_p), ("scratch", C.c_void_p)]


class Totals(C.Structure):
    _fields_ = [("mass", C.c_double * 2), ("momentum", C.c_double * 3), ("time", C.c_int64),
                ("finite", C.c_int32), ("pad", C.c_int32)]


_LIB = None

# every symbol the header declares, with its signature
SIGNATURES = {
    "lbm_required_bytes": (C.c_int, [C.POINTER(Domain), C.POINTER(Params), C.POINTER(Sizes)]),
    "lbm_create": (C.c_int, [C.POINTER(Domain), C.c_void_p, C.c_void_p, C.POINTER(Params),
                             C.POINTER(DeviceBuffers), C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_moments": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Totals)]),
    "lbm_totals_get": (C.c_int, [C.c_void_p, C.POINTER(Totals)]),
    "lbm_get_populations": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_set_populations": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_set_reservoir": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_time": (C.c_int64, [C.c_void_p]),
    "lbm_sync": (C.c_int, [C.c_void_p]),
    "lbm_last_step_ms": (C.c_double, [C.c_void_p]),
    "lbm_destroy": (None, [C.c_void_p]),
    "lbm_strerror": (C.c_char_p, [C.c_int]),
}


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run python -m paper_2206_11524_amd.build)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(code: int, what: str):
    if code != LBM_OK:
        raise LbmError(code, what)


def default_shift(storage: str, ncomp: int, rho_init: np.ndarray):
    """Shift rho0 for the stored populations: zero for the plain FP64/FP32
    formats; for the 16-bit formats the smallest initial density of each
    component (its dissolved density in a two-phase set-up), so populations of
    a component where it is dilute are stored as small numbers with full
    relative precision."""
    if storage in ("f64", "f32"):
        return (0.0, 0.0)
    out = [float(rho_init[s].min()) for s in range(ncomp)]
    return tuple(out + [0.0] * (2 - len(out)))


def make_params(ncomp=2, c_ns=1, tau=(1.0, 1.0), G=0.0, G_ads=(0.0, 0.0), F_ext=(0.0, 0.0, 0.0),
                g_scale=1.0, storage="f64", rho_shift=(0.0, 0.0), store_scale_log2=0,
                reservoirs: Sequence = (), check_every=0) -> Params:
    p = Params()
    p.ncomp, p.c_ns = ncomp, c_ns
    t = list(tau) + [1.0] * (2 - len(tau))
    p.tau[0], p.tau[1] = t[0], t[1]
    p.G_inter = G
    ga = list(G_ads) + [0.0] * (2 - len(G_ads))
    p.G_ads[0], p.G_ads[1] = ga[0], ga[1]
    for a in range(3):
        p.F_ext[a] = F_ext[a]
    p.g_scale = g_scale
    rs = list(rho_shift) + [0.0] * (2 - len(rho_shift))
    p.rho_shift[0], p.rho_shift[1] = rs[0], rs[1]
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.store_scale_log2 = store_scale_log2
    p.n_res = len(reservoirs)
    for k, (axis, lo, hi, rho) in enumerate(reservoirs):
        p.res[k].axis, p.res[k].lo, p.res[k].hi = axis, lo, hi
        rr = list(rho) + [0.0] * (2 - len(rho))
        p.res[k].rho[0], p.res[k].rho[1] = rr[0], rr[1]
    p.check_every = check_every
    return p


def required_bytes(shape, params: Params) -> Sizes:
    d = Domain(*[int(v) for v in shape])
    s = Sizes()
    _check(_lib().lbm_required_bytes(C.byref(d), C.byref(params), C.byref(s)), "lbm_required_bytes")
    return s


class Simulation:
    """One HMCSC domain on the current GPU.

    ``ns``: float32 [c_ns, nz, ny, nx]; ``rho_init``: float64 [ncomp, nz, ny, nx].
    Device buffers are torch tensors owned by this object (``library_alloc=True``
    lets the library allocate instead).
    """

    def __init__(self, shape, ns, rho_init, params: Params, stream=None, library_alloc=False):
        import torch

        self.lib = _lib()
        self.shape = tuple(int(v) for v in shape)
        self.params = params
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.ncomp = params.ncomp
        ns = np.ascontiguousarray(ns, dtype=np.float32)
        rho_init = np.ascontiguousarray(rho_init, dtype=np.float64)
        if ns.size != params.c_ns * self.N or rho_init.size != params.ncomp * self.N:
            raise ValueError("n_s / rho_init sizes do not match the domain")
        self.sizes = required_bytes(self.shape, params)
        self._tensors = []
        bufs = None
        if not library_alloc:
            dev = torch.device("cuda", torch.cuda.current_device())

            def alloc(n):
                t = torch.empty(max(int(n), 256), dtype=torch.uint8, device=dev)
                self._tensors.append(t)
                return t.data_ptr()

            bufs = DeviceBuffers(alloc(self.sizes.pop_bytes), alloc(self.sizes.pop_bytes),
                                 alloc(self.sizes.ns_bytes), alloc(self.sizes.scratch_bytes))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        ctx = C.c_void_p()
        d = Domain(nx, ny, nz)
        _check(self.lib.lbm_create(C.byref(d), ns.ctypes.data, rho_init.ctypes.data, C.byref(params),
                                   C.byref(bufs) if bufs is not None else None, C.c_void_p(stream),
                                   C.byref(ctx)), "lbm_create")
        self.ctx = ctx

    # -- stepping ---------------------------------------------------------
    def step(self, n: int = 1):
        _check(self.lib.lbm_step(self.ctx, int(n)), "lbm_step")

    def sync(self):
        _check(self.lib.lbm_sync(self.ctx), "lbm_sync")

    @property
    def time(self) -> int:
        return int(self.lib.lbm_time(self.ctx))

    def last_step_ms(self) -> float:
        return float(self.lib.lbm_last_step_ms(self.ctx))

    # -- outputs ----------------------------------------------------------
    def moments(self, fields=True):
        nx, ny, nz = self.shape
        tot = Totals()
        if fields:
            rho = np.empty((self.ncomp, nz, ny, nx))
            u = np.empty((3, nz, ny, nx))
            p = np.empty((nz, ny, nx))
            _check(self.lib.lbm_moments(self.ctx, rho.ctypes.data, u.ctypes.data, p.ctypes.data,
                                        C.byref(tot)), "lbm_moments")
        else:
            rho = u = p = None
            _check(self.lib.lbm_totals_get(self.ctx, C.byref(tot)), "lbm_totals_get")
        return {"rho": rho, "u": u, "p": p, "mass": np.array(tot.mass[: self.ncomp]),
                "momentum": np.array(tot.momentum[:]), "time": tot.time, "finite": bool(tot.finite)}

    def totals(self):
        return self.moments(fields=False)

    def populations(self) -> np.ndarray:
        nx, ny, nz = self.shape
        f = np.empty((self.ncomp, Q, nz, ny, nx))
        _check(self.lib.lbm_get_populations(self.ctx, f.ctypes.data), "lbm_get_populations")
        return f

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.size != self.ncomp * Q * self.N:
            raise ValueError("population array has the wrong size")
        _check(self.lib.lbm_set_populations(self.ctx, f.ctypes.data), "lbm_set_populations")

    def set_reservoir(self, r: int, rho):
        arr = (C.c_double * 2)(*(list(rho) + [0.0] * (2 - len(rho))))
        _check(self.lib.lbm_set_reservoir(self.ctx, int(r), arr), "lbm_set_reservoir")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None
        self._tensors = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(w, storage="f32", rho_shift=None, store_scale_log2=0, check_every=0, **kw) -> Simulation:
    """Simulation of an ``inputs.Workload``."""
    if rho_shift is None:
        rho_shift = default_shift(storage, w.ncomp, w.rho)
    p = make_params(ncomp=w.ncomp, c_ns=w.c_ns, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext,
                    g_scale=w.g_scale, storage=storage, rho_shift=rho_shift,
                    store_scale_log2=store_scale_log2, reservoirs=w.reservoirs, check_every=check_every)
    return Simulation(w.shape, w.ns, w.rho, p, **kw)
