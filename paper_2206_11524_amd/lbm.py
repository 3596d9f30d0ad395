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
STORE_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
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
                ("rounding", C.c_int32), ("forcing", C.c_int32), ("res", Reservoir * MAX_RES)]


class Sizes(C.Structure):
    _fields_ = [("pop_bytes", C.c_uint64), ("ns_bytes", C.c_uint64), ("scratch_bytes", C.c_uint64)]


class DeviceBuffers(C.Structure):
    _fields_ = [("f_a", C.c_void_p), ("f_b", C.c_void_p), ("n_s", C.c_void_p), ("scratch", C.c_void_p)]


class FillQuery(C.Structure):
    _fields_ = [("axis", C.c_int32), ("inlet_lo", C.c_int32), ("inlet_hi", C.c_int32),
                ("outlet_lo", C.c_int32), ("outlet_hi", C.c_int32), ("pore_lo", C.c_int32),
                ("pore_hi", C.c_int32), ("comp", C.c_int32), ("threshold", C.c_double)]


class FillState(C.Structure):
    _fields_ = [("dp", C.c_double), ("p_inlet", C.c_double), ("p_outlet", C.c_double),
                ("saturation", C.c_double), ("pore_volume", C.c_double), ("time", C.c_int64)]


class Permeability(C.Structure):
    _fields_ = [("k", C.c_double), ("k_comp", C.c_double * 2), ("momentum", C.c_double), ("nu", C.c_double),
                ("time", C.c_int64)]


class DropletQuery(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("r_core", C.c_double), ("r_far", C.c_double), ("margin", C.c_double),
                ("comp", C.c_int32), ("pad", C.c_int32)]


class DropletState(C.Structure):
    _fields_ = [("R", C.c_double), ("dp", C.c_double), ("gamma", C.c_double), ("p_in", C.c_double),
                ("p_out", C.c_double), ("rho_in", C.c_double), ("rho_out", C.c_double), ("time", C.c_int64)]


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
    "lbm_totals_get_static": (C.c_int, [C.c_void_p, C.POINTER(Totals)]),
    "lbm_fill_state_get": (C.c_int, [C.c_void_p, C.POINTER(FillQuery), C.POINTER(FillState)]),
    "lbm_permeability_get": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Permeability)]),
    "lbm_droplet_get": (C.c_int, [C.c_void_p, C.POINTER(DropletQuery), C.POINTER(DropletState)]),
    "lbm_get_populations": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_set_populations": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_set_reservoir": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_time": (C.c_int64, [C.c_void_p]),
    "lbm_set_time": (C.c_int, [C.c_void_p, C.c_int64]),
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
    """Shift rho0 for the stored populations: zero for FP64; for FP32 and the
    16-bit formats the smallest initial density of each component (its
    dissolved density in a two-phase set-up), so the stored values are the
    deviations f - w_i rho0, small where a component is dilute or the flow is
    slow, and carry full relative precision."""
    if storage == "f64":
        return (0.0, 0.0)
    out = [float(rho_init[s].min()) for s in range(ncomp)]
    return tuple(out + [0.0] * (2 - len(out)))


ROUNDING = {"nearest": 0, "stochastic": 1}
# "shan-chen": the HMCSC; "guo": the GS-WBS with Guo forcing (Eq. GS-WBS)
FORCING = {"shan-chen": 0, "guo": 1}


def default_rounding(storage: str) -> str:
    """Stochastic rounding for the 16-bit formats (unbiased: slow changes are
    not rounded away step after step), nearest otherwise."""
    return "stochastic" if storage in ("f16s", "bf16s") else "nearest"


def make_params(ncomp=2, c_ns=1, tau=(1.0, 1.0), G=0.0, G_ads=(0.0, 0.0), F_ext=(0.0, 0.0, 0.0),
                g_scale=1.0, storage="f64", rho_shift=(0.0, 0.0), store_scale_log2=0,
                reservoirs: Sequence = (), check_every=0, rounding=None, forcing="shan-chen") -> Params:
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
    p.rounding = ROUNDING[rounding or default_rounding(storage)]
    p.forcing = FORCING[forcing]
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

    def set_time(self, t: int):
        _check(self.lib.lbm_set_time(self.ctx, int(t)), "lbm_set_time")

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

    def fill_state(self, axis, inlet, outlet, pore, comp=0, threshold=0.5):
        """Capillary pressure (Eq. CapPressure) and saturation (Eq. Saturation)
        on slabs given as (lo, hi) coordinate ranges along ``axis``."""
        q = FillQuery(axis, inlet[0], inlet[1], outlet[0], outlet[1], pore[0], pore[1], comp, threshold)
        out = FillState()
        _check(self.lib.lbm_fill_state_get(self.ctx, C.byref(q), C.byref(out)), "lbm_fill_state_get")
        return {"dp": out.dp, "p_inlet": out.p_inlet, "p_outlet": out.p_outlet, "saturation": out.saturation,
                "pore_volume": out.pore_volume, "time": out.time}

    def permeability(self, axis=0):
        """Permeability of Eq. (Permeability) along ``axis`` with each
        component's share (see ``lbm_permeability_get``)."""
        out = Permeability()
        _check(self.lib.lbm_permeability_get(self.ctx, axis, C.byref(out)), "lbm_permeability_get")
        return {"k": out.k, "k_comp": (out.k_comp[0], out.k_comp[1]), "momentum": out.momentum, "nu": out.nu,
                "time": out.time}

    def droplet(self, center, r_core, r_far, margin=4.0, comp=0):
        """Static-droplet measurement (Sec. 3.3, see ``lbm_droplet_get``):
        radius from the component's volume, pressure jump and interfacial tension."""
        q = DropletQuery((C.c_double * 3)(*center), r_core, r_far, margin, comp, 0)
        out = DropletState()
        _check(self.lib.lbm_droplet_get(self.ctx, C.byref(q), C.byref(out)), "lbm_droplet_get")
        return {k: getattr(out, k) for k, _ in DropletState._fields_}

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


def from_workload(w, storage="f32", rho_shift=None, store_scale_log2=0, check_every=0, rounding=None,
                  forcing="shan-chen", **kw) -> Simulation:
    """Simulation of an ``inputs.Workload``."""
    if rho_shift is None:
        rho_shift = default_shift(storage, w.ncomp, w.rho)
    p = make_params(ncomp=w.ncomp, c_ns=w.c_ns, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext,
                    g_scale=w.g_scale, storage=storage, rho_shift=rho_shift,
                    store_scale_log2=store_scale_log2, reservoirs=w.reservoirs, check_every=check_every,
                    rounding=rounding, forcing=forcing)
    return Simulation(w.shape, w.ns, w.rho, p, **kw)


# ---------------------------------------------------------------------------
# Batched stepping and serving.

class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_slots", C.c_int32), ("steps_per_tick", C.c_int32),
                ("storage", C.c_int32), ("ncomp", C.c_int32), ("c_ns", C.c_int32), ("max_cells", C.c_int64),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("policy", C.c_int32), ("pad", C.c_int32),
                ("run_cells", C.c_int64)]


SERVE_POLICY = {"fair": 0, "shortest-first": 1}


class Request(C.Structure):
    _fields_ = [("dom", Domain), ("n_s", C.c_void_p), ("rho_init", C.c_void_p), ("params", Params),
                ("max_steps", C.c_int64), ("conv_tol", C.c_double), ("conv_window", C.c_int32),
                ("conv_noise", C.c_int32), ("rho_out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("converged", C.c_int32), ("steps_done", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double), ("totals", Totals)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("queued", C.c_int64), ("active", C.c_int64),
                ("cell_updates", C.c_double), ("busy_seconds", C.c_double), ("uptime_seconds", C.c_double),
                ("bytes_resident", C.c_uint64), ("ticks", C.c_int64)]


SERVE_SIGNATURES = {
    "lbm_group_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "lbm_group_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_group_last_step_ms": (C.c_double, [C.c_void_p]),
    "lbm_group_destroy": (None, [C.c_void_p]),
    "lbm_server_create": (C.c_int, [C.POINTER(ServerCfg), C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_batch_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "lbm_batch_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Result)]),
    "lbm_batch_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double, C.POINTER(Result)]),
    "lbm_server_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "lbm_server_destroy": (None, [C.c_void_p]),
}


def _serve_lib():
    lib = _lib()
    if not getattr(lib, "_serve_ready", False):
        for name, (res, args) in SERVE_SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._serve_ready = True
    return lib


class Group:
    """Several Simulations stepped together, one batched launch per step."""

    def __init__(self, sims):
        self.lib = _serve_lib()
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.ctx.value for s in self.sims])
        g = C.c_void_p()
        _check(self.lib.lbm_group_create(arr, len(self.sims), C.byref(g)), "lbm_group_create")
        self.g = g

    def step(self, n: int):
        _check(self.lib.lbm_group_step(self.g, int(n)), "lbm_group_step")

    def last_step_ms(self) -> float:
        return float(self.lib.lbm_group_last_step_ms(self.g))

    def close(self):
        if getattr(self, "g", None):
            self.lib.lbm_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (worker thread inside the library)."""

    def __init__(self, storage="f16s", ncomp=2, c_ns=1, max_slots=64, steps_per_tick=100, max_cells=192 ** 3,
                 hbm_budget_bytes=0, tile=(0, 0), policy="fair", run_cells=0):
        self.lib = _serve_lib()
        cfg = ServerCfg(int(hbm_budget_bytes), int(max_slots), int(steps_per_tick),
                        STORAGE[storage] if isinstance(storage, str) else int(storage), ncomp, c_ns,
                        int(max_cells), tile[0], tile[1],
                        SERVE_POLICY[policy] if isinstance(policy, str) else int(policy), 0, int(run_cells))
        s = C.c_void_p()
        _check(self.lib.lbm_server_create(C.byref(cfg), None, C.byref(s)), "lbm_server_create")
        self.s = s
        self.storage = storage
        self._keep = {}

    def submit(self, shape, ns, rho_init, params: Params, max_steps: int, conv_tol: float = 0.0,
               want_rho: bool = False, conv_window: int = 0, conv_noise: bool = False) -> int:
        ns = np.ascontiguousarray(ns, dtype=np.float32)
        rho_init = np.ascontiguousarray(rho_init, dtype=np.float64)
        out = np.empty_like(rho_init) if want_rho else None
        rq = Request(Domain(*[int(v) for v in shape]), ns.ctypes.data, rho_init.ctypes.data, params,
                     int(max_steps), float(conv_tol), int(conv_window), int(bool(conv_noise)),
                     out.ctypes.data if out is not None else None)
        t = C.c_uint64()
        _check(self.lib.lbm_batch_submit(self.s, C.byref(rq), C.byref(t)), "lbm_batch_submit")
        if out is not None:
            self._keep[t.value] = out
        return t.value

    def submit_workload(self, w, max_steps, conv_tol=0.0, want_rho=False, rho_shift=None, rounding=None,
                        conv_window=0, conv_noise=False):
        if rho_shift is None:
            rho_shift = default_shift(self.storage, w.ncomp, w.rho)
        p = make_params(ncomp=w.ncomp, c_ns=w.c_ns, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext,
                        g_scale=w.g_scale, storage=self.storage, rho_shift=rho_shift, reservoirs=w.reservoirs,
                        rounding=rounding)
        return self.submit(w.shape, w.ns, w.rho, p, max_steps, conv_tol, want_rho, conv_window, conv_noise)

    def poll(self, ticket):
        r = Result()
        rc = self.lib.lbm_batch_poll(self.s, C.c_uint64(ticket), C.byref(r))
        if rc == LBM_EAGAIN:
            return None
        _check(rc, "lbm_batch_poll")
        return self._result(ticket, r)

    def wait(self, ticket, timeout_s=-1.0):
        r = Result()
        rc = self.lib.lbm_batch_wait(self.s, C.c_uint64(ticket), float(timeout_s), C.byref(r))
        if rc == LBM_EAGAIN:
            return None
        _check(rc, "lbm_batch_wait")
        return self._result(ticket, r)

    def _result(self, ticket, r):
        return {"status": r.status, "converged": bool(r.converged), "steps_done": r.steps_done,
                "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                "mass": list(r.totals.mass), "momentum": list(r.totals.momentum),
                "rho": self._keep.pop(ticket, None)}

    def stats(self):
        st = ServerStats()
        _check(self.lib.lbm_server_stats_get(self.s, C.byref(st)), "lbm_server_stats_get")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "s", None):
            self.lib.lbm_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
