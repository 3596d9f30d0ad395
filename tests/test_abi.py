"""The C ABI library loads and exports every function include/lbm.h declares,
and its host-side validation and sizing behave as documented.  No compute call
is made here (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2206_11524_amd import lbm

from _common import build_c_driver

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_\w+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        pytest.fail("libhmcsc.so is not built (run python -m paper_2206_11524_amd.build)")
    return lbm._lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 12
    for n in sorted(names):
        assert hasattr(lib, n), n
    # and the binding covers all of them
    assert names <= set(lbm.SIGNATURES) | set(getattr(lbm, "SERVE_SIGNATURES", {}))


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert lib.lbm_strerror(code)


def test_required_bytes_matches_layout(lib):
    for storage, b in (("f64", 8), ("f32", 4), ("f16s", 2), ("bf16s", 2)):
        p = lbm.make_params(ncomp=2, c_ns=1, storage=storage)
        s = lbm.required_bytes((256, 256, 256), p)
        assert s.pop_bytes == 2 * 19 * 256 ** 3 * b
        assert s.ns_bytes == 4 * 256 ** 3
        assert s.scratch_bytes >= 8 * (2 + 3 + 1) * 256 ** 3


@pytest.mark.parametrize("bad", [
    dict(ncomp=3), dict(ncomp=1, c_ns=2), dict(tau=(0.5, 1.0)), dict(tau=(1.0, 0.4)),
    dict(storage=7), dict(storage="f32", store_scale_log2=3), dict(G=float("nan")),
    dict(reservoirs=[(3, 0, 1, (1.0, 0.0))]), dict(reservoirs=[(2, 0, 99, (1.0, 0.0))]),
    dict(check_every=-1),
])
def test_invalid_parameters_rejected_before_any_device_work(lib, bad):
    p = lbm.make_params(**{**dict(ncomp=2, c_ns=1, tau=(1.0, 1.0)), **bad})
    d = lbm.Domain(8, 8, 8)
    s = lbm.Sizes()
    assert lib.lbm_required_bytes(C.byref(d), C.byref(p), C.byref(s)) == lbm.LBM_EINVAL
    ns = np.zeros(8 ** 3, np.float32)
    rho = np.ones(2 * 8 ** 3)
    ctx = C.c_void_p(1)
    rc = lib.lbm_create(C.byref(d), ns.ctypes.data, rho.ctypes.data, C.byref(p), None, None, C.byref(ctx))
    assert rc == lbm.LBM_EINVAL
    assert not ctx.value


def test_invalid_rounding_mode_rejected(lib):
    p = lbm.make_params(ncomp=2, c_ns=1, storage="f16s")
    p.rounding = 2
    d, s = lbm.Domain(8, 8, 8), lbm.Sizes()
    assert lib.lbm_required_bytes(C.byref(d), C.byref(p), C.byref(s)) == lbm.LBM_EINVAL


def test_invalid_forcing_scheme_rejected(lib):
    p = lbm.make_params(ncomp=2, c_ns=1, storage="f32", forcing="guo")
    d, s = lbm.Domain(8, 8, 8), lbm.Sizes()
    assert lib.lbm_required_bytes(C.byref(d), C.byref(p), C.byref(s)) == lbm.LBM_OK
    p.forcing = 2
    assert lib.lbm_required_bytes(C.byref(d), C.byref(p), C.byref(s)) == lbm.LBM_EINVAL


@pytest.mark.parametrize("field,value", [("policy", 2), ("policy", -1), ("pad", 1), ("run_cells", -5)])
def test_invalid_server_config_rejected(lib, field, value):
    """Rejected before the library touches a device (so this runs without one)."""
    lbm._serve_lib()
    cfg = lbm.ServerCfg(0, 4, 10, lbm.STORAGE["f32"], 2, 1, 32 ** 3, 64, 8, 0, 0, 0)
    setattr(cfg, field, value)
    s = C.c_void_p()
    assert lib.lbm_server_create(C.byref(cfg), None, C.byref(s)) == lbm.LBM_EINVAL
    assert not s.value


_STRUCTS = ["lbm_domain", "lbm_reservoir", "lbm_params", "lbm_sizes", "lbm_device_buffers", "lbm_totals",
            "lbm_fill_query", "lbm_fill_state", "lbm_permeability", "lbm_droplet_query", "lbm_droplet_state",
            "lbm_server_cfg", "lbm_request",
            "lbm_result", "lbm_server_stats"]


def _ctypes_of(name):
    return {"lbm_domain": lbm.Domain, "lbm_reservoir": lbm.Reservoir, "lbm_params": lbm.Params,
            "lbm_sizes": lbm.Sizes, "lbm_device_buffers": lbm.DeviceBuffers, "lbm_totals": lbm.Totals,
            "lbm_fill_query": lbm.FillQuery, "lbm_fill_state": lbm.FillState,
            "lbm_permeability": lbm.Permeability, "lbm_droplet_query": lbm.DropletQuery,
            "lbm_droplet_state": lbm.DropletState,
            "lbm_server_cfg": lbm.ServerCfg, "lbm_request": lbm.Request, "lbm_result": lbm.Result,
            "lbm_server_stats": lbm.ServerStats}[name]


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every struct of include/lbm.h has, as compiled by the host C compiler,
    the size and field offsets of its ctypes mirror in the binding."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', 'int main(void) {']
    for st in _STRUCTS:
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for fname, _ in _ctypes_of(st)._fields_:
            lines.append(f'printf("{st} {fname} %zu\\n", offsetof({st}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in _STRUCTS:
        cls = _ctypes_of(st)
        assert got[(st, "size")] == C.sizeof(cls), st
        for fname, _ in cls._fields_:
            assert got[(st, fname)] == getattr(cls, fname).offset, (st, fname)


@pytest.mark.parametrize("shape", [(0, 4, 4), (4, -1, 4), (8192, 4096, 1), (65536, 256, 65536)])
def test_bad_domains_rejected(lib, shape):
    """Empty axes, a plane too large for one 32-bit addressed plane block
    (19 * 8 bytes per cell), and 2^40 cells or more are rejected."""
    p = lbm.make_params()
    d = lbm.Domain(*shape)
    s = lbm.Sizes()
    assert lib.lbm_required_bytes(C.byref(d), C.byref(p), C.byref(s)) == lbm.LBM_EINVAL


@pytest.mark.parametrize("storage", ["f16s", "f32", "f64"])
def test_domains_beyond_4_gib_per_component_are_accepted(lib, storage):
    """Each plane block has its own buffer descriptor, so one component's 19
    direction arrays may span more than 4 GiB: 1024^3 cells (8.6e9 cells per
    buffer in FP16 with two components) and 2^31 cells and more are sized
    (whether they fit is decided by the device allocation at creation)."""
    for shape in [(1024, 1024, 1024), (2048, 1024, 1024)]:
        p = lbm.make_params(storage=storage)
        d = lbm.Domain(*shape)
        s = lbm.Sizes()
        assert lib.lbm_required_bytes(C.byref(d), C.byref(p), C.byref(s)) == lbm.LBM_OK
        N = shape[0] * shape[1] * shape[2]
        assert s.pop_bytes >= 2 * 19 * N * lbm.STORE_BYTES[storage] > 1 << 32


def test_bounce_back_fraction_outside_unit_interval_rejected(lib):
    p = lbm.make_params()
    d = lbm.Domain(4, 4, 4)
    ns = np.zeros(64, np.float32)
    ns[5] = 1.5
    rho = np.ones(128)
    ctx = C.c_void_p()
    assert lib.lbm_create(C.byref(d), ns.ctypes.data, rho.ctypes.data, C.byref(p), None, None,
                          C.byref(ctx)) == lbm.LBM_EINVAL
    ns[5] = np.nan
    assert lib.lbm_create(C.byref(d), ns.ctypes.data, rho.ctypes.data, C.byref(p), None, None,
                          C.byref(ctx)) == lbm.LBM_EINVAL


def test_misaligned_caller_buffers_rejected(lib):
    p = lbm.make_params()
    d = lbm.Domain(4, 4, 4)
    ns = np.zeros(64, np.float32)
    rho = np.ones(128)
    bufs = lbm.DeviceBuffers(4096, 4096 + 8, 8192, 16384)
    ctx = C.c_void_p()
    assert lib.lbm_create(C.byref(d), ns.ctypes.data, rho.ctypes.data, C.byref(p), C.byref(bufs), None,
                          C.byref(ctx)) == lbm.LBM_EINVAL


def test_fill_query_rejected_without_context(lib):
    q, out = lbm.FillQuery(2, 0, 4, 60, 64, 4, 60, 0, 0.5), lbm.FillState()
    assert lib.lbm_fill_state_get(None, C.byref(q), C.byref(out)) == lbm.LBM_EINVAL


def test_permeability_rejected_without_context(lib):
    out = lbm.Permeability()
    assert lib.lbm_permeability_get(None, 0, C.byref(out)) == lbm.LBM_EINVAL


def test_droplet_query_rejected_without_context(lib):
    q, out = lbm.DropletQuery((C.c_double * 3)(8, 8, 8), 2.0, 6.0, 4.0, 0, 0), lbm.DropletState()
    assert lib.lbm_droplet_get(None, C.byref(q), C.byref(out)) == lbm.LBM_EINVAL


def test_null_context_calls_are_rejected(lib):
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_sync(None) == lbm.LBM_EINVAL
    assert lib.lbm_time(None) == -1
    lib.lbm_destroy(None)


def test_c_program_compiles_and_links_against_the_header(lib, tmp_path):
    assert os.path.exists(build_c_driver(tmp_path / "abi_driver"))
