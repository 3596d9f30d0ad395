#!/usr/bin/env python3
"""Throughput benchmark of the HMCSC step on one MI355X.

Workload: electrolyte filling of a synthetic electrode, 256^3 voxels, two
components (D3Q19), random overlapping spheres (solid fraction 0.5, n_s = 1),
gray binder (n_s in [0.2, 0.8]) in 20 % of the pore space, 16-layer density
reservoirs at both ends of z, G_inter = 0.9, G_ads = -+0.3 (stencil weights
sum_i W_i c_i c_i = I).  A step is one full time step of the method over the
whole domain (forces, collision, partial bounce-back, streaming, reservoirs).

Headline value: MLUPS of the plain FP32 path.  The same workload is also timed
with shifted FP16 and BF16 storage (FP32 arithmetic), in FP64, and in FP32 with the
GS-WBS of the paper's appendix (Guo forcing, Eq. GS-WBS; same bytes per cell,
both components' forces evaluated per cell).  Each variant reports
its step kernel against the HBM roofline, with the algorithmic bytes per cell
update B = 2*19*2*s + 4 (read and write every population once, read n_s once).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
Q = 19
STORE_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}


def alg_bytes(storage: str, ncomp: int = 2, c_ns: int = 1) -> int:
    return 2 * Q * ncomp * STORE_BYTES[storage] + 4 * c_ns


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_kernels.h"):
        with open(os.path.join(ROOT, "paper_2206_11524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(storage: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "k_step_electrode256_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = d.get("variants", {}).get(storage)
    return None if v is None else v.get("bytes_per_launch")


def run_variant(w, variant, steps, warmup):
    """variant: a storage name, or storage-guo for the GS-WBS with Guo forcing."""
    import torch
    from paper_2206_11524_amd import lbm

    storage, _, scheme = variant.partition("-")
    sim = lbm.from_workload(w, storage=storage, forcing="guo" if scheme == "guo" else "shan-chen")
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kernel_ms = sim.last_step_ms()
    tot = sim.totals()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    N = w.ncells
    mlups = N * steps / dt / 1e6
    B = alg_bytes(storage, w.ncomp, w.c_ns)
    achieved = B * N / (kernel_ms * 1e-3) / 1e9
    traffic = traffic_for(variant)
    return {
        "storage": storage,
        "mlups": mlups,
        "ms_per_step": dt / steps * 1e3,
        "kernel_ms": kernel_ms,
        "finite": tot["finite"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_cell": B, "cells_per_launch": N},
    }


def stream_copy_gbs(mib=2048, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time) on this GPU,
    the practical streaming ceiling the step kernel is compared with."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def ensemble(storage="f16s", ndom=64, steps=100, warmup=10, seed=3000):
    """Batched ensemble: ndom porous domains with edges drawn from
    {32, 48, 64, 96, 128}, stepped together (one batched launch per step) and,
    for comparison, one after the other with the single-domain kernel."""
    import torch
    from paper_2206_11524_amd import inputs, lbm

    g = np.random.Generator(np.random.PCG64(seed))
    edges = g.choice([32, 48, 64, 96, 128], size=ndom)
    ws = [inputs.porous_domain(int(e), seed + 1 + k) for k, e in enumerate(edges)]
    cells = sum(w.ncells for w in ws)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sims = [lbm.from_workload(w, storage=storage) for w in ws]
        grp = lbm.Group(sims)
        grp.step(warmup)
        stream.synchronize()
        t0 = time.perf_counter()
        grp.step(steps)
        stream.synchronize()
        t_group = time.perf_counter() - t0
        launch_ms = grp.last_step_ms()
        t0 = time.perf_counter()
        for sim in sims:
            sim.step(steps)
        stream.synchronize()
        t_seq = time.perf_counter() - t0
        grp.close()
        for sim in sims:
            sim.close()
    del sims
    torch.cuda.empty_cache()
    return {"domains": ndom, "cells": cells, "storage": storage, "steps": steps,
            "grouped_mlups": round(cells * steps / t_group / 1e6, 1),
            "sequential_mlups": round(cells * steps / t_seq / 1e6, 1),
            "grouped_launch_ms": round(launch_ms, 4),
            "edges": {int(e): int((edges == e).sum()) for e in sorted(set(edges.tolist()))}}


def serving(rate=0.5, seconds=30.0, storage="f16s", seed=4000, steps_per_tick=100, drain_s=120.0, tile_x=0,
            policy="fair", run_cells=0, conv_window=8, compare_group=False):
    """Continuous-batching serving: Poisson arrivals at `rate` per second for
    `seconds`, each a porous domain of edge U{48..192} asking for U{2000..20000}
    steps or convergence to 1e-6 relative change of its momentum, tested on
    window means of `conv_window` samples (one per tick) with the noise floor
    of the stochastically rounded state; reports completion latency
    percentiles and the aggregate MLUPS of the server under the given sharing
    policy ("fair" or "shortest-first").  With compare_group the same domains
    are afterwards stepped together as one group (all resident, one batched
    launch per step): the batched rate of that same mix, beside the server's."""
    from paper_2206_11524_amd import inputs, lbm

    g = np.random.Generator(np.random.PCG64(seed))
    n = max(1, int(rate * seconds * 1.5) + 4)
    gaps = g.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < seconds]
    reqs = []
    for k in range(len(arrivals)):
        e = int(g.integers(48, 193))
        reqs.append((inputs.porous_domain(e, seed + 1 + k), int(g.integers(2000, 20001))))
        if (k + 1) % 20 == 0:
            print(f"# serving: generated {k + 1}/{len(arrivals)} requests", file=sys.stderr, flush=True)
    srv = lbm.Server(storage=storage, max_slots=64, steps_per_tick=steps_per_tick, max_cells=192 ** 3,
                     tile=(tile_x, 8 if tile_x else 0), policy=policy,
                     run_cells=run_cells)
    t0 = time.perf_counter()
    tickets = []
    depth = 0
    trace = []  # (seconds since the first arrival, queued, resident), about once a second

    def sample(force=False):
        now = time.perf_counter() - t0
        if not (force or not trace or now - trace[-1][0] >= 1.0):
            return None
        st = srv.stats()
        trace.append((round(now, 1), st["queued"], st["active"]))
        return st

    for (w, steps), ta in zip(reqs, arrivals):
        while time.perf_counter() - t0 < ta:
            sample()
            time.sleep(0.002)
        tickets.append(srv.submit_workload(w, steps, conv_tol=1e-6, conv_window=conv_window,
                                           conv_noise=conv_window > 1))
        st = sample(force=True)
        depth = max(depth, st["queued"] + st["active"])
    # collect results, giving the queue drain_s after the last arrival to finish; a
    # progress line every 15 s (a saturated queue can run for minutes)
    res = [None] * len(tickets)
    pending = list(range(len(tickets)))
    deadline = time.perf_counter() + drain_s
    last = time.perf_counter()
    while pending and time.perf_counter() < deadline:
        r = srv.wait(tickets[pending[0]], 1.0)
        if r is not None:
            res[pending.pop(0)] = r
        for k in list(pending):
            r = srv.poll(tickets[k])
            if r is not None:
                res[k] = r
                pending.remove(k)
        sample()
        if time.perf_counter() - last > 15.0:
            st = srv.stats()
            print(f"# serving: {len(tickets) - len(pending)}/{len(tickets)} done, {st['active']} active, "
                  f"{st['queued']} queued", file=sys.stderr, flush=True)
            last = time.perf_counter()
    st = srv.stats()
    srv.close()
    same_mix = None
    if compare_group:
        # the same domains, all resident, stepped together by one batched launch per step
        sims = [lbm.from_workload(w, storage=storage) for w, _ in reqs]
        grp = lbm.Group(sims)
        grp.step(10)
        sims[0].sync()
        tg = time.perf_counter()
        grp.step(50)
        sims[0].sync()
        tg = time.perf_counter() - tg
        same_mix = round(sum(w.ncells for w, _ in reqs) * 50 / tg / 1e6, 1)
        grp.close()
        for sim in sims:
            sim.close()
        del sims
    done = [r for r in res if r is not None and r["status"] == 0]
    lat = np.array([r["t_done"] - r["t_submit"] for r in done])
    steps_asked = {k: s for k, (_, s) in enumerate(reqs)}
    return {"rate_per_s": rate, "arrival_window_s": seconds, "requests": len(reqs), "completed": len(done),
            "converged": int(sum(r["converged"] for r in done)),
            "steps_saved_by_convergence": int(sum(steps_asked[k] - r["steps_done"] for k, r in enumerate(res)
                                                  if r is not None and r["status"] == 0 and r["converged"])),
            "conv_window": conv_window, "storage": storage, "policy": policy,
            "mean_latency_s": round(float(lat.mean()), 3) if len(lat) else None,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
            "aggregate_mlups": round(st["cell_updates"] / max(st["busy_seconds"], 1e-9) / 1e6, 1),
            "max_in_system": depth, "ticks": st["ticks"],
            **({"grouped_same_mix_mlups": same_mix} if same_mix is not None else {}),
            "depth_trace": {"columns": ["t_s", "queued", "resident"], "rows": trace}}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(w, budget_s=20.0):
    """The FP64 CPU oracle on the same workload, timed on the host cores for a
    bounded number of whole-domain steps."""
    from oracle.ref import Oracle, Reservoir, Setup

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    res = [Reservoir(a, lo, hi, tuple(r)) for (a, lo, hi, r) in w.reservoirs]
    st = Setup(w.shape, ncomp=w.ncomp, c_ns=w.c_ns, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext,
               g_scale=w.g_scale, reservoirs=res, nthreads=threads)
    o = Oracle(st, w.ns.astype(np.float64))
    f = o.init(w.rho)
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = o.step(f)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": round(w.ncells * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} full time steps of the {w.shape[0]}x{w.shape[1]}x{w.shape[2]} workload, "
                      f"FP64, {dt:.1f} s", "cpu_model": cpu_model()}


def cpu_baseline_single_thread(w, planes=16, budget_s=6.0):
    """The FP64 oracle on one host thread: whole steps of a slab of the same
    workload (planes z in [nz/2 - planes/2, nz/2 + planes/2), periodic, away
    from the reservoirs), bounded to a few seconds."""
    from oracle.ref import Oracle, Setup

    nx, ny, nz = w.shape
    z0 = max(0, nz // 2 - planes // 2)
    z1 = min(nz, z0 + planes)
    ns = np.ascontiguousarray(w.ns[:, z0:z1].astype(np.float64))
    rho = np.ascontiguousarray(w.rho[:, z0:z1])
    st = Setup((nx, ny, z1 - z0), ncomp=w.ncomp, c_ns=w.c_ns, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext,
               g_scale=w.g_scale, nthreads=1)
    o = Oracle(st, ns)
    f = o.init(rho)
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = o.step(f)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 20:
            break
    dt = time.perf_counter() - t0
    cells = nx * ny * (z1 - z0)
    return {"value": round(cells * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} full time steps of a {nx}x{ny}x{z1 - z0} slab of the workload, FP64, {dt:.1f} s",
            "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--edge", type=int, default=256)
    ap.add_argument("--variants", default="f32,f16s,bf16s,f64,f32-guo",
                    help="storage formats; storage-guo runs the GS-WBS with Guo forcing")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=0.25, help="arrivals per second (0: no serving run)")
    ap.add_argument("--serve-seconds", type=float, default=40.0)
    ap.add_argument("--serve-burst", type=int, default=24,
                    help="also serve a burst of this many requests arriving within one second (0: none): the "
                         "server saturated, as under the 20/s arrivals of the serving workload")
    ap.add_argument("--serve-drain", type=float, default=120.0,
                    help="seconds after the last arrival for the queue to finish")
    ap.add_argument("--serve-policy", default="fair", choices=("fair", "shortest-first"),
                    help="how the server shares each tick among resident requests")
    ap.add_argument("--serve-run-cells", type=int, default=0,
                    help="shortest-first: cells stepped per tick at least (0: the library default)")
    ap.add_argument("--serve-tile", type=int, default=0, choices=(0, 32, 64),
                    help="tile width of the batched kernel in the server (0: the library default)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_11524_amd import inputs

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_each_way": n * 4, "launches": 10}))
        return

    w = inputs.electrode(n=args.edge)
    variants = [v for v in args.variants.split(",") if v]
    results = {}
    for v in variants:
        results[v] = run_variant(w, v, args.steps, args.warmup)
        print(f"# {v}: {results[v]['mlups']:.0f} MLUPS, kernel {results[v]['kernel_ms']:.3f} ms, "
              f"{results[v]['roofline']['achieved']:.0f} GB/s", file=sys.stderr, flush=True)

    head = results.get("f32") or results[variants[0]]
    line = {
        "metric": "MLUPS (2-comp D3Q19) + % HBM roofline; FP16-store vs FP32; p50/p99 batch latency",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"electrolyte filling, synthetic electrode {args.edge}^3, 2 components, "
                               "D3Q19, sphere packing 0.5 solid + gray binder, z reservoirs",
                   "cells": w.ncells, "storage": head["storage"], "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "variants": {k: {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                         "roofline_frac": r["roofline"]["frac"], "achieved_GBs": r["roofline"]["achieved"],
                         "traffic": r["roofline"]["traffic"], "finite": r["finite"]}
                     for k, r in results.items()},
    }
    if "f32" in results and "f16s" in results:
        line["fp16_gain_over_fp32"] = round(results["f16s"]["mlups"] / results["f32"]["mlups"], 3)
    if not args.no_ensemble:
        line["ensemble"] = ensemble()
        print(f"# ensemble: {line['ensemble']}", file=sys.stderr, flush=True)
    if args.serve_burst > 0:
        line["serving_saturated"] = serving(float(args.serve_burst), 1.0, drain_s=args.serve_drain,
                                            tile_x=args.serve_tile, policy=args.serve_policy,
                                            run_cells=args.serve_run_cells, seed=4500, compare_group=True)
        print(f"# serving (saturated): {line['serving_saturated']}", file=sys.stderr, flush=True)
    if args.serve_rate > 0:
        line["serving"] = serving(args.serve_rate, args.serve_seconds, drain_s=args.serve_drain,
                                  tile_x=args.serve_tile, policy=args.serve_policy,
                                  run_cells=args.serve_run_cells)
        print(f"# serving: {line['serving']}", file=sys.stderr, flush=True)
    copy = stream_copy_gbs()
    line["stream_copy_GBs"] = round(copy, 1)
    line["roofline"]["frac_of_stream_copy"] = round(head["roofline"]["achieved"] / copy, 4)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        print(f"# cpu baseline: {line['cpu_baseline']}", file=sys.stderr, flush=True)
        line["cpu_baseline_1thread"] = cpu_baseline_single_thread(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
