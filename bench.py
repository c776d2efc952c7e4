#!/usr/bin/env python3
"""Benchmark of the fused NDG RHS + RK4 stage path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--precision fp64]
    python bench.py --serve [--requests 2000] [--time-scale 0.01] [--rates 1]
    python bench.py --efficiency

A step is one classical RK4 step (four fused RHS + stage launches) over the
whole mesh of the chosen workload; default: 3-D isothermal Euler, 64^3
elements, N = 4 (125 nodes per element, 131,072,000 unknowns), FP64, seeded
solenoidal velocity at Mach 0.1. The state is resident in HBM before the
timed region. Prints one JSON line:

  value        unknown (DOF) updates per second per RK stage:
               unknowns * 4 stages * K / timed seconds
  roofline     the stage kernel's achieved HBM bandwidth from its algorithmic
               bytes (3.5 state-array passes per launch on average: the RK4
               schedule reads/writes 2, 4, 5 and 3 arrays in its four stages)
               over its average launch time from HIP events on its stream;
               traffic = measured HBM bytes per launch from rocprofv3 counters
               (profiles/), null when the kernel changed since they were taken
  cpu_baseline the CPU oracle (FP64, OpenMP) timed on this host on full-mesh
               RK4 steps of the same workload (a bounded sample, >= 1 step)

--serve measures the continuous-batching server on the seeded request stream
(1-D/2-D advection and 2-D isothermal Euler, N in 1..7, K log-uniform in
[16, 256^2], final times uniform in [0.1, 1] x time-scale, FP64, RK4):
first at saturation (every request arrives at time 0) for the capacity C in
solves/s, then with Poisson arrivals at each rate multiple of C; each run is
repeated one solve at a time (FIFO, dg_step alone) on the same GPU. Prints one
JSON line with solves/s and p50/p99 latency (completion - arrival) per run.

--efficiency repeats the paper's error-versus-computing-time study (Sec. 3.1):
2-D advection with a = (1, 0) over one revolution (T = 1) from
U0 = sum_{k=1}^{40} A_k sin(2 pi k x) (seeded A_k ~ U[0,1)), (a) spatial order
N+1 = 3..8 with RK6 and (b) RK3/RK4/RK6 at order 8, each on a ladder of square
meshes; dt = 0.1 dx_min / |a|. Error = relative L2 distance to U0 after the
revolution (the exact solution); time = GPU time of all steps (HIP events).
Prints one JSON line per run.
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

METRIC = "NDG DOF-updates/s per RK stage + %HBM peak; served solves/s with p50/p99"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD public specification
# state-array passes per step of the fused schedules: RK4 2+4+5+3, RK3 3+3+3,
# RK6 (stage s reads Y_s, U and the k's it combines, writes k_s and Y_s+1)
# 4+5+6+7+8+9+7
PASSES_PER_STEP = {4: 14, 3: 9, 6: 46}
STAGES = {4: 4, 3: 3, 6: 7}
KERNEL_SOURCES = ["paper_2510_05254_amd/csrc/dg_stage.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, precision: str, rk: int, launch_cfg):
    """Measured HBM bytes per stage launch from profiles/, if the kernel, the RK
    scheme and the launch configuration (tile order, z-slab, x-block) are
    those measured."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    if rec.get("rk") != rk:
        return None
    cfg = rec.get("launch_config")
    if cfg is not None and list(cfg) != [launch_cfg[0], launch_cfg[1], launch_cfg[4]]:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, U0, dt, budget_s: float):
    """The oracle as it stands, on the host cores, on full-mesh RK4 steps."""
    import oracle
    oracle.build(force=False)
    threads = oracle.get_threads()
    steps, t0 = 0, time.perf_counter()
    U = U0
    while True:
        U = oracle.step(w.dim, w.N, w.K, w.eq, w.params, U, 4, dt, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            break
        if el / steps * (steps + 1) > 1.5 * budget_s:
            break
    return {"value": w.unknowns * 4 * steps / el, "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} full-mesh RK4 step(s) of {w.name} ({w.unknowns} unknowns), "
                      f"{el:.1f} s, FP64, OpenMP over elements"}


def serve_main(a):
    import math
    import torch
    from paper_2510_05254_amd import serve

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    torch.cuda.init()
    arena = int(a.arena_gib * (1 << 30))
    reqs = serve.request_stream(a.requests, 1.0, time_scale=a.time_scale)
    t0 = time.perf_counter()
    prep = {r.rid: serve.prepare(r) for r in reqs}
    log(f"prepared {len(reqs)} requests in {time.perf_counter() - t0:.1f} s")
    upd = sum(r.unknowns * 4 * prep[r.rid][2] for r in reqs)

    # untimed warm-up over a small stream (kernel loading, first launches)
    wreqs = serve.request_stream(40, 1.0, seed=1, time_scale=0.001, kmax=1024)
    wprep = {r.rid: serve.prepare(r) for r in wreqs}
    with serve.Server(arena, chunk=a.chunk, graph=not a.no_graph) as srv:
        srv.serve(serve.with_rate(wreqs, math.inf, 1), wprep)
    serve.serve_sequential(serve.with_rate(wreqs, math.inf, 1), wprep, 1 << 30)

    def run_batched(rate, seed):
        with serve.Server(arena, chunk=a.chunk, graph=not a.no_graph) as srv:
            done, rej, wall = srv.serve(serve.with_rate(reqs, rate, seed), prep)
        out = serve.summarize(done, wall)
        out["rejected"] = len(rej)
        log(f"batched rate={rate:.4g}: {json.dumps(out)}")
        return out

    def run_seq(rate, seed):
        done, rej, wall = serve.serve_sequential(serve.with_rate(reqs, rate, seed), prep, arena)
        out = serve.summarize(done, wall)
        out["rejected"] = len(rej)
        log(f"sequential rate={rate:.4g}: {json.dumps(out)}")
        return out

    cap_b = run_batched(math.inf, 0)
    cap_s = run_seq(math.inf, 0)
    C = cap_b["solves_per_s"]
    runs = []
    for i, f in enumerate(float(x) for x in a.rates.split(",") if x):
        rate = f * C
        runs.append({"rate_multiple": f, "rate_per_s": rate,
                     "batched": run_batched(rate, 100 + i), "sequential": run_seq(rate, 100 + i)})
    out = {
        "metric": "served solves/s with p50/p99 latency",
        "value": C,
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served_stream_{a.requests}req_timescale{a.time_scale:g}",
                   "requests": a.requests, "time_scale": a.time_scale, "rk": 4,
                   "arena_gib": a.arena_gib, "chunk": a.chunk, "graph": not a.no_graph,
                   "dof_updates": upd},
        "capacity": {"batched": cap_b, "sequential": cap_s,
                     "speedup": C / cap_s["solves_per_s"]},
        "rates": runs,
    }
    print(json.dumps(out), flush=True)


def efficiency_main(a):
    import torch
    from paper_2510_05254_amd import dg
    from paper_2510_05254_amd import workloads as W

    torch.cuda.init()
    ladder = {2: (16, 32, 64, 128, 256, 512), 3: (16, 32, 64, 128, 256, 512),
              4: (8, 16, 32, 64, 128, 256), 5: (8, 16, 32, 64, 128, 256),
              6: (8, 16, 32, 64, 96, 128), 7: (8, 16, 32, 48, 64, 96, 128)}
    runs = [(N, 6, K) for N in range(2, 8) for K in ladder[N]]
    runs += [(7, rk, K) for rk in (3, 4) for K in ladder[7]]
    for N, rk, K in runs:
        w = W.Workload(f"adv2d_Nk40_K{K}_N{N}", 2, N, (K, K), W.ADVECTION, (1.0, 0.0), "fourier1d",
                       W.SEED_BASE + 6, rk=rk, t_final=1.0, ic_args={"nk": 40})
        stream = torch.cuda.Stream()
        with dg.Solver(2, N, (K, K), W.ADVECTION, (1.0, 0.0), hip_stream=stream.cuda_stream) as s:
            ax = s.axis_coords()
            U0 = W.initial_state(w, ax)
            dt, n = W.time_step(w, ax, U0)
            s.set_state(U0)
            s.step(rk, dt, 1)                       # warm-up (kernel load)
            s.set_state(U0)
            s.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(rk, dt, n)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            _, rel = s.l2_error(U0)                  # one revolution: the exact solution is U0
        print(json.dumps({"study": "error_vs_time_adv2d_Nk40", "order": N + 1, "N": N, "rk": rk,
                          "K": [K, K], "steps": n, "dt": dt, "gpu_seconds": ms / 1e3,
                          "rel_l2_error": rel, "unknowns": w.unknowns}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--rk", type=int, choices=[3, 4, 6], default=4)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true", help="served-stream benchmark")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--time-scale", type=float, default=0.01)
    ap.add_argument("--rates", default="1", help="comma-separated multiples of capacity")
    ap.add_argument("--arena-gib", type=float, default=32.0)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--efficiency", action="store_true", help="error vs computing time study")
    ap.add_argument("--launch-config", default=None, metavar="ORDER,SLAB,XBLOCK",
                    help="tile order (0 XCD-contiguous, 1 plain), z-slab, x-block to time")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the launch configuration before timing (the committed traffic "
                         "counters are for the default configuration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.serve:
        serve_main(a)
        return
    if a.efficiency:
        efficiency_main(a)
        return

    import torch
    from paper_2510_05254_amd import dg
    from paper_2510_05254_amd import workloads as W

    w = W.config(a.config)
    prec = dg.DG_FP64 if a.precision == "fp64" else dg.DG_FP32
    rsize = 8 if prec == dg.DG_FP64 else 4
    torch.cuda.init()
    stream = torch.cuda.Stream()
    s = dg.Solver(w.dim, w.N, w.K, w.eq, w.params, precision=prec, hip_stream=stream.cuda_stream)
    ax = s.axis_coords()
    t0 = time.perf_counter()
    U0 = W.initial_state(w, ax)
    dt, _ = W.time_step(w, ax, U0)
    t_ic = time.perf_counter() - t0
    s.set_state(U0)
    m0 = s.mass()
    # launch configuration: the default, or autotuned before the timed region
    # (every candidate computes the same results)
    if a.launch_config:
        order, slab, xblk = (int(x) for x in a.launch_config.split(","))
        c = list(s.launch_config())
        c[0], c[1], c[4] = order, slab, xblk
        s.set_launch_config(c)
    launch_cfg = s.autotune(a.rk, dt, 3) if a.autotune else s.launch_config()

    s.step(a.rk, dt, a.warmup)
    s.synchronize()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    s.step(a.rk, dt, a.steps)
    ev1.record(stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    m1 = s.mass()
    Ufin = s.get_state()
    if not np.all(np.isfinite(Ufin)):
        print("non-finite state after the timed steps", file=sys.stderr)
        sys.exit(1)
    del Ufin

    stages = STAGES[a.rk]
    launches = stages * a.steps
    ms_step = ms / a.steps
    value = w.unknowns * stages * a.steps / (ms / 1e3)
    avg_launch_s = ms / 1e3 / launches
    alg_bytes = PASSES_PER_STEP[a.rk] / stages * w.unknowns * rsize
    achieved = alg_bytes / avg_launch_s / 1e9
    traffic = load_traffic(w.name, a.precision, a.rk, launch_cfg)

    # achievable bandwidth: a plain device-to-device copy of 2 GiB
    src = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    c1.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == dg.DG_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "N": w.N, "K": list(w.K),
                   "equation": "advection" if w.eq == 0 else "isothermal_euler",
                   "rk": a.rk, "unknowns": w.unknowns, "nodes": w.nodes, "dt": dt,
                   "precision": a.precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "stage_kernel", "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_us": avg_launch_s * 1e6},
        "launch_config": {"tile_order": "plain" if launch_cfg[0] else "xcd_contiguous",
                          "z_slab": launch_cfg[1], "halo_divisor_1d": launch_cfg[2],
                          "x_block": launch_cfg[4], "autotuned": bool(launch_cfg[3])},
        "nodes_per_s": w.nodes * stages * a.steps / (ms / 1e3),
        "copy_gbps": copy_gbs,
        "mass_drift": (np.abs(m1 - m0) / np.maximum(np.abs(m0), 1.0)).max(),
        "ic_seconds": t_ic,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, U0, dt, a.cpu_budget)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
