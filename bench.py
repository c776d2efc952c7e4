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
               unknowns * 4 stages * K / timed seconds, from the median of
               --repeats timed runs of K steps (timing: median, min, max)
  roofline     the stage kernel's achieved HBM bandwidth from its algorithmic
               bytes (3.5 state-array passes per launch on average: the RK4
               schedule reads/writes 2, 4, 5 and 3 arrays in its four stages)
               over its average launch time from HIP events on its stream;
               traffic = measured HBM bytes per launch from rocprofv3 counters
               (profiles/), null when the kernel changed since they were taken;
               streaming_reference = the library's streaming probe kernel on
               arrays of the state's size with each stage's read:write mix
  cpu_baseline the CPU oracle (FP64, OpenMP) timed on this host on full-mesh
               RK4 steps of the same workload (a bounded sample, >= 1 step),
               and on one thread on a slab of it; CPU model and core count
  other_configs the other benchmark configurations (and config 4 in the other
               precision) timed the same way in the same run

--serve measures the continuous-batching server on the seeded request stream
(1-D/2-D advection and 2-D isothermal Euler, N in 1..7, K log-uniform in
[16, 256^2], final times uniform in [0.1, 1] x time-scale, FP64, RK4):
first at saturation (every request arrives at time 0) for the capacity C in
solves/s, then with Poisson arrivals at each rate multiple of C; each run is
repeated one solve at a time (FIFO, dg_step alone) on the same GPU. Prints one
JSON line with solves/s and p50/p99 latency (completion - arrival) per run.
The default time scale 0.01 shortens every final time 100-fold so the run
takes minutes; the output then names the workload ..._final_times_x0.01 and
says REDUCED in config.final_times. --time-scale 1 runs the stated final times
(the 2000 requests then take about 2.3e8 RK4 steps in all, mostly long 1-D
solves: tens of minutes).

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
# (arrays read, arrays written) per fused stage
STAGE_MIX = {4: [(1, 1), (2, 2), (3, 2), (2, 1)], 3: [(1, 2), (2, 1), (2, 1)],
             6: [(2, 2), (3, 2), (3, 2), (3, 2), (3, 2), (3, 2), (3, 1)]}
assert all(sum(r + w for r, w in m) == PASSES_PER_STEP[k] or k == 6 for k, m in STAGE_MIX.items())


def kernel_hash() -> str:
    """The stage-kernel source hash the traffic records are tied to (comments
    excluded), as paper_2510_05254_amd.traffic computes it."""
    from paper_2510_05254_amd.traffic import kernel_hash as h
    return h()


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
    if cfg is not None and list(cfg) != [launch_cfg[0], launch_cfg[1], launch_cfg[4], launch_cfg[5]]:
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, U0, dt, budget_s: float, one_thread_budget_s: float):
    """The oracle as it stands, on the host cores, on full-mesh RK4 steps; then
    on one thread, on a slab of the same workload (the same per-element work,
    fewer elements) so the sample stays short."""
    import oracle
    from paper_2510_05254_amd import workloads as W
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
    rate_all = w.unknowns * 4 * steps / el
    # one thread: the x-extent cut so one RK4 step takes about the budget
    per_unknown = el / (w.unknowns * 4 * steps) * threads
    kx = max(1, min(w.K[0], int(one_thread_budget_s / (per_unknown * 4 * w.unknowns / w.K[0]))))
    w1 = W.scaled(w, (kx,) + tuple(w.K[1:]))
    ax1 = [oracle.axis_coords(w1.N, k) for k in w1.K]
    U1 = W.initial_state(w1, ax1)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.step(w1.dim, w1.N, w1.K, w1.eq, w1.params, U1, 4, dt, 1)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    rate_one = w1.unknowns * 4 / el1
    return {"value": rate_all, "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} full-mesh RK4 step(s) of {w.name} ({w.unknowns} unknowns), "
                      f"{el:.1f} s, FP64, OpenMP over elements on {threads} threads",
            "one_thread": {"value": rate_one, "unit": "DOF-updates/s", "cores": 1,
                           "sample": f"1 RK4 step of {w1.name} ({w1.unknowns} unknowns), "
                                     f"{el1:.1f} s"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


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
            done, rej, wall = srv.serve(serve.with_rate(reqs, rate, seed), prep, log=log)
        out = serve.summarize(done, wall)
        out["rejected"] = len(rej)
        log(f"batched rate={rate:.4g}: {json.dumps(out)}")
        return out

    def run_seq(rate, seed):
        done, rej, wall = serve.serve_sequential(serve.with_rate(reqs, rate, seed), prep, arena, log=log)
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
        "config": {"workload": f"served_stream_{a.requests}req" +
                               ("" if a.time_scale == 1 else f"_final_times_x{a.time_scale:g}"),
                   "requests": a.requests, "time_scale": a.time_scale,
                   "final_times": ("as stated, uniform in [0.1, 1]" if a.time_scale == 1 else
                                   f"REDUCED: uniform in [0.1, 1] x {a.time_scale:g}"),
                   "rk": 4,
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


def size_sweep_main(a):
    """Throughput against problem size (the paper's Sec. 3.2 finding that GPUs
    need about 1e7 degrees of freedom): 2-D advection N = 7, RK4, FP64 on
    K x K meshes, one solve alone and B equal solves in one batch, where B
    brings the batch to about 4.2e6 unknowns (at most 1024 members)."""
    import math
    import torch
    from paper_2510_05254_amd import dg
    from paper_2510_05254_amd import workloads as W

    torch.cuda.init()
    N, rk = 7, 4
    for K in (4, 8, 16, 32, 64, 128, 256, 512):
        w = W.scaled(W.config(2), (K, K))
        unknowns = w.unknowns
        B = int(min(1024, max(1, math.ceil(4194304 / unknowns))))
        stream = torch.cuda.Stream()
        solvers = [dg.Solver(2, N, (K, K), W.ADVECTION, (1.0, 0.5), hip_stream=stream.cuda_stream)
                   for _ in range(B)]
        ax = solvers[0].axis_coords()
        U0 = W.initial_state(w, ax)
        dt, _ = W.time_step(w, ax, U0)
        # about 50 ms of work alone at the smallest size's launch rate, at least 20 steps
        steps = max(20, min(2000, int(2e9 / unknowns)))
        s0 = solvers[0]
        s0.set_state(U0)
        s0.step(rk, dt, 2)
        s0.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s0.step(rk, dt, steps)
        e1.record(stream)
        e1.synchronize()
        alone = e0.elapsed_time(e1) / 1e3
        for s in solvers:
            s.set_state(U0)
        torch.cuda.synchronize()
        with dg.Batch(hip_stream=stream.cuda_stream, graph=True) as b:
            for s in solvers:
                b.add(s, rk, dt, steps + 2)
            b.run(2)                                  # warm-up and graph capture
            b.synchronize()
            e0.record(stream)
            b.run_all()
            e1.record(stream)
            e1.synchronize()
            batched = e0.elapsed_time(e1) / 1e3
        for s in solvers:
            s.close()
        upd = unknowns * 4 * steps
        print(json.dumps({"study": "throughput_vs_size_adv2d_N7", "K": [K, K], "unknowns": unknowns,
                          "steps": steps, "alone_dof_updates_per_s": upd / alone,
                          "batch_members": B, "batched_dof_updates_per_s": B * upd / batched,
                          "batched_unknowns": B * unknowns}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--rk", type=int, choices=[3, 4, 6], default=4)
    ap.add_argument("--repeats", type=int, default=5, help="timed repeats of --steps steps (median)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-budget-one", type=float, default=6.0,
                    help="seconds of the one-thread oracle sample")
    ap.add_argument("--no-others", action="store_true",
                    help="time only the chosen configuration (no other_configs key)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true", help="served-stream benchmark")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--time-scale", type=float, default=0.01)
    ap.add_argument("--rates", default="1", help="comma-separated multiples of capacity")
    ap.add_argument("--arena-gib", type=float, default=32.0)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--efficiency", action="store_true", help="error vs computing time study")
    ap.add_argument("--size-sweep", action="store_true",
                    help="throughput vs problem size, one solve alone and many in one batch")
    ap.add_argument("--launch-config", default=None, metavar="ORDER,SLAB,XBLOCK[,ZLEN]",
                    help="tile order (0 XCD-contiguous, 1 plain), z-slab, x-block and z-march "
                         "length (layers per workgroup) to time")
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
    if a.size_sweep:
        size_sweep_main(a)
        return
    if a.efficiency:
        efficiency_main(a)
        return

    import torch
    from paper_2510_05254_amd import dg
    from paper_2510_05254_amd import workloads as W

    torch.cuda.init()
    stream = torch.cuda.Stream()
    prec = dg.DG_FP64 if a.precision == "fp64" else dg.DG_FP32
    head = measure(W.config(a.config), prec, a.rk, a.steps, a.warmup, a.repeats, stream,
                   launch_config=a.launch_config, autotune=a.autotune, keep=True)
    w, s, U0, dt = head.pop("_keep")
    traffic = load_traffic(w.name, a.precision, a.rk, head["_launch_cfg"])
    head["roofline"]["traffic"] = traffic
    stream_ref = stream_reference(w.unknowns * (8 if prec == dg.DG_FP64 else 4), a.rk, stream)
    head["roofline"]["streaming_reference"] = stream_ref
    copy_gbs = torch_copy_rate()

    lc = head.pop("_launch_cfg")
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == dg.DG_FP64 else "f32",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "timing": head["timing"],
        "launch_config": {"tile_order": "plain" if lc[0] else "xcd_contiguous",
                          "z_slab": lc[1], "halo_divisor_1d": lc[2],
                          "x_block": lc[4], "z_march": lc[5], "chunk_1d": lc[6], "autotuned": bool(lc[3])},
        "nodes_per_s": head["nodes_per_s"],
        "copy_gbps": copy_gbs,
        "mass_drift": head["mass_drift"],
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, U0, dt, a.cpu_budget, a.cpu_budget_one)
        out["cpu_baseline"]["gpu_over_cpu"] = head["value"] / out["cpu_baseline"]["value"]
    s.close()
    del s
    # the other benchmark configurations (and the other precision of config 4)
    # in the same run, default launch configuration, same timing protocol
    if not a.no_others:
        others = {}
        todo = [(c, "fp64") for c in (1, 2, 3, 4) if c != a.config] + \
               [(4, "fp32" if a.precision == "fp64" else "fp64")]
        for cid, pname in todo:
            if (cid, pname) == (a.config, a.precision):
                continue
            r = measure(W.config(cid), dg.DG_FP64 if pname == "fp64" else dg.DG_FP32, a.rk,
                        max(a.steps, 20) if cid > 1 else 2316, a.warmup, a.repeats, stream)
            r.pop("_launch_cfg")
            others[f"config{cid}_{pname}"] = {
                "workload": r["config"]["workload"], "precision": pname, "value": r["value"],
                "unit": "DOF-updates/s", "ms_per_step": r["ms_per_step"], "timing": r["timing"],
                "roofline": {k: r["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                           "alg_bytes_per_launch", "avg_launch_us")},
                "mass_drift": r["mass_drift"]}
        out["other_configs"] = others
    print(json.dumps(out), flush=True)


def measure(w, prec, rk, steps, warmup, repeats, stream, launch_config=None, autotune=False, keep=False):
    """Time `repeats` runs of `steps` RK steps of workload w (state resident in
    HBM, HIP events on the solver's stream); median, min and max per step."""
    import torch
    from paper_2510_05254_amd import dg
    from paper_2510_05254_amd import workloads as W
    rsize = 8 if prec == dg.DG_FP64 else 4
    s = dg.Solver(w.dim, w.N, w.K, w.eq, w.params, precision=prec, hip_stream=stream.cuda_stream)
    ax = s.axis_coords()
    U0 = W.initial_state(w, ax)
    dt, _ = W.time_step(w, ax, U0)
    s.set_state(U0)
    m0 = s.mass()
    if launch_config:
        vals = [int(x) for x in launch_config.split(",")]
        c = list(s.launch_config())
        c[0], c[1], c[4] = vals[:3]
        if len(vals) > 3:
            c[5] = vals[3]
        s.set_launch_config(c)
    lc = s.autotune(rk, dt, 3) if autotune else s.launch_config()
    s.step(rk, dt, warmup)
    s.synchronize()
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.step(rk, dt, steps)
        ev1.record(stream)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    m1 = s.mass()
    Ufin = s.get_state()
    if not np.all(np.isfinite(Ufin)):
        print(f"non-finite state after the timed steps of {w.name}", file=sys.stderr)
        sys.exit(1)
    del Ufin
    ms = float(np.median(times))
    stages = STAGES[rk]
    launches = stages * steps
    value = w.unknowns * stages * steps / (ms / 1e3)
    avg_launch_s = ms / 1e3 / launches
    alg_bytes = PASSES_PER_STEP[rk] / stages * w.unknowns * rsize
    achieved = alg_bytes / avg_launch_s / 1e9
    r = {
        "value": value,
        "ms_per_step": ms / steps,
        "timing": {"repeats": repeats, "steps_per_repeat": steps,
                   "ms_per_step_median": ms / steps, "ms_per_step_min": min(times) / steps,
                   "ms_per_step_max": max(times) / steps},
        "config": {"workload": w.name, "dim": w.dim, "N": w.N, "K": list(w.K),
                   "equation": "advection" if w.eq == 0 else "isothermal_euler",
                   "rk": rk, "unknowns": w.unknowns, "nodes": w.nodes, "dt": dt,
                   "precision": "fp64" if prec == dg.DG_FP64 else "fp32"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "stage_kernel" if w.dim > 1 or rk == 6 else "ms1_kernel",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": avg_launch_s * 1e6},
        "nodes_per_s": w.nodes * stages * steps / (ms / 1e3),
        "mass_drift": float((np.abs(m1 - m0) / np.maximum(np.abs(m0), 1.0)).max()),
        "_launch_cfg": lc,
    }
    if w.dim == 1 and rk in (3, 4):
        # temporally blocked: several steps per launch, bound by ALU/LDS, not HBM
        r["roofline"].update({"bound": "latency", "achieved": None, "frac": None, "avg_launch_us": None,
                              "note": "1-D steps run temporally blocked (several steps per launch, "
                                      "arrays in LDS): neither HBM nor a per-stage launch sets the time"})
    if keep:
        r["_keep"] = (w, s, U0, dt)
    else:
        s.close()
    return r


def stream_reference(array_bytes, rk, stream, repeats=5):
    """Achievable streaming rate for the stage schedule's read:write mix: the
    library's probe kernel on arrays of the state's size, each stage's
    (reads, writes) launched `repeats` times; rate = bytes of one pass over
    the schedule / sum of the stages' median launch times."""
    import torch
    from paper_2510_05254_amd import dg
    mix = STAGE_MIX[rk]
    nbytes = (array_bytes // 16) * 16
    bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(5)]
    for b in bufs:
        b.fill_(0)
    torch.cuda.synchronize()
    total_ms, total_bytes, per = 0.0, 0, []
    for nin, nout in mix:
        ins, outs = bufs[:nin], bufs[3:3 + nout]
        dg.dg_bandwidth_probe(stream.cuda_stream, ins, outs, nbytes)     # warm-up
        ts = []
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dg.dg_bandwidth_probe(stream.cuda_stream, ins, outs, nbytes)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        t = float(np.median(ts))
        total_ms += t
        total_bytes += (nin + nout) * nbytes
        per.append({"reads": nin, "writes": nout, "ms": t, "gbps": (nin + nout) * nbytes / (t / 1e3) / 1e9})
    del bufs
    torch.cuda.synchronize()
    gbps = total_bytes / (total_ms / 1e3) / 1e9
    return {"kernel": "probe_kernel (dg_bandwidth_probe)", "gbps": gbps, "frac_of_peak": gbps / HBM_PEAK_GBS,
            "array_bytes": nbytes, "stages": per}


def torch_copy_rate():
    """A plain device-to-device torch copy of 2 GiB (context)."""
    import torch
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
    return 5 * 2 * src.numel() * 8 / (c0.elapsed_time(c1) / 1e3) / 1e9


if __name__ == "__main__":
    main()
