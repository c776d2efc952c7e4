"""Served-stream runs with per-request records, and the report that combines
them (the stream at its stated final times takes longer than one run should,
so the one-at-a-time baseline can be measured in request subsets).

    python -m paper_2510_05254_amd.serve_runs run MODE TIME_SCALE [--rate R] [--subset k/m] --out F.json
    python -m paper_2510_05254_amd.serve_runs report BATCHED.json SEQ.json [SEQ.json ...] [--poisson f,...]

run: serve the seeded 2000-request stream (serve.request_stream) with final
times scaled by TIME_SCALE, batched (serve.Server, 32 GiB arena, chunks of 32
ticks) or one at a time (serve.serve_sequential), every request arriving at
t = 0 or, with --rate, Poisson arrivals at R per second (seed 100); --subset
k/m keeps the requests with rid % m == k. Writes the summary and, per
request, arrival, admission and completion times.

report: the batched run as measured; the one-at-a-time server rebuilt from the
subsets' measured service times (admission to completion of each request,
which does not depend on the other requests when they run one at a time):
FIFO in arrival order, start = max(arrival, previous completion), for the
saturation stream and, with --poisson, Poisson arrivals at those multiples of
the batched capacity (the same arrival draws as run --rate).
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import serve

N_REQUESTS = 2000
ARENA_BYTES = 32 << 30
CHUNK = 32
ARRIVAL_SEED = 100


def _log(msg):
    print(msg, flush=True)


def run(mode: str, time_scale: float, rate: float, subset, out: str):
    import torch
    torch.cuda.init()
    reqs = serve.request_stream(N_REQUESTS, 1.0, time_scale=time_scale)
    if subset:
        k, m = (int(x) for x in subset.split("/"))
        reqs = [r for r in reqs if r.rid % m == k]
    t0 = time.perf_counter()
    prep = {r.rid: serve.prepare(r) for r in reqs}
    _log(f"prepared {len(reqs)} in {time.perf_counter() - t0:.1f} s")
    # warm-up: kernel loading and first launches, on a small stream
    wreqs = serve.request_stream(40, 1.0, seed=1, time_scale=0.001, kmax=1024)
    wprep = {r.rid: serve.prepare(r) for r in wreqs}
    with serve.Server(ARENA_BYTES) as srv:
        srv.serve(serve.with_rate(wreqs, math.inf, 1), wprep)
    serve.serve_sequential(serve.with_rate(wreqs, math.inf, 1), wprep, 1 << 30)
    arr = serve.with_rate(reqs, rate, ARRIVAL_SEED)
    if mode == "batched":
        with serve.Server(ARENA_BYTES, chunk=CHUNK) as srv:
            done, rej, wall = srv.serve(arr, prep, log=_log)
    else:
        done, rej, wall = serve.serve_sequential(arr, prep, ARENA_BYTES, log=_log)
    rec = {"mode": mode, "time_scale": time_scale, "rate": rate, "subset": subset, "wall": wall,
           "summary": serve.summarize(done, wall), "rejected": len(rej),
           "requests": [{"rid": r.rid, "dim": r.dim, "N": r.N, "K": list(r.K), "eq": r.eq,
                         "nsteps": r.nsteps, "unknowns": r.unknowns, "arrival": r.arrival,
                         "admitted": r.admitted, "done": r.done} for r in done]}
    with open(out, "w") as fh:
        json.dump(rec, fh)
    _log(json.dumps(rec["summary"]))


def fifo(services, arrivals):
    """One server, FIFO: (latencies, completion of the last request)."""
    t, lat = 0.0, []
    for s, a in zip(services, arrivals):
        t = max(t, a) + s
        lat.append(t - a)
    return lat, t


def report(batched: str, seq_files, poisson):
    b = json.load(open(batched))
    service = {}
    for f in seq_files:
        for r in json.load(open(f))["requests"]:
            service[r["rid"]] = r["done"] - r["admitted"]
    reqs = serve.request_stream(N_REQUESTS, 1.0, time_scale=b["time_scale"])
    missing = [r.rid for r in reqs if r.rid not in service]
    if missing:
        raise SystemExit(f"no service time for {len(missing)} requests (e.g. rid {missing[0]})")
    out = {"time_scale": b["time_scale"], "batched": dict(b["summary"], rate=b["rate"])}
    upd = sum(r["unknowns"] * 4 * r["nsteps"] for r in b["requests"])
    runs = [("saturation", math.inf)] + [(f"poisson_{f:g}x", f * b["summary"]["solves_per_s"]) for f in poisson]
    for name, rate in runs:
        arr = sorted(serve.with_rate(reqs, rate, ARRIVAL_SEED), key=lambda r: (r.arrival, r.rid))
        lat, wall = fifo([service[r.rid] for r in arr], [r.arrival for r in arr])
        out[f"one_at_a_time_{name}"] = {
            "rate": rate, "solves": len(arr), "wall_s": wall, "solves_per_s": len(arr) / wall,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(np.mean(lat)), "dof_updates_per_s": upd / wall}
    out["sum_of_service_s"] = sum(service.values())
    print(json.dumps(out, indent=1))
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("mode", choices=["batched", "sequential"])
    r.add_argument("time_scale", type=float)
    r.add_argument("--rate", type=float, default=math.inf)
    r.add_argument("--subset", default=None)
    r.add_argument("--out", required=True)
    p = sub.add_parser("report")
    p.add_argument("batched")
    p.add_argument("sequential", nargs="+")
    p.add_argument("--poisson", default="")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.mode, a.time_scale, a.rate, a.subset, a.out)
    else:
        report(a.batched, a.sequential, [float(x) for x in a.poisson.split(",") if x])


if __name__ == "__main__":
    main()
