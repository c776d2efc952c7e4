"""Continuous-batching server for streams of NDG solves on one GPU.

Requests (dimension, equation, degree N, element count K, final time, initial
data) arrive over time. The server keeps every admitted solve resident in
device memory and advances all of them together with dg_batch (one launch per
RK stage per kernel class), admitting new requests between bounded chunks of
ticks as memory and slots free up. Each solve takes exactly the RK steps it
would take alone, so its result is the same alone and in the mix.

Memory: one device arena (a torch allocation made once) carved by a first-fit
allocator into per-solve workspaces (dg_create_ex with a workspace), so
admission never allocates device memory. A request is admitted when its
workspace (dg_workspace_bytes) fits in the arena and a slot is free.

The baseline is the same stream served one solve at a time (FIFO, each solve
stepped alone with dg_step on the same GPU).

Request stream (the served-stream benchmark configuration): seeded requests,
each 1-D advection, 2-D advection or 2-D isothermal Euler with equal
probability, N uniform in 1..7, total element count K log-uniform in
[16, 256^2] (2-D meshes are square), final time uniform in [0.1, 1] times a
stated time scale, random-Fourier initial data, Poisson arrivals at a stated
rate, RK4, dt = 0.1 dx_min / sum of wave speeds, FP64.
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import dg
from . import workloads as W


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    dim: int
    N: int
    K: tuple
    eq: int
    params: tuple
    t_final: float
    seed: int
    # filled while serving
    dt: float = 0.0
    nsteps: int = 0
    admitted: float = -1.0
    done: float = -1.0
    result: np.ndarray | None = field(default=None, repr=False)

    @property
    def unknowns(self) -> int:
        nv = 1 if self.eq == W.ADVECTION else 1 + self.dim
        return int(np.prod(self.K)) * (self.N + 1) ** self.dim * nv


def request_stream(n: int, rate: float, seed: int = W.SEED_BASE + 5, time_scale: float = 1.0,
                   kmin: int = 16, kmax: int = 256 * 256):
    """n seeded requests with Poisson arrivals at `rate` per second."""
    rng = W.SplitMix64(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += -math.log(1.0 - rng.uniform()) / rate
        kind = rng.randint(0, 2)
        N = rng.randint(1, 7)
        ktot = math.exp(math.log(kmin) + rng.uniform() * (math.log(kmax) - math.log(kmin)))
        tf = (0.1 + 0.9 * rng.uniform()) * time_scale
        if kind == 0:
            dim, eq, K, par = 1, W.ADVECTION, (max(1, int(round(ktot))),), (1.0,)
        else:
            side = max(1, int(round(math.sqrt(ktot))))
            if kind == 1:
                dim, eq, K, par = 2, W.ADVECTION, (side, side), (1.0, 0.5)
            else:
                dim, eq, K, par = 2, W.EULER, (side, side), (1.0,)
        out.append(Request(i, t, dim, N, K, eq, par, tf, seed * 1000 + i))
    return out


def _workload(r: Request) -> W.Workload:
    if r.eq == W.ADVECTION:
        return W.Workload(f"req{r.rid}", r.dim, r.N, r.K, r.eq, r.params, "fourier_adv", r.seed,
                          t_final=r.t_final, ic_args={"modes": 4, "kmax": 3})
    return W.Workload(f"req{r.rid}", r.dim, r.N, r.K, r.eq, r.params, "euler_random", r.seed,
                      t_final=r.t_final, ic_args={"modes": 4, "kmax": 3, "noise": 0.01, "mach": 0.1})


class FirstFit:
    """First-fit allocator over [0, nbytes) with 256-byte aligned blocks."""

    ALIGN = 256

    def __init__(self, nbytes: int):
        self.nbytes = int(nbytes)
        self.free = [(0, self.nbytes)] if self.nbytes > 0 else []    # sorted (offset, size)

    def alloc(self, size: int):
        """(offset, size) of a block of at least `size` bytes, or None."""
        size = max(self.ALIGN, (int(size) + self.ALIGN - 1) // self.ALIGN * self.ALIGN)
        for i, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + size, sz - size)
                return off, size
        return None

    def release(self, off: int, size: int):
        """Return a block; adjacent free blocks are merged."""
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def in_use(self) -> int:
        return self.nbytes - sum(s for _, s in self.free)


class Arena(FirstFit):
    """FirstFit over one device allocation made once (a torch tensor)."""

    def __init__(self, nbytes: int):
        import torch
        super().__init__(nbytes)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        self.base = self.buf.data_ptr()


_AXES = {}


def _axis(N: int, k: int):
    """Node coordinates of a periodic axis of k elements, taken from the library
    (a one-axis solver), cached per (N, k)."""
    key = (N, k)
    if key not in _AXES:
        with dg.Solver(1, N, (k,), W.ADVECTION, (1.0,)) as s:
            _AXES[key] = s.axis_coords()[0]
    return _AXES[key]


def prepare(r: Request):
    """(U0, dt, nsteps) of a request: its initial state on the library's nodes
    and the step rule of the workloads module."""
    w = _workload(r)
    ax = [np.asarray(_axis(r.N, k)).reshape(k, r.N + 1) for k in r.K]
    U0 = W.initial_state(w, ax)
    dt, n = W.time_step(w, ax, U0)
    return U0, dt, n


class Server:
    """Continuous batching of requests over one dg_batch on one stream.

    Loop: move arrived requests to the waiting queue; admit waiting requests
    in arrival order while a slot is free and their workspace fits in the
    arena (a request larger than the whole arena is rejected); enqueue up to
    `chunk` ticks (dg_batch_run stops early at the next member to finish);
    retire finished members (their completion time is taken after the
    stream has drained). At most `depth` runs are in flight ahead of the GPU,
    so admission decisions follow the GPU closely.
    """

    def __init__(self, arena_bytes: int, max_slots: int = 4096, chunk: int = 32,
                 graph: bool = True, keep_results: bool = False, depth: int = 2):
        import torch
        self.stream = torch.cuda.Stream()
        self.arena = Arena(arena_bytes)
        self.batch = dg.Batch(hip_stream=self.stream.cuda_stream, graph=graph)
        self.max_slots = max_slots
        self.chunk = chunk
        self.keep = keep_results
        self.depth = depth
        self.active = {}            # rid -> (request, solver, (off, size))
        self.tick = 0               # ticks enqueued so far
        self.finish = []            # heap of (tick at which a member finishes, rid)

    def close(self):
        self.batch.synchronize()
        for r, s, blk in self.active.values():
            s.close()
            self.arena.release(*blk)
        self.active.clear()
        self.batch.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _admit(self, r: Request, prep, now: float) -> bool:
        U0, r.dt, r.nsteps = prep
        ws = dg.dg_workspace_bytes(r.dim, r.N, r.K, r.eq, dg.DG_FP64, 4)
        blk = self.arena.alloc(ws)
        if blk is None:
            return False
        # admitted solvers run their setup on streams of torch's stream pool,
        # not on the batch stream: creating a solver and setting its state
        # then wait for earlier admissions only, not for the ticks in flight
        # (dg_batch_add orders the batch stream after the member's stream; a
        # member's stream waits for the batch only when the member is read)
        import torch
        st = torch.cuda.Stream()
        if st.cuda_stream == self.stream.cuda_stream:     # the pool hands out streams in turn
            st = torch.cuda.Stream()
        s = dg.Solver(r.dim, r.N, r.K, r.eq, r.params, precision=dg.DG_FP64, hip_stream=st.cuda_stream,
                      device_workspace=self.arena.base + blk[0], workspace_bytes=blk[1])
        s._ws = self.arena.buf                  # the arena outlives the solver
        s.set_state(U0)
        self.batch.add(s, 4, r.dt, r.nsteps)
        r.admitted = now
        self.active[r.rid] = (r, s, blk)
        # dg_batch_run never runs past the next member to finish, so a member
        # admitted at tick T with n steps finishes exactly at tick T + n
        heapq.heappush(self.finish, (self.tick + r.nsteps, r.rid))
        return True

    def _retire(self, rids, t):
        out = []
        for rid in rids:
            r, s, blk = self.active.pop(rid)
            if self.keep:
                r.result = s.get_state()
            r.done = t
            self.batch.remove(s)
            s.close()
            self.arena.release(*blk)
            out.append(r)
        return out

    def serve(self, requests, prepared, log=None, log_every: float = 20.0):
        """Serve `requests` (any order; arrival times in seconds from the call).
        prepared[rid] = (U0, dt, nsteps). Returns (completed, rejected, wall).
        log(msg), if given, gets a progress line every log_every seconds."""
        import torch
        from collections import deque
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting = deque()
        inflight = deque()
        done, rejected = [], []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0          # noqa: E731
        last = 0.0
        while pending or waiting or self.active:
            t = now()
            if log and t - last >= log_every:
                last = t
                log(f"{t:.0f} s: {len(done)} done, {len(self.active)} active, {len(waiting)} waiting, "
                    f"{len(pending)} not arrived")
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            while waiting and len(self.active) < self.max_slots:
                if self._admit(waiting[0], prepared[waiting[0].rid], t):
                    waiting.popleft()
                elif not self.active:                   # larger than the whole arena
                    rejected.append(waiting.popleft())
                else:
                    break
            if self.active:
                self.tick += self.batch.run(self.chunk)
                fin = []
                while self.finish and self.finish[0][0] <= self.tick:
                    fin.append(heapq.heappop(self.finish)[1])
                if fin:
                    self.batch.synchronize()
                    inflight.clear()
                    done.extend(self._retire(fin, now()))
                else:
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    inflight.append(ev)
                    if len(inflight) > self.depth:
                        inflight.popleft().synchronize()
            elif pending:
                time.sleep(max(0.0, min(pending[0].arrival - now(), 0.005)))
        return done, rejected, now()


def serve_sequential(requests, prepared, arena_bytes: int, keep_results: bool = False, log=None,
                     log_every: float = 20.0):
    """Baseline on the same GPU: FIFO, one solve at a time, each stepped alone
    with dg_step on one stream from one arena (no per-request allocation).
    Returns (completed, rejected, wall). log as for Server.serve."""
    import torch
    stream = torch.cuda.Stream()
    arena = Arena(arena_bytes)
    done, rejected = [], []
    order = sorted(requests, key=lambda r: (r.arrival, r.rid))
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0              # noqa: E731
    last = 0.0
    for r in order:
        if log and now() - last >= log_every:
            last = now()
            log(f"{last:.0f} s: {len(done)} of {len(order)} done")
        while now() < r.arrival:
            time.sleep(min(r.arrival - now(), 0.005))
        U0, r.dt, r.nsteps = prepared[r.rid]
        ws = dg.dg_workspace_bytes(r.dim, r.N, r.K, r.eq, dg.DG_FP64, 4)
        if ws > arena.nbytes:
            rejected.append(r)
            continue
        r.admitted = now()
        with dg.Solver(r.dim, r.N, r.K, r.eq, r.params, hip_stream=stream.cuda_stream,
                       device_workspace=arena.base, workspace_bytes=arena.nbytes) as s:
            s.set_state(U0)
            s.step(4, r.dt, r.nsteps)
            s.synchronize()
            if keep_results:
                r.result = s.get_state()
        r.done = now()
        done.append(r)
    return done, rejected, now()


def summarize(done, wall):
    """Throughput and latency (completion - arrival) of a served stream."""
    if not done:
        return {"solves": 0, "wall_s": wall}
    lat = np.array([r.done - r.arrival for r in done])
    upd = sum(r.unknowns * 4 * r.nsteps for r in done)
    return {"solves": len(done), "wall_s": round(wall, 4),
            "solves_per_s": len(done) / wall,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "dof_updates_per_s": upd / wall}


def with_rate(requests, rate: float, seed: int):
    """Copies of `requests` with Poisson arrivals at `rate` per second
    (rate = inf: all arrive at time 0)."""
    rng = W.SplitMix64(seed)
    t = 0.0
    out = []
    for r in requests:
        if math.isfinite(rate):
            t += -math.log(1.0 - rng.uniform()) / rate
        out.append(Request(r.rid, t, r.dim, r.N, r.K, r.eq, r.params, r.t_final, r.seed))
    return out
