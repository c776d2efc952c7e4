"""Continuous-batching server on the GPU: every served result is bitwise the
result of the same request stepped alone with dg_step, admission respects the
memory arena and the slot limit, and over-budget requests are rejected."""
import math

import numpy as np
import pytest

import oracle
from paper_2510_05254_amd import dg, serve
from _helpers import parity

pytestmark = pytest.mark.gpu


def _stream(n, seed, kmax=1024, ts=0.004):
    reqs = serve.request_stream(n, 1.0, seed=seed, time_scale=ts, kmin=16, kmax=kmax)
    return reqs, {r.rid: serve.prepare(r) for r in reqs}


def _ws(r):
    return dg.dg_workspace_bytes(r.dim, r.N, r.K, r.eq, dg.DG_FP64, 4)


@pytest.mark.parametrize("graph,arena_factor,slots", [(True, 100.0, 64), (False, 2.5, 3)])
def test_served_results_equal_solo_results(graph, arena_factor, slots):
    reqs, prep = _stream(24, 11)
    big = max(_ws(r) for r in reqs)
    arena = int(arena_factor * big)
    sat = serve.with_rate(reqs, math.inf, 1)
    with serve.Server(arena, max_slots=slots, chunk=8, graph=graph, keep_results=True) as srv:
        done, rejected, wall = srv.serve(sat, prep)
        assert srv.arena.in_use() == 0 and not srv.active
    assert not rejected and len(done) == len(reqs)
    solo, rej2, _ = serve.serve_sequential(serve.with_rate(reqs, math.inf, 1), prep, arena,
                                           keep_results=True)
    assert not rej2
    by_id = {r.rid: r for r in solo}
    for r in done:
        assert r.done >= r.admitted >= r.arrival
        np.testing.assert_array_equal(r.result, by_id[r.rid].result)
    # the oracle on the three smallest requests
    for r in sorted(done, key=lambda r: r.unknowns * r.nsteps)[:3]:
        U0, dt, n = prep[r.rid]
        Uo = oracle.step(r.dim, r.N, r.K, r.eq, r.params, U0, 4, dt, n)
        parity(r.result, Uo, what=f"served request {r.rid}")
    s = serve.summarize(done, wall)
    assert s["solves"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_over_budget_request_is_rejected():
    reqs, prep = _stream(6, 12)
    blk = lambda r: -(-_ws(r) // serve.FirstFit.ALIGN) * serve.FirstFit.ALIGN   # noqa: E731
    arena = blk(max(reqs, key=blk)) - serve.FirstFit.ALIGN     # the largest cannot fit
    too_big = sorted(r.rid for r in reqs if blk(r) > arena)
    assert too_big and len(too_big) < len(reqs)
    sat = serve.with_rate(reqs, math.inf, 2)
    with serve.Server(arena, chunk=4) as srv:
        done, rejected, _ = srv.serve(sat, prep)
    assert sorted(r.rid for r in rejected) == too_big
    assert len(done) == len(reqs) - len(too_big)


def test_arrivals_over_time():
    """Requests arriving while others run are admitted and finish after arriving."""
    reqs, prep = _stream(10, 13, kmax=256)
    timed = serve.with_rate(reqs, 200.0, 3)
    with serve.Server(1 << 28, chunk=2) as srv:
        done, rejected, wall = srv.serve(timed, prep)
    assert not rejected and len(done) == 10
    for r in done:
        assert r.admitted >= r.arrival and r.done > r.admitted
    assert wall >= timed[-1].arrival
