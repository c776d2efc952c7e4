"""Host logic of the continuous-batching server: the seeded request stream and
the first-fit arena allocator (no GPU needed)."""
import math

import numpy as np
import pytest

from paper_2510_05254_amd import serve
from paper_2510_05254_amd import workloads as W


def test_stream_is_seeded_and_deterministic():
    a = serve.request_stream(50, 3.0)
    b = serve.request_stream(50, 3.0)
    assert [(r.arrival, r.dim, r.N, r.K, r.eq, r.t_final, r.seed) for r in a] == \
           [(r.arrival, r.dim, r.N, r.K, r.eq, r.t_final, r.seed) for r in b]
    c = serve.request_stream(50, 3.0, seed=7)
    assert [r.K for r in a] != [r.K for r in c]


def test_stream_distribution():
    n, rate = 2000, 4.0
    reqs = serve.request_stream(n, rate)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    # Poisson arrivals: mean gap 1/rate (standard error 1/(rate sqrt(n)))
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 1 / rate) < 4 / (rate * math.sqrt(n))
    assert abs(np.median(gaps) - math.log(2) / rate) < 0.1 / rate
    Ns = np.array([r.N for r in reqs])
    assert Ns.min() == 1 and Ns.max() == 7
    assert np.all(np.abs(np.bincount(Ns)[1:] / n - 1 / 7) < 0.03)
    kinds = np.array([(r.dim, r.eq) for r in reqs])
    for kind in [(1, W.ADVECTION), (2, W.ADVECTION), (2, W.EULER)]:
        frac = np.mean(np.all(kinds == kind, axis=1))
        assert abs(frac - 1 / 3) < 0.04
    ktot = np.array([np.prod(r.K) for r in reqs], dtype=float)
    assert ktot.min() >= 16 * 0.9 and ktot.max() <= 256 * 256 * 1.01
    # log-uniform: log K spread evenly over [log 16, log 65536]
    u = (np.log(ktot) - math.log(16)) / (math.log(65536) - math.log(16))
    for q in (0.25, 0.5, 0.75):
        assert abs(np.quantile(u, q) - q) < 0.05
    for r in reqs:
        assert len(r.K) == r.dim
        if r.dim == 2:
            assert r.K[0] == r.K[1]
        assert 0.1 <= r.t_final <= 1.0
    tf = np.array([r.t_final for r in reqs])
    assert abs(tf.mean() - 0.55) < 0.03


def test_stream_time_scale_and_kmax():
    reqs = serve.request_stream(100, 1.0, time_scale=0.01, kmax=256)
    assert all(0.001 <= r.t_final <= 0.01 for r in reqs)
    assert all(np.prod(r.K) <= 256 * 1.2 for r in reqs)


def test_with_rate():
    base = serve.request_stream(30, 1.0)
    sat = serve.with_rate(base, math.inf, 1)
    assert all(r.arrival == 0.0 for r in sat)
    assert [(r.rid, r.K, r.N) for r in sat] == [(r.rid, r.K, r.N) for r in base]
    fast = serve.with_rate(base, 100.0, 1)
    assert np.all(np.diff([r.arrival for r in fast]) > 0)
    assert fast[-1].arrival < base[-1].arrival


def test_request_unknowns():
    r = serve.Request(0, 0.0, 2, 3, (5, 4), W.EULER, (1.0,), 0.5, 1)
    assert r.unknowns == 20 * 16 * 3
    r = serve.Request(0, 0.0, 1, 7, (9,), W.ADVECTION, (1.0,), 0.5, 1)
    assert r.unknowns == 9 * 8


def test_first_fit_basics():
    a = serve.FirstFit(4096)
    b1 = a.alloc(100)
    assert b1 == (0, 256)
    b2 = a.alloc(256)
    assert b2 == (256, 256)
    b3 = a.alloc(3000)
    assert b3 == (512, 3072)
    assert a.alloc(1024) is None and a.alloc(513) is None
    assert a.alloc(512) == (3584, 512)
    assert a.in_use() == 4096
    a.release(*b2)
    assert a.alloc(300) is None                 # the hole is 256 bytes
    a.release(*b1)                              # merges with b2's hole
    assert a.free == [(0, 512)]
    assert a.alloc(300) == (0, 512)
    assert serve.FirstFit(0).alloc(1) is None


def test_first_fit_random_no_overlap():
    rng = np.random.default_rng(5)
    a = serve.FirstFit(1 << 20)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            a.release(*live.pop(int(rng.integers(len(live)))))
        else:
            blk = a.alloc(int(rng.integers(1, 40000)))
            if blk is not None:
                assert blk[0] % 256 == 0 and blk[0] + blk[1] <= a.nbytes
                live.append(blk)
        spans = sorted(live + a.free)
        pos = 0
        for off, size in spans:                 # live and free blocks tile the arena
            assert off == pos and size > 0
            pos += size
        assert pos == a.nbytes
        for (o1, s1), (o2, s2) in zip(a.free, a.free[1:]):
            assert o1 + s1 < o2                 # free blocks are merged
    for blk in live:
        a.release(*blk)
    assert a.free == [(0, a.nbytes)]


def test_fifo_rebuild_of_one_at_a_time_server():
    """The one-at-a-time timeline rebuilt from service times: a request starts
    when it has arrived and the previous one has finished."""
    from paper_2510_05254_amd.serve_runs import fifo
    lat, end = fifo([1.0, 2.0, 3.0], [0.0, 0.0, 0.0])
    assert lat == [1.0, 3.0, 6.0] and end == 6.0
    lat, end = fifo([1.0, 1.0, 1.0], [0.0, 5.0, 5.5])     # idle gap, then a queue
    assert lat == [1.0, 1.0, 1.5] and end == 7.0
