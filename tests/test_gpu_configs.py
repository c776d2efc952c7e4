"""GPU parity at the benchmark configurations' full sizes, in the launch
configuration bench.py times.

* Config 1 (1-D advection, K=64, N=3, to t=1 in 2316 RK4 steps): every output
  against the oracle, and both against the exact translated solution.
* Configs 2-4 at full mesh size: every output against the oracle after a
  reduced number of steps the oracle finishes in seconds (2-D advection 10,
  2-D Euler 5, 3-D Euler 1 step); then the full step count on the GPU alone,
  checked by properties that hold at any size: mass conservation and, for
  advection, the exact translated solution.
* A mesh whose state arrays exceed 2 GiB (the stage kernels' 64-bit
  addressing path, which none of the configurations reaches): every output
  against the oracle after one RK4 and one RK6 step.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_2510_05254_amd import dg
from paper_2510_05254_amd import workloads as W
from _helpers import PARITY_RTOL, rel_l2_per_var

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=1)
def _inputs(cid):
    w = W.config(cid)
    ax = [oracle.axis_coords(w.N, k) for k in w.K]
    U0 = W.initial_state(w, ax)
    dt, n = W.time_step(w, ax, U0)
    return w, ax, U0, dt, n


def test_config1_full_run():
    w, ax, U0, dt, n = _inputs(1)
    _say(f"config 1: {n} RK4 steps dt={dt}")
    with dg.Solver(w.dim, w.N, w.K, w.eq, w.params) as s:
        s.set_state(U0)
        s.step(4, dt, n)
        Ug = s.get_state()
        gpu_err = s.l2_error(U0)
    Uo = oracle.step(w.dim, w.N, w.K, w.eq, w.params, U0, 4, dt, n)
    assert np.all(rel_l2_per_var(Ug, Uo) <= PARITY_RTOL)
    # after one revolution both equal U_0 up to the discretisation error
    o_abs, o_rel = oracle.l2_error(w.dim, w.N, w.K, w.eq, Uo, U0)
    # | |Ug - U0| - |Uo - U0| | <= |Ug - Uo| <= PARITY_RTOL |U0| (triangle inequality)
    norm0 = o_abs / o_rel
    assert abs(gpu_err[0] - o_abs) <= 2 * PARITY_RTOL * norm0
    assert 1e-8 < o_rel < 1e-4, o_rel


@pytest.mark.parametrize("cid,steps", [(2, 10), (3, 5), (4, 1)])
def test_config_full_size_parity(cid, steps):
    w, ax, U0, dt, n = _inputs(cid)
    _say(f"config {cid}: {w.unknowns} unknowns, {steps} RK4 steps on GPU")
    with dg.Solver(w.dim, w.N, w.K, w.eq, w.params) as s:
        s.set_state(U0)
        s.step(4, dt, steps)
        Ug = s.get_state()
    _say(f"config {cid}: oracle ({oracle.get_threads()} threads)")
    Uo = oracle.step(w.dim, w.N, w.K, w.eq, w.params, U0, 4, dt, steps)
    err = rel_l2_per_var(Ug, Uo)
    _say(f"config {cid}: rel L2 per var {err}")
    assert np.all(err <= PARITY_RTOL), err


@pytest.mark.parametrize("cid", [2, 3, 4])
def test_config_full_run_properties(cid):
    w, ax, U0, dt, n = _inputs(cid)
    _say(f"config {cid}: full {n} RK4 steps on GPU")
    with dg.Solver(w.dim, w.N, w.K, w.eq, w.params) as s:
        s.set_state(U0)
        m0 = s.mass()
        s.step(4, dt, n)
        m1 = s.mass()
        Ug = s.get_state()
        if w.eq == W.ADVECTION:
            exact = W.translated_advection(w, ax, n * dt)
            a, r = s.l2_error(exact)
    assert np.all(np.isfinite(Ug))
    scale = np.maximum(np.abs(U0).max(axis=1), 1.0)
    assert np.all(np.abs(m1 - m0) <= 1e-12 * scale), (m0, m1)
    if w.eq == W.ADVECTION:
        _say(f"config {cid}: L2 vs exact {a} rel {r}")
        assert r < 1e-8, r


# FP32 path at the configurations' sizes against the FP64 oracle. Single
# precision rounds each stage's arithmetic at u = 6e-8; over a few steps the
# relative error stays at a few hundred u (bar 1e-5). For the 2316-step run of
# config 1 the error is measured against |U0| and may grow linearly with the
# 9264 stages (bar 1e-4). Measured values are printed for the record.
@pytest.mark.parametrize("cid,steps,bar", [(1, None, 1e-4), (2, 10, 1e-5), (3, 5, 1e-5), (4, 1, 1e-5)])
def test_config_fp32_against_fp64_oracle(cid, steps, bar):
    w, ax, U0, dt, n = _inputs(cid)
    steps = n if steps is None else steps
    with dg.Solver(w.dim, w.N, w.K, w.eq, w.params, precision=dg.DG_FP32) as s:
        s.set_state(U0)
        s.step(4, dt, steps)
        Ug = s.get_state()
    Uo = oracle.step(w.dim, w.N, w.K, w.eq, w.params, U0, 4, dt, steps)
    if cid == 1:
        err = np.array([np.linalg.norm(Ug - Uo) / np.linalg.norm(U0)])
    else:
        err = rel_l2_per_var(Ug, Uo)
    _say(f"config {cid} FP32, {steps} RK4 steps: rel L2 per var vs FP64 oracle {err}")
    assert np.all(err <= bar), err


# 3-D Euler N = 4 on 84 x 81 x 80 elements: 2.18 GB per state array, so the
# stage kernels address it with 64-bit pointers; tiles of 2 x 2 elements with
# a ragged last row.
@pytest.mark.parametrize("rk", [4, 6])
def test_64bit_addressing_parity(rk):
    from _helpers import EUL, case, params
    K = (84, 81, 80)
    w, ax, U0, dt = case(3, 4, K, EUL, 31)
    assert U0.nbytes >= 2 ** 31
    _say(f"64-bit path: K={K}, {U0.nbytes / 1e9:.2f} GB per array, rk={rk}")
    with dg.Solver(3, 4, K, EUL, params(3, EUL)) as s:
        s.set_state(U0)
        s.step(rk, dt, 1)
        Ug = s.get_state()
    Uo = oracle.step(3, 4, K, EUL, params(3, EUL), U0, rk, dt, 1)
    err = rel_l2_per_var(Ug, Uo)
    _say(f"rel L2 per var {err}")
    assert np.all(err <= PARITY_RTOL), err
    assert rel_l2_per_var(Uo, U0).max() > 1e3 * PARITY_RTOL
