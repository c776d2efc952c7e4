"""Batched stepping (dg_batch_*) on the GPU.

A member of a batch must end exactly where dg_step on the same solver alone
ends (same stage programs and kernel bodies), and within the parity
bar of the oracle. Covered: mixed kernel classes (1-D/2-D/3-D, advection and
Euler, several N), different meshes and time steps in one class, members with
different step counts, members admitted while others run (continuous
batching), hipGraph replay of a tick with host work between replays, and the
error paths.
"""
import numpy as np
import pytest

import oracle
from paper_2510_05254_amd import dg
from _helpers import ADV, EUL, PARITY_RTOL, case, params, parity, rel_l2_per_var

pytestmark = pytest.mark.gpu

MIX = [  # (dim, N, K, eq, rk, nsteps)
    (1, 3, (37,), ADV, 4, 5),
    (1, 3, (64,), ADV, 4, 9),      # same class as the first, other mesh and dt
    (2, 2, (9, 5), EUL, 4, 4),
    (2, 2, (3, 11), EUL, 4, 13),   # gaps of >= 4 steps: graph replays
    (2, 7, (5, 4), ADV, 3, 6),
    (3, 2, (4, 3, 5), EUL, 4, 3),
    (3, 4, (3, 2, 2), EUL, 4, 18),
    (3, 4, (2, 3, 1), EUL, 4, 7),  # same class: 2 x 2 tiles, ragged last row
    # classes with the velocity LDS layout and/or the six-wave register target
    (3, 1, (40, 3, 2), EUL, 4, 3),
    (3, 6, (2, 2, 1), EUL, 3, 2),
    (3, 7, (2, 1, 2), EUL, 4, 2),
    (3, 8, (1, 2, 1), EUL, 4, 2),
    (1, 5, (10,), EUL, 3, 5),
    (1, 7, (1500,), ADV, 4, 27),   # 1-D, chunked: several multi-step launches
    (1, 7, (90,), ADV, 4, 9),      # same class, held whole by one workgroup
    # RK6 members: fused stages with further inputs, one launch per stage
    (1, 4, (50,), ADV, 6, 3),
    (2, 3, (6, 5), EUL, 6, 2),
    (2, 3, (4, 7), EUL, 6, 5),     # same class, other mesh, dt and step count
    (3, 2, (3, 2, 2), EUL, 6, 2),
]


def _solver_with_state(dim, N, K, eq, seed):
    w, ax, U0, dt = case(dim, N, K, eq, seed)
    s = dg.Solver(dim, N, K, eq, params(dim, eq))
    s.set_state(U0)
    return s, U0, dt


def _alone(dim, N, K, eq, U0, rk, dt, n):
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        s.step(rk, dt, n)
        return s.get_state()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_single_solves(graph):
    solvers, refs = [], []
    with dg.Batch(graph=graph) as b:
        for i, (dim, N, K, eq, rk, n) in enumerate(MIX):
            s, U0, dt = _solver_with_state(dim, N, K, eq, 100 + i)
            b.add(s, rk, dt, n)
            solvers.append((s, U0, dt))
        assert b.size() == (len(MIX), len(MIX))
        calls = b.run_all()
        assert calls == len(set(m[5] for m in MIX))     # one run per distinct finish time
        assert b.size() == (len(MIX), 0)
        for (dim, N, K, eq, rk, n), (s, U0, dt) in zip(MIX, solvers):
            assert b.remaining(s) == 0
            Ub = s.get_state()
            Ua = _alone(dim, N, K, eq, U0, rk, dt, n)
            np.testing.assert_array_equal(Ub, Ua)
            Uo = oracle.step(dim, N, K, eq, params(dim, eq), U0, rk, dt, n)
            parity(Ub, Uo, what=f"batch member dim={dim} N={N} K={K} eq={eq} rk={rk}")
    for s, _, _ in solvers:
        s.close()


# FP32 members (1-D chunked and whole, 2-D, 3-D with 2 x 2 tiles and a ragged
# last row; RK3 and RK4): bitwise the FP32 dg_step result, and within the
# FP32 bar of the FP64 oracle.
MIX32 = [  # (dim, N, K, eq, rk, nsteps)
    (1, 5, (3000,), EUL, 4, 9),
    (1, 3, (50,), ADV, 3, 6),
    (2, 3, (9, 5), EUL, 4, 5),
    (2, 7, (6, 4), ADV, 4, 5),
    (3, 4, (3, 3, 2), EUL, 4, 5),
    (3, 2, (5, 3, 2), ADV, 3, 4),
]
FP32_BAR = 2e-5      # relative L2 per variable after <= 9 steps (u = 6e-8 per stage operation)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_fp32_matches_single_solves(graph):
    made = []
    with dg.Batch(graph=graph) as b:
        for i, (dim, N, K, eq, rk, n) in enumerate(MIX32):
            w, ax, U0, dt = case(dim, N, K, eq, 300 + i)
            s = dg.Solver(dim, N, K, eq, params(dim, eq), precision=dg.DG_FP32)
            s.set_state(U0)
            b.add(s, rk, dt, n)
            made.append((s, U0, dt))
        b.run_all()
        for (dim, N, K, eq, rk, n), (s, U0, dt) in zip(MIX32, made):
            Ub = s.get_state()
            with dg.Solver(dim, N, K, eq, params(dim, eq), precision=dg.DG_FP32) as a:
                a.set_state(U0)
                a.step(rk, dt, n)
                np.testing.assert_array_equal(Ub, a.get_state())
            Uo = oracle.step(dim, N, K, eq, params(dim, eq), U0, rk, dt, n)
            err = rel_l2_per_var(Ub, Uo)
            print(f"fp32 batch member dim={dim} N={N} K={K} rk={rk}: rel L2 {err}")
            assert np.all(err <= FP32_BAR), err
    for s, _, _ in made:
        s.close()


def test_continuous_admission_and_graph_replays():
    """Members join while others run; graph ticks replayed with host work between."""
    specs = [(2, 3, (6, 5), EUL, 4, 12), (1, 4, (20,), ADV, 4, 7), (2, 3, (4, 4), EUL, 4, 9)]
    made = [_solver_with_state(*sp[:4], seed=7 + i) for i, sp in enumerate(specs)]
    with dg.Batch(graph=True) as b:
        b.add(made[0][0], 4, made[0][2], specs[0][5])
        assert b.run(3) == 3
        mid = made[0][0].get_state()                       # host work between replays
        np.testing.assert_array_equal(mid, _alone(*specs[0][:4], made[0][1], 4, made[0][2], 3))
        b.add(made[1][0], 4, made[1][2], specs[1][5])       # joins the running batch
        assert b.run(2) == 2
        b.add(made[2][0], 4, made[2][2], specs[2][5])
        while b.run(1 << 40):
            pass
        for sp, (s, U0, dt) in zip(specs, made):
            np.testing.assert_array_equal(s.get_state(), _alone(*sp[:4], U0, 4, dt, sp[5]))
        for s, _, _ in made:
            b.remove(s)
        assert b.size() == (0, 0)
    for s, _, _ in made:
        s.close()


def test_batch_error_paths():
    s, U0, dt = _solver_with_state(2, 2, (3, 3), ADV, 3)
    fresh = dg.Solver(2, 2, (3, 3), ADV, params(2, ADV))
    # an RK6 member needs the RK6 stage store: an external workspace sized
    # for RK4 cannot hold it
    import torch
    ws4 = dg.dg_workspace_bytes(2, 2, (3, 3), ADV, dg.DG_FP64, 4)
    buf = torch.empty(ws4, dtype=torch.uint8, device="cuda")
    small = dg.Solver(2, 2, (3, 3), ADV, params(2, ADV), device_workspace=buf.data_ptr(), workspace_bytes=ws4)
    small.set_state(U0)
    with dg.Batch() as b:
        with pytest.raises(dg.DgError) as e:
            b.add(small, 6, dt, 2)
        assert e.value.status == dg.DG_ENOMEM
        with pytest.raises(dg.DgError) as e:
            b.add(fresh, 4, dt, 2)
        assert e.value.status == dg.DG_ESTATE
        for bad in ((5, dt, 2), (4, -dt, 2), (4, dt, 0)):
            with pytest.raises(dg.DgError) as e:
                b.add(s, *bad)
            assert e.value.status == dg.DG_EINVAL
        b.add(s, 4, dt, 2)
        with pytest.raises(dg.DgError) as e:
            b.add(s, 4, dt, 2)
        assert e.value.status == dg.DG_ESTATE
        with pytest.raises(dg.DgError) as e:
            s.step(4, dt, 1)                  # a member is stepped by its batch only
        assert e.value.status == dg.DG_ESTATE
        with pytest.raises(dg.DgError) as e:
            s.set_state(U0)
        assert e.value.status == dg.DG_ESTATE
        with pytest.raises(dg.DgError) as e:
            b.remove(fresh)
        assert e.value.status == dg.DG_EINVAL
        assert b.run(0) == 0
        s.close()                             # destroying a member removes it
        assert b.size() == (0, 0)
        assert b.run(10) == 0
    fresh.close()
    small.close()


def test_reading_an_active_member_mid_run():
    """A member read on the device while the batch still has steps for it sees
    the state after the steps enqueued so far, and the batch's later steps
    (which rewrite its arrays, including the staging the read converts
    through) wait for that read."""
    import torch
    specs = [(2, 3, (6, 5), EUL, 11), (1, 6, (900,), ADV, 11), (3, 2, (3, 2, 2), EUL, 11)]
    made = [_solver_with_state(*sp[:4], 300 + i) for i, sp in enumerate(specs)]
    with dg.Batch() as b:
        for (s, U0, dt), sp in zip(made, specs):
            b.add(s, 4, dt, sp[4])
        assert b.run(4) == 4
        mids = []
        for s, U0, dt in made:
            out = torch.empty(U0.size, dtype=torch.float64, device="cuda")
            s.get_state_device(out)                 # asynchronous, on the member's stream
            mids.append(out)
        b.run(1 << 40)                              # the remaining 7 steps, enqueued after the reads
        b.synchronize()
        for (s, U0, dt), sp, out in zip(made, specs, mids):
            s.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy().reshape(U0.shape), _alone(*sp[:4], U0, 4, dt, 4))
            np.testing.assert_array_equal(s.get_state(), _alone(*sp[:4], U0, 4, dt, sp[4]))
    for s, _, _ in made:
        s.close()
