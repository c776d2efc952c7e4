"""dg_step_static (stepping with no device allocation, work memory in the
library's static scratch) against the allocating path on the same inputs,
through the C ABI: dg_create_ex (library-owned memory) + dg_set_state_device +
dg_step + dg_get_state_device. The kernels and stage schedules are shared, so
results must agree bit for bit. Calls follow each other on one stream with
shrinking inputs, so later calls run on scratch the earlier, larger ones left
behind; the sequence changes kernel class (tables re-uploaded), scheme (RK3,
RK4, RK6), precision and the 1-D temporally blocked path."""
import sys

import numpy as np
import pytest
import torch

from paper_2510_05254_amd import dg
from _helpers import ADV, EUL, case, params

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _allocating(dim, N, K, eq, prec, U0_dev, rk, dt, nsteps, stream):
    """The existing entry points, library-owned workspace."""
    out = torch.empty_like(U0_dev)
    h = dg.dg_create_ex(dim, N, K, eq, params(dim, eq), prec, stream.cuda_stream)
    try:
        dg.dg_set_state_device(h, U0_dev)
        dg.dg_step(h, rk, dt, nsteps)
        dg.dg_get_state_device(h, out)
        dg.dg_synchronize(h)
    finally:
        dg.dg_destroy(h)
    return out


# (dim, N, K, eq, precision, rk, steps): each call's state is no larger than
# the one before; the first is the largest 2-D advection N = 7 mesh of the
# benchmark configurations (256^2, 3 x 33.6 MB of RK work arrays)
SEQUENCE = [
    (2, 7, (256, 256), ADV, dg.DG_FP64, 4, 3),
    (2, 7, (19, 13), ADV, dg.DG_FP64, 4, 5),
    (3, 4, (5, 3, 2), EUL, dg.DG_FP64, 4, 3),
    (3, 2, (6, 5, 4), EUL, dg.DG_FP64, 6, 2),
    (1, 3, (300,), EUL, dg.DG_FP64, 4, 7),
    (2, 3, (9, 5), EUL, dg.DG_FP32, 3, 4),
    (1, 5, (13,), ADV, dg.DG_FP64, 3, 9),
]


def test_static_matches_allocating_path_in_sequence():
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    prev = None
    for i, (dim, N, K, eq, prec, rk, steps) in enumerate(SEQUENCE):
        w, ax, U0, dt = case(dim, N, K, eq, seed=100 + i)
        size = U0.size
        assert prev is None or size <= prev, "inputs must not grow along the sequence"
        prev = size
        _say(f"call {i}: dim={dim} N={N} K={K} eq={eq} prec={prec} rk={rk} steps={steps} "
             f"unknowns={size}")
        U64 = torch.from_numpy(np.ascontiguousarray(U0.reshape(-1))).to("cuda")
        ref = _allocating(dim, N, K, eq, prec, U64, rk, dt, steps, stream)
        if prec == dg.DG_FP64:
            u = U64.clone()
        else:
            u = U64.to(torch.float32)
        torch.cuda.synchronize()
        dg.dg_step_static(dim, N, K, eq, params(dim, eq), prec, stream.cuda_stream, u, rk, dt, steps)
        stream.synchronize()
        got = u.to(torch.float64).cpu().numpy()
        want = ref.cpu().numpy()
        assert np.all(np.isfinite(got))
        moved = np.abs(want - U0.reshape(-1)).max()
        assert moved > 0.0, "the state did not move"
        diff = np.abs(got - want).max()
        _say(f"call {i}: max |static - dg_step| = {diff:.3e} (state moved by {moved:.3e})")
        assert np.array_equal(got, want), f"call {i}: static path differs from dg_step by {diff}"


def test_static_zero_steps_and_oversize_leave_state_untouched():
    torch.cuda.set_device(0)
    w, ax, U0, dt = case(2, 3, (7, 4), EUL, seed=7)
    u = torch.from_numpy(np.ascontiguousarray(U0.reshape(-1))).to("cuda")
    before = u.clone()
    dg.dg_step_static(2, 3, (7, 4), EUL, params(2, EUL), dg.DG_FP64, None, u, 4, dt, 0)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
    # a mesh whose RK work arrays exceed the static scratch is refused before
    # anything runs (the state array itself need not exist at that size: the
    # size check precedes every device access)
    K = (512, 512)
    n = 512 * 512 * 8 * 8
    with pytest.raises(dg.DgError) as e:
        dg.dg_step_static(2, 7, K, ADV, params(2, ADV), dg.DG_FP64, None, u.data_ptr(), 4, dt, 1,
                          count=n)
    assert e.value.status == dg.DG_ENOMEM
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
