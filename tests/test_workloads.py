"""Checks of the seeded input generators (no method arithmetic involved)."""
import os

import numpy as np
import pytest

from paper_2510_05254_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_outputs():
    ref = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
           if l.strip() and not l.startswith("#")]
    r = W.SplitMix64(0)
    assert [r.next_u64() for _ in range(len(ref))] == ref
    u = W.SplitMix64(123).uniforms(1000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.05


def _direct(axes, kvec, phase, coef):
    """Node-by-node evaluation in canonical order (element x fastest, node x fastest)."""
    dim = len(axes)
    K = [a.shape[0] for a in axes]
    n1 = axes[0].shape[1]
    out = []
    for e in np.ndindex(*reversed(K)):
        e = tuple(reversed(e))
        for n in np.ndindex(*([n1] * dim)):
            n = tuple(reversed(n))
            x = np.array([axes[d][e[d], n[d]] for d in range(dim)])
            out.append(sum(c * np.sin(2 * np.pi * np.dot(k, x) + 2 * np.pi * p)
                           for k, p, c in zip(kvec, phase, coef)))
    return np.array(out)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_fourier_sum_matches_direct_evaluation(dim):
    rng = W.SplitMix64(dim)
    K = [3, 2, 2][:dim]
    N = 2
    axes = [np.sort(rng.uniforms(k * (N + 1))).reshape(k, N + 1) for k in K]
    kvec = [[rng.randint(-3, 3) for _ in range(dim)] for _ in range(4)]
    ph = rng.uniforms(4)
    co = rng.uniforms(4)
    np.testing.assert_allclose(W.fourier_sum(axes, kvec, ph, co)[0], _direct(axes, kvec, ph, co),
                               atol=1e-12)


def test_config_shapes_and_steps(oracle):
    w1 = W.config(1)
    ax = [oracle.axis_coords(w1.N, w1.K[0])]
    U0 = W.initial_state(w1, ax)
    dt, n = W.time_step(w1, ax, U0)
    assert n == 2316 and abs(dt - 1 / 2316) < 1e-18
    np.testing.assert_allclose(U0[0], np.sin(2 * np.pi * ax[0].reshape(-1)), atol=1e-14)
    assert (W.config(2).unknowns, W.config(3).unknowns, W.config(4).unknowns) == (
        4194304, 12582912, 131072000)


@pytest.mark.parametrize("cid,K", [(3, (8, 6)), (4, (4, 3, 5))])
def test_euler_initial_fields(oracle, cid, K):
    w = W.scaled(W.config(cid), K)
    ax = [oracle.axis_coords(w.N, k) for k in w.K]
    U = W.initial_state(w, ax)
    rho = U[0]
    vel = U[1:] / rho
    speed = np.sqrt((vel ** 2).sum(axis=0))
    assert abs(speed.max() - 0.1) < 1e-14
    if cid == 3:
        assert abs(np.abs(rho - 1).max() - 1e-2) < 1e-14
    else:
        assert np.all(rho == 1.0)
    # same seed, same field
    np.testing.assert_array_equal(U, W.initial_state(w, ax))
