"""Whole-solver pins for the oracle (RHS + RK together).

* Periodic linear advection has the exact solution U_0(x - a t) (Sec. 3.1, the
  paper's one-revolution test); the L2 error converges at order N+1 (the
  expected convergence the paper reports for its Fig. convergence, with RK6
  and a small time step).
* Mass (the integral of every conserved variable) is conserved to roundoff.
* A constant isothermal Euler state is a steady solution.
* A small acoustic wave travels at c_s: a right-running wave returns to its
  initial state after t = 1/c_s along x, y or z.
* The nodal quadrature integrates polynomials of degree <= 2N-1 per direction
  exactly (mass and L2 functions).
"""
import numpy as np
import pytest

from paper_2510_05254_amd import workloads as W

ADV, EUL = 0, 1


@pytest.mark.parametrize("N,Ks", [(1, (128, 256)), (2, (32, 64)), (3, (16, 32)), (4, (16, 32)),
                                  (5, (8, 16)), (6, (8, 16)), (7, (8, 16))])
def test_advection_convergence_order(oracle, N, Ks):
    errs = []
    for K in Ks:
        w = W.Workload("conv", 1, N, (K,), ADV, (1.0,), "fourier1d", 7, rk=6, t_final=1.0,
                       ic_args={"nk": 3})
        ax = [oracle.axis_coords(N, K)]
        U0 = W.initial_state(w, ax)
        dt, n = W.time_step(w, ax, U0)
        U = oracle.step(1, N, [K], ADV, [1.0], U0, 6, dt, n)
        errs.append(oracle.l2_error(1, N, [K], ADV, U, U0)[0])
    rate = np.log2(errs[0] / errs[1])
    assert rate >= N + 1 - 0.3, (N, errs, rate)
    assert 1e-11 < errs[1] < 2e-2


@pytest.mark.parametrize("rk", [3, 4, 6])
def test_advection_2d_translated_solution(oracle, rk):
    """2-D advection with a = (1, 0.5) after t = 0.2 against U_0(x - a t); the
    error falls at order N+1 = 6 when the mesh is refined."""
    errs = []
    for K in (6, 12):
        w = W.Workload("adv2d", 2, 5, (K, K), ADV, (1.0, 0.5), "fourier_adv", 3, rk=rk,
                       t_final=0.2, ic_args={"modes": 3, "kmax": 2})
        ax = [oracle.axis_coords(5, K), oracle.axis_coords(5, K)]
        U0 = W.initial_state(w, ax)
        dt, n = W.time_step(w, ax, U0)
        U = oracle.step(2, 5, [K, K], ADV, [1.0, 0.5], U0, rk, dt, n)
        exact = W.translated_advection(w, ax, n * dt)
        errs.append(oracle.l2_error(2, 5, [K, K], ADV, U, exact)[1])
    assert errs[0] < 3e-4, errs
    if rk == 6:
        assert np.log2(errs[0] / errs[1]) >= 5.7, errs


@pytest.mark.parametrize("dim,N,K", [(1, 3, (8,)), (2, 2, (4, 3)), (3, 2, (2, 3, 2))])
def test_euler_mass_conservation(oracle, dim, N, K):
    rng = W.SplitMix64(41)
    n = int(np.prod(K)) * (N + 1) ** dim
    rho = 1.0 + 0.1 * (rng.uniforms(n) - 0.5)
    U0 = np.array([rho] + [rho * 0.1 * (rng.uniforms(n) - 0.5) for _ in range(dim)])
    m0 = oracle.mass(dim, N, K, EUL, U0)
    U = oracle.step(dim, N, K, EUL, [1.0], U0, 4, 1e-3, 100)
    m1 = oracle.mass(dim, N, K, EUL, U)
    assert np.all(np.isfinite(U))
    np.testing.assert_allclose(m1, m0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_constant_euler_state_is_steady(oracle, dim):
    N, K = 3, (3,) * dim
    n = int(np.prod(K)) * (N + 1) ** dim
    vals = np.array([1.2, 0.3, -0.2, 0.1][:dim + 1])
    U0 = np.repeat(vals[:, None], n, axis=1)
    U = oracle.step(dim, N, K, EUL, [1.0], U0, 4, 2e-3, 20)
    assert np.abs(U - U0).max() <= 1e-13


@pytest.mark.parametrize("dim,axis", [(1, 0), (2, 1), (3, 2)])
def test_acoustic_wave_returns(oracle, dim, axis):
    """rho = 1 + eps s, m_axis = c eps s with s = sin(2 pi x_axis): a right-running
    isothermal sound wave; after t = 1/c it is back where it started."""
    N, Ka, eps, c = 5, 8, 1e-6, 1.0
    K = [2] * dim
    K[axis] = Ka
    ax = [oracle.axis_coords(N, k) for k in K]
    w = W.Workload("s", dim, N, tuple(K), ADV, (1.0,) * dim, "fourier1d", 1)
    ks = [0] * dim
    ks[axis] = 1
    s = W.fourier_sum(ax, [ks], [0.0], [1.0])[0]
    U0 = np.zeros((dim + 1, w.nodes))
    U0[0] = 1.0 + eps * s
    U0[1 + axis] = c * eps * s
    dx = min(np.diff(a, axis=1).min() for a in ax)
    n = int(np.ceil(1.0 / (0.2 * dx / (c * 1.001))))
    U = oracle.step(dim, N, K, EUL, [c], U0, 4, 1.0 / (c * n), n)
    err = np.abs(U - U0).max()
    assert err <= 1e-3 * eps, err


def test_quadrature_integrals(oracle):
    """mass/l2 integrate tensor polynomials of degree <= 2N-1 per direction exactly."""
    N, K = 3, (2, 3, 2)
    ax = [oracle.axis_coords(N, k) for k in K]
    n = int(np.prod(K)) * (N + 1) ** 3
    X = W.fourier_sum(ax, [[1, 0, 0]], [0.0], [1.0])[0]   # only for the grid shape
    # build x, y, z at every node in canonical order
    G = [np.zeros_like(X) for _ in range(3)]
    for d in range(3):
        vals = ax[d]
        if d == 0:
            arr = np.broadcast_to(vals[None, None, :, None, None, :], (K[2], K[1], K[0], N + 1, N + 1, N + 1))
        elif d == 1:
            arr = np.broadcast_to(vals[None, :, None, None, :, None], (K[2], K[1], K[0], N + 1, N + 1, N + 1))
        else:
            arr = np.broadcast_to(vals[:, None, None, :, None, None], (K[2], K[1], K[0], N + 1, N + 1, N + 1))
        G[d] = np.ascontiguousarray(arr).reshape(-1)
    x, y, z = G
    f = x ** 5 * y ** 2 + z ** 3 - 2 * x * y * z      # per-direction degree <= 5 = 2N-1
    exact = 1 / 18 + 1 / 4 - 2 / 8
    U = np.array([f, 0 * f, 0 * f, 0 * f])
    m = oracle.mass(3, N, K, EUL, U)
    assert abs(m[0] - exact) <= 1e-15 and np.all(m[1:] == 0)
    se, sr = oracle.l2(3, N, K, EUL, U, np.zeros_like(U))
    g = x ** 2 * y + z          # squared: per-direction degree <= 4
    se2, _ = oracle.l2(3, N, K, EUL, np.array([g, g, g, g]), np.zeros((4, n)))
    exact_sq = 1 / 5 * 1 / 3 + 2 * (1 / 3 * 1 / 2 * 1 / 2) + 1 / 3
    np.testing.assert_allclose(se2, exact_sq, rtol=1e-14)
    assert np.all(sr == 0)
