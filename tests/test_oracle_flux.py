"""Pins for the oracle's physical and numerical fluxes (eqs. advection2d,
eulerIso2d, LF).

The isothermal Euler flux is pinned by properties of the PDE rather than by
retyping it: the eigenvalues of its Jacobian are u_d - c, u_d (dim-1 times),
u_d + c; a fluid at rest only carries pressure rho c^2 normal to the face; the
momentum flux tensor is symmetric; and an axis permutation maps the fluxes
onto each other. The Lax-Friedrichs flux is pinned by consistency
(Fhat(U, U) = F(U)), by its reduction to exact upwinding for advection, and by
its dissipation term.
"""
import numpy as np
import pytest

from paper_2510_05254_amd.workloads import SplitMix64

ADV, EUL = 0, 1


def _random_euler_state(rng, dim):
    rho = 0.5 + rng.uniform()
    u = [0.6 * (2 * rng.uniform() - 1) for _ in range(dim)]
    return np.array([rho] + [rho * x for x in u]), rho, np.array(u)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_euler_jacobian_eigenvalues(oracle, dim):
    rng = SplitMix64(11 + dim)
    c = 0.7
    for _ in range(10):
        U, rho, u = _random_euler_state(rng, dim)
        for d in range(dim):
            h = 1e-6
            J = np.zeros((dim + 1, dim + 1))
            for j in range(dim + 1):
                e = np.zeros(dim + 1)
                e[j] = h
                J[:, j] = (oracle.flux(dim, d, EUL, [c], U + e) - oracle.flux(dim, d, EUL, [c], U - e)) / (2 * h)
            ev = np.sort(np.linalg.eigvals(J).real)
            ref = np.sort([u[d] - c, u[d] + c] + [u[d]] * (dim - 1))
            np.testing.assert_allclose(ev, ref, atol=1e-7)
            assert abs(oracle.max_speed(dim, d, EUL, [c], U) - (abs(u[d]) + c)) <= 1e-15


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_euler_flux_at_rest_and_symmetry(oracle, dim):
    c = 1.3
    rho = 0.8
    U = np.zeros(dim + 1)
    U[0] = rho
    for d in range(dim):
        F = oracle.flux(dim, d, EUL, [c], U)
        ref = np.zeros(dim + 1)
        ref[1 + d] = rho * c * c
        np.testing.assert_allclose(F, ref, rtol=1e-15, atol=0)
    rng = SplitMix64(5)
    U, rho, u = _random_euler_state(rng, dim)
    for d in range(dim):
        Fd = oracle.flux(dim, d, EUL, [c], U)
        assert Fd[0] == U[1 + d]                      # mass flux = momentum
        for k in range(dim):
            Fk = oracle.flux(dim, k, EUL, [c], U)
            assert abs(Fd[1 + k] - Fk[1 + d]) <= 1e-15  # symmetric momentum flux


def test_euler_flux_axis_permutation(oracle):
    rng = SplitMix64(9)
    c = 1.0
    U, _, _ = _random_euler_state(rng, 3)
    perm = [2, 0, 1]            # new axis a is old axis perm[a]
    Up = np.array([U[0]] + [U[1 + perm[a]] for a in range(3)])
    for a in range(3):
        F = oracle.flux(3, perm[a], EUL, [c], U)
        Fp = oracle.flux(3, a, EUL, [c], Up)
        np.testing.assert_allclose(Fp, [F[0]] + [F[1 + perm[b]] for b in range(3)], rtol=1e-15)


@pytest.mark.parametrize("dim,eq", [(1, ADV), (3, ADV), (1, EUL), (2, EUL), (3, EUL)])
def test_numflux_consistency(oracle, dim, eq):
    rng = SplitMix64(21)
    par = [0.7, -1.1, 0.3] if eq == ADV else [1.0]
    for _ in range(10):
        U = _random_euler_state(rng, dim)[0] if eq == EUL else np.array([rng.uniform() - 0.5])
        for d in range(dim):
            np.testing.assert_array_equal(oracle.numflux(dim, d, eq, par, U, U),
                                          oracle.flux(dim, d, eq, par, U))


def test_numflux_advection_is_upwind(oracle):
    for a in (1.0, -0.5, 2.5):
        UL, UR = np.array([0.3]), np.array([-1.7])
        F = oracle.numflux(1, 0, ADV, [a], UL, UR)
        up = a * (UL if a > 0 else UR)
        assert abs(F[0] - up[0]) <= 2e-16 * abs(up[0]) + 1e-300


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_numflux_euler_dissipation(oracle, dim):
    rng = SplitMix64(33)
    c = 1.0
    UL, _, uL = _random_euler_state(rng, dim)
    UR, _, uR = _random_euler_state(rng, dim)
    for d in range(dim):
        F = oracle.numflux(dim, d, EUL, [c], UL, UR)
        central = 0.5 * (oracle.flux(dim, d, EUL, [c], UL) + oracle.flux(dim, d, EUL, [c], UR))
        alpha = max(abs(uL[d]), abs(uR[d])) + c
        np.testing.assert_allclose(F - central, -0.5 * alpha * (UR - UL), atol=1e-15)
