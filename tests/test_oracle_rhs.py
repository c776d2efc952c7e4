"""Pins for the oracle's NDG right-hand side (Sec. 2.1 evolution equation).

Each check is a property the discrete operator must have, chosen so that a
plausible mistake (a dropped face term, a wrong sign, a transposed D, a wrong
neighbour index or Jacobian) fails at least one of them:

* hand-derived values on a 2-element mesh (tests/golden);
* conservation: the quadrature integral of R vanishes for every variable;
* the upwind energy identity for advection (exact for random data);
* free stream: R(constant state) = 0;
* weak and strong forms agree (summation by parts);
* periodic shift, axis permutation, reduction of 2-D/3-D to 1-D;
* linearity for advection;
* consistency: R of the interpolant of a smooth field tends to -div F at rate N.
"""
import os

import numpy as np
import pytest

from paper_2510_05254_amd.workloads import SplitMix64

ADV, EUL = 0, 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(seed, n, lo=-1.0, hi=1.0):
    r = SplitMix64(seed)
    return lo + (hi - lo) * r.uniforms(n)


def _state(dim, N, K, eq, seed):
    n = int(np.prod(K)) * (N + 1) ** dim
    if eq == ADV:
        return _rand(seed, n).reshape(1, n)
    rho = _rand(seed, n, 0.6, 1.4)
    U = [rho] + [rho * _rand(seed + 1 + d, n, -0.4, 0.4) for d in range(dim)]
    return np.array(U)


def _par(dim, eq):
    return [0.8, -0.45, 0.3][:dim] if eq == ADV else [1.2]


def _weights(oracle, dim, N, K):
    """Nodal quadrature weights prod_d (dx_d/2) w_{n_d} in canonical order."""
    _, w = oracle.lgl(N)
    Kl = list(K) + [1] * (3 - dim)
    wn = np.ones(1)
    for d in range(dim):                       # node index n = i + n1 (j + n1 k)
        wn = np.kron(w * (0.5 / Kl[d]), wn) if d > 0 else w * (0.5 / Kl[d])
    # np.kron above builds x fastest: wn[i + n1*j] = w_i w_j (scaled)
    return np.tile(wn, int(np.prod(K)))


def _grid(U, dim, N, K):
    """(nvar, E*Np) -> (nvar, Kz, Ky, Kx, n1z, n1y, n1x) with unit extents padded."""
    n1 = N + 1
    Kl = list(K) + [1] * (3 - dim)
    nl = [n1 if d < dim else 1 for d in range(3)]
    return U.reshape(U.shape[0], Kl[2], Kl[1], Kl[0], nl[2], nl[1], nl[0])


def _flat(G):
    return G.reshape(G.shape[0], -1)


CASES = [(1, 1, (4,)), (1, 4, (3,)), (1, 8, (2,)), (2, 2, (3, 2)), (2, 5, (2, 3)),
         (3, 1, (2, 3, 2)), (3, 3, (2, 2, 3)), (3, 4, (1, 2, 2))]


def test_golden_two_element_advection(oracle):
    rows = np.loadtxt(os.path.join(GOLDEN, "adv1d_N1_K2_rhs.txt"))
    u = np.array([1.0, 2.0, 3.0, 4.0])
    for row in rows:
        a, ref = row[0], row[1:]
        for form in ("weak", "strong"):
            R = oracle.rhs(1, 1, [2], ADV, [a], u, form=form)[0]
            np.testing.assert_allclose(R, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,N,K", CASES)
@pytest.mark.parametrize("eq", [ADV, EUL])
def test_conservation(oracle, dim, N, K, eq):
    U = _state(dim, N, K, eq, 100 + N)
    R = oracle.rhs(dim, N, K, eq, _par(dim, eq), U)
    W = _weights(oracle, dim, N, K)
    for v in range(U.shape[0]):
        total = np.dot(W, R[v])
        scale = np.dot(W, np.abs(R[v]))
        assert abs(total) <= 1e-14 * scale, (v, total, scale)


@pytest.mark.parametrize("dim,N,K", CASES)
def test_advection_energy_identity(oracle, dim, N, K):
    """sum M U R = -1/2 sum_d |a_d| sum_{faces perp d} (face weight) [U]^2."""
    par = _par(dim, ADV)
    U = _state(dim, N, K, ADV, 7 + N)
    R = oracle.rhs(dim, N, K, ADV, par, U)
    W = _weights(oracle, dim, N, K)
    lhs = np.dot(W, U[0] * R[0])
    _, w = oracle.lgl(N)
    G = _grid(U, dim, N, K)[0]                  # (Kz, Ky, Kx, n1z, n1y, n1x)
    Kl = list(K) + [1] * (3 - dim)
    rhs = 0.0
    for d in range(dim):
        eax, nax = 2 - d, 5 - d                  # element / node axis of direction d
        upper = np.take(G, [N], axis=nax)        # this element's upper trace
        lower_next = np.take(np.roll(G, -1, axis=eax), [0], axis=nax)
        jump2 = (lower_next - upper) ** 2
        wts = np.ones(jump2.shape)
        for d2 in range(dim):
            if d2 == d:
                continue
            s = [1] * 6
            s[5 - d2] = N + 1
            wts = wts * (w * 0.5 / Kl[d2]).reshape(s)
        rhs += -0.5 * abs(par[d]) * float((wts * jump2).sum())
    assert abs(lhs - rhs) <= 1e-13 * max(abs(rhs), 1e-300), (lhs, rhs)


@pytest.mark.parametrize("dim,N,K", CASES)
def test_free_stream(oracle, dim, N, K):
    n = int(np.prod(K)) * (N + 1) ** dim
    for eq, vals in ((ADV, [0.73]), (EUL, [1.3, 0.2, -0.15, 0.05][:dim + 1])):
        U = np.repeat(np.array(vals)[:, None], n, axis=1)
        R = oracle.rhs(dim, N, K, eq, _par(dim, eq), U)
        # natural size of one volume or lift term: (2/dx) (1/w_0) max|F|
        fmax = max(abs(vals[0]), 1.0) * (1.0 + 1.2 ** 2)
        scale = 2.0 * max(K) * N * (N + 1) / 2.0 * fmax
        assert np.abs(R).max() <= 2e-15 * scale, (eq, np.abs(R).max(), scale)


@pytest.mark.parametrize("dim,N,K", CASES)
@pytest.mark.parametrize("eq", [ADV, EUL])
def test_weak_equals_strong(oracle, dim, N, K, eq):
    U = _state(dim, N, K, eq, 300 + N)
    Rw = oracle.rhs(dim, N, K, eq, _par(dim, eq), U, form="weak")
    Rs = oracle.rhs(dim, N, K, eq, _par(dim, eq), U, form="strong")
    assert np.abs(Rw - Rs).max() <= 1e-13 * np.abs(Rw).max()


@pytest.mark.parametrize("dim,N,K", [(1, 3, (5,)), (2, 2, (3, 4)), (3, 2, (2, 3, 4))])
@pytest.mark.parametrize("eq", [ADV, EUL])
def test_periodic_shift(oracle, dim, N, K, eq):
    U = _state(dim, N, K, eq, 55)
    R = oracle.rhs(dim, N, K, eq, _par(dim, eq), U)
    for d in range(dim):
        ax = 3 - d                                # element axis of direction d in _grid
        Us = _flat(np.roll(_grid(U, dim, N, K), 1, axis=ax))
        Rs = oracle.rhs(dim, N, K, eq, _par(dim, eq), Us)
        np.testing.assert_array_equal(Rs, _flat(np.roll(_grid(R, dim, N, K), 1, axis=ax)))


@pytest.mark.parametrize("eq", [ADV, EUL])
def test_axis_permutation_2d(oracle, eq):
    N, K = 3, (3, 5)
    U = _state(2, N, K, eq, 77)
    par = [0.6, -0.9] if eq == ADV else [1.1]
    R = oracle.rhs(2, N, K, eq, par, U)
    G = _grid(U, 2, N, K)                         # (v, 1, Ky, Kx, 1, n1y, n1x)
    Gt = G.transpose(0, 1, 3, 2, 4, 6, 5)
    if eq == EUL:
        Gt = Gt[[0, 2, 1]]
    part = [par[1], par[0]] if eq == ADV else par
    Rt = oracle.rhs(2, N, (K[1], K[0]), eq, part, _flat(np.ascontiguousarray(Gt)))
    H = _grid(R, 2, N, K).transpose(0, 1, 3, 2, 4, 6, 5)
    if eq == EUL:
        H = H[[0, 2, 1]]
    np.testing.assert_allclose(Rt, _flat(np.ascontiguousarray(H)), rtol=0,
                               atol=1e-14 * np.abs(R).max())


def test_axis_permutation_3d_euler(oracle):
    N, K = 2, (2, 3, 4)
    U = _state(3, N, K, EUL, 88)
    R = oracle.rhs(3, N, K, EUL, [1.0], U)
    # cyclic relabel: new x = old y, new y = old z, new z = old x
    G = _grid(U, 3, N, K)                         # (v, Kz, Ky, Kx, n1z, n1y, n1x)
    Gp = G.transpose(0, 3, 1, 2, 6, 4, 5)[[0, 2, 3, 1]]
    Rp = oracle.rhs(3, N, (K[1], K[2], K[0]), EUL, [1.0], _flat(np.ascontiguousarray(Gp)))
    H = _grid(R, 3, N, K).transpose(0, 3, 1, 2, 6, 4, 5)[[0, 2, 3, 1]]
    np.testing.assert_allclose(Rp, _flat(np.ascontiguousarray(H)), rtol=0,
                               atol=1e-14 * np.abs(R).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_advection_reduces_to_1d(oracle, dim):
    N, Kx = 4, 5
    K = (Kx,) + (2,) * (dim - 1)
    u1 = _rand(3, Kx * (N + 1))
    R1 = oracle.rhs(1, N, [Kx], ADV, [0.9], u1)[0]
    G = np.zeros(_grid(np.zeros((1, int(np.prod(K)) * (N + 1) ** dim)), dim, N, K).shape)
    G[...] = u1.reshape(Kx, N + 1)[None, None, None, :, None, None, :].reshape(
        1, 1, 1, Kx, 1, 1, N + 1)
    U = _flat(G)
    R = oracle.rhs(dim, N, K, ADV, [0.9] + [0.0] * (dim - 1), U)
    Rg = _grid(R, dim, N, K)[0]
    for idx in np.ndindex(Rg.shape[0], Rg.shape[1], Rg.shape[3], Rg.shape[4]):
        z, y, k, j = idx
        np.testing.assert_allclose(Rg[z, y, :, k, j, :].reshape(-1), R1, rtol=0,
                                   atol=1e-14 * np.abs(R1).max())


def test_euler_2d_reduces_to_1d(oracle):
    N, Kx, Ky = 3, 4, 2
    n1 = N + 1
    rho = _rand(4, Kx * n1, 0.7, 1.3)
    m = rho * _rand(5, Kx * n1, -0.3, 0.3)
    R1 = oracle.rhs(1, N, [Kx], EUL, [1.0], np.array([rho, m]))
    G = np.zeros((3, 1, Ky, Kx, 1, n1, n1))
    G[0] = rho.reshape(Kx, n1)[None, None, :, None, None, :]
    G[1] = m.reshape(Kx, n1)[None, None, :, None, None, :]
    R = _grid(oracle.rhs(2, N, (Kx, Ky), EUL, [1.0], _flat(G)), 2, N, (Kx, Ky))
    scale = np.abs(R1).max()
    for ey in range(Ky):
        for j in range(n1):
            for v in range(2):
                np.testing.assert_allclose(R[v, 0, ey, :, 0, j, :].reshape(-1), R1[v], rtol=0,
                                           atol=2e-14 * scale)
            assert np.abs(R[2, 0, ey, :, 0, j, :]).max() <= 2e-14 * scale


def test_advection_linearity(oracle):
    dim, N, K = 2, 3, (3, 2)
    par = _par(dim, ADV)
    U, V = _state(dim, N, K, ADV, 1), _state(dim, N, K, ADV, 2)
    RU, RV = oracle.rhs(dim, N, K, ADV, par, U), oracle.rhs(dim, N, K, ADV, par, V)
    R = oracle.rhs(dim, N, K, ADV, par, 0.3 * U - 1.7 * V)
    np.testing.assert_allclose(R, 0.3 * RU - 1.7 * RV, rtol=0, atol=1e-13 * np.abs(R).max())


@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_consistency_rate(oracle, N):
    """R(interpolant of sin 2 pi x) -> -a d/dx sin(2 pi x), pointwise error O(dx^N)."""
    a = 1.0
    errs = []
    Ks = [8, 16]
    for K in Ks:
        x = oracle.axis_coords(N, K).reshape(-1)
        R = oracle.rhs(1, N, [K], ADV, [a], np.sin(2 * np.pi * x))[0]
        errs.append(np.abs(R + a * 2 * np.pi * np.cos(2 * np.pi * x)).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate >= N - 0.3, (N, errs, rate)
