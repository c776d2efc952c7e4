"""Pins for the oracle's LGL nodes, weights and differentiation matrix.

The paper defines the nodes as the solutions of (1 - xi^2) P_N'(xi) = 0 and uses
the Lagrange cardinal polynomials on them (Sec. 2.1, eqs. lagrange_pol and
ortho_at_roots) with the matching quadrature (eq. lag_coefs). The pins below
do not use the oracle's formulas: closed forms for small N, a 50-digit mpmath
brute force (polynomial roots, exact integrals and derivatives of the
Lagrange polynomials), polynomial exactness of the rule, and the
summation-by-parts identity.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

NS = list(range(1, 9))


def _legendre_coeffs(n):
    """Exact monomial coefficients (ascending) of P_n via Bonnet's recurrence."""
    p0, p1 = [Fraction(1)], [Fraction(0), Fraction(1)]
    if n == 0:
        return p0
    for k in range(1, n):
        nxt = [Fraction(0)] * (k + 2)
        for i, c in enumerate(p1):
            nxt[i + 1] += Fraction(2 * k + 1, k + 1) * c
        for i, c in enumerate(p0):
            nxt[i] -= Fraction(k, k + 1) * c
        p0, p1 = p1, nxt
    return p1


def _mp_lgl(N, dps=50):
    """Nodes and weights at dps digits: roots of P_N', weights = integral of h_k."""
    with mpmath.workdps(dps):
        P = _legendre_coeffs(N)
        dP = [i * c for i, c in enumerate(P)][1:]
        roots = mpmath.polyroots([mpmath.mpf(c.numerator) / c.denominator for c in reversed(dP)],
                                 maxsteps=200, extraprec=200) if N > 1 else []
        nodes = sorted([mpmath.mpf(-1)] + [mpmath.re(r) for r in roots] + [mpmath.mpf(1)])
        weights = []
        for k in range(N + 1):
            poly = [mpmath.mpf(1)]
            for m in range(N + 1):
                if m == k:
                    continue
                den = nodes[k] - nodes[m]
                new = [mpmath.mpf(0)] * (len(poly) + 1)
                for i, c in enumerate(poly):
                    new[i + 1] += c / den
                    new[i] -= c * nodes[m] / den
                poly = new
            weights.append(sum(c * (1 - (-1) ** (i + 1)) / (i + 1) for i, c in enumerate(poly)))
        return nodes, weights


def _mp_dmat(N, nodes, dps=50):
    """D[i, l] = h_l'(xi_i) by differentiating the product form at dps digits."""
    with mpmath.workdps(dps):
        D = [[mpmath.mpf(0)] * (N + 1) for _ in range(N + 1)]
        for l in range(N + 1):
            others = [m for m in range(N + 1) if m != l]
            den = mpmath.fprod(nodes[l] - nodes[m] for m in others)
            for i in range(N + 1):
                s = mpmath.mpf(0)
                for skip in others:
                    s += mpmath.fprod(nodes[i] - nodes[m] for m in others if m != skip)
                D[i][l] = s / den
        return D


@pytest.mark.parametrize("N,xi_ref,w_ref", [
    (1, [-1, 1], [1, 1]),
    (2, [-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_lgl_closed_forms(oracle, N, xi_ref, w_ref):
    xi, w = oracle.lgl(N)
    np.testing.assert_allclose(xi, xi_ref, rtol=0, atol=4.5e-16)
    np.testing.assert_allclose(w, w_ref, rtol=4.5e-16, atol=0)


@pytest.mark.parametrize("N", NS)
def test_lgl_mpmath_brute_force(oracle, N):
    xi, w = oracle.lgl(N)
    nodes, weights = _mp_lgl(N)
    ulp = np.finfo(np.float64).eps
    for a, b in zip(xi, nodes):
        assert abs(a - float(b)) <= 2 * ulp, (N, a, b)
    for a, b in zip(w, weights):
        assert abs(a - float(b)) <= 4 * ulp * abs(float(b)), (N, a, b)


@pytest.mark.parametrize("N", NS)
def test_lgl_symmetry_and_sum(oracle, N):
    xi, w = oracle.lgl(N)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    assert np.all(np.diff(xi) > 0)
    np.testing.assert_array_equal(xi, -xi[::-1])
    np.testing.assert_allclose(w, w[::-1], rtol=2e-16)
    assert abs(w.sum() - 2.0) <= 1e-15
    # end weights 2/(N(N+1)) (P_N(+-1) = +-1)
    assert abs(w[0] - 2.0 / (N * (N + 1))) <= 2e-16


@pytest.mark.parametrize("N", NS)
def test_quadrature_exact_to_degree_2N_minus_1(oracle, N):
    xi, w = oracle.lgl(N)
    for m in range(0, 2 * N):
        exact = (1 - (-1) ** (m + 1)) / (m + 1)
        assert abs(np.dot(w, xi ** m) - exact) <= 4.5e-16, (N, m)
    # the (N+1)-point Lobatto rule is not exact for degree 2N
    m = 2 * N
    err = np.dot(w, xi ** m) - 2.0 / (m + 1)
    assert abs(err) > 1e-6
    if N == 3:
        assert abs(err - 0.0609523809523809) < 1e-12   # 2(1/6 + (5/6)/125) - 2/7
    if N == 4:
        assert abs(err - 0.0145124716553288) < 1e-12   # 2(1/10 + (49/90)(3/7)^4) - 2/9


@pytest.mark.parametrize("N", NS)
def test_dmat_mpmath_brute_force(oracle, N):
    xi, _ = oracle.lgl(N)
    D = oracle.dmat(N)
    nodes, _ = _mp_lgl(N)
    Dm = _mp_dmat(N, nodes)
    scale = max(abs(float(x)) for row in Dm for x in row)
    for i in range(N + 1):
        for l in range(N + 1):
            assert abs(D[i, l] - float(Dm[i][l])) <= 2e-15 * scale, (N, i, l)


@pytest.mark.parametrize("N", NS)
def test_dmat_exact_on_polynomials(oracle, N):
    xi, _ = oracle.lgl(N)
    D = oracle.dmat(N)
    scale = np.abs(D).max()
    for m in range(0, N + 1):
        exact = m * xi ** (m - 1) if m > 0 else np.zeros_like(xi)
        assert np.abs(D @ xi ** m - exact).max() <= 1e-13 * scale, (N, m)
    # row sums vanish (derivative of a constant), corner entries -+N(N+1)/4
    assert np.abs(D.sum(axis=1)).max() <= 1e-14 * scale
    assert abs(D[0, 0] + N * (N + 1) / 4) <= 1e-14 * scale
    assert abs(D[N, N] - N * (N + 1) / 4) <= 1e-14 * scale


@pytest.mark.parametrize("N", NS)
def test_summation_by_parts(oracle, N):
    """W D + D^T W = diag(-1, 0, ..., 0, 1) for the LGL rule (exact for degree 2N-1)."""
    xi, w = oracle.lgl(N)
    D = oracle.dmat(N)
    Q = np.diag(w) @ D
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.abs(Q + Q.T - B).max() <= 5e-15


@pytest.mark.parametrize("K,N", [(1, 1), (3, 4), (5, 8)])
def test_axis_coords(oracle, K, N):
    x = oracle.axis_coords(N, K)
    xi, _ = oracle.lgl(N)
    dx = 1.0 / K
    assert x.shape == (K, N + 1)
    for e in range(K):
        np.testing.assert_allclose(x[e, 0], e * dx, atol=1e-16)
        np.testing.assert_allclose(x[e, -1], (e + 1) * dx, atol=2e-16)
        np.testing.assert_allclose(x[e], e * dx + dx * (xi + 1) / 2, atol=2e-16)
