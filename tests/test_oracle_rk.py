"""Pins for the oracle's Runge-Kutta schemes (Sec. 2.3, eqs. RK3, RK4, RK6).

* Order conditions: for every rooted tree t with |t| <= p, b . Phi(t) = 1/gamma(t)
  (Butcher's elementary weights), generated here from the trees themselves;
  RK3 (Heun reading) p = 3, RK4 p = 4, RK6 p = 6 (37 trees), and RK6 must fail
  at order 7.
* Observed order of the oracle's stepping routine on the logistic equation
  y' = y(1-y) against its closed form 1/(1 + 9 e^{-t}).
* On a linear PDE one step must equal the scheme's stability polynomial
  1 + sum_m z^m b^T A^{m-1} 1 applied to the assembled operator, and its
  first p+1 coefficients are 1/m!.
"""
import math

import numpy as np
import pytest

ORDER = {3: 3, 4: 4, 6: 6}


def _canon(t):
    return tuple(sorted(_canon(c) for c in t))


def _grow(t):
    out = [_canon(t + ((),))]
    for i, c in enumerate(t):
        for g in _grow(c):
            out.append(_canon(t[:i] + (g,) + t[i + 1:]))
    return out


def trees(order):
    """All rooted trees with `order` vertices (a tree = sorted tuple of child trees)."""
    level = {()}
    for _ in range(order - 1):
        level = {g for t in level for g in _grow(t)}
    return sorted(level)


def _size(t):
    return 1 + sum(_size(c) for c in t)


def _gamma(t):
    return _size(t) * math.prod(_gamma(c) for c in t)


def _phi(t, A):
    v = np.ones(A.shape[0])
    for c in t:
        v = v * (A @ _phi(c, A))
    return v


def test_tree_counts():
    assert [len(trees(n)) for n in range(1, 8)] == [1, 1, 2, 4, 9, 20, 48]


@pytest.mark.parametrize("rk", [3, 4, 6])
def test_order_conditions(oracle, rk):
    S, A, b = oracle.rk_tableau(rk)
    assert S == {3: 3, 4: 4, 6: 7}[rk]
    assert np.all(np.triu(A) == 0)                       # explicit
    p = ORDER[rk]
    for n in range(1, p + 1):
        for t in trees(n):
            assert abs(b @ _phi(t, A) - 1.0 / _gamma(t)) <= 2e-14, (rk, t)
    worst = max(abs(b @ _phi(t, A) - 1.0 / _gamma(t)) for t in trees(p + 1))
    assert worst > 1e-6, (rk, worst)                      # exactly order p


@pytest.mark.parametrize("rk", [3, 4, 6])
def test_observed_order_logistic(oracle, rk):
    T, y0 = 2.0, 0.1
    exact = 1.0 / (1.0 + 9.0 * math.exp(-T))
    steps = {3: [8, 16, 32], 4: [8, 16, 32], 6: [4, 8, 16]}[rk]
    errs = [abs(oracle.ode_solve(rk, "logistic", y0, T / n, n) - exact) for n in steps]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(rates[-1] - ORDER[rk]) <= 0.25, (rk, errs, rates)


@pytest.mark.parametrize("rk", [3, 4, 6])
def test_linear_ode_stability_function(oracle, rk):
    S, A, b = oracle.rk_tableau(rk)
    for z in (-0.7, 0.3, -2.0):
        coeff = [1.0] + [b @ np.linalg.matrix_power(A, m - 1) @ np.ones(S) for m in range(1, S + 1)]
        Rz = sum(c * z ** m for m, c in enumerate(coeff))
        y = oracle.ode_solve(rk, "linear", 1.0, 1.0, 1, lam=z)
        assert abs(y - Rz) <= 1e-14 * max(1.0, abs(Rz))
        for m in range(ORDER[rk] + 1):
            assert abs(coeff[m] - 1.0 / math.factorial(m)) <= 1e-15
    if rk == 6:
        # the z^7 term of Luther's scheme: b^T A^6 1 = -1/2160 (exact arithmetic)
        assert abs(coeff[7] + 1.0 / 2160.0) <= 1e-16


@pytest.mark.parametrize("rk", [3, 4, 6])
def test_pde_step_is_stability_polynomial(oracle, rk):
    """One RK step of linear advection equals P(dt L) U with L assembled column by column."""
    dim, N, K, a = 1, 2, [3], [1.0]
    n = K[0] * (N + 1)
    L = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        L[:, j] = oracle.rhs(dim, N, K, 0, a, e)[0]
    S, A, b = oracle.rk_tableau(rk)
    dt = 0.05
    U = np.sin(2 * np.pi * oracle.axis_coords(N, K[0]).reshape(-1)) + 0.3
    P = np.eye(n)
    Z = dt * L
    Zm = np.eye(n)
    for m in range(1, S + 1):
        Zm = Zm @ Z
        P = P + (b @ np.linalg.matrix_power(A, m - 1) @ np.ones(S)) * Zm
    U1 = oracle.step(dim, N, K, 0, a, U, rk, dt, 1)[0]
    np.testing.assert_allclose(U1, P @ U, rtol=0, atol=1e-13)
