"""CPU FP64 oracle for the nodal discontinuous Galerkin (NDG) Runge-Kutta path.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers. The oracle is plain C in
``dg_oracle.c`` (double precision, no FMA contraction, OpenMP over elements
only) loaded through ctypes. It shares no code with the GPU library and never
imports it.

What each function follows (Sporykhin & Homann, arXiv:2510.05254):

=================  ============================================  ==============================
function           passage                                       pinned by
=================  ============================================  ==============================
lgl                Sec. 2.1 node definition (1-x^2)P_N'=0,       closed forms N<=4, mpmath
                   eq. lag_coefs weights                         50-digit brute force N<=8,
                                                                 exactness to degree 2N-1
dmat               Sec. 2.1 dh_l/dx of eq. lagrange_pol          exact on degree<=N, SBP
axis_coords        Sec. 2.1 partition + eq. transformation       closed form
flux / numflux     eqs. advection2d, eulerIso2d, LF              Jacobian eigenvalues,
                                                                 consistency, upwind reduction
rhs (weak/strong)  Sec. 2.1 evolution equation, tensor product   conservation, energy identity,
                                                                 free stream, weak=strong,
                                                                 shift/permutation/reduction
step               Sec. 2.3 eqs. RK3 (Heun reading), RK4, RK6    order conditions, ODE orders,
                                                                 stability polynomial, exact
                                                                 advection convergence N+1
l2 / mass          Sec. 3.1 L2 norm, LGL quadrature              polynomial integrals
=================  ============================================  ==============================
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.path.join(_HERE, "libdg_oracle.so")

ADVECTION = 0
EULER = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile dg_oracle.c into libdg_oracle.so with gcc (FP64, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    d, i32, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
    vp = ctypes.c_void_p
    lib.or_lgl.argtypes = [i32, vp, vp]
    lib.or_dmat.argtypes = [i32, vp, vp]
    lib.or_axis_coords.argtypes = [i32, i64, vp]
    lib.or_flux.argtypes = [i32, i32, i32, vp, vp, vp]
    lib.or_numflux.argtypes = [i32, i32, i32, vp, vp, vp, vp]
    lib.or_max_speed.argtypes = [i32, i32, i32, vp, vp]
    lib.or_max_speed.restype = d
    lib.or_rhs.argtypes = [i32, i32, vp, i32, vp, i32, vp, vp]
    lib.or_step.argtypes = [i32, i32, vp, i32, vp, i32, d, i64, vp]
    lib.or_rk_tableau.argtypes = [i32, P(i32), vp, vp]
    lib.or_ode_solve.argtypes = [i32, i32, d, d, d, i64, P(d)]
    lib.or_l2.argtypes = [i32, i32, vp, i32, vp, vp, vp, vp]
    lib.or_mass.argtypes = [i32, i32, vp, i32, vp, vp]
    lib.or_set_threads.argtypes = [i32]
    lib.or_get_threads.restype = i32
    for name in ("or_lgl", "or_dmat", "or_axis_coords", "or_flux", "or_numflux", "or_rhs",
                 "or_step", "or_rk_tableau", "or_ode_solve", "or_l2", "or_mass"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed (rc={rc})")


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _K(dim, K):
    K = np.atleast_1d(np.asarray(K, dtype=np.int64))
    if K.size == 1 and dim > 1:
        K = np.repeat(K, dim)
    if K.size != dim:
        raise ValueError("K must have dim entries")
    return np.ascontiguousarray(K)


def nvar(dim: int, eq: int) -> int:
    return 1 if eq == ADVECTION else 1 + dim


def n_nodes(dim: int, N: int, K) -> int:
    return int(np.prod(_K(dim, K))) * (N + 1) ** dim


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def lgl(N: int):
    """LGL nodes xi (ascending) and weights w, N+1 each."""
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    _check(_load().or_lgl(N, _ptr(xi), _ptr(w)), "lgl")
    return xi, w


def dmat(N: int, xi=None):
    """D[i, l] = h_l'(xi_i) (Lagrange derivative at the nodes)."""
    if xi is None:
        xi, _ = lgl(N)
    xi = _f64(xi, N + 1)
    D = np.zeros((N + 1, N + 1))
    _check(_load().or_dmat(N, _ptr(xi), _ptr(D)), "dmat")
    return D


def axis_coords(N: int, K: int):
    """1-D node coordinates along one axis, shape (K, N+1)."""
    x = np.zeros((int(K), N + 1))
    _check(_load().or_axis_coords(N, int(K), _ptr(x)), "axis_coords")
    return x


def _par(dim, eq, params):
    p = np.zeros(3)
    params = np.atleast_1d(np.asarray(params, dtype=np.float64))
    if eq == ADVECTION:
        p[:dim] = params[:dim]
    else:
        p[0] = params[0]
    return p


def flux(dim, d, eq, params, U):
    U = _f64(U, nvar(dim, eq))
    F = np.zeros(nvar(dim, eq))
    _check(_load().or_flux(dim, d, eq, _ptr(_par(dim, eq, params)), _ptr(U), _ptr(F)), "flux")
    return F


def numflux(dim, d, eq, params, UL, UR):
    nv = nvar(dim, eq)
    UL, UR = _f64(UL, nv), _f64(UR, nv)
    F = np.zeros(nv)
    _check(_load().or_numflux(dim, d, eq, _ptr(_par(dim, eq, params)), _ptr(UL), _ptr(UR),
                              _ptr(F)), "numflux")
    return F


def max_speed(dim, d, eq, params, U):
    U = _f64(U, nvar(dim, eq))
    return float(_load().or_max_speed(dim, d, eq, _ptr(_par(dim, eq, params)), _ptr(U)))


def rhs(dim, N, K, eq, params, U, form: str = "weak"):
    """dU/dt of the NDG system; U in the canonical layout (nvar, E*(N+1)^dim)."""
    K = _K(dim, K)
    n = nvar(dim, eq) * n_nodes(dim, N, K)
    U = _f64(U, n)
    R = np.zeros(n)
    f = {"weak": 0, "strong": 1}[form]
    _check(_load().or_rhs(dim, N, _ptr(K), eq, _ptr(_par(dim, eq, params)), f, _ptr(U), _ptr(R)),
           "rhs")
    return R.reshape(nvar(dim, eq), -1)


def step(dim, N, K, eq, params, U, rk: int, dt: float, nsteps: int):
    """nsteps Runge-Kutta steps (rk in 3, 4, 6); returns a new array."""
    K = _K(dim, K)
    n = nvar(dim, eq) * n_nodes(dim, N, K)
    V = _f64(U, n).copy()
    _check(_load().or_step(dim, N, _ptr(K), eq, _ptr(_par(dim, eq, params)), int(rk), float(dt),
                           int(nsteps), _ptr(V)), "step")
    return V.reshape(nvar(dim, eq), -1)


def rk_tableau(rk: int):
    """(stages, A 7x7, b 7) Butcher coefficients of the scheme."""
    s = ctypes.c_int(0)
    A = np.zeros((7, 7))
    b = np.zeros(7)
    _check(_load().or_rk_tableau(int(rk), ctypes.byref(s), _ptr(A), _ptr(b)), "rk_tableau")
    S = s.value
    return S, A[:S, :S].copy(), b[:S].copy()


def ode_solve(rk: int, kind: str, y0: float, dt: float, nsteps: int, lam: float = 0.0) -> float:
    """Scalar ODE stepped by the oracle's RK routine: 'linear' y'=lam y, 'logistic' y'=y(1-y)."""
    out = ctypes.c_double(0.0)
    k = {"linear": 0, "logistic": 1}[kind]
    _check(_load().or_ode_solve(int(rk), k, float(lam), float(y0), float(dt), int(nsteps),
                                ctypes.byref(out)), "ode_solve")
    return out.value


def l2(dim, N, K, eq, U, Uref):
    """Per-variable integrals of (U-Uref)^2 and Uref^2 (nodal LGL quadrature)."""
    K = _K(dim, K)
    nv = nvar(dim, eq)
    n = nv * n_nodes(dim, N, K)
    U, Uref = _f64(U, n), _f64(Uref, n)
    se, sr = np.zeros(nv), np.zeros(nv)
    _check(_load().or_l2(dim, N, _ptr(K), eq, _ptr(U), _ptr(Uref), _ptr(se), _ptr(sr)), "l2")
    return se, sr


def l2_error(dim, N, K, eq, U, Uref):
    """(absolute, relative) L2 error over all variables."""
    se, sr = l2(dim, N, K, eq, U, Uref)
    a = float(np.sqrt(se.sum()))
    return a, a / float(np.sqrt(sr.sum()))


def mass(dim, N, K, eq, U):
    K = _K(dim, K)
    nv = nvar(dim, eq)
    U = _f64(U, nv * n_nodes(dim, N, K))
    m = np.zeros(nv)
    _check(_load().or_mass(dim, N, _ptr(K), eq, _ptr(U), _ptr(m)), "mass")
    return m
