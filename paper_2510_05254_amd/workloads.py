"""Seeded synthetic inputs for the NDG Runge-Kutta path.

This module holds no part of the method's arithmetic: it draws random numbers
(SplitMix64), evaluates Fourier-mode initial fields at node coordinates handed
to it, and applies the time-step rule of the benchmark configurations. The
same arrays feed the GPU library and the CPU oracle; node coordinates come from
whichever side asks (the library's ``dg_get_axis_coords`` or the oracle's
``axis_coords``).

Workloads follow the paper's synthetic random-Fourier initial conditions
(Sec. 3.1, eq. initialCond: U_0 = sum_k A_k sin(2 pi k x), A_k in [0, 1]) at the
shapes of the benchmark configurations:

====  ===================================================================
id    workload
====  ===================================================================
1     1-D advection, a = 1, K = 64, N = 3, U_0 = sin(2 pi x), RK4,
      dt = 0.1 dx_min, to t = 1
2     2-D advection, a = (1, 0.5), 256 x 256, N = 7, 8 random Fourier modes,
      RK4, 100 steps
3     2-D isothermal Euler, c_s = 1, 512 x 512, N = 3, rho = 1 + 1e-2 noise
      (16 modes), velocity from a 16-mode stream function at Mach 0.1, RK4,
      200 steps
4     3-D isothermal Euler, c_s = 1, 64^3, N = 4, rho = 1, solenoidal velocity
      from 32 modes at Mach 0.1, RK4, 50 steps
====  ===================================================================

Layout of a state array: (nvar, E * (N+1)^dim) float64, element index
e = ex + Kx (ey + Ky ez) and node index n = i + (N+1)(j + (N+1) k).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ADVECTION = 0
EULER = 1
SEED_BASE = 20251005
_M64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), exact 64-bit arithmetic."""

    def __init__(self, seed: int):
        self.state = int(seed) & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniforms(self, n: int) -> np.ndarray:
        return np.array([self.uniform() for _ in range(n)])

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform in [lo, hi] (inclusive)."""
        return lo + min(int(self.uniform() * (hi - lo + 1)), hi - lo)


@dataclass
class Workload:
    """One synthetic solve: mesh, equation, initial-condition recipe and stepping."""
    name: str
    dim: int
    N: int
    K: tuple
    eq: int
    params: tuple            # advection: a[dim]; Euler: (c_s,)
    ic: str                  # sine1d | fourier_adv | fourier1d | euler2d | euler3d | constant
    seed: int
    rk: int = 4
    steps: int | None = None
    t_final: float | None = None
    cfl: float = 0.1
    ic_args: dict = field(default_factory=dict)

    @property
    def nvar(self) -> int:
        return 1 if self.eq == ADVECTION else 1 + self.dim

    @property
    def elements(self) -> int:
        return int(np.prod(self.K))

    @property
    def nodes(self) -> int:
        return self.elements * (self.N + 1) ** self.dim

    @property
    def unknowns(self) -> int:
        return self.nodes * self.nvar


def config(cid: int) -> Workload:
    """The benchmark configurations 1-4 (see the module docstring)."""
    if cid == 1:
        return Workload("adv1d_K64_N3", 1, 3, (64,), ADVECTION, (1.0,), "sine1d",
                        SEED_BASE + 1, rk=4, t_final=1.0)
    if cid == 2:
        return Workload("adv2d_256x256_N7", 2, 7, (256, 256), ADVECTION, (1.0, 0.5),
                        "fourier_adv", SEED_BASE + 2, rk=4, steps=100,
                        ic_args={"modes": 8, "kmax": 8})
    if cid == 3:
        return Workload("euler2d_512x512_N3", 2, 3, (512, 512), EULER, (1.0,), "euler2d",
                        SEED_BASE + 3, rk=4, steps=200,
                        ic_args={"modes": 16, "kmax": 4, "noise": 1e-2, "mach": 0.1})
    if cid == 4:
        return Workload("euler3d_64x64x64_N4", 3, 4, (64, 64, 64), EULER, (1.0,), "euler3d",
                        SEED_BASE + 4, rk=4, steps=50,
                        ic_args={"modes": 32, "kmax": 4, "mach": 0.1})
    raise ValueError(f"unknown configuration {cid}")


def scaled(w: Workload, K) -> Workload:
    """The same recipe on a different element grid (for small parity cases)."""
    K = tuple(int(k) for k in (K if np.ndim(K) else [K] * w.dim))
    return Workload(w.name + "_K" + "x".join(map(str, K)), w.dim, w.N, K, w.eq, w.params,
                    w.ic, w.seed, w.rk, w.steps, w.t_final, w.cfl, dict(w.ic_args))


# ---------------------------------------------------------------------------
# Field evaluation on the tensor grid of 1-D axis coordinates
# ---------------------------------------------------------------------------

def _to_canonical(F: np.ndarray, dim: int, K, n1: int) -> np.ndarray:
    """(L_z, L_y, L_x) grid values with L_d = K_d (N+1) -> canonical (E*Np,) order."""
    if dim == 1:
        return F.reshape(-1)
    if dim == 2:
        Ky, Kx = K[1], K[0]
        G = F.reshape(Ky, n1, Kx, n1).transpose(0, 2, 1, 3)
        return np.ascontiguousarray(G).reshape(-1)
    Kz, Ky, Kx = K[2], K[1], K[0]
    G = F.reshape(Kz, n1, Ky, n1, Kx, n1).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(G).reshape(-1)


def fourier_sum(axes, kvec, phase, coef) -> np.ndarray:
    """sum_m coef[m, c] sin(2 pi k_m . x + 2 pi phase_m) for each component c.

    axes: list of per-axis coordinate arrays of shape (K_d, N+1), x first.
    kvec: (M, dim) integer wave vectors; phase: (M,); coef: (M, ncomp).
    Returns (ncomp, E*Np) in canonical layout. Separable evaluation: each mode
    is a product of per-axis complex exponentials, summed by a matrix product.
    """
    dim = len(axes)
    K = [a.shape[0] for a in axes]
    n1 = axes[0].shape[1]
    kvec = np.asarray(kvec, dtype=np.float64).reshape(-1, dim)
    coef = np.asarray(coef, dtype=np.float64)
    if coef.ndim == 1:
        coef = coef[:, None]
    M, nc = coef.shape
    amp = coef * np.exp(2j * np.pi * np.asarray(phase))[:, None]         # (M, nc)
    E = [np.exp(2j * np.pi * kvec[:, d][:, None] * axes[d].reshape(1, -1)) for d in range(dim)]
    out = np.empty((nc, int(np.prod(K)) * n1 ** dim))
    for c in range(nc):
        if dim == 1:
            F = (amp[:, c] @ E[0]).imag
        elif dim == 2:
            F = ((amp[:, c][:, None] * E[1]).T @ E[0]).imag
        else:
            T = (amp[:, c][:, None, None] * E[2][:, :, None] * E[1][:, None, :])
            F = (T.reshape(M, -1).T @ E[0]).imag
        out[c] = _to_canonical(F, dim, K, n1)
    return out


def _draw_k(rng: SplitMix64, dim: int, kmax: int):
    while True:
        k = [rng.randint(-kmax, kmax) for _ in range(dim)]
        if any(k):
            return k


def initial_state(w: Workload, axes) -> np.ndarray:
    """Seeded initial state (nvar, E*Np) at the given per-axis coordinates."""
    dim = w.dim
    axes = [np.asarray(a, dtype=np.float64).reshape(w.K[d], w.N + 1) for d, a in enumerate(axes)]
    rng = SplitMix64(w.seed)
    a = w.ic_args
    if w.ic == "sine1d":
        return fourier_sum(axes, [[1] + [0] * (dim - 1)], [0.0], [1.0])
    if w.ic == "constant":
        vals = np.asarray(a["values"], dtype=np.float64)
        return np.repeat(vals[:, None], w.nodes, axis=1)
    if w.ic == "fourier1d":
        # eq. initialCond: sum_{k=1}^{Nk} A_k sin(2 pi k x), A_k ~ U[0, 1); x-only in >1-D
        nk = int(a.get("nk", 40))
        A = rng.uniforms(nk)
        kv = [[k] + [0] * (dim - 1) for k in range(1, nk + 1)]
        return fourier_sum(axes, kv, np.zeros(nk), A)
    if w.ic == "fourier_adv":
        M, kmax = int(a["modes"]), int(a["kmax"])
        kv, ph, A = [], [], []
        for _ in range(M):
            kv.append(_draw_k(rng, dim, kmax))
            A.append(rng.uniform())
            ph.append(rng.uniform())
        return fourier_sum(axes, kv, ph, A)
    if w.ic in ("euler2d", "euler3d"):
        return _euler_ic(w, axes, rng)
    if w.ic == "euler_random":
        return _euler_random(w, axes, rng)
    raise ValueError(f"unknown initial condition {w.ic}")


def _euler_random(w: Workload, axes, rng: SplitMix64) -> np.ndarray:
    """Any dimension: rho = 1 + noise * delta (max |delta| = 1) and each velocity
    component a sum of random modes, scaled to max speed mach * c_s."""
    dim, a = w.dim, w.ic_args
    M, kmax = int(a.get("modes", 4)), int(a.get("kmax", 2))
    cs = float(w.params[0])

    def modes(ncomp):
        kv, ph, C = [], [], []
        for _ in range(M):
            kv.append(_draw_k(rng, dim, kmax))
            ph.append(rng.uniform())
            C.append([rng.uniform() for _ in range(ncomp)])
        return fourier_sum(axes, kv, ph, np.array(C))

    delta = modes(1)[0]
    delta /= np.abs(delta).max()
    rho = 1.0 + float(a.get("noise", 0.2)) * delta
    vel = modes(dim)
    vel *= float(a.get("mach", 0.3)) * cs / np.sqrt((vel ** 2).sum(axis=0)).max()
    U = np.empty((1 + dim, w.nodes))
    U[0] = rho
    U[1:] = rho[None, :] * vel
    return U


def _euler_ic(w: Workload, axes, rng: SplitMix64) -> np.ndarray:
    dim, a = w.dim, w.ic_args
    M, kmax = int(a["modes"]), int(a["kmax"])
    mach = float(a.get("mach", 0.1))
    cs = float(w.params[0])
    if dim == 2:
        # density noise: rho = 1 + noise * delta, max |delta| = 1
        kv, ph, A = [], [], []
        for _ in range(M):
            kv.append(_draw_k(rng, 2, kmax)); A.append(rng.uniform()); ph.append(rng.uniform())
        delta = fourier_sum(axes, kv, ph, A)[0]
        delta /= np.abs(delta).max()
        rho = 1.0 + float(a.get("noise", 1e-2)) * delta
        # velocity from a stream function psi = sum B sin(2 pi q.x + 2 pi th):
        # u = d psi/dy, v = -d psi/dx (cos written as a quarter-period phase shift)
        kv, ph, C = [], [], []
        for _ in range(M):
            q = _draw_k(rng, 2, kmax)
            B = rng.uniform()
            th = rng.uniform()
            kv.append(q); ph.append(th + 0.25)
            C.append([2 * np.pi * B * q[1], -2 * np.pi * B * q[0]])
        vel = fourier_sum(axes, kv, ph, np.array(C))
    elif dim == 3:
        rho = np.ones(w.nodes)
        # solenoidal: u = sum (b_m x k_m) sin(2 pi k_m.x + 2 pi phi_m)
        kv, ph, C = [], [], []
        for _ in range(M):
            k = _draw_k(rng, 3, kmax)
            b = [2.0 * rng.uniform() - 1.0 for _ in range(3)]
            ph.append(rng.uniform())
            kv.append(k)
            C.append(np.cross(b, k))
        vel = fourier_sum(axes, kv, ph, np.array(C, dtype=np.float64))
    else:
        raise ValueError("Euler initial fields are defined for 2-D and 3-D")
    speed = np.sqrt((vel ** 2).sum(axis=0)).max()
    vel *= (mach * cs) / speed
    U = np.empty((1 + dim, w.nodes))
    U[0] = rho
    U[1:] = rho[None, :] * vel
    return U


# ---------------------------------------------------------------------------
# Time-step rule
# ---------------------------------------------------------------------------

def dx_min(axes) -> float:
    """Smallest node spacing inside an element over all axes."""
    return float(min(np.diff(np.asarray(a), axis=1).min() for a in axes))


def max_speeds(w: Workload, U: np.ndarray):
    """Largest signal speed along each direction of the initial state."""
    if w.eq == ADVECTION:
        return [abs(float(w.params[d])) for d in range(w.dim)]
    rho = U[0]
    cs = float(w.params[0])
    return [float(np.abs(U[1 + d] / rho).max()) + cs for d in range(w.dim)]


def time_step(w: Workload, axes, U0: np.ndarray):
    """(dt, nsteps): dt0 = cfl * dx_min / sum_d lambda_d; with a final time,
    nsteps = ceil(T / dt0) and dt = T / nsteps; otherwise the fixed step count."""
    dt0 = w.cfl * dx_min(axes) / sum(max_speeds(w, U0))
    if w.t_final is not None:
        n = int(math.ceil(w.t_final / dt0 - 1e-12))
        return w.t_final / n, n
    return dt0, int(w.steps)


def translated_advection(w: Workload, axes, t: float) -> np.ndarray:
    """Exact advection solution U_0(x - a t) for the Fourier initial conditions."""
    shifted = [np.asarray(ax) - float(w.params[d]) * t for d, ax in enumerate(axes)]
    return initial_state(w, shifted)
