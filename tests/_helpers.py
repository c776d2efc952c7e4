"""Shared helpers for the GPU tests: seeded inputs on oracle coordinates,
time-step choice and the parity metric. Test infrastructure only."""
import numpy as np

from paper_2510_05254_amd import workloads as W

ADV, EUL = 0, 1
PARITY_RTOL = 1e-12          # FP64 GPU vs oracle, relative L2 per variable


def epb(dim, N):
    """Elements per workgroup tile the stage kernel uses (mesh choice only)."""
    return max(1, 256 // (N + 1) ** dim)


def ragged_K(dim, N):
    """A small mesh with several x-tiles, a ragged last tile and K_y != K_z."""
    e = epb(dim, N)
    if dim == 1:
        return (e + 3,)
    if dim == 2:
        return (e + 3 if e > 1 else 3, 3)
    return (e + 1 if e > 1 else 2, 3, 2)


def params(dim, eq):
    return (0.9, -0.55, 0.35)[:dim] if eq == ADV else (1.0,)


def case(dim, N, K, eq, seed=1234, **ic):
    """(workload, oracle axis coordinates, U0, dt) for a smooth random state."""
    if eq == ADV:
        w = W.Workload("adv", dim, N, tuple(K), ADV, params(dim, eq), "fourier_adv", seed,
                       ic_args={"modes": ic.get("modes", 4), "kmax": ic.get("kmax", 2)})
    else:
        w = W.Workload("eul", dim, N, tuple(K), EUL, params(dim, eq), "euler_random", seed,
                       ic_args={"modes": 4, "kmax": 2, "noise": 0.2, "mach": 0.3})
    import oracle
    ax = [oracle.axis_coords(N, k) for k in K]
    U0 = W.initial_state(w, ax)
    dt = 0.1 * W.dx_min(ax) / sum(W.max_speeds(w, U0))
    return w, ax, U0, dt


def rel_l2_per_var(A, B):
    A = np.asarray(A).reshape(B.shape[0], -1)
    B = np.asarray(B).reshape(B.shape[0], -1)
    return np.array([np.linalg.norm(A[v] - B[v]) / max(np.linalg.norm(B[v]), 1e-300)
                     for v in range(B.shape[0])])
