"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Bar: FP64 relative L2 per variable <= 1e-12 after a few full RK steps, for
every (equation, dimension, degree 1..8, RK scheme). Meshes have several
workgroup tiles along x with a ragged last tile, K_y != K_z, and the special
cases K_d = 1 (an element is its own periodic neighbour), K_x below the tile
width (the periodic wrap stays inside one tile) and K_z split into XCD slabs.
"""
import numpy as np
import pytest

import oracle
from paper_2510_05254_amd import dg
from _helpers import ADV, EUL, PARITY_RTOL, case, params, parity, ragged_K, rel_l2_per_var

pytestmark = pytest.mark.gpu

ALL = [(dim, N, eq) for dim in (1, 2, 3) for N in range(1, 9) for eq in (ADV, EUL)]


def _run_both(dim, N, K, eq, rk, nsteps, seed=1234):
    w, ax, U0, dt = case(dim, N, K, eq, seed)
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        s.step(rk, dt, nsteps)
        Ug = s.get_state()
    Uo = oracle.step(dim, N, K, eq, params(dim, eq), U0, rk, dt, nsteps)
    return U0, Ug, Uo


@pytest.mark.parametrize("dim,N,eq", ALL)
def test_parity_rk4(dim, N, eq):
    K = ragged_K(dim, N, eq)
    U0, Ug, Uo = _run_both(dim, N, K, eq, 4, 3)
    parity(Ug, Uo, what=f"dim={dim} N={N} eq={eq} K={K}")
    assert rel_l2_per_var(Uo, U0).max() > 1e3 * PARITY_RTOL     # the state really moved


@pytest.mark.parametrize("rk", [3, 6])
@pytest.mark.parametrize("dim,N,eq", ALL)
def test_parity_rk3_rk6(dim, N, eq, rk):
    K = ragged_K(dim, N, eq)
    U0, Ug, Uo = _run_both(dim, N, K, eq, rk, 3)
    parity(Ug, Uo, what=f"rk={rk} dim={dim} N={N} eq={eq}")
    assert rel_l2_per_var(Uo, U0).max() > 1e3 * PARITY_RTOL


@pytest.mark.parametrize("dim,N,K,eq", [
    (1, 3, (1,), ADV), (1, 3, (1,), EUL), (2, 2, (1, 1), EUL), (3, 2, (1, 1, 1), EUL),
    (2, 3, (5, 1), ADV), (3, 3, (2, 1, 3), EUL),      # K_d = 1 in some directions
    (1, 2, (7,), EUL), (2, 1, (10, 4), ADV),          # K_x < tile width: wrap inside a tile
    (3, 1, (3, 2, 16), EUL), (3, 4, (2, 2, 24), ADV),  # K_z split into XCD slabs
    (2, 7, (4, 9), EUL), (3, 5, (4, 1, 2), ADV),
    # 3-D N = 4 tiles hold 2 x 2 elements: one row (its y-neighbours are
    # itself), a ragged last row, one element, one layer
    (3, 4, (3, 1, 2), EUL), (3, 4, (1, 5, 3), ADV), (3, 4, (1, 1, 1), EUL), (3, 4, (4, 3, 1), EUL),
])
def test_parity_special_meshes(dim, N, K, eq):
    U0, Ug, Uo = _run_both(dim, N, K, eq, 4, 2)
    parity(Ug, Uo, what=f"dim={dim} N={N} K={K} eq={eq}")


# 1-D RK3/RK4 run temporally blocked (several steps per launch, arrays in
# LDS). Meshes too large for one workgroup are split into chunks with halos:
# these cases have several chunks with a ragged last one and step counts above
# the per-launch limit, so several launches run back to back.
@pytest.mark.parametrize("N,K,eq,rk,nsteps", [
    (7, 1500, ADV, 4, 30), (1, 5000, ADV, 4, 70), (3, 700, EUL, 4, 9),
    (8, 400, EUL, 3, 11), (4, 450, ADV, 3, 40), (2, 1201, EUL, 4, 5),
])
def test_parity_1d_chunked_multistep(N, K, eq, rk, nsteps):
    w, ax, U0, dt = case(1, N, (K,), eq, 77)
    with dg.Solver(1, N, (K,), eq, params(1, eq)) as s:
        s.set_state(U0)
        m0 = s.mass()
        s.step(rk, dt, nsteps)
        Ug = s.get_state()
        m1 = s.mass()
    Uo = oracle.step(1, N, (K,), eq, params(1, eq), U0, rk, dt, nsteps)
    parity(Ug, Uo, what=f"1-D N={N} K={K} eq={eq} rk={rk}")
    assert rel_l2_per_var(Uo, U0).max() > 1e3 * PARITY_RTOL
    scale = np.abs(U0).reshape(U0.shape[0], -1).max(axis=1)
    assert np.all(np.abs(m1 - m0) <= 1e-14 * np.maximum(scale, 1.0))


# Chunked meshes are cut into about one chunk per CU, so small meshes run as
# many workgroups that each own a few elements and carry halos several times
# wider. Launches read one state array and write the other, so a workgroup
# never loads a halo that a neighbouring chunk has already advanced: every
# steps-per-launch bound and chunk length (a chunk per CU, the halo-bound
# plan, a few elements, the whole mesh in one chunk; odd or even launch counts,
# single-step launches ending in a copy launch) ends bitwise at the same state,
# equal to the oracle.
@pytest.mark.parametrize("N,K,eq,nsteps", [(3, 700, ADV, 25), (7, 300, ADV, 13), (2, 2000, EUL, 9), (5, 129, ADV, 1)])
def test_1d_chunkings_bitwise(N, K, eq, nsteps):
    w, ax, U0, dt = case(1, N, (K,), eq, 31)
    ref = None
    with dg.Solver(1, N, (K,), eq, params(1, eq)) as s:
        base = s.launch_config()
        assert base[6] == 0                     # a chunk per CU by default
        for div, chunk in ((10, 0), (6, 0), (24, 0), (40, 0), (1024, 0), (10, -1), (6, 3), (16, 17), (40, K)):
            c = list(base)
            c[2], c[6] = div, chunk
            s.set_launch_config(c)
            assert s.launch_config()[6] == chunk
            s.set_state(U0)
            s.step(4, dt, nsteps)
            got = s.get_state()
            if ref is None:
                ref = got
            np.testing.assert_array_equal(got, ref, err_msg=f"halo divisor {div}, chunk {chunk}")
    Uo = oracle.step(1, N, (K,), eq, params(1, eq), U0, 4, dt, nsteps)
    parity(ref, Uo, what=f"1-D N={N} K={K} eq={eq} chunked")


def test_parity_1d_whole_mesh_many_steps():
    """A mesh held by one workgroup, stepped past the per-launch step limit.
    Over 4100 steps the N = 1 solution decays by about 1e5, so rounding is
    measured against the initial state's norm (as for the full-length 1-D
    configuration run)."""
    N, K, eq = 1, (8,), ADV
    w, ax, U0, dt = case(1, N, K, eq, 5)
    with dg.Solver(1, N, K, eq, params(1, eq)) as s:
        s.set_state(U0)
        s.step(4, dt, 4100)
        Ug = s.get_state()
    Uo = oracle.step(1, N, K, eq, params(1, eq), U0, 4, dt, 4100)
    assert np.linalg.norm(Ug - Uo) <= PARITY_RTOL * np.linalg.norm(U0)
    assert np.max(np.abs(Ug - Uo)) <= PARITY_RTOL * np.max(np.abs(U0))
    assert np.linalg.norm(Uo) < 0.1 * np.linalg.norm(U0)        # the long run really happened


@pytest.mark.parametrize("dim,N,eq", [(1, 5, EUL), (2, 3, EUL), (3, 4, EUL), (3, 2, ADV)])
def test_conservation_and_determinism(dim, N, eq):
    K = ragged_K(dim, N, eq)
    w, ax, U0, dt = case(dim, N, K, eq)
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        m0 = s.mass()
        np.testing.assert_allclose(m0, oracle.mass(dim, N, K, eq, U0), rtol=1e-13, atol=1e-15)
        s.step(4, dt, 20)
        m1 = s.mass()
        U1 = s.get_state()
        s.set_state(U0)
        s.step(4, dt, 20)
        U2 = s.get_state()
    scale = np.abs(U0).reshape(U0.shape[0], -1).max(axis=1) * 1.0
    assert np.all(np.abs(m1 - m0) <= 1e-14 * np.maximum(scale, 1.0)), (m0, m1)
    np.testing.assert_array_equal(U1, U2)            # bitwise repeatable


@pytest.mark.parametrize("dim,N,K,eq", [(2, 4, (5, 3), EUL), (1, 7, (1500,), ADV)])
def test_checkpoint_split_is_bitwise(dim, N, K, eq):
    w, ax, U0, dt = case(dim, N, K, eq)
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        s.step(4, dt, 7)
        Ua = s.get_state()
        s.set_state(U0)
        s.step(4, dt, 3)
        mid = s.get_state()
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s2:
        s2.set_state(mid)
        s2.step(4, dt, 4)
        Ub = s2.get_state()
    np.testing.assert_array_equal(Ua, Ub)


def test_reductions_match_oracle():
    dim, N, K, eq = 3, 3, (3, 2, 2), EUL
    w, ax, U0, dt = case(dim, N, K, eq)
    ref = U0 * (1.0 + 1e-3 * np.sin(np.arange(U0.size)).reshape(U0.shape))
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        se, sr = s.l2_error_vars(ref)
        a, r = s.l2_error(ref)
        m = s.mass()
    ose, osr = oracle.l2(dim, N, K, eq, U0, ref)
    np.testing.assert_allclose(se, ose, rtol=1e-12)
    np.testing.assert_allclose(sr, osr, rtol=1e-13)
    oa, orr = oracle.l2_error(dim, N, K, eq, U0, ref)
    assert abs(a - oa) <= 1e-12 * oa and abs(r - orr) <= 1e-12 * orr
    np.testing.assert_allclose(m, oracle.mass(dim, N, K, eq, U0), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("dim,N,K", [(1, 8, (5,)), (2, 3, (4, 3)), (3, 4, (2, 3, 5))])
def test_axis_coords_and_roundtrip(dim, N, K):
    with dg.Solver(dim, N, K, EUL, (1.0,)) as s:
        for d, x in enumerate(s.axis_coords()):
            np.testing.assert_allclose(x, oracle.axis_coords(N, K[d]), rtol=0, atol=4.5e-16)
        # all node coordinates: the tensor product of the oracle's per-axis
        # coordinates in the canonical (element x fastest, node x fastest) order
        xyz = s.coords()
        assert xyz.shape == (dim, s.nodes)
        oax = [oracle.axis_coords(N, K[d]).reshape(K[d], N + 1) for d in range(dim)]
        n1 = N + 1
        for node in np.random.default_rng(3).integers(0, s.nodes, 200).tolist() + [0, s.nodes - 1]:
            e, n = divmod(node, n1 ** dim)
            ee, nn = [], []
            for d in range(dim):
                ee.append(e % K[d]); e //= K[d]
                nn.append(n % n1); n //= n1
            for d in range(dim):
                assert abs(xyz[d, node] - oax[d][ee[d], nn[d]]) <= 4.5e-16, (node, d)
        with pytest.raises(dg.DgError) as e:
            dg._call("dg_get_coords", s.h, np.zeros(3).ctypes.data_as(dg.ctypes.c_void_p), 3)
        assert e.value.status == dg.DG_EINVAL
        U = np.random.default_rng(1).standard_normal((s.nvar, s.nodes))
        s.set_state(U)
        np.testing.assert_array_equal(s.get_state(), U)
        s.step(4, 1e-9, 0)                   # nsteps = 0 is a no-op
        np.testing.assert_array_equal(s.get_state(), U)


def test_error_paths_on_device():
    with dg.Solver(2, 3, (4, 4), ADV, (1.0, 0.5)) as s:
        with pytest.raises(dg.DgError) as e:
            s.step(4, 0.01, 1)
        assert e.value.status == dg.DG_ESTATE
        with pytest.raises(dg.DgError) as e:
            s.set_state(np.zeros(10))
        assert e.value.status == dg.DG_EINVAL
        s.set_state(np.zeros((1, s.nodes)))
        for bad in ((5, 0.01, 1), (4, 0.0, 1), (4, float("nan"), 1), (4, 0.01, -1)):
            with pytest.raises(dg.DgError) as e:
                s.step(*bad)
            assert e.value.status == dg.DG_EINVAL
        U = s.get_state()
        assert np.all(U == 0)


def test_device_arrays_stream_and_workspace():
    import torch
    dim, N, K, eq = 3, 2, (4, 3, 2), EUL
    w, ax, U0, dt = case(dim, N, K, eq)
    nbytes = dg.dg_workspace_bytes(dim, N, K, eq, dg.DG_FP64, 6)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    with dg.Solver(dim, N, K, eq, params(dim, eq), hip_stream=stream.cuda_stream,
                   device_workspace=ws, workspace_bytes=nbytes) as s:
        assert s.stream == stream.cuda_stream
        u = torch.from_numpy(U0).to("cuda")
        torch.cuda.synchronize()
        s.set_state_device(u)
        s.step(6, dt, 2)
        out = torch.empty_like(u)
        s.get_state_device(out)
        s.synchronize()
        Ug = out.cpu().numpy()
    Uo = oracle.step(dim, N, K, eq, params(dim, eq), U0, 6, dt, 2)
    parity(Ug, Uo, what="device arrays, external stream and workspace, RK6")


def test_workspace_too_small_for_rk6():
    import torch
    dim, N, K, eq = 2, 2, (3, 3), ADV
    nbytes = dg.dg_workspace_bytes(dim, N, K, eq, dg.DG_FP64, 4)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    with dg.Solver(dim, N, K, eq, params(dim, eq), device_workspace=ws, workspace_bytes=nbytes) as s:
        s.set_state(np.ones((1, s.nodes)))
        s.step(4, 0.01, 1)
        with pytest.raises(dg.DgError) as e:
            s.step(6, 0.01, 1)
        assert e.value.status == dg.DG_ENOMEM
    with pytest.raises(dg.DgError) as e:
        dg.Solver(dim, N, K, eq, params(dim, eq), device_workspace=ws, workspace_bytes=nbytes // 2)
    assert e.value.status == dg.DG_ENOMEM


@pytest.mark.parametrize("dim,N,eq", [(1, 3, ADV), (2, 7, ADV), (2, 3, EUL), (3, 4, EUL), (3, 8, EUL)])
def test_fp32_against_fp64_oracle(dim, N, eq):
    """FP32 state/RHS path: error against the FP64 oracle after 3 RK4 steps."""
    K = ragged_K(dim, N, eq)
    w, ax, U0, dt = case(dim, N, K, eq)
    with dg.Solver(dim, N, K, eq, params(dim, eq), precision=dg.DG_FP32) as s:
        s.set_state(U0)
        s.step(4, dt, 3)
        Ug = s.get_state()
        m = s.mass()
    Uo = oracle.step(dim, N, K, eq, params(dim, eq), U0, 4, dt, 3)
    err = rel_l2_per_var(Ug, Uo)
    print(f"fp32 dim={dim} N={N} eq={eq} rel L2 per var {err}")
    assert np.all(err <= 2e-6), err
    np.testing.assert_allclose(m, oracle.mass(dim, N, K, eq, Uo), rtol=1e-6, atol=1e-7)


# FP32 on the other paths: 1-D chunked meshes (temporally blocked kernel,
# several launches), RK3 and RK6, 3-D N = 4 tiles of 2 x 2 elements.
@pytest.mark.parametrize("dim,N,K,eq,rk,nsteps,bar", [
    (1, 5, (3000,), EUL, 4, 20, 1e-5), (1, 2, (700,), ADV, 3, 30, 1e-5),
    (2, 4, (9, 7), EUL, 6, 3, 1e-5), (3, 4, (5, 3, 2), EUL, 3, 3, 1e-5), (3, 4, (3, 2, 3), ADV, 6, 2, 1e-5),
])
def test_fp32_other_paths(dim, N, K, eq, rk, nsteps, bar):
    w, ax, U0, dt = case(dim, N, K, eq, 44)
    with dg.Solver(dim, N, K, eq, params(dim, eq), precision=dg.DG_FP32) as s:
        s.set_state(U0)
        s.step(rk, dt, nsteps)
        Ug = s.get_state()
    Uo = oracle.step(dim, N, K, eq, params(dim, eq), U0, rk, dt, nsteps)
    err = rel_l2_per_var(Ug, Uo)
    print(f"fp32 dim={dim} N={N} K={K} rk={rk} steps={nsteps}: rel L2 per var {err}")
    assert np.all(err <= bar), err
    assert rel_l2_per_var(Uo, U0).max() > 10 * bar     # the state really moved


# The autotuner times launch configurations that all compute the same bits:
# afterwards the state is the one set, and stepping gives bitwise what the
# default configuration gives.
@pytest.mark.parametrize("dim,N,K,eq,rk", [(3, 4, (6, 4, 8), EUL, 4), (2, 3, (20, 9), EUL, 4),
                                           (1, 7, (1500,), ADV, 4), (2, 5, (7, 6), ADV, 6),
                                           (1, 3, (40,), EUL, 3)])
def test_autotune_keeps_state_and_results(dim, N, K, eq, rk):
    w, ax, U0, dt = case(dim, N, K, eq, 21)
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        s.step(rk, dt, 3)
        ref = s.get_state()
        s.set_state(U0)
        cfg = s.autotune(rk, dt, 2)
        assert cfg[3] == 1 and cfg[0] in (0, 1) and cfg[1] >= 1 and cfg[2] >= 3 and cfg[4] >= 1 and cfg[5] >= 1
        np.testing.assert_array_equal(s.get_state(), U0)
        s.step(rk, dt, 3)
        np.testing.assert_array_equal(s.get_state(), ref)


# Every launch configuration (tile order, z-slab, x-block, z-march length)
# visits the same tiles in another order: the results are bitwise those of the
# default one, also with a ragged last x-tile, x-blocks of one tile, z-march
# chunks with a ragged last chunk and whole-column chunks (the first layer's
# lower neighbour is then the column's top layer, across the periodic wrap).
@pytest.mark.parametrize("N,K,eq,cfgs", [
    (4, (16, 5, 6), EUL, [(0, 1, 2, 1), (0, 3, 4, 1), (1, 6, 1, 1), (0, 2, 8, 1), (1, 1, 4, 1),
                          (0, 1, 4, 2), (0, 2, 2, 4), (1, 1, 8, 6), (0, 1, 4, 5), (0, 3, 1, 2)]),
    (4, (15, 3, 4), ADV, [(0, 4, 2, 1), (0, 1, 1, 1), (1, 2, 4, 1), (0, 1, 4, 4), (0, 2, 1, 3)]),
    (1, (70, 3, 4), EUL, [(0, 2, 1, 1), (1, 4, 3, 1), (0, 1, 3, 1), (0, 1, 1, 4), (0, 2, 3, 2)]),
    (2, (9, 4, 7), EUL, [(0, 1, 1, 7), (0, 1, 1, 3), (1, 2, 1, 2)]),
])
def test_launch_configs_bitwise(N, K, eq, cfgs):
    w, ax, U0, dt = case(3, N, K, eq, 22)
    with dg.Solver(3, N, K, eq, params(3, eq)) as s:
        base = s.launch_config()
        assert base[3] == 0 and base[4] >= 1 and base[5] >= 1
        refs = {}
        for rk in (4, 3):
            s.set_state(U0)
            s.step(rk, dt, 2)
            refs[rk] = s.get_state()
        for order, slab, xblk, zlen in cfgs:
            c = list(base)
            c[0], c[1], c[4], c[5] = order, slab, xblk, zlen
            s.set_launch_config(c)
            got = s.launch_config()
            assert (got[0], got[1], got[4], got[5], got[3]) == (order, slab, xblk, zlen, 0)
            for rk in (4, 3, 6):
                s.set_state(U0)
                s.step(rk, dt, 2)
                if rk not in refs:
                    refs[rk] = s.get_state()
                np.testing.assert_array_equal(s.get_state(), refs[rk],
                                              err_msg=f"{(order, slab, xblk, zlen)} rk{rk}")


def test_set_launch_config_errors():
    w, ax, U0, dt = case(3, 4, (8, 3, 6), EUL, 5)
    with dg.Solver(3, 4, (8, 3, 6), EUL, params(3, EUL)) as s:
        base = list(s.launch_config())
        assert base[4] == 4            # 8 elements, 2 per tile
        for i, v in ((0, 2), (0, -1), (1, 4), (1, 0), (2, 0), (2, 2000), (4, 3), (4, 0), (5, 0), (5, 7), (6, -2),
                     (6, (1 << 30) + 1)):
            c = list(base)
            c[i] = v
            with pytest.raises(dg.DgError) as e:
                s.set_launch_config(c)
            assert e.value.status == dg.DG_EINVAL, (i, v)
            assert s.launch_config() == tuple(base)
        with pytest.raises(ValueError):
            s.set_launch_config(base[:4])
        with pytest.raises(dg.DgError) as e:
            dg._call("dg_set_launch_config", s.h, (dg.ctypes.c_int64 * 7)(*base), 6)
        assert e.value.status == dg.DG_EINVAL
        # the z-slab counts z-units: with chunks of 4 layers K_z = 6 has 2
        c = list(base)
        c[5], c[1] = 4, 3
        with pytest.raises(dg.DgError) as e:
            s.set_launch_config(c)
        assert e.value.status == dg.DG_EINVAL
        c[1] = 2
        s.set_launch_config(c)
        assert s.launch_config()[5] == 4 and s.launch_config()[1] == 2
        s.set_launch_config(base)
    with dg.Solver(2, 3, (5, 4), ADV, params(2, ADV)) as s:
        base = list(s.launch_config())
        for i, v in ((1, 2), (4, base[4] + 1), (5, 2)):
            c = list(base)
            c[i] = v
            with pytest.raises(dg.DgError) as e:
                s.set_launch_config(c)
            assert e.value.status == dg.DG_EINVAL
        c = list(base)
        c[0] = 1
        s.set_launch_config(c)
        assert s.launch_config()[0] == 1
        w2, ax2, U2, dt2 = case(2, 3, (5, 4), ADV, 6)
        s.set_state(U2)
        with dg.Batch() as b:
            b.add(s, 4, dt2, 2)
            with pytest.raises(dg.DgError) as e:
                s.set_launch_config(base)
            assert e.value.status == dg.DG_ESTATE
            b.run_all()
            b.synchronize()


def test_autotune_error_paths():
    import torch
    w, ax, U0, dt = case(2, 2, (4, 3), ADV, 3)
    with dg.Solver(2, 2, (4, 3), ADV, params(2, ADV)) as s:
        with pytest.raises(dg.DgError) as e:
            s.autotune(4, dt)
        assert e.value.status == dg.DG_ESTATE
        s.set_state(U0)
        for bad in ((5, dt, 2), (4, -dt, 2), (4, dt, 0)):
            with pytest.raises(dg.DgError) as e:
                s.autotune(*bad)
            assert e.value.status == dg.DG_EINVAL
    ws = dg.dg_workspace_bytes(2, 2, (4, 3), ADV)
    buf = torch.empty(ws, dtype=torch.uint8, device="cuda")
    with dg.Solver(2, 2, (4, 3), ADV, params(2, ADV), device_workspace=buf, workspace_bytes=ws) as s:
        s.set_state(U0)
        with pytest.raises(dg.DgError) as e:
            s.autotune(4, dt)
        assert e.value.status == dg.DG_ENOTSUP


# An external workspace with one state array to spare: the tuner keeps its
# copy of the state there, restores the state, and stepping afterwards is
# bitwise the untuned result (also for RK6, whose store precedes the copy).
@pytest.mark.parametrize("dim,N,K,eq,rk", [(3, 4, (6, 3, 4), EUL, 4), (3, 2, (5, 4, 4), ADV, 6),
                                           (2, 3, (9, 7), EUL, 3)])
def test_autotune_with_external_workspace(dim, N, K, eq, rk):
    import torch
    w, ax, U0, dt = case(dim, N, K, eq, 23)
    with dg.Solver(dim, N, K, eq, params(dim, eq)) as s:
        s.set_state(U0)
        s.step(rk, dt, 3)
        ref = s.get_state()
    arr = -(-U0.size * 8 // 256) * 256
    ws = dg.dg_workspace_bytes(dim, N, K, eq, dg.DG_FP64, rk) + arr
    buf = torch.empty(ws, dtype=torch.uint8, device="cuda")
    with dg.Solver(dim, N, K, eq, params(dim, eq), device_workspace=buf, workspace_bytes=ws) as s:
        s.set_state(U0)
        cfg = s.autotune(rk, dt, 2)
        assert cfg[3] == 1
        np.testing.assert_array_equal(s.get_state(), U0)
        s.step(rk, dt, 3)
        np.testing.assert_array_equal(s.get_state(), ref)
