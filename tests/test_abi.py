"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/dg.h declares, and validates arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_05254_amd import dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", text)))


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("dg_create", "dg_set_state", "dg_step", "dg_get_state", "dg_l2_error"):
        assert must in names
    assert set(names) == set(dg.SIGNATURES), set(names) ^ set(dg.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = dg.load()
    for name in _declared():
        assert hasattr(lib, name), name
    # the .so is a shared library built for gfx950 (the offload bundle names the target)
    blob = open(dg.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


@pytest.mark.parametrize("args,why", [
    ((0, 3, [4], 0, [1.0]), "dim"),
    ((4, 3, [4], 0, [1.0]), "dim"),
    ((1, 0, [4], 0, [1.0]), "N"),
    ((1, 9, [4], 0, [1.0]), "N"),
    ((2, 3, [4, 0], 0, [1.0, 1.0]), "K"),
    ((1, 3, [4], 2, [1.0]), "equation"),
    ((1, 3, [4], 1, [0.0]), "sound speed"),
    ((1, 3, [4], 1, [-1.0]), "sound speed"),
    ((2, 3, [4, 4], 0, [1.0, float("nan")]), "velocity"),
    ((1, 3, [4], 1, [float("inf")]), "sound speed"),
    ((1, 3, [2 ** 30 + 1], 0, [1.0]), "K"),                        # maximum size per direction
    ((3, 1, [2 ** 11, 2 ** 11, 2 ** 10], 1, [1.0]), "elements"),   # more than 4e9 elements
])
def test_create_rejects_invalid_arguments(args, why):
    with pytest.raises(dg.DgError) as e:
        dg.dg_create(*args)
    assert e.value.status == dg.DG_EINVAL
    assert why.split()[0].lower() in str(e.value).lower() or why in str(e.value)


def test_create_rejects_bad_precision_and_null_out():
    lib = dg.load()
    K = np.array([4], dtype=np.int64)
    p = np.array([1.0])
    h = ctypes.c_void_p()
    rc = lib.dg_create_ex(1, 3, K.ctypes.data_as(ctypes.c_void_p), 0, p.ctypes.data_as(ctypes.c_void_p),
                          7, None, None, 0, ctypes.byref(h))
    assert rc == dg.DG_EINVAL
    rc = lib.dg_create(1, 3, K.ctypes.data_as(ctypes.c_void_p), 0, p.ctypes.data_as(ctypes.c_void_p), None)
    assert rc == dg.DG_EINVAL


def test_null_handle_calls_fail_cleanly():
    lib = dg.load()
    assert lib.dg_step(None, 4, 0.1, 1) == dg.DG_EINVAL
    assert lib.dg_sizes(None, None, None) == dg.DG_EINVAL
    assert lib.dg_get_coords(None, None, 0) == dg.DG_EINVAL
    assert lib.dg_destroy(None) == dg.DG_OK
    assert lib.dg_stream(None) is None
    assert "NULL" in dg.dg_last_error() or dg.dg_last_error() == ""


def test_bandwidth_probe_validates_arguments():
    lib = dg.load()
    arr = (ctypes.c_void_p * 3)(16, 32, 48)
    assert lib.dg_bandwidth_probe(None, arr, 0, arr, 1, 1024) == dg.DG_EINVAL
    assert lib.dg_bandwidth_probe(None, arr, 4, arr, 1, 1024) == dg.DG_EINVAL
    assert lib.dg_bandwidth_probe(None, arr, 1, arr, 3, 1024) == dg.DG_EINVAL
    assert lib.dg_bandwidth_probe(None, arr, 1, arr, 1, 1000) == dg.DG_EINVAL
    assert lib.dg_bandwidth_probe(None, None, 1, arr, 1, 1024) == dg.DG_EINVAL
    bad = (ctypes.c_void_p * 1)(8)
    assert lib.dg_bandwidth_probe(None, bad, 1, arr, 1, 1024) == dg.DG_EINVAL


def test_workspace_bytes():
    b4 = dg.dg_workspace_bytes(3, 4, [64, 64, 64], 1, dg.DG_FP64, 4)
    b6 = dg.dg_workspace_bytes(3, 4, [64, 64, 64], 1, dg.DG_FP64, 6)
    b4f = dg.dg_workspace_bytes(3, 4, [64, 64, 64], 1, dg.DG_FP32, 4)
    arr = 131072000 * 8
    assert 4 * arr <= b4 < 4 * arr + 2 ** 20
    assert b6 - b4 == 5 * arr
    assert 4 * arr // 2 <= b4f < b4
    with pytest.raises(dg.DgError):
        dg.dg_workspace_bytes(3, 4, [64, 64, 64], 1, dg.DG_FP64, 5)
    # the largest meshes the validation admits are sized without overflow
    big = dg.dg_workspace_bytes(1, 8, [2 ** 30], 1, dg.DG_FP64, 4)
    assert big >= 4 * 2 ** 30 * 9 * 2 * 8
    big3 = dg.dg_workspace_bytes(3, 8, [2 ** 11, 2 ** 11, 953], 1, dg.DG_FP64, 6)
    assert big3 >= 9 * (2 ** 22 * 953) * 729 * 4 * 8


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_valid_create_without_gpu_reports_edevice():
    with pytest.raises(dg.DgError) as e:
        dg.dg_create(1, 3, [64], 0, [1.0])
    assert e.value.status == dg.DG_EDEVICE


def test_single_hip_runtime_in_process():
    """libdg.so must bind to the HIP runtime torch loads (same SONAME), never a second copy."""
    dg.load()
    import torch  # noqa: F401
    maps = open("/proc/self/maps").read()
    hip = set(re.findall(r"\S*libamdhip64\S*", maps))
    hsa = set(re.findall(r"\S*libhsa-runtime64\S*", maps))
    assert len(hip) == 1 and len(hsa) == 1, (hip, hsa)


def test_step_static_validates_before_touching_a_device():
    """dg_step_static's argument and size checks need no GPU."""
    lib = dg.load()
    K = np.array([16, 16], dtype=np.int64)
    p = np.array([1.0, 0.5])
    kp, pp = K.ctypes.data_as(ctypes.c_void_p), p.ctypes.data_as(ctypes.c_void_p)
    n = 16 * 16 * 16
    fake = ctypes.c_void_p(1 << 20)          # never dereferenced: every call below fails a check
    assert lib.dg_step_static(4, 3, kp, 0, pp, 0, None, fake, n, 4, 0.1, 1) == dg.DG_EINVAL
    assert lib.dg_step_static(2, 3, kp, 0, pp, 0, None, None, n, 4, 0.1, 1) == dg.DG_EINVAL
    assert lib.dg_step_static(2, 3, kp, 0, pp, 0, None, fake, n + 1, 4, 0.1, 1) == dg.DG_EINVAL
    assert lib.dg_step_static(2, 3, kp, 0, pp, 0, None, fake, n, 5, 0.1, 1) == dg.DG_EINVAL
    assert lib.dg_step_static(2, 3, kp, 0, pp, 0, None, fake, n, 4, -0.1, 1) == dg.DG_EINVAL
    assert lib.dg_step_static(2, 3, kp, 0, pp, 0, None, fake, n, 4, 0.1, -1) == dg.DG_EINVAL
    assert lib.dg_step_static(2, 3, kp, 0, pp, 2, None, fake, n, 4, 0.1, 1) == dg.DG_EINVAL
    odd = ctypes.c_void_p((1 << 20) + 4)
    assert lib.dg_step_static(2, 3, kp, 0, pp, 0, None, odd, n, 4, 0.1, 1) == dg.DG_EINVAL
    # larger than the static scratch: 3 RK work arrays of 2-D 512^2 N = 7 FP64
    Kb = np.array([512, 512], dtype=np.int64)
    nb = 512 * 512 * 64
    assert 3 * nb * 8 > dg.DG_STATIC_SCRATCH_BYTES
    rc = lib.dg_step_static(2, 7, Kb.ctypes.data_as(ctypes.c_void_p), 0, pp, 0, None, fake, nb, 4, 0.1, 1)
    assert rc == dg.DG_ENOMEM
    assert "static scratch" in dg.dg_last_error()
    # the RK6 limit is lower (8 work arrays): a mesh that fits RK4 but not RK6
    Km = np.array([256, 256], dtype=np.int64)
    nm = 256 * 256 * 64
    assert 3 * nm * 8 < dg.DG_STATIC_SCRATCH_BYTES < 8 * nm * 8
    rc = lib.dg_step_static(2, 7, Km.ctypes.data_as(ctypes.c_void_p), 0, pp, 0, None, fake, nm, 6, 0.1, 1)
    assert rc == dg.DG_ENOMEM
