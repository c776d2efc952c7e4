"""Tile geometry of the stage kernels (csrc/dg_stage.hpp, Geo) against the
rule the host-side tests rely on: the face-table emulation and the ragged
parity meshes assume EPB = max(1, 256 NPL / (N+1)^dim) elements along x,
two rows for 3-D N = 4 and one otherwise, lanes of NPL = 2 nodes for 2-D
advection and 1 otherwise, and THREADS lanes covering the tile in whole
waves. The check is made by the compiler: a host-only syntax pass over a
file of static_asserts that includes the kernel header. It also bounds every
class's face table by the library's reserved 16 KB and its workgroup by 1024
lanes. Test infrastructure only; no GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_05254_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
FACE_TABLE_BYTES = 16384          # kFaceTableBytes, csrc/dg_host.hpp


def expected(dim, N, eq):
    """(NPL, EPB, EPY, THREADS, NF) of the rule above."""
    npl = 2 if dim == 2 and eq == 0 else 1
    np_ = (N + 1) ** dim
    epb = max(1, 256 * npl // np_)
    epy = 2 if dim == 3 and N == 4 else 1
    tn = epb * epy * np_
    threads = -(-(-(-tn // npl)) // 64) * 64
    nf1 = (N + 1) ** (dim - 1)
    nf = epy * (epb + 1) * nf1 + (epb * (epy + 1) * nf1 if dim > 1 else 0) + \
        (epb * epy * 2 * nf1 if dim > 2 else 0)
    return npl, epb, epy, threads, nf


CLASSES = [(d, n, e) for d in (1, 2, 3) for n in range(1, 9) for e in (0, 1)]


def test_rule_bounds():
    for dim, N, eq in CLASSES:
        npl, epb, epy, threads, nf = expected(dim, N, eq)
        tn = epb * epy * (N + 1) ** dim
        assert threads * npl >= tn and threads <= 1024, (dim, N, eq)
        assert 16 * nf <= FACE_TABLE_BYTES, (dim, N, eq, nf)
        assert epb <= 255, "the face table packs plane indices in 8 bits"


def test_kernel_geometry_matches_rule(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    lines = ['#include "dg_stage.hpp"']
    for dim, N, eq in CLASSES:
        npl, epb, epy, threads, nf = expected(dim, N, eq)
        g = f"dg::Geo<{dim}, {N}, {eq}>"
        for field, want in (("NPL", npl), ("EPB", epb), ("EPY", epy), ("THREADS", threads), ("NF", nf)):
            lines.append(f'static_assert({g}::{field} == {want}, "{g}::{field}");')
    src = tmp_path / "geometry.hip"
    src.write_text("\n".join(lines) + "\n")
    r = subprocess.run([HIPCC, "-std=c++17", "--offload-arch=gfx950", "--cuda-host-only", "-fsyntax-only",
                        "-I", CSRC, str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
