"""Host logic of the stage kernel's face-point table (csrc/dg_tables.cpp).

The table is compiled here with g++ (host code only, behind a stub of its
header) and read through an emulation of the kernel's addressing: the same
field decoding, neighbour bases and activity rules as the face phase of
csrc/dg_stage.hpp. For every tile of small meshes (ragged last tiles along x
and y, K_d = 1 self-neighbours, tiles of one and two rows) it checks that
* every node the face phase reads lies in the state array;
* the two sides of a face point are the two elements sharing that face
  (periodic neighbours along d), at the face's nodes (i_d = N below, 0 above)
  with the same tangential indices;
* every element face node receives its lift exactly once (per direction and
  side), in the slot the node-parallel phase reads for it.
Test infrastructure only; no GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2510_05254_amd", "csrc", "dg_tables.cpp")

STUB = """#pragma once
#include <cstddef>
#include <cstdint>
namespace dg {
int face_table_size(int dim, int N, int epb, int epy);
void build_face_table(int dim, int N, int epb, int epy, int nv, uint32_t *tab);
}
"""
DUMP = """#include <cstdio>
#include <cstdlib>
#include <vector>
#include "dg_host.hpp"
int main(int argc, char **argv) {
    const int dim = atoi(argv[1]), N = atoi(argv[2]), epb = atoi(argv[3]), epy = atoi(argv[4]);
    const int nv = atoi(argv[5]);
    const int n = dg::face_table_size(dim, N, epb, epy);
    std::vector<uint32_t> t(4 * (size_t)n);
    dg::build_face_table(dim, N, epb, epy, nv, t.data());
    for (int f = 0; f < n; ++f) printf("%u %u %u %u\\n", t[4 * f], t[4 * f + 1], t[4 * f + 2], t[4 * f + 3]);
    return 0;
}
"""


@pytest.fixture(scope="module")
def dump(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("face_table")
    shutil.copy(SRC, d / "dg_tables.cpp")
    (d / "dg_host.hpp").write_text(STUB)
    (d / "dump.cpp").write_text(DUMP)
    exe = d / "dump"
    subprocess.run(["g++", "-O1", "-std=c++17", "-o", str(exe), str(d / "dump.cpp"), str(d / "dg_tables.cpp")],
                   check=True, capture_output=True)

    def table(dim, N, epb, epy, nv=1):
        out = subprocess.run([str(exe), str(dim), str(N), str(epb), str(epy), str(nv)], check=True,
                             capture_output=True, text=True).stdout
        return [tuple(int(x) for x in line.split()) for line in out.splitlines()]
    return table


def tile_shape(dim, N, nv):
    """(elements along x, rows along y) of the kernel's tile: Geo::EPB, tile_rows
    (2-D advection, nv = 1: lanes of two nodes, twice the elements)."""
    npl = 2 if dim == 2 and nv == 1 else 1
    epb = max(1, 256 * npl // (N + 1) ** dim)
    return epb, 2 if (dim == 3 and N == 4) else 1


def emulate(tab, dim, N, K, epb, epy, nv=1):
    """Walk every tile as the face phase does; return the set of written lifts.
    Global indices are those of the element-interleaved state arrays (element
    stride nv * Np values; variable 0 of node n of element e at e * nv * Np + n)."""
    N1 = N + 1
    NP, NF1, NS = N1 ** dim, N1 ** (dim - 1), epb * epy
    ES = nv * NP
    K0, K1, K2 = (tuple(K) + (1, 1))[:3]
    nodes = K0 * K1 * K2 * NP
    wrap = lambda e, k: (e + k) % k

    def where(g):                     # global value index -> element (ex, ey, ez), node (i, j, k)
        e, n = divmod(g, ES)
        assert n < NP, "index is not variable 0 of a node"
        return (e % K0, (e // K0) % K1, e // (K0 * K1)), (n % N1, (n // N1) % N1, n // (N1 * N1))

    def lift_slot(q, d, side):        # the slot the node-parallel phase reads
        s, n = divmod(q, NP)
        i, j, k = n % N1, (n // N1) % N1, n // (N1 * N1)
        t = {0: j + N1 * k, 1: i + N1 * k, 2: i + N1 * j}[d] if dim > 1 else 0
        return ((d * NS + s) * 2 + side) * NF1 + t

    lifts = set()
    for ez in range(K2):
        for ty in range(-(-K1 // epy)):
            for tx in range(-(-K0 // epb)):
                ex0, ey0 = tx * epb, ty * epy
                nact, nacty = min(epb, K0 - ex0), min(epy, K1 - ey0)
                ebase = K0 * (ey0 + K1 * ez)
                nb = [(ebase + wrap(ex0 - 1, K0)) * ES, (ebase + wrap(ex0 + nact, K0)) * ES,
                      (ex0 + K0 * (wrap(ey0 - 1, K1) + K1 * ez)) * ES,
                      (ex0 + K0 * (wrap(ey0 + nacty, K1) + K1 * ez)) * ES,
                      (ex0 + K0 * (ey0 + K1 * wrap(ez - 1, K2))) * ES,
                      (ex0 + K0 * (ey0 + K1 * wrap(ez + 1, K2))) * ES]

                def in_tile(q):
                    s, n = divmod(q, NP)
                    sy, sx = divmod(s, epb)
                    assert sx < nact and sy < nacty, "in-tile side on an inactive slot"
                    return (ebase + K0 * sy + ex0 + sx) * ES + n

                for w0, w1, w2, w3 in tab:
                    if not ((w0 >> 8) & 0xff) <= nact or not ((w0 >> 24) & 0xf) <= nacty:
                        continue
                    d, oth_lower, bsel = w0 & 3, (w0 >> 2) & 1, (w0 >> 3) & 7
                    outside = ((w0 >> 6) & 1) == 0 or ((w0 >> 16) & 0xff) == nact or (w0 >> 28) == nacty
                    own_q, oth_q, own_l, oth_l = w1 & 0xffff, w1 >> 16, w3 & 0xffff, w3 >> 16
                    g_own = in_tile(own_q)
                    g_oth = nb[bsel] + ((w0 >> 7) & 1) * K0 * ES + w2 if outside else in_tile(oth_q)
                    assert 0 <= g_oth < nodes * nv, "outside read out of bounds"
                    (e_o, n_o), (e_t, n_t) = where(g_own), where(g_oth)
                    (e_lo, n_lo), (e_hi, n_hi) = ((e_t, n_t), (e_o, n_o)) if oth_lower else ((e_o, n_o), (e_t, n_t))
                    assert e_hi[d] == wrap(e_lo[d] + 1, (K0, K1, K2)[d]), "sides are not neighbours"
                    assert all(e_hi[a] == e_lo[a] for a in range(3) if a != d)
                    assert n_lo[d] == N and n_hi[d] == 0, "sides are not the face nodes"
                    assert all(n_lo[a] == n_hi[a] for a in range(dim) if a != d), "tangential mismatch"
                    own_side = 0 if oth_lower else 1
                    assert own_l == lift_slot(own_q, d, own_side)
                    key = (g_own, d, own_side)
                    assert key not in lifts, "lift written twice"
                    lifts.add(key)
                    if d == 2 and oth_lower:
                        # z-marching kernels read the layer below's upper face
                        # from their LDS buffer at slot * NF1 + t, where the
                        # layer below stored node (i, j, N) of the same slot
                        s_own, n_own = divmod(own_q, NP)
                        assert oth_l == s_own * NF1 + n_own, "z-march buffer index"
                        assert n_own < NF1
                    if not outside:
                        assert oth_l == lift_slot(oth_q, d, 1 - own_side)
                        key = (g_oth, d, 1 - own_side)
                        assert key not in lifts, "lift written twice"
                        lifts.add(key)
    # every face node of every element, once per direction and side
    want = set()
    for g in (e * ES + n for e in range(K0 * K1 * K2) for n in range(NP)):
        _, ijk = where(g)
        for d in range(dim):
            if ijk[d] == 0:
                want.add((g, d, 0))
            if ijk[d] == N:
                want.add((g, d, 1))
    assert lifts == want
    return len(lifts)


def meshes(dim, epb, epy):
    if dim == 1:
        return [(1,), (epb + 3,), (2 * epb,)]
    if dim == 2:
        return [(1, 1), (epb + 3, 3), (epb, 2 * epy + 1), (2, 1)]
    return [(1, 1, 1), (epb + 1, 3, 2), (2 * epb, 2 * epy + 1, 1), (1, epy + 1, 3)]


@pytest.mark.parametrize("dim,N", [(d, n) for d in (1, 2, 3) for n in range(1, 9)])
def test_kernel_tile_tables(dump, dim, N):
    for nv in (1, 1 + dim):                                 # advection, isothermal Euler
        epb, epy = tile_shape(dim, N, nv)
        if dim == 3 and N >= 5:
            meshes_ = [(1, 1, 1), (2, 3, 2), (3, 1, 2)]    # keep the emulation small
        else:
            meshes_ = meshes(dim, epb, epy)
        tab = dump(dim, N, epb, epy, nv)
        for K in meshes_:
            emulate(tab, dim, N, K, epb, epy, nv)


# The builder for tile shapes the kernels do not use (two rows in 2-D, other
# widths): the same properties, so a change of tile shape keeps them.
@pytest.mark.parametrize("dim,N,epb,epy,K", [
    (2, 3, 4, 2, (7, 5)), (2, 1, 2, 2, (3, 3)), (2, 2, 3, 2, (7, 1)),
    (3, 3, 4, 2, (5, 3, 2)), (3, 2, 2, 2, (3, 5, 2)), (3, 4, 1, 2, (3, 3, 1)), (3, 4, 2, 1, (5, 3, 2)),
])
def test_other_tile_shapes(dump, dim, N, epb, epy, K):
    for nv in (1, 1 + dim):
        emulate(dump(dim, N, epb, epy, nv), dim, N, K, epb, epy, nv)


def test_table_sizes(dump):
    # x-planes per row, y-planes per column, z-faces per slot
    for dim, N, epb, epy in [(1, 3, 64, 1), (2, 7, 4, 1), (2, 7, 8, 1), (2, 1, 128, 1), (3, 4, 2, 2),
                             (3, 1, 32, 1), (2, 3, 16, 2)]:
        nf1 = (N + 1) ** (dim - 1)
        want = epy * (epb + 1) * nf1 + (epb * (epy + 1) * nf1 if dim > 1 else 0) + \
            (epb * epy * 2 * nf1 if dim > 2 else 0)
        assert len(dump(dim, N, epb, epy)) == want
        assert 16 * want <= 16384          # the library's face-table budget


def test_emulation_rejects_a_table_for_another_layout(dump):
    """The y/z outside offsets depend on the values per element: a table built
    for one variable, read with the Euler layout's element stride, must fail."""
    epb, epy = tile_shape(3, 4, 4)
    with pytest.raises(AssertionError):
        emulate(dump(3, 4, epb, epy, 1), 3, 4, (epb + 1, 3, 2), epb, epy, 4)
