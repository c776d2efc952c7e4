// dg_tables.cpp -- host-built descriptor table of the face points of one
// workgroup tile (EPB elements along x), used by the stage kernel's
// face-parallel Lax-Friedrichs phase. The table depends only on (dim, N, EPB).
//
// Face point f of a tile, f in [0, NF):
//   f <  NFX: x-plane pl = f / NF1 (0..EPB) at tangential node t = f % NF1,
//             between slot pl-1 (its x-upper face) and slot pl (x-lower face);
//             slot -1 / EPB are the neighbouring tiles (global memory);
//   f >= NFX: direction d = 1, 2: the lower (side 0) or upper (side 1) face of
//             slot s at tangential node t; the other side is the neighbouring
//             element along d (global memory).
// Entry (4 x uint32):
//   w0 = d | (lslot+1) << 2 | (rslot+1) << 10 | kind << 18
//        (slot+1 = 0: that side is not in the tile; kind 0 x-plane,
//         1 lower face of slot s, 2 upper face of slot s)
//   w1 = lnode | rnode << 16   node of the left/right side inside its element
//   w2 = pl or s               (plane or slot, for the ragged-tile test)
//   w3 = liftL | liftR << 16   lift slots written for the in-tile sides
#include <cstdint>
#include <vector>

#include "dg_host.hpp"

namespace dg {

static int ipow_h(int b, int e) { return e == 0 ? 1 : b * ipow_h(b, e - 1); }

int face_table_size(int dim, int N, int epb)
{
    const int nf1 = ipow_h(N + 1, dim - 1);
    return (epb + 1) * nf1 + (dim - 1) * epb * 2 * nf1;
}

void build_face_table(int dim, int N, int epb, uint32_t *tab)
{
    const int N1 = N + 1, NF1 = ipow_h(N1, dim - 1);
    const int NFX = (epb + 1) * NF1, NFO = epb * 2 * NF1;
    const int NF = face_table_size(dim, N, epb);
    auto lift = [&](int d, int slot, int side, int t) {
        return (uint32_t)(((d * epb + slot) * 2 + side) * NF1 + t);
    };
    for (int f = 0; f < NF; ++f) {
        uint32_t d, kind, ps, lnode, rnode, liftL = 0xffff, liftR = 0xffff;
        int lslot, rslot;
        if (f < NFX) {
            const int pl = f / NF1, t = f % NF1;
            d = 0; kind = 0; ps = (uint32_t)pl;
            lslot = pl - 1;
            rslot = pl < epb ? pl : -1;
            lnode = (uint32_t)(N + N1 * t);
            rnode = (uint32_t)(N1 * t);
            if (lslot >= 0) liftL = lift(0, lslot, 1, t);
            if (rslot >= 0) liftR = lift(0, rslot, 0, t);
        } else {
            const int g = f - NFX;
            d = (uint32_t)(1 + g / NFO);
            const int r = g % NFO;
            const int s = r / (2 * NF1), side = (r / NF1) % 2, t = r % NF1;
            const int ta = t % N1, tb = t / N1;
            const uint32_t nlo = d == 1 ? (uint32_t)(ta + N1 * (0 + N1 * tb)) : (uint32_t)(ta + N1 * (tb + N1 * 0));
            const uint32_t nhi = d == 1 ? (uint32_t)(ta + N1 * (N + N1 * tb)) : (uint32_t)(ta + N1 * (tb + N1 * N));
            ps = (uint32_t)s;
            lnode = nhi;
            rnode = nlo;
            if (side == 0) {
                kind = 1; lslot = -1; rslot = s;
                liftR = lift((int)d, s, 0, t);
            } else {
                kind = 2; lslot = s; rslot = -1;
                liftL = lift((int)d, s, 1, t);
            }
        }
        tab[4 * f + 0] = d | (uint32_t)(lslot + 1) << 2 | (uint32_t)(rslot + 1) << 10 | kind << 18;
        tab[4 * f + 1] = lnode | rnode << 16;
        tab[4 * f + 2] = ps;
        tab[4 * f + 3] = liftL | liftR << 16;
    }
}

}  // namespace dg
