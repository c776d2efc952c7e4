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
// Each face point has an "own" side inside the tile and an "other" side
// (inside the tile only for x-planes between two tile slots). Entry (4 x uint32):
//   w0 = d | other_is_lower << 2 | bsel << 3 | other_in_tile << 6 | need << 8 | xplane << 16
//        need:   the point is active iff need <= nact, the tile's active slots
//                (x-plane pl: need = pl; face of slot s: need = s + 1);
//        xplane: pl for x-planes, 0xff otherwise; the other side of plane nact
//                of a ragged tile lies outside the tile;
//        bsel:   which neighbour element base holds an outside other side:
//                2 d + (1 if that element is the upper neighbour);
//   w1 = own_q | other_q << 16   tile node index (slot * Np + node) of each side
//   w2 = goff                    node offset of an outside other side from its
//                                neighbour base (x: node; y/z: s * Np + node)
//   w3 = own_lift | other_lift << 16   lift slots of the two sides
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
        uint32_t d, kind, ps, own_node, oth_node, own_lift, oth_lift = 0xffff, oth_lower;
        int own_slot, oth_slot;
        if (f < NFX) {
            const int pl = f / NF1, t = f % NF1;
            d = 0; kind = 0; ps = (uint32_t)pl;
            const uint32_t lnode = (uint32_t)(N + N1 * t), rnode = (uint32_t)(N1 * t);
            if (pl == 0) {            // own: slot 0 (upper side), other: tile to the left
                own_slot = 0; own_node = rnode; own_lift = lift(0, 0, 0, t);
                oth_slot = -1; oth_node = lnode; oth_lower = 1;
            } else {                  // own: slot pl-1 (lower side), other: slot pl or outside
                own_slot = pl - 1; own_node = lnode; own_lift = lift(0, pl - 1, 1, t);
                oth_node = rnode; oth_lower = 0;
                oth_slot = pl < epb ? pl : -1;
                if (oth_slot >= 0) oth_lift = lift(0, pl, 0, t);
            }
        } else {
            const int g = f - NFX;
            d = (uint32_t)(1 + g / NFO);
            const int r = g % NFO;
            const int s = r / (2 * NF1), side = (r / NF1) % 2, t = r % NF1;
            const int ta = t % N1, tb = t / N1;
            const uint32_t nlo = d == 1 ? (uint32_t)(ta + N1 * (0 + N1 * tb)) : (uint32_t)(ta + N1 * (tb + N1 * 0));
            const uint32_t nhi = d == 1 ? (uint32_t)(ta + N1 * (N + N1 * tb)) : (uint32_t)(ta + N1 * (tb + N1 * N));
            ps = (uint32_t)s;
            own_slot = s;
            oth_slot = -1;
            if (side == 0) {          // lower face: own is the upper side of the face
                kind = 1; own_node = nlo; oth_node = nhi; oth_lower = 1;
                own_lift = lift((int)d, s, 0, t);
            } else {                  // upper face: own is the lower side of the face
                kind = 2; own_node = nhi; oth_node = nlo; oth_lower = 0;
                own_lift = lift((int)d, s, 1, t);
            }
        }
        const uint32_t NP = (uint32_t)ipow_h(N1, dim);
        const uint32_t in_tile = oth_slot >= 0 ? 1u : 0u;
        const uint32_t upper_nb = oth_lower ? 0u : 1u;
        const uint32_t bsel = 2 * d + upper_nb;
        const uint32_t need = kind == 0 ? ps : ps + 1;
        const uint32_t xplane = kind == 0 ? ps : 0xffu;
        const uint32_t own_q = (uint32_t)own_slot * NP + own_node;
        const uint32_t oth_q = in_tile ? (uint32_t)oth_slot * NP + oth_node : 0u;
        const uint32_t goff = kind == 0 ? oth_node : ps * NP + oth_node;
        tab[4 * f + 0] = d | oth_lower << 2 | bsel << 3 | in_tile << 6 | need << 8 | xplane << 16;
        tab[4 * f + 1] = own_q | oth_q << 16;
        tab[4 * f + 2] = goff;
        tab[4 * f + 3] = own_lift | oth_lift << 16;
    }
}

}  // namespace dg
