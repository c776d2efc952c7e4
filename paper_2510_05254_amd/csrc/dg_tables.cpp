// dg_tables.cpp -- host-built descriptor table of the face points of one
// workgroup tile (EPB elements along x times EPY rows along y; slot
// s = sx + EPB sy), used by the stage kernel's face-parallel Lax-Friedrichs
// phase. The table depends only on (dim, N, EPB, EPY): offsets that depend on
// the mesh (a row of elements) are applied in the kernel.
//
// Face points, in table order (t: tangential node of the face):
//   x-planes: row sy, plane pl = 0..EPB, t; plane pl lies between slot
//             (pl-1, sy) (its x-upper face) and slot (pl, sy) (x-lower face);
//             slots -1 / EPB are the neighbouring tiles (global memory);
//   y-planes: column sx, plane py = 0..EPY, t; between rows py-1 and py of
//             the column, rows -1 / EPY in the neighbouring tiles;
//   z-faces:  slot, side (0 lower, 1 upper), t; the other side is always the
//             neighbouring element along z (global memory).
// Each face point has an "own" side inside the tile and an "other" side
// (inside the tile only for planes between two tile slots). Entry (4 x uint32):
//   w0 = d | other_is_lower << 2 | bsel << 3 | other_in_tile << 6 | row << 7 |
//        need << 8 | xplane << 16 | needy << 24 | yplane << 28
//        need, needy: the point is active iff need <= nact and needy <= nacty,
//                the tile's active x slots and rows;
//        xplane, yplane: pl / py of an in-tile plane (0xff / 0xf otherwise):
//                the other side of plane nact (nacty) of a ragged tile lies
//                outside the tile;
//        bsel:   which neighbour base holds an outside other side:
//                2 d + (1 if it is the upper neighbour);
//        row:    the outside element lies in tile row 1 (x and z faces): one
//                row of elements further than the base (so EPY <= 2);
//   w1 = own_q | other_q << 16   tile node index (slot * Np + node) of each side
//   w2 = goff                    value offset of an outside other side from its
//                                base in the element-interleaved state arrays
//                                (x: node; y, z: sx * nv * Np + node)
//   w3 = own_lift | other_lift << 16   lift slots of the two sides; for a
//                                lower z-face point (other side outside the
//                                tile, no lift) other_lift is instead the
//                                point's index slot * NF1 + t in the
//                                z-marching kernel's buffer of the layer
//                                below's upper-face state
#include <cstdint>
#include <vector>

#include "dg_host.hpp"

namespace dg {

static int ipow_h(int b, int e) { return e == 0 ? 1 : b * ipow_h(b, e - 1); }

int face_table_size(int dim, int N, int epb, int epy)
{
    const int nf1 = ipow_h(N + 1, dim - 1);
    const int nfx = epy * (epb + 1) * nf1;
    const int nfy = dim > 1 ? epb * (epy + 1) * nf1 : 0;
    const int nfz = dim > 2 ? epb * epy * 2 * nf1 : 0;
    return nfx + nfy + nfz;
}

namespace {

struct FacePoint {
    uint32_t d = 0, oth_lower = 0, bsel = 0, in_tile = 0, row = 0;
    uint32_t need = 0, xplane = 0xff, needy = 1, yplane = 0xf;
    uint32_t own_q = 0, oth_q = 0, goff = 0, own_lift = 0, oth_lift = 0xffff;
};

void put(const FacePoint &p, uint32_t *e)
{
    e[0] = p.d | p.oth_lower << 2 | p.bsel << 3 | p.in_tile << 6 | p.row << 7 | p.need << 8 |
           p.xplane << 16 | p.needy << 24 | p.yplane << 28;
    e[1] = p.own_q | p.oth_q << 16;
    e[2] = p.goff;
    e[3] = p.own_lift | p.oth_lift << 16;
}

}  // namespace

void build_face_table(int dim, int N, int epb, int epy, int nv, uint32_t *tab)
{
    const int N1 = N + 1, NF1 = ipow_h(N1, dim - 1);
    const uint32_t NP = (uint32_t)ipow_h(N1, dim);
    const uint32_t ES = NP * (uint32_t)nv;       // values per element in the state arrays
    const int ns = epb * epy;
    auto slot = [&](int sx, int sy) { return (uint32_t)(sx + epb * sy); };
    auto lift = [&](int d, uint32_t s, int side, int t) {
        return (uint32_t)(((d * ns + (int)s) * 2 + side) * NF1 + t);
    };
    uint32_t *e = tab;
    // x-planes; face node t = j + N1 k, lower side at i = N, upper side at i = 0
    for (int sy = 0; sy < epy; ++sy)
        for (int pl = 0; pl <= epb; ++pl)
            for (int t = 0; t < NF1; ++t, e += 4) {
                const uint32_t lnode = (uint32_t)(N + N1 * t), rnode = (uint32_t)(N1 * t);
                FacePoint p;
                p.d = 0;
                p.need = (uint32_t)pl;
                p.needy = (uint32_t)(sy + 1);
                p.xplane = (uint32_t)pl;
                p.row = (uint32_t)sy;
                if (pl == 0) {        // own: slot (0, sy) (upper side), other: tile to the left
                    p.own_q = slot(0, sy) * NP + rnode;
                    p.own_lift = lift(0, slot(0, sy), 0, t);
                    p.oth_lower = 1;
                    p.bsel = 0;
                    p.goff = lnode;
                } else {              // own: slot (pl-1, sy) (lower side), other: slot (pl, sy) or outside
                    p.own_q = slot(pl - 1, sy) * NP + lnode;
                    p.own_lift = lift(0, slot(pl - 1, sy), 1, t);
                    p.oth_lower = 0;
                    p.bsel = 1;
                    p.goff = rnode;
                    if (pl < epb) {
                        p.in_tile = 1;
                        p.oth_q = slot(pl, sy) * NP + rnode;
                        p.oth_lift = lift(0, slot(pl, sy), 0, t);
                    }
                }
                put(p, e);
            }
    // y-planes; face node t = i + N1 k, lower side at j = N, upper side at j = 0
    if (dim > 1)
        for (int sx = 0; sx < epb; ++sx)
            for (int py = 0; py <= epy; ++py)
                for (int t = 0; t < NF1; ++t, e += 4) {
                    const int ta = t % N1, tb = t / N1;
                    const uint32_t nlo = (uint32_t)(ta + N1 * N1 * tb);           // j = 0
                    const uint32_t nhi = (uint32_t)(ta + N1 * (N + N1 * tb));     // j = N
                    FacePoint p;
                    p.d = 1;
                    p.need = (uint32_t)(sx + 1);
                    p.needy = (uint32_t)(py == 0 ? 1 : py);
                    if (py == 0) {    // own: row 0 (upper side), other: the row below the tile
                        p.own_q = slot(sx, 0) * NP + nlo;
                        p.own_lift = lift(1, slot(sx, 0), 0, t);
                        p.oth_lower = 1;
                        p.bsel = 2;
                        p.goff = (uint32_t)sx * ES + nhi;
                    } else {          // own: row py-1 (lower side), other: row py or outside
                        p.own_q = slot(sx, py - 1) * NP + nhi;
                        p.own_lift = lift(1, slot(sx, py - 1), 1, t);
                        p.oth_lower = 0;
                        p.bsel = 3;
                        p.goff = (uint32_t)sx * ES + nlo;
                        if (py < epy) {
                            p.in_tile = 1;
                            p.yplane = (uint32_t)py;
                            p.oth_q = slot(sx, py) * NP + nlo;
                            p.oth_lift = lift(1, slot(sx, py), 0, t);
                        }
                    }
                    put(p, e);
                }
    // z-faces; face node t = i + N1 j
    if (dim > 2)
        for (int sy = 0; sy < epy; ++sy)
            for (int sx = 0; sx < epb; ++sx)
                for (int side = 0; side < 2; ++side)
                    for (int t = 0; t < NF1; ++t, e += 4) {
                        const uint32_t nlo = (uint32_t)t, nhi = (uint32_t)(t + N1 * N1 * N);
                        FacePoint p;
                        p.d = 2;
                        p.need = (uint32_t)(sx + 1);
                        p.needy = (uint32_t)(sy + 1);
                        p.row = (uint32_t)sy;
                        p.own_q = slot(sx, sy) * NP + (side == 0 ? nlo : nhi);
                        p.own_lift = lift(2, slot(sx, sy), side, t);
                        p.oth_lower = side == 0 ? 1 : 0;
                        p.bsel = side == 0 ? 4 : 5;
                        p.goff = (uint32_t)sx * ES + (side == 0 ? nhi : nlo);
                        if (side == 0) p.oth_lift = slot(sx, sy) * (uint32_t)NF1 + (uint32_t)t;
                        put(p, e);
                    }
}

}  // namespace dg
