// dg_stage.hpp -- fused NDG right-hand side + Runge-Kutta stage kernel for
// gfx950 (CDNA4), templated on precision, dimension, degree and equation.
//
// What one launch computes (Sporykhin & Homann, arXiv:2510.05254, Sec. 2.1):
// for every node l of every element, the strong form of the semi-discrete
// NDG operator, which equals the paper's weak form by the LGL
// summation-by-parts identity W D + D^T W = diag(-1, 0, .., 0, 1):
//
//   R_l = sum_d (2/dx_d) [ - sum_m D_{l_d m} F_d(U)_{..m..}
//                          + delta_{l_d,0} (1/w_0) (Fhat_lower - F_d(U_l))
//                          - delta_{l_d,N} (1/w_N) (Fhat_upper - F_d(U_l)) ]
//
// with F_d the physical flux (eqs. advection2d, eulerIso2d), Fhat the
// Lax-Friedrichs flux of eq. LF, alpha the larger of the two traces' wave
// speeds, periodic neighbours, and w_0 = w_N = 2/(N(N+1)). The Runge-Kutta
// stage update is applied in the same pass (StageParams).
//
// Work decomposition (MI355X-specific, not from the paper). A workgroup owns
// a tile of EPB consecutive elements along x (EPB * (N+1)^dim nodes, ~256
// threads), times two rows along y for 3-D N = 4 (512 threads), and runs
// three phases separated by barriers:
//  1. node-parallel: load the stage input (one thread per node, variables in
//     registers), stage it in LDS together with, for Euler, either 1/rho and
//     the symmetric momentum-flux tensor m_a m_b / rho + delta_ab rho c^2 or
//     the velocities m_k / rho (StageLds);
//  2. face-parallel: one thread per face point of the tile (a host-built
//     descriptor table lists them). Faces inside the tile read both sides from
//     LDS and are evaluated once; faces to neighbouring tiles read the other
//     side from global memory (prefetched before the first barrier). The
//     lift (2/dx)(1/w_0)(Fhat - F) of each in-tile side goes to LDS;
//  3. node-parallel: volume term (D held in LDS), plus the lifts, plus the RK
//     combination, stored with one coalesced store per variable and output.
// Fluxes are evaluated through one set of functions with FMA contraction off
// and a fixed reciprocal sequence, so a face shared by two tiles gets the same
// Fhat bits on both sides and the scheme conserves to roundoff.
//
// Layout of the state arrays on the device (element-interleaved): element e
// holds its variables one after another, value (v, e, n) at e * NV * NP +
// v * NP + n, so a tile's variables are one contiguous run per row of
// elements (the ABI's variable-major layout is converted at set/get).
// Addressing: when every state array fits the 32-bit buffer range, loads and
// stores are raw buffer instructions with one 32-bit offset per node (the
// variable offset rides in the scalar offset); otherwise 64-bit pointers.
//
// Tile order: virtual block b runs on XCD b % 8 (private L2 per XCD); tiles
// are renumbered so each XCD owns a contiguous range, in the order x-tile
// fastest within an x-block of `xblk` tiles, then z inside a slab of `slab`
// layers, then y-tile, then slab, then x-block, which keeps the y- and
// z-neighbours of a tile among recently visited tiles (xblk slab and xblk
// tiles back inside a slab).
#pragma once

#include <type_traits>

#include "dg_internal.hpp"

namespace dg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// LDS layout and register target of the single-solve stage kernel, by class
// (3-D isothermal Euler, FP64, 32-bit addressing; all others keep the tensor
// layout and four waves per SIMD). The velocity layout shrinks the
// workgroup's LDS so that more workgroups share a CU: N = 1 by itself
// (4 instead of 3 workgroups of 256 threads), N = 4, 7, 8 together with a
// six-waves-per-SIMD register target (3 instead of 2, 3 instead of 2, 2
// instead of 1); N = 6 needs only the register target (3 instead of 2).
// Six-wave kernels load the RK inputs in phase 3.
constexpr bool stage_big_euler(int DIM, int EQ, int rbytes, bool BUF)
{
    return DIM == 3 && EQ == 1 && rbytes == 8 && BUF;
}
constexpr int stage_waves(int DIM, int N, int EQ, int rbytes, bool BUF)
{
    return stage_big_euler(DIM, EQ, rbytes, BUF) && (N == 4 || N >= 6) ? 6 : 4;
}
constexpr bool stage_vel(int DIM, int N, int EQ, int rbytes, bool BUF)
{
    return stage_big_euler(DIM, EQ, rbytes, BUF) && (N == 1 || N == 4 || N == 7 || N == 8);
}

// Rows of elements along y per tile: two for 3-D N = 4, whose tile of 2 x 2
// elements (512 threads) reads half the y-face traces per element of a 2 x 1
// tile and has its 500 face points in one pass.
constexpr int tile_rows(int DIM, int N) { return DIM == 3 && N == 4 ? 2 : 1; }

// Nodes per lane of the stage kernels: two for 2-D advection, one otherwise.
// A 2-D advection tile moves few bytes per node and its lanes spend most of
// the tile waiting on global loads, with the CU already at eight waves per
// SIMD; two nodes per lane put twice the loads in flight per wave (and twice
// the elements per workgroup) for 46-78 VGPRs: still eight waves at N >= 6,
// six to eight below, where the gain is smaller. Euler tiles (more registers
// per node) lose occupancy at two nodes per lane and get slower. Every choice
// computes the same bits: a node's arithmetic does not depend on the lane or
// the tile that holds it.
constexpr int stage_npl(int DIM, int EQ) { return DIM == 2 && EQ == 0 ? 2 : 1; }

// A tile is EPB elements along x times EPY along y; TM scales it along x:
// EPB = max(1, 256 TM NPL / (N+1)^dim), and THREADS lanes of NPL nodes cover
// it (lane t holds tile nodes t, t + THREADS, ...).
template <int DIM, int N, int EQ, int TM = 1>
struct Geo {
    static constexpr int N1 = N + 1;
    static constexpr int NP = ipow(N1, DIM);          // nodes per element
    static constexpr int NF1 = ipow(N1, DIM - 1);     // nodes per face
    static constexpr int NPL = stage_npl(DIM, EQ);     // nodes per lane
    static constexpr int EPB = (256 * TM * NPL / NP) < 1 ? 1 : (256 * TM * NPL / NP);
    static constexpr int EPY = tile_rows(DIM, N);
    static_assert(EPY == 1 || EPY == 2, "the face table encodes one bit of tile row");
    static constexpr int NS = EPB * EPY;              // element slots, slot = sx + EPB sy
    static constexpr int TN = NS * NP;
    static constexpr int THREADS = (((TN + NPL - 1) / NPL + 63) / 64) * 64;
    static constexpr int NFX = EPY * (EPB + 1) * NF1;                 // x-plane points
    static constexpr int NFY = DIM > 1 ? EPB * (EPY + 1) * NF1 : 0;   // y-plane points
    static constexpr int NFZ = DIM > 2 ? NS * 2 * NF1 : 0;            // z-face points
    static constexpr int NF = NFX + NFY + NFZ;
    static constexpr int NL = DIM * NS * 2 * NF1;     // lift slots per variable
};

template <int EQ, int DIM>
struct Vars {
    static constexpr int NV = EQ == 0 ? 1 : 1 + DIM;
    static constexpr int NSYM = EQ == 0 ? 0 : DIM * (DIM + 1) / 2;
};

__device__ __forceinline__ constexpr int sym_index(int d, int k, int dim)
{
    const int a = d < k ? d : k, b = d < k ? k : d;
    return a * dim - (a * (a - 1)) / 2 + (b - a);
}

// 1/x: hardware reciprocal estimate refined by Newton-Raphson steps
// e = 1 - x r, r <- r + r e, written with explicit FMAs.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// Momentum-flux tensor entry m_a (m_b / rho) + delta_ab rho c^2, canonical
// order a <= b, contraction off: LDS copies and recomputations agree bitwise.
template <typename real>
__device__ __forceinline__ real sym_flux(real ma, real mb, real rho, real rinv, real c2, bool diag)
{
#pragma clang fp contract(off)
    real f = ma * (mb * rinv);
    if (diag) f = f + rho * c2;
    return f;
}

// The same entry from m_a and the velocity v_b = m_b (1/rho) that phase 1
// stores: the operations of sym_flux in its order, so the same bits.
template <typename real>
__device__ __forceinline__ real sym_flux_v(real ma, real vb, real rho, real c2, bool diag)
{
#pragma clang fp contract(off)
    real f = ma * vb;
    if (diag) f = f + rho * c2;
    return f;
}

// a b + c rounded once
template <typename real>
__device__ __forceinline__ real fmadd(real a, real b, real c)
{
    if constexpr (sizeof(real) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// largest absolute eigenvalue of the isothermal Euler flux Jacobian along d
template <typename real>
__device__ __forceinline__ real wave_speed(real md, real rinv, real c)
{
#pragma clang fp contract(off)
    return fabs(md * rinv) + c;
}

// flux along D and wave speed of a state U held in registers (same rounding
// as the LDS copies made in phase 1)
template <typename real, int DIM, int EQ, int D>
__device__ __forceinline__ void flux_of(const real *U, const real *par, real *F, real &lam)
{
    if constexpr (EQ == 0) {
#pragma clang fp contract(off)
        F[0] = par[D] * U[0];
        lam = fabs(par[D]);
    } else {
        const real c = par[0];
        const real c2 = c * c;
        const real rinv = recip(U[0]);
        F[0] = U[1 + D];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const int a = D < k ? D : k, b = D < k ? k : D;
            F[1 + k] = sym_flux(U[1 + a], U[1 + b], U[0], rinv, c2, a == b);
        }
        lam = wave_speed(U[1 + D], rinv, c);
    }
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// State-array access: raw buffer (32-bit offsets) or 64-bit pointer.
template <typename real, bool BUF>
struct Arr;

template <typename real>
struct Arr<real, true> {
    using idx_t = uint32_t;
    __amdgpu_buffer_rsrc_t r;
    uint32_t vbytes;   // bytes between variables
    // nodes: nodes per variable; vstride: values between the variables of a
    // node (the element's node count in the element-interleaved layout)
    __device__ __forceinline__ Arr(const void *p, int64_t nodes, int nvar, int vstride)
    {
        vbytes = uint32_t(vstride * (int64_t)sizeof(real));
        r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0,
                                              (int)(uint32_t(nvar) * uint32_t(nodes) * uint32_t(sizeof(real))),
                                              0x00020000);
    }
    // (last argument: the instruction's cache-policy bits, default policy)
    __device__ __forceinline__ real ld(int v, idx_t node) const
    {
        if constexpr (sizeof(real) == 8)
            return __builtin_bit_cast(real, __builtin_amdgcn_raw_buffer_load_b64(
                                                r, node * (uint32_t)sizeof(real), v * vbytes, 0));
        else
            return __builtin_bit_cast(real, __builtin_amdgcn_raw_buffer_load_b32(
                                                r, node * (uint32_t)sizeof(real), v * vbytes, 0));
    }
    __device__ __forceinline__ void st(int v, idx_t node, real x) const
    {
        if constexpr (sizeof(real) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r,
                                                  node * (uint32_t)sizeof(real), v * vbytes, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r,
                                                  node * (uint32_t)sizeof(real), v * vbytes, 0);
    }
};

template <typename real>
struct Arr<real, false> {
    using idx_t = int64_t;
    real *p;
    int64_t stride;
    __device__ __forceinline__ Arr(const void *ptr, int64_t, int, int vstride)
        : p(static_cast<real *>(const_cast<void *>(ptr))), stride(vstride) {}
    __device__ __forceinline__ real ld(int v, idx_t node) const { return p[v * stride + node]; }
    __device__ __forceinline__ void st(int v, idx_t node, real x) const { p[v * stride + node] = x; }
};

// LDS of one stage-kernel workgroup. Per node, Euler keeps either the
// symmetric momentum-flux tensor and 1/rho (VEL = false: fewest LDS reads and
// flops in the volume term) or the velocities m_k (1/rho) (VEL = true:
// smaller, so that more workgroups share a CU; the tensor entries are rebuilt
// from them with the same operations, so the results are the same bits).
template <typename real, int DIM, int N, int EQ, int TM, bool VEL, bool ZM = false>
struct StageLds {
    using G = Geo<DIM, N, EQ, TM>;
    static constexpr int NV = Vars<EQ, DIM>::NV, NSYM = Vars<EQ, DIM>::NSYM;
    static constexpr int NE = EQ == 0 ? 1 : (VEL ? DIM : NSYM + 1);
    real sY[NV][G::TN];
    real sE[NE][EQ == 1 ? G::TN : 1];   // VEL: v_k; otherwise tensor (sym_index order), then 1/rho
    real sL[NV][G::NL];
    real sD[G::N1 * G::N1];
    // ZM (z-march): the previous layer's upper z-face state, slot * NF1 + t
    real sZ[NV][ZM ? G::NS * G::NF1 : 1];
};

// Whether the single-solve 3-D stage kernel keeps each layer's upper z-face
// state in LDS for the next layer of its chunk (a z-marching workgroup runs
// consecutive layers of one tile column; without the buffer the lower faces
// read the layer below from global memory, which the same workgroup has just
// loaded): for every 3-D class whose workgroups per CU do not drop with the
// extra buffer. Workgroups per CU: the smaller of the LDS limit (160 KB per
// CU) and the register target (`waves` waves per SIMD, four SIMDs).
template <typename real, int DIM, int N, int EQ, int TM, bool VEL, int WAVES>
constexpr bool stage_zm()
{
    constexpr long lds = 160 * 1024;
    constexpr long wg_waves = Geo<DIM, N, EQ, TM>::THREADS / 64;
    constexpr long cap = 4 * WAVES / wg_waves;
    constexpr long with = lds / (long)sizeof(StageLds<real, DIM, N, EQ, TM, VEL, true>);
    constexpr long without = lds / (long)sizeof(StageLds<real, DIM, N, EQ, TM, VEL, false>);
    return DIM == 3 && (with < cap ? with : cap) == (without < cap ? without : cap);
}

// per-thread constants of a workgroup (independent of the tile), for each
// of the lane's nodes
template <int DIM, int N, int EQ, int TM>
struct ThreadSetup {
    static constexpr int NPL = Geo<DIM, N, EQ, TM>::NPL;
    int tid, slot[NPL], sx[NPL], sy[NPL], n[NPL], ijk[NPL][3];
    __device__ __forceinline__ ThreadSetup()
    {
        using G = Geo<DIM, N, EQ, TM>;
        tid = threadIdx.x;
#pragma unroll
        for (int u = 0; u < NPL; ++u) {
            const int vt = tid + u * G::THREADS;
            slot[u] = vt / G::NP;
            sy[u] = slot[u] / G::EPB;
            sx[u] = slot[u] - sy[u] * G::EPB;
            n[u] = vt - slot[u] * G::NP;
            ijk[u][0] = n[u] % G::N1;
            ijk[u][1] = DIM > 1 ? (n[u] / G::N1) % G::N1 : 0;
            ijk[u][2] = DIM > 2 ? n[u] / (G::N1 * G::N1) : 0;
        }
    }
};

// Tile coordinates of tile (unit) L in the launch order: x-tile, y-tile and
// z (the layer, or for a z-marching launch the chunk of layers) from the
// host's magic-number reciprocals: x-tile within an x-block fastest, then z
// within a slab, then y-tile, then slab, then x-block (3-D).
template <int DIM>
__device__ __forceinline__ void decode_tile(const StageParams &p, uint32_t L, int64_t &tx, int64_t &ty,
                                            int64_t &ez)
{
    if constexpr (DIM == 1) {
        tx = L; ty = 0; ez = 0;
    } else if constexpr (DIM == 2) {
        const uint32_t r1 = fast_div(L, p.fd_tx);
        tx = L - r1 * p.fd_tx.div; ty = r1; ez = 0;
    } else {
        const uint32_t r1 = fast_div(L, p.fd_xb);
        const uint32_t r2 = fast_div(r1, p.fd_slab);
        const uint32_t r3 = fast_div(r2, p.fd_ty);
        const uint32_t r4 = fast_div(r3, p.fd_nslab);
        const uint32_t xi = L - r1 * p.fd_xb.div;
        const uint32_t zs = r1 - r2 * p.fd_slab.div;
        ty = r2 - r3 * p.fd_ty.div;
        ez = int64_t(r3 - r4 * p.fd_nslab.div) * p.fd_slab.div + zs;
        tx = int64_t(r4) * p.fd_xb.div + xi;
    }
}

// One tile (EPB x EPY elements) of one RHS + RK stage: the tile at x-tile tx,
// y-tile ty, layer ez of the solve described by p. NIN >= 0 fixes the
// number of RK inputs (p.nin) at compile time, so their loads are issued in
// phase 1 behind the outside traces with exact waits; NIN = -1 reads p.nin and
// loads the inputs in phase 3. ZM: z-marching kernel; zl: the layer below
// was the previous tile of this workgroup, so the lower z-faces take the
// other side's state from lds.sZ (written by that tile) instead of global
// memory, and this tile leaves its upper z-face state there in turn.
template <typename real, int DIM, int N, int EQ, bool BUF, int TM, bool XIN = false, int NIN = -1,
          int WAVES = 4, bool VEL = false, bool ZM = false>
__device__ __forceinline__ void stage_tile_at(const StageParams &p, int64_t tx, int64_t ty, int64_t ez,
                                              bool zl, StageLds<real, DIM, N, EQ, TM, VEL, ZM> &lds,
                                              const ThreadSetup<DIM, N, EQ, TM> &ts, real dval,
                                              const ExtraIn *x = nullptr)
{
    using G = Geo<DIM, N, EQ, TM>;
    constexpr int N1 = G::N1, NP = G::NP, NF1 = G::NF1, EPB = G::EPB, EPY = G::EPY, NS = G::NS;
    constexpr int THREADS = G::THREADS, NF = G::NF;
    constexpr int NV = Vars<EQ, DIM>::NV;
    constexpr int ES = NP * NV;      // values per element (element-interleaved layout)
    constexpr real INVW0 = real(N * (N + 1)) / real(2);     // 1/w_0 = 1/w_N
    using A = Arr<real, BUF>;
    using idx_t = typename A::idx_t;
    auto &sY = lds.sY;
    auto &sE = lds.sE;
    constexpr int NSYM = Vars<EQ, DIM>::NSYM;
    auto &sL = lds.sL;
    auto &sD = lds.sD;
    constexpr int NPL = G::NPL;
    const int tid = ts.tid;

    const A yin(p.yin, p.stride, NV, NP);
    real par[3], rdx2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        par[d] = real(p.par[d]);
        rdx2[d] = real(p.rdx2[d]);
    }
    const real c2 = par[0] * par[0];
    const int64_t K0 = p.K[0], K1 = p.K[1], K2 = p.K[2];

    (void)zl;
    const int64_t ex0 = tx * EPB, ey0 = ty * EPY;
    const int nact = (int)((K0 - ex0) < EPB ? (K0 - ex0) : EPB);      // active x slots
    const int nacty = EPY == 1 ? 1 : (int)((K1 - ey0) < EPY ? (K1 - ey0) : EPY);     // active rows
    const int64_t ebase = K0 * (ey0 + K1 * ez);    // element index of (0, ey0, ez)

    // Neighbour element bases (node offsets) of this tile, uniform: bsel =
    // 2 d + 1 for the upper neighbour along d, 2 d for the lower one (x: the
    // elements left of the tile's first slot and right of its last active
    // slot in row 0; y: the rows below the tile and above its last active
    // row; z: the layers below/above the tile, at its first element). Faces
    // of tile row sy add sy rows (rstride nodes) to an x or z base.
    auto wrap = [](int64_t e, int64_t K) { return e < 0 ? e + K : (e >= K ? e - K : e); };
    // named values, not an array: a select over array elements becomes a
    // dynamically indexed (scratch) load
    const idx_t nb0 = idx_t((ebase + wrap(ex0 - 1, K0)) * ES);
    const idx_t nb1 = idx_t((ebase + wrap(ex0 + nact, K0)) * ES);
    const idx_t rstride = idx_t(K0 * ES);
    idx_t nb2 = 0, nb3 = 0, nb4 = 0, nb5 = 0;
    if constexpr (DIM > 1) {
        nb2 = idx_t((ex0 + K0 * (wrap(ey0 - 1, K1) + K1 * ez)) * ES);
        nb3 = idx_t((ex0 + K0 * (wrap(ey0 + nacty, K1) + K1 * ez)) * ES);
    }
    if constexpr (DIM > 2) {
        nb4 = idx_t((ex0 + K0 * (ey0 + K1 * wrap(ez - 1, K2))) * ES);
        nb5 = idx_t((ex0 + K0 * (ey0 + K1 * wrap(ez + 1, K2))) * ES);
    }
    // Face point fields (see dg_tables.cpp): w0 = d | other_is_lower << 2 |
    // bsel << 3 | other_in_tile << 6 | row << 7 | need << 8 | xplane << 16 |
    // needy << 24 | yplane << 28, w1 = own_q | other_q << 16, w2 = outside
    // node offset, w3 = lift slots.
    // (one-row tiles: every point has needy = 1 and no in-tile y-plane)
    auto face_valid = [nact, nacty](uint32_t w0) {
        const bool x = ((w0 >> 8) & 0xffu) <= uint32_t(nact);
        (void)nacty;
        if constexpr (EPY == 1) return x;
        else return x && ((w0 >> 24) & 0xfu) <= uint32_t(nacty);
    };
    auto other_outside = [nact, nacty](uint32_t w0) {
        const bool o = ((w0 >> 6) & 1u) == 0 || ((w0 >> 16) & 0xffu) == uint32_t(nact);
        (void)nacty;
        if constexpr (EPY == 1) return o;
        else return o || (w0 >> 28) == uint32_t(nacty);
    };
    // blend of the six bases by masks (bitwise, so it stays in registers)
    auto outside_node = [nb0, nb1, nb2, nb3, nb4, nb5, rstride](uint32_t w0, uint32_t w2) -> idx_t {
        using U = typename std::make_unsigned<idx_t>::type;
        (void)nb2, (void)nb3, (void)nb4, (void)nb5, (void)rstride;     // unused in 1-D
        const uint32_t bsel = (w0 >> 3) & 7u;
        auto m = [bsel](uint32_t k) { return U(0) - U(bsel == k); };
        U b = (U(nb0) & m(0)) | (U(nb1) & m(1));
        if constexpr (DIM > 1) b |= (U(nb2) & m(2)) | (U(nb3) & m(3));
        if constexpr (DIM > 2) b |= (U(nb4) & m(4)) | (U(nb5) & m(5));
        if constexpr (EPY > 1) b += U(rstride) & (U(0) - U((w0 >> 7) & 1u));
        return idx_t(b) + idx_t(w2);
    };

    // lower z-face point whose other side (the layer below) is in lds.sZ
    auto z_in_lds = [zl](uint32_t w0) {
        (void)zl;
        if constexpr (!ZM) return false;
        else return zl && (w0 & 3u) == 2u && ((w0 >> 2) & 1u);
    };

    // ---- phase 1: state, 1/rho and flux tensor into LDS; the outside trace
    // of this thread's first face point is prefetched behind the own state.
    bool active[NPL];
    int ln[NPL];
    idx_t gi[NPL];
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        const int slot = ts.slot[u], n = ts.n[u];
        active[u] = EPY == 1 ? slot < nact : ts.sx[u] < nact && ts.sy[u] < nacty;
        ln[u] = slot * NP + n;
        gi[u] = EPY == 1 ? idx_t((ebase + ex0 + slot) * ES + n)
                         : idx_t((ebase + K0 * ts.sy[u] + ex0 + ts.sx[u]) * ES + n);
    }
    // both groups are loaded unconditionally (inactive lanes read node 0) so
    // the wait before the LDS stores covers only the first group
    // Issue order matters (vector loads retire in order): this thread's first
    // face-point descriptor, then the own state, then (once the descriptor is
    // in) the outside trace; phase 1 then waits for the own state only.
    uint32_t fw0 = 0, fw1 = 0, fw2 = 0, fw3 = 0;
    if (tid < NF) {
        fw0 = p.ftab[4 * tid + 0];
        fw1 = p.ftab[4 * tid + 1];
        fw2 = p.ftab[4 * tid + 2];
        fw3 = p.ftab[4 * tid + 3];
    }
    // the second face point of threads that have one (tiles with more face
    // points than threads), read and prefetched here too so phase 2 does not
    // wait on two dependent global loads
    constexpr bool PASS2 = NF > THREADS;
    uint32_t fx0 = 0, fx1 = 0, fx2 = 0, fx3 = 0;
    if (PASS2 && tid + THREADS < NF) {
        fx0 = p.ftab[4 * (tid + THREADS) + 0];
        fx1 = p.ftab[4 * (tid + THREADS) + 1];
        fx2 = p.ftab[4 * (tid + THREADS) + 2];
        fx3 = p.ftab[4 * (tid + THREADS) + 3];
    }
    real y[NPL][NV], g[NV];
    idx_t gy[NPL];
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        gy[u] = active[u] ? gi[u] : idx_t(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) y[u][v] = yin.ld(v, gy[u]);
    }
    const bool pre = tid < NF && face_valid(fw0) && other_outside(fw0) && !z_in_lds(fw0);
    const idx_t gn0 = pre ? outside_node(fw0, fw2) : idx_t(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = yin.ld(v, gn0);
    real g2[NV];
    if constexpr (PASS2) {
        const bool pre2 = tid + THREADS < NF && face_valid(fx0) && other_outside(fx0) && !z_in_lds(fx0);
        const idx_t gn2 = pre2 ? outside_node(fx0, fx2) : idx_t(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) g2[v] = yin.ld(v, gn2);
    }
    // RK inputs, issued last: the waits for the own state and the traces do
    // not cover them. Kernels built for six waves per SIMD load them in
    // phase 3 instead, so they are not held in registers across the phases.
    constexpr bool EARLY = NIN >= 0 && WAVES == 4;
    real a0[NPL][NV], a1[NPL][NV];
    if constexpr (EARLY && NIN >= 1) {
        const A in0(p.in0, p.stride, NV, NP);
#pragma unroll
        for (int u = 0; u < NPL; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v) a0[u][v] = in0.ld(v, gy[u]);
    }
    if constexpr (EARLY && NIN >= 2) {
        const A in1(p.in1, p.stride, NV, NP);
#pragma unroll
        for (int u = 0; u < NPL; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v) a1[u][v] = in1.ld(v, gy[u]);
    }
    const bool has0 = NIN < 0 ? p.nin > 0 : NIN >= 1;
    const bool has1 = NIN < 0 ? p.nin > 1 : NIN >= 2;
    // D (loaded at kernel entry into dval, stored here so the entry does not
    // wait for it before the tile's loads are issued)
    if (tid < N1 * N1) sD[tid] = dval;
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        if (!active[u]) continue;
        const real *yu = y[u];
        const int lnu = ln[u];
#pragma unroll
        for (int v = 0; v < NV; ++v) sY[v][lnu] = yu[v];
        if constexpr (EQ == 1) {
            const real rinv = recip(yu[0]);
            if constexpr (VEL) {
                // m_b (1/rho) as sym_flux and wave_speed form it; the tensor
                // entries are rebuilt from these where they are needed
#pragma unroll
                for (int k = 0; k < DIM; ++k) sE[k][lnu] = yu[1 + k] * rinv;
            } else {
                sE[NSYM][lnu] = rinv;
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int b = a; b < DIM; ++b)
                        sE[sym_index(a, b, DIM)][lnu] = sym_flux(yu[1 + a], yu[1 + b], yu[0], rinv, c2, a == b);
            }
        }
    }
    __syncthreads();

    // ---- phase 2: Lax-Friedrichs flux at the tile's face points, lifts to LDS.
    // With sigma = -1 when the other side is the lower one,
    //   Fhat = 1/2 [(F_own + F_oth) - (sigma alpha)(U_oth - U_own)]
    // is eq. LF with (U^-, U^+) = (lower, upper); two tiles sharing a face
    // evaluate it with the roles swapped and get the same bits (the sum
    // commutes and both factors of the product change sign exactly).
    for (int f = tid; f < NF; f += THREADS) {
        uint32_t w0 = fw0, w1 = fw1, w2 = fw2, w3 = fw3;
        if (PASS2 && f >= THREADS && f < 2 * THREADS) {
            w0 = fx0; w1 = fx1; w2 = fx2; w3 = fx3;
#pragma unroll
            for (int v = 0; v < NV; ++v) g[v] = g2[v];
        } else if (f >= 2 * THREADS) {
            w0 = p.ftab[4 * f + 0];
            w1 = p.ftab[4 * f + 1];
            w2 = p.ftab[4 * f + 2];
            w3 = p.ftab[4 * f + 3];
        }
        if (!face_valid(w0)) continue;
        const bool oglob = other_outside(w0);
        const bool ozl = z_in_lds(w0);
        if (f >= 2 * THREADS && oglob && !ozl) {
            const idx_t gn = outside_node(w0, w2);
#pragma unroll
            for (int v = 0; v < NV; ++v) g[v] = yin.ld(v, gn);
        }
        if constexpr (ZM) {
            // the layer below's upper face node, left in LDS by the previous
            // tile of this workgroup (slot * NF1 + t: the table's other-lift
            // field of a lower z-face point)
            if (ozl) {
#pragma unroll
                for (int v = 0; v < NV; ++v) g[v] = lds.sZ[v][w3 >> 16];
            }
        }
        const int own_q = int(w1 & 0xffffu);
        const int oth_q = int(w1 >> 16);
        const bool oth_lower = (w0 >> 2) & 1u;
        const int own_l = int(w3 & 0xffffu), oth_l = int(w3 >> 16);
        auto face = [&](auto dconst) {
            constexpr int D = decltype(dconst)::value;
            real Uo[NV], Fo[NV], Ut[NV], Ft[NV], lo, lt;
            auto from_lds = [&](int q, real *U, real *F, real &lam) {
#pragma unroll
                for (int v = 0; v < NV; ++v) U[v] = sY[v][q];
                if constexpr (EQ == 0) {
#pragma clang fp contract(off)
                    F[0] = par[D] * U[0];
                    lam = fabs(par[D]);
                } else {
                    F[0] = U[1 + D];
                    if constexpr (VEL) {
#pragma unroll
                        for (int k = 0; k < DIM; ++k) {
                            const int a = D < k ? D : k, b = D < k ? k : D;
                            F[1 + k] = sym_flux_v(U[1 + a], sE[b][q], U[0], c2, a == b);
                        }
                        // |m_D (1/rho)| + c, as wave_speed forms it
                        lam = fabs(sE[D][q]) + par[0];
                    } else {
#pragma unroll
                        for (int k = 0; k < DIM; ++k) F[1 + k] = sE[sym_index(D, k, DIM)][q];
                        lam = wave_speed(F[0], sE[NSYM][q], par[0]);
                    }
                }
            };
            from_lds(own_q, Uo, Fo, lo);
            if (oglob) {
#pragma unroll
                for (int v = 0; v < NV; ++v) Ut[v] = g[v];
                flux_of<real, DIM, EQ, D>(Ut, par, Ft, lt);
            } else {
                from_lds(oth_q, Ut, Ft, lt);
            }
            const real alpha = lo > lt ? lo : lt;
            const real sa = oth_lower ? -alpha : alpha;
            const real sl = rdx2[D] * INVW0;
            const real so = oth_lower ? sl : -sl;     // lift sign of the own side
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const real fh = real(0.5) * ((Fo[v] + Ft[v]) - sa * (Ut[v] - Uo[v]));
                sL[v][own_l] = so * (fh - Fo[v]);
                if (!oglob) sL[v][oth_l] = -so * (fh - Ft[v]);
            }
        };
        const int d = int(w0 & 3u);
        if (d == 0) face(std::integral_constant<int, 0>());
        if constexpr (DIM > 1) if (d == 1) face(std::integral_constant<int, 1>());
        if constexpr (DIM > 2) if (d == 2) face(std::integral_constant<int, 2>());
    }
    __syncthreads();

    // ---- phase 3: volume term + lifts, RK stage combination, store
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        if (!active[u]) continue;
        const int slot = ts.slot[u], n = ts.n[u];
        const int *ijk = ts.ijk[u];
        real R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) R[v] = real(0);
        const int base = slot * NP;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int id = ijk[d];
            const int sd = d == 0 ? 1 : (d == 1 ? N1 : N1 * N1);
            const int line0 = base + n - id * sd;
            real acc[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = real(0);
#pragma unroll 1
            for (int m = 0; m < N1; ++m) {
                const real dm = sD[id * N1 + m];
                const int q = line0 + m * sd;
                if constexpr (EQ == 0) {
                    acc[0] += dm * sY[0][q];
                } else {
                    acc[0] += dm * sY[1 + d][q];
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        if constexpr (VEL) {
                            const int a = d < k ? d : k, b = d < k ? k : d;
                            acc[1 + k] += dm * sym_flux_v(sY[1 + a][q], sE[b][q], sY[0][q], c2, a == b);
                        } else {
                            acc[1 + k] += dm * sE[sym_index(d, k, DIM)][q];
                        }
                    }
                }
            }
            if constexpr (EQ == 0) {
                R[0] -= rdx2[d] * (par[d] * acc[0]);
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) R[v] -= rdx2[d] * acc[v];
            }
            if (id == 0 || id == N) {
                const int t = d == 0 ? (DIM > 1 ? ijk[1] + N1 * ijk[2] : 0)
                                     : (d == 1 ? ijk[0] + N1 * ijk[2] : ijk[0] + N1 * ijk[1]);
                const int li = ((d * NS + slot) * 2 + (id == N ? 1 : 0)) * NF1 + t;
#pragma unroll
                for (int v = 0; v < NV; ++v) R[v] += sL[v][li];
            }
        }
        if constexpr (ZM) {
            // this layer's upper z-face state, for the next layer's lower faces
            if (ijk[2] == N) {
#pragma unroll
                for (int v = 0; v < NV; ++v) lds.sZ[v][slot * NF1 + ijk[0] + N1 * ijk[1]] = y[u][v];
            }
        }
        if (!EARLY && has0) {
            const A in0(p.in0, p.stride, NV, NP);
#pragma unroll
            for (int v = 0; v < NV; ++v) a0[u][v] = in0.ld(v, gi[u]);
        }
        if (!EARLY && has1) {
            const A in1(p.in1, p.stride, NV, NP);
#pragma unroll
            for (int v = 0; v < NV; ++v) a1[u][v] = in1.ld(v, gi[u]);
        }
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            // RK combination in one fixed rounding sequence, cy y, then fused
            // multiply-adds of the inputs in order, R last, whatever the
            // kernel variant knows about the inputs at compile time
#pragma clang fp contract(off)
            if (o < p.nout) {
                const real cy = real(p.cy[o]), c0 = real(p.c0[o]), c1 = real(p.c1[o]),
                           cr = real(p.cr[o]);
                const A out(o == 0 ? p.out0 : p.out1, p.stride, NV, NP);
                if constexpr (!XIN) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        real val = cy * y[u][v];
                        if (has0) val = fmadd(c0, a0[u][v], val);
                        if (has1) val = fmadd(c1, a1[u][v], val);
                        out.st(v, gi[u], fmadd(cr, R[v], val));
                    }
                } else {
                    // fused RK6 stages: also the stored k's with nonzero weights
                    real val[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        val[v] = cy * y[u][v];
                        if (has0) val[v] = fmadd(c0, a0[u][v], val[v]);
                        if (has1) val[v] = fmadd(c1, a1[u][v], val[v]);
                    }
                    for (int j = 0; j < x->n; ++j) {
                        if (x->c[o][j] == 0.0) continue;
                        const real cj = real(x->c[o][j]);
                        const A in(x->in[j], p.stride, NV, NP);
#pragma unroll
                        for (int v = 0; v < NV; ++v) val[v] = fmadd(cj, in.ld(v, gi[u]), val[v]);
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) out.st(v, gi[u], fmadd(cr, R[v], val[v]));
                }
            }
        }
    }
}

// stage_tile_at on tile L of the launch order (one layer per tile)
template <typename real, int DIM, int N, int EQ, bool BUF, int TM, bool XIN = false, int NIN = -1,
          int WAVES = 4, bool VEL = false>
__device__ __forceinline__ void stage_tile(const StageParams &p, uint32_t L,
                                           StageLds<real, DIM, N, EQ, TM, VEL> &lds,
                                           const ThreadSetup<DIM, N, EQ, TM> &ts, real dval,
                                           const ExtraIn *x = nullptr)
{
    int64_t tx, ty, ez;
    decode_tile<DIM>(p, L, tx, ty, ez);
    stage_tile_at<real, DIM, N, EQ, BUF, TM, XIN, NIN, WAVES, VEL>(p, tx, ty, ez, false, lds, ts, dval, x);
}

// Single-solve stage kernel. Virtual block b is unit L of the launch order
// (XCD-contiguous renumbering: b runs on XCD b % 8): the chunk of p.zlen
// layers (1 in 1-D and 2-D) of one tile column that decode_tile's z
// coordinate names, run bottom to top (z-march). Classes with stage_zm take
// the lower z-faces' other side of every layer after the chunk's first from
// the LDS copy of the layer below.
template <typename real, int DIM, int N, int EQ, bool BUF, int NIN, int TM = 1>
__global__ void __launch_bounds__((Geo<DIM, N, EQ, TM>::THREADS))
__attribute__((amdgpu_waves_per_eu(stage_waves(DIM, N, EQ, (int)sizeof(real), BUF))))
stage_kernel(const StageParams p)
{
    using G = Geo<DIM, N, EQ, TM>;
    constexpr int W = stage_waves(DIM, N, EQ, (int)sizeof(real), BUF);
    constexpr bool VEL = stage_vel(DIM, N, EQ, (int)sizeof(real), BUF);
    constexpr bool ZM = stage_zm<real, DIM, N, EQ, TM, VEL, W>();
    __shared__ StageLds<real, DIM, N, EQ, TM, VEL, ZM> lds;
    const ThreadSetup<DIM, N, EQ, TM> ts;
    const real dval = ts.tid < G::N1 * G::N1 ? static_cast<const real *>(p.D)[ts.tid] : real(0);
    for (uint32_t vb = blockIdx.x; vb < p.ntiles32; vb += gridDim.x) {
        const uint32_t xb = vb & (kXcds - 1), jb = vb / kXcds;
        const uint32_t L = p.plain_order ? vb : xb * p.xq + (xb < p.xr ? xb : p.xr) + jb;
        int64_t tx, ty, ez;
        decode_tile<DIM>(p, L, tx, ty, ez);
        // (32-bit: K_z <= 2^30)
        const uint32_t z0 = uint32_t(ez) * p.zlen;
        const uint32_t kz = uint32_t(p.K[2]);
        const uint32_t z1 = z0 + p.zlen < kz ? z0 + p.zlen : kz;
        for (uint32_t z = z0; z < z1; ++z) {
            stage_tile_at<real, DIM, N, EQ, BUF, TM, false, NIN, W, VEL, ZM>(p, tx, ty, z, ZM && z > z0, lds,
                                                                           ts, dval);
            __syncthreads();
        }
    }
}

// Single-solve stage kernel with further inputs (fused RK6 stages).
template <typename real, int DIM, int N, int EQ, bool BUF>
__global__ void __launch_bounds__((Geo<DIM, N, EQ>::THREADS)) __attribute__((amdgpu_waves_per_eu(4)))
stage_kernel_x(const StageParams p, const ExtraIn x)
{
    using G = Geo<DIM, N, EQ>;
    __shared__ StageLds<real, DIM, N, EQ, 1, false> lds;
    const ThreadSetup<DIM, N, EQ, 1> ts;
    const real dval = ts.tid < G::N1 * G::N1 ? static_cast<const real *>(p.D)[ts.tid] : real(0);
    for (uint32_t vb = blockIdx.x; vb < p.ntiles32; vb += gridDim.x) {
        const uint32_t xb = vb & (kXcds - 1), jb = vb / kXcds;
        const uint32_t L = p.plain_order ? vb : xb * p.xq + (xb < p.xr ? xb : p.xr) + jb;
        stage_tile<real, DIM, N, EQ, BUF, 1, true>(p, L, lds, ts, dval, &x);
        __syncthreads();
    }
}

// A batch member's stage parameters (and its first virtual tile, and for the
// fused RK6 stages its further inputs) copied into LDS by the workgroup:
// stage_tile reads them many times, and from LDS a read is a broadcast
// instead of a dependent global load.
template <bool XIN>
struct MemberLds {
    StageParams p;
    ExtraIn x[XIN ? 1 : 0 + 1];
    uint32_t base;
};

template <bool XIN, int THREADS>
__device__ __forceinline__ void load_member(const BatchLaunch &b, uint32_t s, MemberLds<XIN> &m, int tid)
{
    static_assert(sizeof(StageParams) % 4 == 0 && sizeof(ExtraIn) % 4 == 0, "copied as dwords");
    constexpr int NP4 = sizeof(StageParams) / 4, NX4 = XIN ? (int)sizeof(ExtraIn) / 4 : 0;
    static_assert(NP4 + NX4 + 1 <= THREADS, "one dword per thread");
    if (tid < NP4) {
        reinterpret_cast<uint32_t *>(&m.p)[tid] = reinterpret_cast<const uint32_t *>(b.params + s)[tid];
    } else if (tid < NP4 + NX4) {
        reinterpret_cast<uint32_t *>(&m.x[0])[tid - NP4] = reinterpret_cast<const uint32_t *>(b.extra + s)[tid - NP4];
    } else if (tid == NP4 + NX4) {
        m.base = b.tile_base[s];
    }
}

// Batched stage: one launch advances every solve of one kernel class (same
// precision, equation, dimension, degree; meshes, arrays and time steps
// differ). Virtual tile T (XCD-contiguous numbering over all solves) belongs
// to solve tile_solve[T] and is that solve's tile T - tile_base[solve].
// The LDS layout is the single-solve kernel's for the class (stage_vel; not
// for N = 1, whose batch kernel then needs more registers than four waves
// per SIMD leave); the register target stays at four waves per SIMD (the
// batch's own per-tile state does not fit the six-wave budget without
// spilling).
template <typename real, int DIM, int N, int EQ, bool BUF, int NIN>
__global__ void __launch_bounds__((Geo<DIM, N, EQ>::THREADS)) __attribute__((amdgpu_waves_per_eu(4)))
stage_kernel_batch(const BatchLaunch b)
{
    using G = Geo<DIM, N, EQ>;
    constexpr int W = 4;
    constexpr bool VEL = stage_vel(DIM, N, EQ, (int)sizeof(real), BUF) && N > 1;
    __shared__ StageLds<real, DIM, N, EQ, 1, VEL> lds;
    __shared__ MemberLds<false> mem;
    const ThreadSetup<DIM, N, EQ, 1> ts;
    const real dval = ts.tid < G::N1 * G::N1 ? static_cast<const real *>(b.D)[ts.tid] : real(0);
    for (uint32_t vb = blockIdx.x; vb < b.ntiles; vb += gridDim.x) {
        const uint32_t xb = vb & (kXcds - 1), jb = vb / kXcds;
        const uint32_t T = xb * b.xq + (xb < b.xr ? xb : b.xr) + jb;
        load_member<false, G::THREADS>(b, b.tile_solve[T], mem, ts.tid);
        __syncthreads();
        stage_tile<real, DIM, N, EQ, BUF, 1, false, NIN, W, VEL>(mem.p, T - mem.base, lds, ts, dval);
        __syncthreads();
    }
}

template <typename real, int DIM, int N, int EQ, bool BUF>
void launch_stage_nin(const StageParams &p, int64_t grid, hipStream_t s)
{
    const dim3 g((unsigned)grid), b(Geo<DIM, N, EQ>::THREADS);
    switch (p.nin) {
    case 0: hipLaunchKernelGGL((stage_kernel<real, DIM, N, EQ, BUF, 0>), g, b, 0, s, p); break;
    case 1: hipLaunchKernelGGL((stage_kernel<real, DIM, N, EQ, BUF, 1>), g, b, 0, s, p); break;
    default: hipLaunchKernelGGL((stage_kernel<real, DIM, N, EQ, BUF, 2>), g, b, 0, s, p); break;
    }
}

template <typename real, int DIM, int N, int EQ>
hipError_t launch_stage(const StageParams &p, int64_t grid, hipStream_t s)
{
    if (p.nin < 0 || p.nin > 2) return hipErrorInvalidValue;
    const int64_t bytes = p.stride * Vars<EQ, DIM>::NV * (int64_t)sizeof(real);
    if (bytes < (int64_t(1) << 31))
        launch_stage_nin<real, DIM, N, EQ, true>(p, grid, s);
    else
        launch_stage_nin<real, DIM, N, EQ, false>(p, grid, s);
    return hipGetLastError();
}

// Batched fused RK6 stage: stage_kernel_x's body per member, the member's
// further inputs from b.extra.
template <typename real, int DIM, int N, int EQ, bool BUF>
__global__ void __launch_bounds__((Geo<DIM, N, EQ>::THREADS)) __attribute__((amdgpu_waves_per_eu(4)))
stage_kernel_batch_x(const BatchLaunch b)
{
    using G = Geo<DIM, N, EQ>;
    __shared__ StageLds<real, DIM, N, EQ, 1, false> lds;
    __shared__ MemberLds<true> mem;
    const ThreadSetup<DIM, N, EQ, 1> ts;
    const real dval = ts.tid < G::N1 * G::N1 ? static_cast<const real *>(b.D)[ts.tid] : real(0);
    for (uint32_t vb = blockIdx.x; vb < b.ntiles; vb += gridDim.x) {
        const uint32_t xb = vb & (kXcds - 1), jb = vb / kXcds;
        const uint32_t T = xb * b.xq + (xb < b.xr ? xb : b.xr) + jb;
        load_member<true, G::THREADS>(b, b.tile_solve[T], mem, ts.tid);
        __syncthreads();
        stage_tile<real, DIM, N, EQ, BUF, 1, true>(mem.p, T - mem.base, lds, ts, dval, &mem.x[0]);
        __syncthreads();
    }
}

template <typename real, int DIM, int N, int EQ>
hipError_t launch_stage_batch_x(const BatchLaunch &b, bool buf, int64_t grid, hipStream_t s)
{
    const dim3 g((unsigned)grid), t(Geo<DIM, N, EQ>::THREADS);
    if (buf)
        hipLaunchKernelGGL((stage_kernel_batch_x<real, DIM, N, EQ, true>), g, t, 0, s, b);
    else
        hipLaunchKernelGGL((stage_kernel_batch_x<real, DIM, N, EQ, false>), g, t, 0, s, b);
    return hipGetLastError();
}

template <typename real, int DIM, int N, int EQ, bool BUF>
void launch_stage_batch_nin(const BatchLaunch &b, int nin, int64_t grid, hipStream_t s)
{
    const dim3 g((unsigned)grid), t(Geo<DIM, N, EQ>::THREADS);
    switch (nin) {
    case 0: hipLaunchKernelGGL((stage_kernel_batch<real, DIM, N, EQ, BUF, 0>), g, t, 0, s, b); break;
    case 1: hipLaunchKernelGGL((stage_kernel_batch<real, DIM, N, EQ, BUF, 1>), g, t, 0, s, b); break;
    default: hipLaunchKernelGGL((stage_kernel_batch<real, DIM, N, EQ, BUF, 2>), g, t, 0, s, b); break;
    }
}

template <typename real, int DIM, int N, int EQ>
hipError_t launch_stage_batch(const BatchLaunch &b, bool buf, int nin, int64_t grid, hipStream_t s)
{
    if (nin < 0 || nin > 2) return hipErrorInvalidValue;
    if (buf)
        launch_stage_batch_nin<real, DIM, N, EQ, true>(b, nin, grid, s);
    else
        launch_stage_batch_nin<real, DIM, N, EQ, false>(b, nin, grid, s);
    return hipGetLastError();
}

template <typename real, int DIM, int N, int EQ>
hipError_t launch_stage_x(const StageParams &p, const ExtraIn &x, int64_t grid, hipStream_t s)
{
    const int64_t bytes = p.stride * Vars<EQ, DIM>::NV * (int64_t)sizeof(real);
    if (bytes < (int64_t(1) << 31))
        hipLaunchKernelGGL((stage_kernel_x<real, DIM, N, EQ, true>), dim3((unsigned)grid),
                           dim3(Geo<DIM, N, EQ>::THREADS), 0, s, p, x);
    else
        hipLaunchKernelGGL((stage_kernel_x<real, DIM, N, EQ, false>), dim3((unsigned)grid),
                           dim3(Geo<DIM, N, EQ>::THREADS), 0, s, p, x);
    return hipGetLastError();
}

template <typename real, int DIM, int EQ>
StageXFn pick_stage_x_n(int N)
{
    switch (N) {
    case 1: return &launch_stage_x<real, DIM, 1, EQ>;
    case 2: return &launch_stage_x<real, DIM, 2, EQ>;
    case 3: return &launch_stage_x<real, DIM, 3, EQ>;
    case 4: return &launch_stage_x<real, DIM, 4, EQ>;
    case 5: return &launch_stage_x<real, DIM, 5, EQ>;
    case 6: return &launch_stage_x<real, DIM, 6, EQ>;
    case 7: return &launch_stage_x<real, DIM, 7, EQ>;
    case 8: return &launch_stage_x<real, DIM, 8, EQ>;
    default: return nullptr;
    }
}

template <typename real, int DIM, int EQ>
BatchFn pick_batch_n(int N)
{
    switch (N) {
    case 1: return &launch_stage_batch<real, DIM, 1, EQ>;
    case 2: return &launch_stage_batch<real, DIM, 2, EQ>;
    case 3: return &launch_stage_batch<real, DIM, 3, EQ>;
    case 4: return &launch_stage_batch<real, DIM, 4, EQ>;
    case 5: return &launch_stage_batch<real, DIM, 5, EQ>;
    case 6: return &launch_stage_batch<real, DIM, 6, EQ>;
    case 7: return &launch_stage_batch<real, DIM, 7, EQ>;
    case 8: return &launch_stage_batch<real, DIM, 8, EQ>;
    default: return nullptr;
    }
}

template <typename real, int DIM, int EQ>
BatchXFn pick_batch_x_n(int N)
{
    switch (N) {
    case 1: return &launch_stage_batch_x<real, DIM, 1, EQ>;
    case 2: return &launch_stage_batch_x<real, DIM, 2, EQ>;
    case 3: return &launch_stage_batch_x<real, DIM, 3, EQ>;
    case 4: return &launch_stage_batch_x<real, DIM, 4, EQ>;
    case 5: return &launch_stage_batch_x<real, DIM, 5, EQ>;
    case 6: return &launch_stage_batch_x<real, DIM, 6, EQ>;
    case 7: return &launch_stage_batch_x<real, DIM, 7, EQ>;
    case 8: return &launch_stage_batch_x<real, DIM, 8, EQ>;
    default: return nullptr;
    }
}

template <typename real, int DIM, int EQ>
StageFn pick_stage_n(int N)
{
    switch (N) {
    case 1: return &launch_stage<real, DIM, 1, EQ>;
    case 2: return &launch_stage<real, DIM, 2, EQ>;
    case 3: return &launch_stage<real, DIM, 3, EQ>;
    case 4: return &launch_stage<real, DIM, 4, EQ>;
    case 5: return &launch_stage<real, DIM, 5, EQ>;
    case 6: return &launch_stage<real, DIM, 6, EQ>;
    case 7: return &launch_stage<real, DIM, 7, EQ>;
    case 8: return &launch_stage<real, DIM, 8, EQ>;
    default: return nullptr;
    }
}

}  // namespace dg
