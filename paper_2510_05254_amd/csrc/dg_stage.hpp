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
// Lax-Friedrichs flux of eq. LF from the (lower, upper) traces of each face,
// periodic neighbours, and w_0 = w_N = 2/(N(N+1)). The RK stage update is
// applied in the same pass (StageParams).
//
// Work decomposition (MI355X-specific, not from the paper):
//  - a workgroup takes a tile of EPB consecutive elements along x, one thread
//    per node, variables in registers; the canonical layout u[v][e][n] makes
//    each variable of a tile one contiguous, coalesced run;
//  - the state of the tile and, for Euler, the symmetric momentum-flux tensor
//    m_d u_k + delta_dk rho c^2 (dim(dim+1)/2 arrays instead of dim*nvar) are
//    staged in LDS; the D contractions read them there, D itself sits in LDS;
//  - face traces of x-neighbours inside the tile come from LDS, all other
//    neighbour traces from global memory (L2-resident: see the tile order);
//  - tiles are ordered so that each XCD (private L2) sweeps a compact region:
//    virtual block b runs on XCD b % 8, and tile index L is remapped so XCD x
//    owns a contiguous range of L; in 3-D the L order is x-tile fastest, then
//    z inside a slab of `slab` layers, then y, then slab, which keeps the
//    y- and z-neighbours of a tile within a short window of recent tiles.
#pragma once

#include "dg_internal.hpp"

namespace dg {

template <int DIM, int N>
struct Shape {
    static constexpr int N1 = N + 1;
    static constexpr int NP = DIM == 1 ? N1 : (DIM == 2 ? N1 * N1 : N1 * N1 * N1);
    static constexpr int EPB = (256 / NP) < 1 ? 1 : (256 / NP);
    static constexpr int THREADS = ((EPB * NP + 63) / 64) * 64;
};

template <int EQ, int DIM>
struct Vars {
    static constexpr int NV = EQ == 0 ? 1 : 1 + DIM;
    static constexpr int NSYM = EQ == 0 ? 0 : DIM * (DIM + 1) / 2;
};

// index of the symmetric pair (d, k) in the packed momentum-flux tensor
__device__ __forceinline__ constexpr int sym_index(int d, int k, int dim)
{
    const int a = d < k ? d : k, b = d < k ? k : d;
    // row-major upper triangle: (0,0)..(0,dim-1),(1,1)..
    return a * dim - (a * (a - 1)) / 2 + (b - a);
}

// Physical flux along D of state U and its largest absolute eigenvalue.
template <typename real, int EQ, int DIM, int D>
__device__ __forceinline__ void flux_and_speed(const real *U, const real *par, real *F, real &lam)
{
    if constexpr (EQ == 0) {
        F[0] = par[D] * U[0];
        lam = fabs(par[D]);
    } else {
        const real c = par[0];
        const real rinv = real(1) / U[0];
        F[0] = U[1 + D];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            real f = U[1 + D] * (U[1 + k] * rinv);
            if (k == D) f += U[0] * (c * c);
            F[1 + k] = f;
        }
        lam = fabs(U[1 + D] * rinv) + c;
    }
}

// Lax-Friedrichs flux (eq. LF) from the lower trace UL and upper trace UR.
// Both elements sharing a face call this with the same (UL, UR), so the two
// sides get bitwise-identical Fhat and the scheme conserves to roundoff.
template <typename real, int EQ, int DIM, int D>
__device__ __forceinline__ void lf_flux(const real *UL, const real *UR, const real *par, real *Fh)
{
    constexpr int NV = Vars<EQ, DIM>::NV;
    real FL[NV], FR[NV], aL, aR;
    flux_and_speed<real, EQ, DIM, D>(UL, par, FL, aL);
    flux_and_speed<real, EQ, DIM, D>(UR, par, FR, aR);
    const real alpha = aL > aR ? aL : aR;
#pragma unroll
    for (int v = 0; v < NV; ++v) Fh[v] = real(0.5) * ((FL[v] + FR[v]) - alpha * (UR[v] - UL[v]));
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t x = b % kXcds, j = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + j;
}

template <int DIM>
__device__ __forceinline__ void tile_coords(int64_t L, const StageParams &p, int64_t &tx,
                                            int64_t &ey, int64_t &ez)
{
    if constexpr (DIM == 1) {
        tx = L; ey = 0; ez = 0;
    } else if constexpr (DIM == 2) {
        tx = L % p.tiles_x; ey = L / p.tiles_x; ez = 0;
    } else {
        tx = L % p.tiles_x;
        int64_t r = L / p.tiles_x;
        const int64_t zs = r % p.slab;
        r /= p.slab;
        ey = r % p.K[1];
        ez = (r / p.K[1]) * p.slab + zs;
    }
}

template <int DIM, int N, int D>
__device__ __forceinline__ int node_with(const int *ijk, int val)
{
    constexpr int N1 = N + 1;
    int q[3] = {ijk[0], ijk[1], ijk[2]};
    q[D] = val;
    if constexpr (DIM == 1) return q[0];
    else if constexpr (DIM == 2) return q[0] + N1 * q[1];
    else return q[0] + N1 * (q[1] + N1 * q[2]);
}

template <typename real, int DIM, int N, int EQ>
__global__ void __launch_bounds__((Shape<DIM, N>::THREADS))
stage_kernel(const StageParams p)
{
    using S = Shape<DIM, N>;
    constexpr int N1 = S::N1, NP = S::NP, EPB = S::EPB, TN = EPB * NP;
    constexpr int NV = Vars<EQ, DIM>::NV, NSYM = Vars<EQ, DIM>::NSYM;
    constexpr real INVW0 = real(N * (N + 1)) / real(2);   // 1/w_0 = 1/w_N

    __shared__ real sY[NV][TN];
    __shared__ real sP[NSYM > 0 ? NSYM : 1][TN];
    __shared__ real sD[N1 * N1];

    const real *yin = static_cast<const real *>(p.yin);
    const real *in0 = static_cast<const real *>(p.in0);
    const real *in1 = static_cast<const real *>(p.in1);
    real *out0 = static_cast<real *>(p.out0);
    real *out1 = static_cast<real *>(p.out1);
    const int64_t stride = p.stride;

    real par[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) par[d] = real(p.par[d]);
    real rdx2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) rdx2[d] = real(p.rdx2[d]);

    const int tid = threadIdx.x;
    if (tid < N1 * N1) sD[tid] = static_cast<const real *>(p.D)[tid];

    const int slot = tid / NP;
    const int n = tid - slot * NP;
    int ijk[3];
    ijk[0] = n % N1;
    ijk[1] = DIM > 1 ? (n / N1) % N1 : 0;
    ijk[2] = DIM > 2 ? n / (N1 * N1) : 0;

    for (int64_t vb = blockIdx.x; vb < p.ntiles; vb += gridDim.x) {
        const int64_t L = xcd_remap(vb, p.ntiles);
        int64_t tx, ey, ez;
        tile_coords<DIM>(L, p, tx, ey, ez);
        const int64_t ex = tx * EPB + slot;
        const bool active = slot < EPB && ex < p.K[0];
        const int64_t ec[3] = {ex, ey, ez};
        const int64_t e = ex + p.K[0] * (ey + p.K[1] * ez);
        const int64_t gi = e * NP + n;

        real y[NV], a0[NV], a1[NV];
        // neighbour traces fetched from global memory: tr[d][v]
        real tr[DIM][NV];
        bool glob[DIM];
        if (active) {
#pragma unroll
            for (int v = 0; v < NV; ++v) y[v] = yin[v * stride + gi];
            if (p.nin > 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v) a0[v] = in0[v * stride + gi];
            }
            if (p.nin > 1) {
#pragma unroll
                for (int v = 0; v < NV; ++v) a1[v] = in1[v * stride + gi];
            }
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const int id = ijk[d];
                const bool lo = id == 0, hi = id == N;
                glob[d] = false;
                if (lo || hi) {
                    int64_t c = ec[d] + (hi ? 1 : -1);
                    if (c < 0) c += p.K[d];
                    if (c >= p.K[d]) c -= p.K[d];
                    bool in_tile = false;
                    if (d == 0) in_tile = (c / EPB) == tx;
                    if (!in_tile) {
                        glob[d] = true;
                        int64_t cc[3] = {ec[0], ec[1], ec[2]};
                        cc[d] = c;
                        const int64_t enb = cc[0] + p.K[0] * (cc[1] + p.K[1] * cc[2]);
                        int nn;
                        if (d == 0) nn = node_with<DIM, N, 0>(ijk, hi ? 0 : N);
                        else if (d == 1) nn = node_with<DIM, N, (DIM > 1 ? 1 : 0)>(ijk, hi ? 0 : N);
                        else nn = node_with<DIM, N, (DIM > 2 ? 2 : 0)>(ijk, hi ? 0 : N);
                        const int64_t gn = enb * NP + nn;
#pragma unroll
                        for (int v = 0; v < NV; ++v) tr[d][v] = yin[v * stride + gn];
                    }
                }
            }
        }

        // stage state and fluxes in LDS
        const int ln = slot * NP + n;
        real Fown[DIM][NV];
        if (active) {
#pragma unroll
            for (int v = 0; v < NV; ++v) sY[v][ln] = y[v];
            if constexpr (EQ == 0) {
#pragma unroll
                for (int d = 0; d < DIM; ++d) Fown[d][0] = par[d] * y[0];
            } else {
                const real c = par[0];
                const real rinv = real(1) / y[0];
                const real pr = y[0] * (c * c);
                real u[DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k) u[k] = y[1 + k] * rinv;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    Fown[d][0] = y[1 + d];
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        real f = y[1 + d] * u[k];
                        if (k == d) f += pr;
                        Fown[d][1 + k] = f;
                    }
                }
#pragma unroll
                for (int d = 0; d < DIM; ++d)
#pragma unroll
                    for (int k = d; k < DIM; ++k) sP[sym_index(d, k, DIM)][ln] = Fown[d][1 + k];
            }
        }
        __syncthreads();

        if (active) {
            real R[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) R[v] = real(0);
            const int base = slot * NP;

            // volume term: -(2/dx_d) sum_m D_{l_d m} F_d(..m..)
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const int id = ijk[d];
                const int sd = d == 0 ? 1 : (d == 1 ? N1 : N1 * N1);
                const int line0 = base + n - id * sd;   // node with l_d = 0 on this line
                real acc[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = real(0);
#pragma unroll
                for (int m = 0; m < N1; ++m) {
                    const real dm = sD[id * N1 + m];
                    const int q = line0 + m * sd;
                    if constexpr (EQ == 0) {
                        acc[0] += dm * sY[0][q];
                    } else {
                        acc[0] += dm * sY[1 + d][q];
#pragma unroll
                        for (int k = 0; k < DIM; ++k) acc[1 + k] += dm * sP[sym_index(d, k, DIM)][q];
                    }
                }
                if constexpr (EQ == 0) {
                    R[0] -= rdx2[d] * (par[d] * acc[0]);
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[v] -= rdx2[d] * acc[v];
                }
            }

            // face terms: Lax-Friedrichs flux and lift at l_d = 0 and l_d = N
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const int id = ijk[d];
                const bool lo = id == 0, hi = id == N;
                if (lo || hi) {
                    real unb[NV];
                    if (glob[d]) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) unb[v] = tr[d][v];
                    } else {
                        // x-neighbour inside this tile (d == 0 only)
                        int64_t c = ex + (hi ? 1 : -1);
                        if (c < 0) c += p.K[0];
                        if (c >= p.K[0]) c -= p.K[0];
                        const int nslot = int(c - tx * EPB);
                        const int nn = node_with<DIM, N, 0>(ijk, hi ? 0 : N);
#pragma unroll
                        for (int v = 0; v < NV; ++v) unb[v] = sY[v][nslot * NP + nn];
                    }
                    real UL[NV], UR[NV], Fh[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        UL[v] = lo ? unb[v] : y[v];
                        UR[v] = lo ? y[v] : unb[v];
                    }
                    if (d == 0) lf_flux<real, EQ, DIM, 0>(UL, UR, par, Fh);
                    else if (d == 1) lf_flux<real, EQ, DIM, (DIM > 1 ? 1 : 0)>(UL, UR, par, Fh);
                    else lf_flux<real, EQ, DIM, (DIM > 2 ? 2 : 0)>(UL, UR, par, Fh);
                    const real s = lo ? rdx2[d] * INVW0 : -rdx2[d] * INVW0;
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[v] += s * (Fh[v] - Fown[d][v]);
                }
            }

            // Runge-Kutta stage combination
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                if (o < p.nout) {
                    const real cy = real(p.cy[o]), c0 = real(p.c0[o]), c1 = real(p.c1[o]),
                               cr = real(p.cr[o]);
                    real *out = o == 0 ? out0 : out1;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        real val = cy * y[v];
                        if (p.nin > 0) val += c0 * a0[v];
                        if (p.nin > 1) val += c1 * a1[v];
                        val += cr * R[v];
                        out[v * stride + gi] = val;
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <typename real, int DIM, int N, int EQ>
hipError_t launch_stage(const StageParams &p, int64_t grid, hipStream_t s)
{
    hipLaunchKernelGGL((stage_kernel<real, DIM, N, EQ>), dim3((unsigned)grid),
                       dim3(Shape<DIM, N>::THREADS), 0, s, p);
    return hipGetLastError();
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
