// dg_multistep.hpp -- temporally blocked 1-D NDG stepping for gfx950: one
// launch advances a 1-D solve by several whole RK3/RK4 steps.
//
// The arithmetic per node is that of the fused RHS + RK stage kernel
// (Sporykhin & Homann, arXiv:2510.05254, Sec. 2.1 strong form with the
// Lax-Friedrichs flux of eq. LF, Sec. 2.3 RK schedules): volume term
// -(2/dx) sum_m D_im F(U_m), lifts +-(2/dx)(1/w_0)(Fhat - F) at the two end
// nodes, and the same fused stage programs (out = cy y + c0 in0 + c1 in1 +
// cr R over the arrays U, A, Ya, Yb).
//
// What differs is where the arrays live. A workgroup keeps its elements'
// four RK arrays in LDS and runs all stages of `nsteps` steps there, in two
// phases per stage (the face fluxes, once per face, and for Euler the nodal
// fluxes; then every node), so HBM sees one read and one write of U per
// launch instead of 3.5 array passes per stage, and the step loop issues one
// launch per `nsteps` steps instead of one per stage. One thread owns one node
// (and keeps row i of D in registers); a workgroup of 1024 (or 512) threads
// covers 1024 / (N+1) elements per pass, so even a small mesh has N+1 times
// more threads in flight than elements. The RK3 and RK4 stage programs are
// compile-time constants (kMsProgRk3, kMsProgRk4).
//   whole mode:   the workgroup holds the entire periodic mesh; neighbours
//                 wrap inside LDS; any number of steps per launch.
//   chunked mode: the workgroup owns T consecutive elements and loads a halo
//                 of H = stages * nsteps elements on each side. The RHS of an
//                 element needs its two neighbours, so the range on which a
//                 stage's result is valid shrinks by one element per side per
//                 stage; after nsteps steps exactly the owned elements are
//                 valid and are written back. Halo work is redundant: every
//                 copy of an element computes the same values.
// Each face's Fhat is evaluated once (contraction off) and lifted into both
// of its elements, so the scheme conserves to roundoff.
#pragma once

#include "dg_internal.hpp"

namespace dg {
namespace ms {

template <typename real, int N, int EQ>
struct Geo1 {
    static constexpr int N1 = N + 1;
    static constexpr int NV = EQ == 0 ? 1 : 2;
    // an element's nodes sit at an odd stride S >= N+1 (in reals) so that
    // lanes reading one node of consecutive elements hit distinct banks
    static constexpr int S = (N1 % 2) ? N1 : N1 + 1;
    // U, A, Ya, Yb, and for Euler the nodal fluxes of the stage input; one
    // face flux per element
    static constexpr int NARR = EQ == 0 ? 4 : 5;
    static constexpr int PER_ELEM = NARR * NV * S * (int)sizeof(real) + NV * (int)sizeof(real);
    // elements held: two workgroups share a CU's 160 KiB of LDS (512 bytes
    // stay for the stage coefficients and the last face)
    static constexpr int CAP_E = (80 * 1024 - 512) / PER_ELEM;
    // 1024 threads in at most 64 VGPRs (two workgroups, eight waves per SIMD)
    // where the kernel fits in them without spilling, else 512 threads in at
    // most 128 VGPRs; a multiple of N+1, so a thread keeps its node on every
    // pass
    static constexpr bool BIG = sizeof(real) == 4 ? (EQ == 0 || N <= 6) : (EQ == 0 && N <= 7);
    static constexpr int WAVES = BIG ? 8 : 4;
    static constexpr int THREADS = N1 * ((BIG ? 1024 : 512) / N1);
    static constexpr int EPP = THREADS / N1;                           // elements per pass
    // advection meshes held whole take a one-barrier stage (where the extra
    // code path fits the register budget without spilling)
    static constexpr bool WHOLE1 = EQ == 0 && (sizeof(real) == 4 || N <= 4);
};

__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// A value that is the same in every lane, moved to scalar registers (the
// per-solve constants are read through a generic pointer, which would
// otherwise hold them in vector registers).
__device__ __forceinline__ float uni(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uni(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// physical flux and wave speed of a 1-D state (advection: a u; isothermal
// Euler: (m, m^2/rho + rho c^2), |m/rho| + c)
template <typename real, int EQ>
__device__ __forceinline__ void flux1(const real *U, real par, real *F, real &lam)
{
#pragma clang fp contract(off)
    if constexpr (EQ == 0) {
        F[0] = par * U[0];
        lam = fabs(par);
    } else {
        const real rinv = rcp_nr(U[0]);
        F[0] = U[1];
        F[1] = U[1] * (U[1] * rinv) + U[0] * (par * par);
        lam = fabs(U[1] * rinv) + par;
    }
}

// eq. LF with (U^-, U^+) = (lower, upper): Fhat = 1/2 [(F^- + F^+) - alpha (U^+ - U^-)]
template <typename real, int NV>
__device__ __forceinline__ void lf_flux(const real *UL, const real *FL, real lamL, const real *UR,
                                        const real *FR, real lamR, real *Fh)
{
#pragma clang fp contract(off)
    const real alpha = lamL > lamR ? lamL : lamR;
#pragma unroll
    for (int v = 0; v < NV; ++v) Fh[v] = real(0.5) * ((FL[v] + FR[v]) - alpha * (UR[v] - UL[v]));
}

template <typename real, int N, int EQ, int RK>
__global__ void __launch_bounds__((Geo1<real, N, EQ>::THREADS)) __attribute__((amdgpu_waves_per_eu(Geo1<real, N, EQ>::WAVES)))
ms1_kernel(const MsLaunch l)
{
    using G = Geo1<real, N, EQ>;
    constexpr int N1 = G::N1, NV = G::NV, S = G::S, CAP_E = G::CAP_E, THREADS = G::THREADS;
    constexpr int EPP = G::EPP;
    constexpr MsProgram PG = RK == 4 ? kMsProgRk4 : kMsProgRk3;
    constexpr real INVW0 = real(N * (N + 1)) / real(2);    // 1/w_0 = 1/w_N
    __shared__ real sA[4][NV][CAP_E * S];                   // U, A, Ya, Yb
    __shared__ real sF[EQ == 0 ? 1 : NV][EQ == 0 ? 1 : CAP_E * S];
    __shared__ real sH[NV][CAP_E + 1];                      // Fhat of face f (elements f-1, f)
    __shared__ real sC[4][2][4];                            // stage coefficients cy, c0, c1, cr

    const int tid = threadIdx.x;
    const int i = tid % N1, e0 = tid / N1;                  // this thread's node, first element
    uint32_t s = 0, chunk = blockIdx.x;
    if (l.solves) {
        s = l.wg_solve[blockIdx.x];
        chunk = blockIdx.x - l.wg_base[s];
    }
    const MsSolve *P = l.solves ? l.solves + s : &l.one;
    const real *Uin = static_cast<const real *>(l.flip ? P->V : P->U);
    real *Uout = static_cast<real *>(l.flip ? P->U : P->V);
    const int64_t K = P->K;
    const bool whole = P->whole != 0;
    const int H = whole ? 0 : PG.stages * l.nsteps;
    const int64_t own0 = whole ? 0 : int64_t(chunk) * P->T;
    const int town = int(whole ? K : (K - own0 < P->T ? K - own0 : P->T));
    const int L = town + 2 * H;                             // local elements
    const int64_t gfirst = own0 - H;                        // global element of local 0
    const real par = uni(real(P->par)), rdx2 = uni(real(P->rdx2));
    const real sl = rdx2 * INVW0;
    // lift weight and face of this thread's node: node 0 lifts +sl from face
    // le, node N -sl from face le + 1, interior nodes nothing
    const real lw = i == 0 ? sl : (i == N ? -sl : real(0));
    const int fo = i == N ? 1 : 0;

    // the stage coefficients, read once
    if (tid < 32) sC[tid >> 3][(tid >> 2) & 1][tid & 3] = real(P->coef[tid >> 3][(tid >> 2) & 1][tid & 3]);
    real d[N1];                                             // row i of D
#pragma unroll
    for (int m = 0; m < N1; ++m) d[m] = static_cast<const real *>(l.D)[i * N1 + m];
    // ---- load U over the local range (node-parallel, coalesced; periodic
    // wrap by one period at most)
    for (int idx = tid; idx < L * N1; idx += THREADS) {
        const int le = idx / N1, n = idx - le * N1;
        int64_t ge = gfirst + le;
        if (ge < 0) ge += K;
        if (ge >= K) ge -= K;
#pragma unroll
        for (int v = 0; v < NV; ++v) sA[0][v][le * S + n] = Uin[(ge * NV + v) * N1 + n];
    }
    __syncthreads();

    int a = 0, b = L;          // elements on which the current stage input is valid
    for (int step = 0; step < l.nsteps; ++step) {
#pragma unroll
        for (int st = 0; st < PG.stages; ++st) {
            const int yi = PG.yin[st], nin = PG.nin[st], nout = PG.nout[st];
            const int i0 = PG.in0[st], i1 = PG.in1[st];
            const int lo = whole ? 0 : a + 1, hi = whole ? L : b - 1;
            real cy[2], c0[2], c1[2], cr[2];
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                cy[o] = uni(sC[st][o][0]);
                c0[o] = uni(sC[st][o][1]);
                c1[o] = uni(sC[st][o][2]);
                cr[o] = uni(sC[st][o][3]);
            }
            if constexpr (G::WHOLE1) {
                if (whole) {
                    // a whole advection mesh: each end node evaluates its face
                    // itself from the face's (lower, upper) pair (the bits of
                    // the face phase), so the stage needs one barrier
                    for (int le = e0; le < L; le += EPP) {
                        const int base = le * S;
                        real acc = real(0);
#pragma unroll
                        for (int m = 0; m < N1; ++m) acc += d[m] * sA[yi][0][base + m];
                        real u[1] = {sA[yi][0][base + i]}, R = real(0), F[1], lam;
                        R -= rdx2 * (par * acc);
                        flux1<real, EQ>(u, par, F, lam);
                        real Fh[1] = {F[0]};
                        if (i == 0 || i == N) {
                            const int el = i == 0 ? (le == 0 ? L - 1 : le - 1) : le;
                            const int eu = i == 0 ? le : (le == L - 1 ? 0 : le + 1);
                            real UL[1] = {sA[yi][0][el * S + N]}, UR[1] = {sA[yi][0][eu * S]};
                            real FL[1], FR[1], lamL, lamR;
                            flux1<real, EQ>(UL, par, FL, lamL);
                            flux1<real, EQ>(UR, par, FR, lamR);
                            lf_flux<real, 1>(UL, FL, lamL, UR, FR, lamR, Fh);
                        }
                        R += lw * (Fh[0] - F[0]);
                        const real a0 = nin > 0 ? sA[i0][0][base + i] : real(0);
                        const real a1 = nin > 1 ? sA[i1][0][base + i] : real(0);
#pragma unroll
                        for (int o = 0; o < 2; ++o) {
                            if (o < nout) {
                                real val = cy[o] * u[0];
                                if (nin > 0) val += c0[o] * a0;
                                if (nin > 1) val += c1[o] * a1;
                                val += cr[o] * R;
                                sA[PG.out[st][o]][0][base + i] = val;
                            }
                        }
                    }
                    __syncthreads();
                    continue;
                }
            }
            // ---- phase 1: eq. LF on every face the stage needs, once per face
            // from its (lower, upper) pair (face f joins elements f-1 and f;
            // whole mode: faces 0..L-1, face 0 wrapping to element L-1), and
            // for Euler the nodal fluxes of the stage input
            const int fhi = whole ? L - 1 : hi;
            for (int f = lo + tid; f <= fhi; f += THREADS) {
                const int el = f == 0 ? L - 1 : f - 1;
                real UL[NV], UR[NV], FL[NV], FR[NV], lamL, lamR, Fh[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    UL[v] = sA[yi][v][el * S + N];
                    UR[v] = sA[yi][v][f * S];
                }
                flux1<real, EQ>(UL, par, FL, lamL);
                flux1<real, EQ>(UR, par, FR, lamR);
                lf_flux<real, NV>(UL, FL, lamL, UR, FR, lamR, Fh);
#pragma unroll
                for (int v = 0; v < NV; ++v) sH[v][f] = Fh[v];
            }
            if constexpr (EQ != 0) {
                for (int le = lo + e0; le < hi; le += EPP) {
                    real u[NV], F[NV], lam;
#pragma unroll
                    for (int v = 0; v < NV; ++v) u[v] = sA[yi][v][le * S + i];
                    flux1<real, EQ>(u, par, F, lam);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sF[v][le * S + i] = F[v];
                }
            }
            __syncthreads();
            // ---- phase 2: node i of each element
            for (int le = lo + e0; le < hi; le += EPP) {
                const int base = le * S;
                // volume term: -(2/dx) sum_m D_im F(U_m)
                real acc[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = real(0);
#pragma unroll
                for (int m = 0; m < N1; ++m) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[v] += d[m] * (EQ == 0 ? sA[yi][v][base + m] : sF[v][base + m]);
                }
                real R[NV], u[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    R[v] = real(0);
                    u[v] = sA[yi][v][base + i];
                }
                if constexpr (EQ == 0) {
                    R[0] -= rdx2 * (par * acc[0]);
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[v] -= rdx2 * acc[v];
                }
                // lifts at the end nodes: +-(2/dx)(1/w_0)(Fhat - F), taken by
                // every lane without a branch (lw = 0 off the end nodes)
                {
                    real F[NV];
                    if constexpr (EQ == 0) {
                        real lam;
                        flux1<real, EQ>(u, par, F, lam);
                    } else {
#pragma unroll
                        for (int v = 0; v < NV; ++v) F[v] = sF[v][base + i];
                    }
                    int fi = le + fo;
                    fi = whole && fi == L ? 0 : fi;
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[v] += lw * (sH[v][fi] - F[v]);
                }
                // RK stage combination at node i (the outputs never alias the
                // stage input; an output that is also an input is this node's)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const real a0 = nin > 0 ? sA[i0][v][base + i] : real(0);
                    const real a1 = nin > 1 ? sA[i1][v][base + i] : real(0);
#pragma unroll
                    for (int o = 0; o < 2; ++o) {
                        if (o < nout) {
                            real val = cy[o] * u[v];
                            if (nin > 0) val += c0[o] * a0;
                            if (nin > 1) val += c1[o] * a1;
                            val += cr[o] * R[v];
                            sA[PG.out[st][o]][v][base + i] = val;
                        }
                    }
                }
            }
            __syncthreads();
            if (!whole) {
                ++a;
                --b;
            }
        }
    }
    // ---- write back the owned elements
    for (int idx = H * N1 + tid; idx < (H + town) * N1; idx += THREADS) {
        const int le = idx / N1, n = idx - le * N1;
        const int64_t ge = gfirst + le;
#pragma unroll
        for (int v = 0; v < NV; ++v) Uout[(ge * NV + v) * N1 + n] = sA[0][v][le * S + n];
    }
}

template <typename real, int N, int EQ>
hipError_t launch_ms1(const MsLaunch &l, hipStream_t s)
{
    if (l.rk == 3)
        hipLaunchKernelGGL((ms1_kernel<real, N, EQ, 3>), dim3(l.nwg), dim3(Geo1<real, N, EQ>::THREADS), 0, s, l);
    else
        hipLaunchKernelGGL((ms1_kernel<real, N, EQ, 4>), dim3(l.nwg), dim3(Geo1<real, N, EQ>::THREADS), 0, s, l);
    return hipGetLastError();
}

template <typename real, int EQ>
MsFn pick_ms1(int N)
{
    switch (N) {
    case 1: return &launch_ms1<real, 1, EQ>;
    case 2: return &launch_ms1<real, 2, EQ>;
    case 3: return &launch_ms1<real, 3, EQ>;
    case 4: return &launch_ms1<real, 4, EQ>;
    case 5: return &launch_ms1<real, 5, EQ>;
    case 6: return &launch_ms1<real, 6, EQ>;
    case 7: return &launch_ms1<real, 7, EQ>;
    case 8: return &launch_ms1<real, 8, EQ>;
    default: return nullptr;
    }
}

template <typename real, int EQ>
int cap1(int N)
{
    switch (N) {
#define DG_CASE(n) \
    case n: return Geo1<real, n, EQ>::CAP_E;
        DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return 0;
    }
}

}  // namespace ms
}  // namespace dg
