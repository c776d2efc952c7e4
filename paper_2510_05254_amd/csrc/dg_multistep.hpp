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
// four RK arrays in LDS and runs all stages of `nsteps` steps there, with one
// barrier per stage, so HBM sees one read and one write of U per launch
// instead of 3.5 array passes per stage, and the step loop issues one launch
// per `nsteps` steps instead of one per stage.
//   whole mode:   the workgroup holds the entire periodic mesh; neighbours
//                 wrap inside LDS; any number of steps per launch.
//   chunked mode: the workgroup owns T consecutive elements and loads a halo
//                 of H = stages * nsteps elements on each side. The RHS of an
//                 element needs its two neighbours, so the range on which a
//                 stage's result is valid shrinks by one element per side per
//                 stage; after nsteps steps exactly the owned elements are
//                 valid and are written back. Halo work is redundant: every
//                 copy of an element computes the same values.
// Both sides of a face evaluate Fhat from the same (lower, upper) trace pair
// with contraction off, so they get the same bits and the scheme conserves
// to roundoff.
#pragma once

#include "dg_internal.hpp"

namespace dg {
namespace ms {

template <typename real, int N, int EQ>
struct Geo1 {
    static constexpr int N1 = N + 1;
    static constexpr int NV = EQ == 0 ? 1 : 2;
    // one thread per element: an element's nodes sit at an odd stride S >= N+1
    // (in doubles) so lanes reading element-strided LDS hit distinct banks
    static constexpr int S = (N1 % 2) ? N1 : N1 + 1;
    static constexpr int PER_ELEM = 4 * NV * S * (int)sizeof(real);    // U, A, Ya, Yb
    static constexpr int BUDGET = 80 * 1024 - N1 * N1 * (int)sizeof(real);
    // elements held (a multiple of 64); threads take one element per pass
    static constexpr int CAP_E = ((BUDGET / PER_ELEM) / 64) * 64;
    static constexpr int THREADS = CAP_E < 256 ? CAP_E : 256;
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

template <typename real, int N, int EQ>
__global__ void __launch_bounds__((Geo1<real, N, EQ>::THREADS)) ms1_kernel(const MsLaunch l)
{
    using G = Geo1<real, N, EQ>;
    constexpr int N1 = G::N1, NV = G::NV, S = G::S, CAP_E = G::CAP_E, THREADS = G::THREADS;
    constexpr real INVW0 = real(N * (N + 1)) / real(2);    // 1/w_0 = 1/w_N
    __shared__ real sA[4][NV][CAP_E * S];                   // U, A, Ya, Yb
    __shared__ real sD[N1 * N1];

    const int tid = threadIdx.x;
    uint32_t s = 0, chunk = blockIdx.x;
    if (l.solves) {
        s = l.wg_solve[blockIdx.x];
        chunk = blockIdx.x - l.wg_base[s];
    }
    const MsSolve *P = l.solves ? l.solves + s : &l.one;
    real *U = static_cast<real *>(P->U);
    const int64_t K = P->K;
    const bool whole = P->whole != 0;
    const int stages = l.prog.stages;
    const int H = whole ? 0 : stages * l.nsteps;
    const int64_t own0 = whole ? 0 : int64_t(chunk) * P->T;
    const int town = int(whole ? K : (K - own0 < P->T ? K - own0 : P->T));
    const int L = town + 2 * H;                             // local elements
    const int64_t gfirst = own0 - H;                        // global element of local 0
    const real par = real(P->par), rdx2 = real(P->rdx2);
    const real sl = rdx2 * INVW0;

    if (tid < N1 * N1) sD[tid] = static_cast<const real *>(l.D)[tid];
    // ---- load U over the local range (node-parallel, coalesced; periodic
    // wrap by one period at most)
    for (int idx = tid; idx < L * N1; idx += THREADS) {
        const int le = idx / N1, i = idx - le * N1;
        int64_t ge = gfirst + le;
        if (ge < 0) ge += K;
        if (ge >= K) ge -= K;
#pragma unroll
        for (int v = 0; v < NV; ++v) sA[0][v][le * S + i] = U[(ge * NV + v) * N1 + i];
    }
    __syncthreads();

    int a = 0, b = L;          // elements on which the current stage input is valid
    for (int step = 0; step < l.nsteps; ++step) {
        for (int st = 0; st < stages; ++st) {
            const int yi = l.prog.yin[st], nin = l.prog.nin[st], nout = l.prog.nout[st];
            const int i0 = l.prog.in0[st], i1 = l.prog.in1[st];
            const int lo = whole ? 0 : a + 1, hi = whole ? L : b - 1;
            real cy[2], c0[2], c1[2], cr[2];
            int oi[2];
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                cy[o] = real(P->coef[st][o][0]);
                c0[o] = real(P->coef[st][o][1]);
                c1[o] = real(P->coef[st][o][2]);
                cr[o] = real(P->coef[st][o][3]);
                oi[o] = l.prog.out[st][o];
            }
            for (int le = lo + tid; le < hi; le += THREADS) {
                const int base = le * S;
                // the element's stage input and fluxes, in registers
                real u[N1][NV], F[N1][NV], lam0, lamN;
#pragma unroll
                for (int m = 0; m < N1; ++m) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) u[m][v] = sA[yi][v][base + m];
                    real lam;
                    flux1<real, EQ>(u[m], par, F[m], lam);
                    if (m == 0) lam0 = lam;
                    if (m == N) lamN = lam;
                }
                // volume term
                real R[N1][NV];
#pragma unroll
                for (int i = 0; i < N1; ++i) {
                    real acc[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[v] = real(0);
#pragma unroll
                    for (int m = 0; m < N1; ++m) {
                        const real dm = sD[i * N1 + m];
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[v] += dm * (EQ == 0 ? u[m][v] : F[m][v]);
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[i][v] = real(0);
                    if constexpr (EQ == 0) {
                        R[i][0] -= rdx2 * (par * acc[0]);
                    } else {
#pragma unroll
                        for (int v = 0; v < NV; ++v) R[i][v] -= rdx2 * acc[v];
                    }
                }
                // lower face (with element le-1) and upper face (with le+1);
                // each face is evaluated by both elements from the same
                // (lower, upper) pair
                {
                    const int ln = le == 0 ? L - 1 : le - 1;       // chunked: le >= 1
                    const int un = le == L - 1 ? 0 : le + 1;       // chunked: le <= L-2
                    real Un[NV], Fn[NV], lamn, Fh[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) Un[v] = sA[yi][v][ln * S + N];
                    flux1<real, EQ>(Un, par, Fn, lamn);
                    lf_flux<real, NV>(Un, Fn, lamn, u[0], F[0], lam0, Fh);
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[0][v] += sl * (Fh[v] - F[0][v]);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Un[v] = sA[yi][v][un * S];
                    flux1<real, EQ>(Un, par, Fn, lamn);
                    lf_flux<real, NV>(u[N], F[N], lamN, Un, Fn, lamn, Fh);
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[N][v] += -sl * (Fh[v] - F[N][v]);
                }
                // RK stage combination
#pragma unroll
                for (int i = 0; i < N1; ++i) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const real a0 = nin > 0 ? sA[i0][v][base + i] : real(0);
                        const real a1 = nin > 1 ? sA[i1][v][base + i] : real(0);
#pragma unroll
                        for (int o = 0; o < 2; ++o) {
                            if (o < nout) {
                                real val = cy[o] * u[i][v];
                                if (nin > 0) val += c0[o] * a0;
                                if (nin > 1) val += c1[o] * a1;
                                val += cr[o] * R[i][v];
                                sA[oi[o]][v][base + i] = val;
                            }
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
        const int le = idx / N1, i = idx - le * N1;
        const int64_t ge = gfirst + le;
#pragma unroll
        for (int v = 0; v < NV; ++v) U[(ge * NV + v) * N1 + i] = sA[0][v][le * S + i];
    }
}

template <typename real, int N, int EQ>
hipError_t launch_ms1(const MsLaunch &l, hipStream_t s)
{
    hipLaunchKernelGGL((ms1_kernel<real, N, EQ>), dim3(l.nwg), dim3(Geo1<real, N, EQ>::THREADS), 0, s, l);
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
