// dg_internal.hpp -- types shared by the host runtime (dg_api.cpp) and the
// gfx950 kernels. Not part of the public ABI (include/dg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dg {

constexpr int kMaxN = 8;
constexpr int kMaxNP1 = kMaxN + 1;
constexpr int kXcds = 8;                 // MI355X: 8 accelerator complex dies
constexpr int64_t kMaxGrid = 1 << 20;    // launch cap; blocks loop beyond it
constexpr int kMaxExtraIn = 5;           // extra stage inputs (RK6 k-store)

// Unsigned 32-bit division by an invariant divisor d as a multiply-high, add
// and shift ("round-up" magic-number method, Granlund & Montgomery, PLDI 1994):
//   n / d = (umulhi(n, mul) + n) >> shift  for all n < 2^32,
// with shift = ceil(log2 d) and mul = floor(2^32 (2^shift - d) / d) + 1 (mod 2^32).
struct FastDiv {
    uint32_t div, mul, shift, pad;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return FastDiv{d, uint32_t(m), l, 0};
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv &f)
{
    const uint32_t hi = __umulhi(n, f.mul);
    return uint32_t((uint64_t(hi) + n) >> f.shift);
}

// Parameters of one fused RHS + Runge-Kutta stage launch.
//
// The kernel evaluates R = RHS(yin) (the NDG right-hand side: volume term,
// Lax-Friedrichs face flux and lift) and writes, for o < nout,
//   out_o = cy[o] * yin + c0[o] * in0 + c1[o] * in1 + cr[o] * R
// elementwise (terms with a zero count are skipped: in0 needs nin >= 1, in1
// needs nin >= 2). out_o may alias in0/in1 (each node is read before it is
// written, by the same thread) but never yin, which neighbouring elements
// read during the launch.
struct StageParams {
    const void *yin;
    const void *in0;
    const void *in1;
    void *out0;
    void *out1;
    double cy[2], c0[2], c1[2], cr[2];
    int nin, nout;
    int64_t K[3];          // elements per direction (1 for unused directions)
    int64_t stride;        // nodes = prod(K) * Np (distance between variables)
    double rdx2[3];        // 2 / dx_d = 2 K_d
    double par[3];         // advection a_d, or {c_s} for isothermal Euler
    const void *D;         // (N+1)^2 differentiation matrix, row-major, in the
                           // state's precision: D[i*(N+1)+m] = h_m'(xi_i)
    int64_t tiles_x;       // ceil(K[0] / elements per tile along x)
    int64_t tiles_y;       // ceil(K[1] / element rows per tile)
    int64_t slab;          // 3-D: z-layers per XCD slab (divides K[2])
    int64_t xblk;          // 3-D: x-tiles per x-block (divides tiles_x)
    int64_t ntiles;        // number of element tiles (virtual blocks)
    // 32-bit tile decoding: virtual block b runs on XCD b % 8; tiles are
    // renumbered L = x * xq + min(x, xr) + b / 8 so each XCD owns a contiguous
    // range, then L -> (x-tile, y-tile) in 2-D and (x-tile in x-block, z in
    // slab, y-tile, slab, x-block) in 3-D by the divisions below.
    uint32_t ntiles32, xq, xr;
    uint32_t plain_order;  // 1: tile L = virtual block (no XCD renumbering)
    uint32_t zlen;         // 3-D z-marching kernels: layers per unit (the
                           // decoded z is then a chunk index); 1 elsewhere
    FastDiv fd_tx, fd_slab, fd_ty, fd_xb, fd_nslab;
    const uint32_t *ftab;  // face-point descriptors of a tile (dg_tables.cpp)
};

// One batched stage launch over the solves of one kernel class.
struct BatchLaunch {
    const StageParams *params;   // per solve, this stage's parameters (device)
    const uint32_t *tile_solve;  // solve owning each virtual tile (device)
    const uint32_t *tile_base;   // first virtual tile of each solve (device)
    const void *D;               // differentiation matrix of the class (device)
    const uint32_t *ftab;        // face-point table of the class (device)
    const struct ExtraIn *extra; // per solve, this stage's further inputs (RK6; device)
    uint32_t ntiles, xq, xr, nsolves;
};

// Quadrature reductions (state element-interleaved, reference variable-major):
// per-block FP64 partial sums of
//   mode 0 (mass): sum q_n U_v
//   mode 1 (L2):   sum q_n (U_v - Uref_v)^2  and  sum q_n Uref_v^2
// with q_n = prod_d (dx_d/2) w_{n_d}.
struct ReduceParams {
    const void *u;
    const double *uref;
    double *partial;       // [block][2*nvar]
    const double *w;       // LGL weights, N+1
    double jac;            // prod_d dx_d/2
    int64_t stride;        // nodes
    int nvar, n1, np, dim, mode;
};

// Conversion between the ABI's variable-major layout and the device's
// element-interleaved layout (to_internal: variable-major src, interleaved
// dst; otherwise the reverse), with the precisions of the launch.
struct LayoutParams {
    const void *src;
    void *dst;
    int64_t nodes;         // nodes per variable
    int nvar, np;          // variables; nodes per element
    int to_internal;
};

// ---------------------------------------------------------------------------
// Temporally blocked 1-D stepping (dg_multistep.hpp): one launch advances
// 1-D solves by nsteps whole RK3/RK4 steps with the RK arrays held in LDS.
// Array indices in a program: 0 = U, 1 = A, 2 = Ya, 3 = Yb.
// ---------------------------------------------------------------------------
struct MsProgram {
    int stages;
    int8_t yin[4], nin[4], in0[4], in1[4], nout[4], out[4][2];
};
// The fused stage programs of the RK3 and RK4 schedules in those indices.
// The multi-step kernel takes them at compile time; the host uses that kernel
// only while its own stage programs equal these.
constexpr MsProgram kMsProgRk3 = {3, {0, 2, 3, 0}, {0, 1, 1, 0}, {0, 0, 1, 0}, {0, 0, 0, 0}, {2, 1, 1, 0},
                                  {{2, 1}, {3, 0}, {0, 0}, {0, 0}}};
constexpr MsProgram kMsProgRk4 = {4, {0, 3, 2, 3}, {0, 1, 2, 1}, {0, 0, 0, 1}, {0, 0, 1, 0}, {1, 2, 2, 1},
                                  {{3, 0}, {1, 2}, {1, 3}, {0, 0}}};

struct MsSolve {
    // The state, canonical layout, in two arrays: a launch reads one and
    // writes the other (MsLaunch::flip), so no workgroup reads a halo that a
    // neighbouring chunk has already advanced; V == U for a mesh held by one
    // workgroup, which reads everything before it writes.
    void *U;
    void *V;
    int64_t K;             // elements
    int64_t T;             // owned elements per workgroup (chunked mode)
    int whole;             // 1: one workgroup holds the whole periodic mesh
    int pad;
    double rdx2;           // 2 / dx
    double par;            // advection speed a, or sound speed c_s
    double coef[4][2][4];  // per stage and output: cy, c0, c1, cr
};

struct MsLaunch {
    const MsSolve *solves;     // device array (batched), or nullptr: use `one`
    const uint32_t *wg_solve;  // batched: solve of each workgroup
    const uint32_t *wg_base;   // batched: first workgroup of each solve
    const void *D;             // (N+1)^2 differentiation matrix (state precision)
    MsSolve one;
    int rk;                    // 3 or 4: the stage program kMsProgRk3 / kMsProgRk4
    uint32_t nwg;              // workgroups
    int nsteps;                // steps per launch (halo = stages * nsteps); 0: copy
    int flip;                  // 0: read U, write V; 1: read V, write U
};

typedef hipError_t (*MsFn)(const MsLaunch &l, hipStream_t s);
// Multi-step launcher for 1-D (precision, equation, N); nullptr if not built.
MsFn ms_fn(int precision, int equation, int N);
// Elements one multi-step workgroup holds in LDS (halo included).
int ms_capacity(int precision, int equation, int N);

// Further stage inputs of the fused RK6 stages (the stored k's), after
// in0/in1:  out_o += sum_{j < n} c[o][j] * in[j]  (zero coefficients skipped).
// A separate kernel argument, so the RK3/RK4 kernels do not carry it.
struct ExtraIn {
    const void *in[kMaxExtraIn];
    double c[2][kMaxExtraIn];
    int n;
};

typedef hipError_t (*StageFn)(const StageParams &p, int64_t grid, hipStream_t s);
typedef hipError_t (*StageXFn)(const StageParams &p, const ExtraIn &x, int64_t grid, hipStream_t s);
// nin: the stage's number of RK inputs, the same for every solve of the launch
typedef hipError_t (*BatchFn)(const BatchLaunch &b, bool buf, int nin, int64_t grid, hipStream_t s);
// batched stage with further inputs (fused RK6 stages; b.extra set)
typedef hipError_t (*BatchXFn)(const BatchLaunch &b, bool buf, int64_t grid, hipStream_t s);

// Stage launcher for (precision, equation, dim, N); nullptr if not built.
StageFn stage_fn(int precision, int equation, int dim, int N);
StageXFn stage_x_fn(int precision, int equation, int dim, int N);
BatchFn batch_fn(int precision, int equation, int dim, int N);
BatchXFn batch_x_fn(int precision, int equation, int dim, int N);
// Threads per block, elements per tile along x and element rows per tile of
// the stage kernel for (dim, N, equation).
int stage_threads(int dim, int N, int eq);
int stage_epb(int dim, int N, int eq);
int stage_epy(int dim, int N, int eq);

hipError_t launch_reduce(int precision, const ReduceParams &p, int64_t blocks, hipStream_t s);
hipError_t launch_layout(int to_precision, int from_precision, const LayoutParams &p, hipStream_t s);
// tile_solve[t] = j for tile_base[j] <= t < tile_base[j+1], j < nsolves
// (tile_base holds nsolves + 1 entries, the last one the total tile count).
hipError_t launch_fill_tile_map(const uint32_t *tile_base, uint32_t nsolves, uint32_t *tile_solve,
                                hipStream_t s);
constexpr int kReduceThreads = 256;

}  // namespace dg
