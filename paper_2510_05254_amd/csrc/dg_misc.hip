// dg_misc.hip -- stage-kernel dispatch, FP64 quadrature reductions (mass, L2),
// precision casts between the canonical FP64 layout and the state type, and
// the batch tile-map fill.
#include "dg_stage.hpp"

namespace dg {

StageFn stage_fn_f64_d1_adv(int N);
StageFn stage_fn_f64_d1_euler(int N);
StageFn stage_fn_f64_d2_adv(int N);
StageFn stage_fn_f64_d2_euler(int N);
StageFn stage_fn_f64_d3_adv(int N);
StageFn stage_fn_f64_d3_euler(int N);
StageFn stage_fn_f32_d1_adv(int N);
StageFn stage_fn_f32_d1_euler(int N);
StageFn stage_fn_f32_d2_adv(int N);
StageFn stage_fn_f32_d2_euler(int N);
StageFn stage_fn_f32_d3_adv(int N);
StageFn stage_fn_f32_d3_euler(int N);

StageXFn stage_x_fn_f64_d1_adv(int N);
StageXFn stage_x_fn_f64_d1_euler(int N);
StageXFn stage_x_fn_f64_d2_adv(int N);
StageXFn stage_x_fn_f64_d2_euler(int N);
StageXFn stage_x_fn_f64_d3_adv(int N);
StageXFn stage_x_fn_f64_d3_euler(int N);
StageXFn stage_x_fn_f32_d1_adv(int N);
StageXFn stage_x_fn_f32_d1_euler(int N);
StageXFn stage_x_fn_f32_d2_adv(int N);
StageXFn stage_x_fn_f32_d2_euler(int N);
StageXFn stage_x_fn_f32_d3_adv(int N);
StageXFn stage_x_fn_f32_d3_euler(int N);
BatchFn batch_fn_f64_d1_adv(int N);
BatchFn batch_fn_f64_d1_euler(int N);
BatchFn batch_fn_f64_d2_adv(int N);
BatchFn batch_fn_f64_d2_euler(int N);
BatchFn batch_fn_f64_d3_adv(int N);
BatchFn batch_fn_f64_d3_euler(int N);
BatchFn batch_fn_f32_d1_adv(int N);
BatchFn batch_fn_f32_d1_euler(int N);
BatchFn batch_fn_f32_d2_adv(int N);
BatchFn batch_fn_f32_d2_euler(int N);
BatchFn batch_fn_f32_d3_adv(int N);
BatchFn batch_fn_f32_d3_euler(int N);
BatchXFn batch_x_fn_f64_d1_adv(int N);
BatchXFn batch_x_fn_f64_d1_euler(int N);
BatchXFn batch_x_fn_f64_d2_adv(int N);
BatchXFn batch_x_fn_f64_d2_euler(int N);
BatchXFn batch_x_fn_f64_d3_adv(int N);
BatchXFn batch_x_fn_f64_d3_euler(int N);
BatchXFn batch_x_fn_f32_d1_adv(int N);
BatchXFn batch_x_fn_f32_d1_euler(int N);
BatchXFn batch_x_fn_f32_d2_adv(int N);
BatchXFn batch_x_fn_f32_d2_euler(int N);
BatchXFn batch_x_fn_f32_d3_adv(int N);
BatchXFn batch_x_fn_f32_d3_euler(int N);

MsFn ms_fn_f64_adv(int N);
MsFn ms_fn_f64_euler(int N);
MsFn ms_fn_f32_adv(int N);
MsFn ms_fn_f32_euler(int N);
int ms_cap_f64_adv(int N);
int ms_cap_f64_euler(int N);
int ms_cap_f32_adv(int N);
int ms_cap_f32_euler(int N);

MsFn ms_fn(int precision, int equation, int N)
{
    if (precision < 0 || precision > 1 || equation < 0 || equation > 1) return nullptr;
    if (precision == 0) return equation == 0 ? ms_fn_f64_adv(N) : ms_fn_f64_euler(N);
    return equation == 0 ? ms_fn_f32_adv(N) : ms_fn_f32_euler(N);
}

int ms_capacity(int precision, int equation, int N)
{
    if (precision < 0 || precision > 1 || equation < 0 || equation > 1) return 0;
    if (precision == 0) return equation == 0 ? ms_cap_f64_adv(N) : ms_cap_f64_euler(N);
    return equation == 0 ? ms_cap_f32_adv(N) : ms_cap_f32_euler(N);
}

BatchFn batch_fn(int precision, int equation, int dim, int N)
{
    typedef BatchFn (*Pick)(int);
    static const Pick table[2][3][2] = {
        {{batch_fn_f64_d1_adv, batch_fn_f64_d1_euler},
         {batch_fn_f64_d2_adv, batch_fn_f64_d2_euler},
         {batch_fn_f64_d3_adv, batch_fn_f64_d3_euler}},
        {{batch_fn_f32_d1_adv, batch_fn_f32_d1_euler},
         {batch_fn_f32_d2_adv, batch_fn_f32_d2_euler},
         {batch_fn_f32_d3_adv, batch_fn_f32_d3_euler}}};
    if (precision < 0 || precision > 1 || equation < 0 || equation > 1 || dim < 1 || dim > 3)
        return nullptr;
    return table[precision][dim - 1][equation](N);
}

BatchXFn batch_x_fn(int precision, int equation, int dim, int N)
{
    typedef BatchXFn (*Pick)(int);
    static const Pick table[2][3][2] = {
        {{batch_x_fn_f64_d1_adv, batch_x_fn_f64_d1_euler},
         {batch_x_fn_f64_d2_adv, batch_x_fn_f64_d2_euler},
         {batch_x_fn_f64_d3_adv, batch_x_fn_f64_d3_euler}},
        {{batch_x_fn_f32_d1_adv, batch_x_fn_f32_d1_euler},
         {batch_x_fn_f32_d2_adv, batch_x_fn_f32_d2_euler},
         {batch_x_fn_f32_d3_adv, batch_x_fn_f32_d3_euler}}};
    if (precision < 0 || precision > 1 || equation < 0 || equation > 1 || dim < 1 || dim > 3)
        return nullptr;
    return table[precision][dim - 1][equation](N);
}

StageXFn stage_x_fn(int precision, int equation, int dim, int N)
{
    typedef StageXFn (*Pick)(int);
    static const Pick table[2][3][2] = {
        {{stage_x_fn_f64_d1_adv, stage_x_fn_f64_d1_euler},
         {stage_x_fn_f64_d2_adv, stage_x_fn_f64_d2_euler},
         {stage_x_fn_f64_d3_adv, stage_x_fn_f64_d3_euler}},
        {{stage_x_fn_f32_d1_adv, stage_x_fn_f32_d1_euler},
         {stage_x_fn_f32_d2_adv, stage_x_fn_f32_d2_euler},
         {stage_x_fn_f32_d3_adv, stage_x_fn_f32_d3_euler}}};
    if (precision < 0 || precision > 1 || equation < 0 || equation > 1 || dim < 1 || dim > 3)
        return nullptr;
    return table[precision][dim - 1][equation](N);
}

StageFn stage_fn(int precision, int equation, int dim, int N)
{
    typedef StageFn (*Pick)(int);
    static const Pick table[2][3][2] = {
        {{stage_fn_f64_d1_adv, stage_fn_f64_d1_euler},
         {stage_fn_f64_d2_adv, stage_fn_f64_d2_euler},
         {stage_fn_f64_d3_adv, stage_fn_f64_d3_euler}},
        {{stage_fn_f32_d1_adv, stage_fn_f32_d1_euler},
         {stage_fn_f32_d2_adv, stage_fn_f32_d2_euler},
         {stage_fn_f32_d3_adv, stage_fn_f32_d3_euler}}};
    if (precision < 0 || precision > 1 || equation < 0 || equation > 1 || dim < 1 || dim > 3)
        return nullptr;
    return table[precision][dim - 1][equation](N);
}

// what: 0 threads per workgroup, 1 elements per tile along x, 2 element rows
template <int DIM, int EQ>
static int threads_n(int N, int what)
{
    switch (N) {
#define DG_CASE(n)                                                                             \
    case n:                                                                                    \
        return what == 0 ? Geo<DIM, n, EQ>::THREADS : what == 1 ? Geo<DIM, n, EQ>::EPB : Geo<DIM, n, EQ>::EPY;
        DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return 0;
    }
}

template <int EQ>
static int geo_of(int dim, int N, int what)
{
    return dim == 1 ? threads_n<1, EQ>(N, what) : dim == 2 ? threads_n<2, EQ>(N, what) : threads_n<3, EQ>(N, what);
}

static int geo_q(int dim, int N, int eq, int what)
{
    return eq == 0 ? geo_of<0>(dim, N, what) : geo_of<1>(dim, N, what);     // 0: advection
}

int stage_threads(int dim, int N, int eq) { return geo_q(dim, N, eq, 0); }
int stage_epb(int dim, int N, int eq) { return geo_q(dim, N, eq, 1); }
int stage_epy(int dim, int N, int eq) { return geo_q(dim, N, eq, 2); }

static int64_t grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    if (g > kMaxGrid) g = kMaxGrid;
    return g < 1 ? 1 : g;
}

// ---------------------------------------------------------------------------
// FP64 quadrature reductions: per-block partial sums (block tree in LDS); the
// host adds the partials in block order, so results are deterministic.
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const ReduceParams p)
{
    constexpr int T = kReduceThreads;
    __shared__ double qn[kMaxNP1 * kMaxNP1 * kMaxNP1];
    __shared__ double red[2 * 4][T];
    // quadrature weight of each node of an element, jac * prod_d w_{n_d}
    // (products in the same order for every node, once per block)
    for (int n = threadIdx.x; n < p.np; n += T) {
        int m = n;
        double q = p.jac;
        for (int d = 0; d < p.dim; ++d) {
            q *= p.w[m % p.n1];
            m /= p.n1;
        }
        qn[n] = q;
    }
    __syncthreads();
    const real *u = static_cast<const real *>(p.u);
    double acc[2 * 4];
    for (int k = 0; k < 2 * 4; ++k) acc[k] = 0.0;
    // grid-stride over nodes; the node index within the element advances by
    // the stride modulo np (one division per thread instead of one per node)
    const int64_t G = (int64_t)gridDim.x * T;
    int64_t i = blockIdx.x * (int64_t)T + threadIdx.x;
    int n = int(i % p.np);
    const int step = int(G % p.np);
    for (; i < p.stride; i += G) {
        const double q = qn[n];
        // u: element-interleaved (element of node i, then variable, then
        // node); uref: variable-major
        const int64_t ui = (i - n) * p.nvar + n;
        n += step;
        if (n >= p.np) n -= p.np;
        for (int v = 0; v < p.nvar; ++v) {
            const double x = double(u[ui + (int64_t)v * p.np]);
            if (p.mode == 0) {
                acc[v] += q * x;
            } else {
                const double r = p.uref[v * p.stride + i];
                const double df = x - r;
                acc[v] += q * df * df;
                acc[4 + v] += q * r * r;
            }
        }
    }
    for (int k = 0; k < 2 * 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = T / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 2 * 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 2 * 4; ++k) p.partial[blockIdx.x * 8 + k] = red[k][0];
}

hipError_t launch_reduce(int precision, const ReduceParams &p, int64_t blocks, hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(reduce_kernel<double>, dim3((unsigned)blocks), dim3(kReduceThreads), 0, s, p);
    else
        hipLaunchKernelGGL(reduce_kernel<float>, dim3((unsigned)blocks), dim3(kReduceThreads), 0, s, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout and precision conversion between the ABI's variable-major arrays
// (v * nodes + e * np + n) and the element-interleaved device arrays
// (e * nvar * np + v * np + n); one thread per destination value, so the
// writes are coalesced. Off the stepping path (set/get state).
// ---------------------------------------------------------------------------
template <typename To, typename From>
__global__ void __launch_bounds__(256) layout_kernel(const LayoutParams p)
{
    const From *src = static_cast<const From *>(p.src);
    To *dst = static_cast<To *>(p.dst);
    const int64_t es = (int64_t)p.nvar * p.np, total = p.nodes * p.nvar;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = j;
        if (p.nvar > 1) {
            if (p.to_internal) {                       // j internal -> k variable-major
                const int64_t e = j / es, r = j - e * es;
                const int64_t v = r / p.np, n = r - v * p.np;
                k = v * p.nodes + e * p.np + n;
            } else {                                   // j variable-major -> k internal
                const int64_t v = j / p.nodes, r = j - v * p.nodes;
                const int64_t e = r / p.np, n = r - e * p.np;
                k = e * es + v * p.np + n;
            }
        }
        dst[j] = To(src[k]);
    }
}

hipError_t launch_layout(int to_precision, int from_precision, const LayoutParams &p, hipStream_t s)
{
    const int64_t g = grid_for(p.nodes * p.nvar, 256);
    const dim3 G((unsigned)g), B(256);
    if (to_precision == 0 && from_precision == 0)
        hipLaunchKernelGGL((layout_kernel<double, double>), G, B, 0, s, p);
    else if (to_precision == 1 && from_precision == 0)
        hipLaunchKernelGGL((layout_kernel<float, double>), G, B, 0, s, p);
    else if (to_precision == 0 && from_precision == 1)
        hipLaunchKernelGGL((layout_kernel<double, float>), G, B, 0, s, p);
    else if (to_precision == 1 && from_precision == 1)
        hipLaunchKernelGGL((layout_kernel<float, float>), G, B, 0, s, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched-launch tile map: one workgroup per solve writes its tile range.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) fill_tile_map_kernel(const uint32_t *base, uint32_t *solve)
{
    const uint32_t j = blockIdx.x;
    const uint32_t lo = base[j], hi = base[j + 1];
    for (uint32_t t = lo + threadIdx.x; t < hi; t += blockDim.x) solve[t] = j;
}

hipError_t launch_fill_tile_map(const uint32_t *tile_base, uint32_t nsolves, uint32_t *tile_solve,
                                hipStream_t s)
{
    if (nsolves == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_tile_map_kernel, dim3(nsolves), dim3(256), 0, s, tile_base, tile_solve);
    return hipGetLastError();
}

}  // namespace dg
