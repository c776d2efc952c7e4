// dg_api.cpp -- host runtime behind the C ABI of include/dg.h: argument
// validation, workspace carve-up, operator tables, the Runge-Kutta stage
// schedules and the launch loop, reductions and host/device copies.
//
// Stage schedules (Sec. 2.3). Every scheme below is algebraically the
// Butcher-form scheme of the paper; they differ only in which combinations of
// stage vectors are kept in memory, chosen to minimise HBM passes.
//
// RK4 (eq. RK4), arrays U, A (accumulator), Ya, Yb, 14 array passes per step:
//   s1: R1 = F(U);   Yb = U + dt/2 R1
//   s2: R2 = F(Yb);  A  = U + (Yb - U)/3 + dt/3 R2  (= U + dt/6 R1 + dt/3 R2)
//                    Ya = U + dt/2 R2
//   s3: R3 = F(Ya);  A += dt/3 R3;  Yb = U + dt R3
//   s4: R4 = F(Yb);  U  = A + dt/6 R4
// RK3 (eq. RK3, Heun reading), 9 passes per step:
//   s1: R1 = F(U);   Ya = U + dt/3 R1;  A = U + dt/4 R1
//   s2: R2 = F(Ya);  Yb = U + 2dt/3 R2
//   s3: R3 = F(Yb);  U  = A + 3dt/4 R3
// RK6 (eq. RK6, Luther): k_s = dt F(Y_s) stored for s = 1..7, each followed
//   by Y_{s+1} = U + (sum_j num_{s+1,j} k_j)/den_{s+1}, and finally
//   U = U + (9k1 + 64k3 + 49k5 + 49k6 + 9k7)/180.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "dg_host.hpp"

using namespace dg;

namespace {
thread_local std::string g_last_error;
}

namespace dg {

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(DG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

Layout layout_for(int dim, int N, const int64_t *K, int eq, int prec)
{
    Layout L;
    int64_t nodes = 1;
    for (int d = 0; d < dim; ++d) nodes *= K[d];
    for (int d = 0; d < dim; ++d) nodes *= (N + 1);
    const int nvar = eq == DG_ADVECTION ? 1 : 1 + dim;
    const size_t sz = prec == DG_FP64 ? 8 : 4;
    L.tables = round_up(sizeof(double) * kMaxNP1 * kMaxNP1) + round_up(sizeof(double) * kMaxNP1) +
               round_up(sizeof(double) * 8 * kReduceBlocks) + round_up(kFaceTableBytes);
    L.array = round_up(sz * (size_t)nvar * (size_t)nodes);
    L.base = L.tables + 4 * L.array;
    L.rk6 = L.base + 5 * L.array;
    return L;
}

int validate(int dim, int N, const int64_t *K, int eq, const double *params, int prec)
{
    if (dim < 1 || dim > 3) return fail(DG_EINVAL, "dim must be 1, 2 or 3");
    if (N < 1 || N > kMaxN) return fail(DG_EINVAL, "N must be in 1..8");
    if (!K) return fail(DG_EINVAL, "K is NULL");
    double total = 1.0;
    for (int d = 0; d < dim; ++d) {
        if (K[d] < 1) return fail(DG_EINVAL, "K[d] must be >= 1");
        if (K[d] > (int64_t(1) << 30)) return fail(DG_EINVAL, "K[d] must be <= 2^30");
        total *= (double)K[d];
    }
    if (total > 4.0e9) return fail(DG_EINVAL, "at most 4e9 elements");
    if (total * std::pow(N + 1.0, dim) * (1 + dim) > 9.0e18 / 8)
        return fail(DG_EINVAL, "mesh too large");
    if (eq != DG_ADVECTION && eq != DG_EULER_ISOTHERMAL)
        return fail(DG_EINVAL, "equation must be DG_ADVECTION or DG_EULER_ISOTHERMAL");
    if (!params) return fail(DG_EINVAL, "params is NULL");
    if (eq == DG_ADVECTION) {
        for (int d = 0; d < dim; ++d)
            if (!std::isfinite(params[d])) return fail(DG_EINVAL, "advection velocity must be finite");
    } else if (!std::isfinite(params[0]) || !(params[0] > 0.0)) {
        return fail(DG_EINVAL, "sound speed c_s must be finite and > 0");
    }
    if (prec != DG_FP64 && prec != DG_FP32) return fail(DG_EINVAL, "precision must be DG_FP64 or DG_FP32");
    return DG_OK;
}


int select_device(const dg_solver *h)
{
    DG_HIP(hipSetDevice(h->device), "hipSetDevice");
    return DG_OK;
}

int64_t z_units(const dg_solver *h) { return (h->K[2] + h->zlen - 1) / h->zlen; }

StageParams base_params(const dg_solver *h, bool zmarch)
{
    StageParams p;
    std::memset(&p, 0, sizeof(p));
    for (int d = 0; d < 3; ++d) {
        p.K[d] = h->K[d];
        p.rdx2[d] = d < h->dim ? 2.0 * (double)h->K[d] : 0.0;
        p.par[d] = h->par[d];
    }
    p.stride = h->nodes;
    p.D = h->Dtab;
    p.tiles_x = h->tiles_x;
    p.tiles_y = h->tiles_y;
    // units along z: chunks of zlen layers for the z-marching kernel, layers
    // otherwise (a z-slab that divides the chunk count but not K_z then
    // falls back to 1 for the one-layer kernels)
    const bool zm = zmarch && h->dim == 3 && h->zlen > 1;
    const int64_t nz = zm ? z_units(h) : h->K[2];
    const int64_t slab = nz % h->slab == 0 ? h->slab : 1;
    const int64_t units = h->tiles_x * h->tiles_y * nz;
    p.zlen = zm ? (uint32_t)h->zlen : 1u;
    p.slab = slab;
    p.xblk = h->xblk;
    p.ntiles = units;
    p.ntiles32 = (uint32_t)units;
    p.xq = (uint32_t)(units / kXcds);
    p.xr = (uint32_t)(units % kXcds);
    p.fd_tx = make_fastdiv((uint32_t)h->tiles_x);
    p.fd_slab = make_fastdiv((uint32_t)slab);
    p.fd_ty = make_fastdiv((uint32_t)h->tiles_y);
    p.fd_xb = make_fastdiv((uint32_t)h->xblk);
    p.fd_nslab = make_fastdiv((uint32_t)(nz / slab));
    p.ftab = h->ftab;
    p.plain_order = (uint32_t)h->plain_order;
    return p;
}

int stage_count(int rk) { return rk == DG_RK4 ? 4 : rk == DG_RK3 ? 3 : rk == DG_RK6 ? 7 : 0; }

namespace {
void set_out(StageParams &p, int o, void *ptr, double cy, double c0, double c1, double cr)
{
    (o == 0 ? p.out0 : p.out1) = ptr;
    p.cy[o] = cy;
    p.c0[o] = c0;
    p.c1[o] = c1;
    p.cr[o] = cr;
    p.nout = o + 1;
}
}  // namespace

// Fused-stage programs of the RK3 and RK4 schedules (see the file comment):
// stage s reads yin (and in0/in1), writes out0/out1 = cy yin + c0 in0 + c1 in1 + cr R.
StageParams stage_program(const dg_solver *h, int rk, int s, double dt, bool zmarch)
{
    StageParams p = base_params(h, zmarch);
    if (rk == DG_RK4) {
        switch (s) {
        case 0:
            p.yin = h->U; p.nin = 0;
            set_out(p, 0, h->Yb, 1.0, 0.0, 0.0, dt / 2);
            break;
        case 1:
            p.yin = h->Yb; p.in0 = h->U; p.nin = 1;
            set_out(p, 0, h->A, 1.0 / 3.0, 2.0 / 3.0, 0.0, dt / 3);
            set_out(p, 1, h->Ya, 0.0, 1.0, 0.0, dt / 2);
            break;
        case 2:
            p.yin = h->Ya; p.in0 = h->U; p.in1 = h->A; p.nin = 2;
            set_out(p, 0, h->A, 0.0, 0.0, 1.0, dt / 3);
            set_out(p, 1, h->Yb, 0.0, 1.0, 0.0, dt);
            break;
        default:
            p.yin = h->Yb; p.in0 = h->A; p.nin = 1;
            set_out(p, 0, h->U, 0.0, 1.0, 0.0, dt / 6);
            break;
        }
    } else {   // RK3, Heun
        switch (s) {
        case 0:
            p.yin = h->U; p.nin = 0;
            set_out(p, 0, h->Ya, 1.0, 0.0, 0.0, dt / 3);
            set_out(p, 1, h->A, 1.0, 0.0, 0.0, dt / 4);
            break;
        case 1:
            p.yin = h->Ya; p.in0 = h->U; p.nin = 1;
            set_out(p, 0, h->Yb, 0.0, 1.0, 0.0, 2.0 * dt / 3);
            break;
        default:
            p.yin = h->Yb; p.in0 = h->A; p.nin = 1;
            set_out(p, 0, h->U, 0.0, 1.0, 0.0, 3.0 * dt / 4);
            break;
        }
    }
    return p;
}

int device_cus(int device)
{
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return 256;
    }
    return n;
}

MsPlan ms_plan(const dg_solver *h, int rk, int64_t tcap)
{
    if (h->dim != 1 || (rk != DG_RK3 && rk != DG_RK4) || !ms_fn(h->prec, h->eq, h->N) ||
        !ms_program_matches(ms_program(h, rk), rk))
        return MsPlan();
    return ms_plan_for(h->K[0], h->n1, ms_capacity(h->prec, h->eq, h->N), stage_count(rk), h->ms_div, tcap);
}

MsProgram ms_program(const dg_solver *h, int rk)
{
    MsProgram g;
    std::memset(&g, 0, sizeof(g));
    g.stages = stage_count(rk);
    const void *arr[4] = {h->U, h->A, h->Ya, h->Yb};
    auto index = [&](const void *q) -> int8_t {
        for (int i = 0; i < 4; ++i)
            if (arr[i] == q) return (int8_t)i;
        return 0;
    };
    for (int st = 0; st < g.stages; ++st) {
        const StageParams p = stage_program(h, rk, st, 1.0);
        g.yin[st] = index(p.yin);
        g.nin[st] = (int8_t)p.nin;
        g.in0[st] = p.nin > 0 ? index(p.in0) : 0;
        g.in1[st] = p.nin > 1 ? index(p.in1) : 0;
        g.nout[st] = (int8_t)p.nout;
        g.out[st][0] = index(p.out0);
        g.out[st][1] = p.nout > 1 ? index(p.out1) : 0;
    }
    return g;
}

bool ms_program_matches(const MsProgram &g, int rk)
{
    const MsProgram &t = rk == DG_RK4 ? kMsProgRk4 : kMsProgRk3;
    if (g.stages != t.stages) return false;
    for (int st = 0; st < t.stages; ++st) {
        if (g.yin[st] != t.yin[st] || g.nin[st] != t.nin[st] || g.nout[st] != t.nout[st]) return false;
        if (t.nin[st] > 0 && g.in0[st] != t.in0[st]) return false;
        if (t.nin[st] > 1 && g.in1[st] != t.in1[st]) return false;
        for (int o = 0; o < t.nout[st]; ++o)
            if (g.out[st][o] != t.out[st][o]) return false;
    }
    return true;
}

MsSolve ms_solve(const dg_solver *h, int rk, double dt, const MsPlan &pl, bool pingpong)
{
    MsSolve m;
    std::memset(&m, 0, sizeof(m));
    m.U = h->U;
    m.V = pingpong ? h->Ya : h->U;
    m.K = h->K[0];
    m.T = pl.T;
    m.whole = pl.whole;
    m.rdx2 = 2.0 * (double)h->K[0];
    m.par = h->par[0];
    for (int st = 0; st < stage_count(rk); ++st) {
        const StageParams p = stage_program(h, rk, st, dt);
        for (int o = 0; o < p.nout; ++o) {
            m.coef[st][o][0] = p.cy[o];
            m.coef[st][o][1] = p.c0[o];
            m.coef[st][o][2] = p.c1[o];
            m.coef[st][o][3] = p.cr[o];
        }
    }
    return m;
}

int setup_solver(dg_solver *h, int dim, int N, const int64_t *K, int equation, const double *params,
                 int precision)
{
    h->dim = dim;
    h->N = N;
    h->eq = equation;
    h->prec = precision;
    h->nvar = equation == DG_ADVECTION ? 1 : 1 + dim;
    h->n1 = N + 1;
    h->np = 1;
    for (int d = 0; d < dim; ++d) h->np *= h->n1;
    int64_t E = 1;
    for (int d = 0; d < 3; ++d) {
        h->K[d] = d < dim ? K[d] : 1;
        E *= h->K[d];
    }
    h->nodes = E * h->np;
    h->unknowns = h->nodes * h->nvar;
    if (equation == DG_ADVECTION)
        for (int d = 0; d < dim; ++d) h->par[d] = params[d];
    else
        h->par[0] = params[0];
    lgl_operator(N, h->xi, h->w, h->D);
    h->lay = layout_for(dim, N, K, equation, precision);
    h->stage = stage_fn(precision, equation, dim, N);
    if (!h->stage) return fail(DG_ENOTSUP, "no stage kernel built for this configuration");
    h->epb = stage_epb(dim, N, equation);
    h->tiles_x = (h->K[0] + h->epb - 1) / h->epb;
    h->epy = stage_epy(dim, N, equation);
    h->tiles_y = (h->K[1] + h->epy - 1) / h->epy;
    // default 3-D tile order: x-blocks of about an eighth of the x-tiles (the
    // largest divisor in [4, max(4, tiles_x / 8)], else whole rows), walked
    // y-tile by y-tile, then layer by layer: each XCD's contiguous range
    // is then an x-column of the mesh, whose y- and z-neighbour traces stay
    // in that XCD's L2 (z-slab 1)
    h->slab = 1;
    h->xblk = h->tiles_x;
    if (dim == 3) {
        for (int64_t xb = std::max<int64_t>(4, h->tiles_x / kXcds); xb >= 4; --xb)
            if (h->tiles_x % xb == 0) { h->xblk = xb; break; }
        // FP32 3-D: units of up to four layers per workgroup (z-march; -5 %
        // per launch on 64^3 N = 4, where FP64 is fastest with one layer)
        if (precision == DG_FP32) h->zlen = std::min<int64_t>(4, h->K[2]);
    }
    // default 2-D tile order: plain when the x-tile count is a multiple of
    // the XCD count (tile L runs on XCD L mod 8, so every XCD holds whole
    // columns of tiles and meets a tile's y-neighbours one row apart, while
    // the eight XCDs sweep the same band of rows): -6.8 % per launch on 2-D
    // Euler 512^2 N = 3, unchanged on 2-D advection 256^2 N = 7; otherwise
    // XCD-contiguous ranges of tiles
    if (dim == 2 && h->tiles_x % kXcds == 0) h->plain_order = 1;
    h->ntiles = h->tiles_x * h->tiles_y * h->K[2];
    h->grid = std::min<int64_t>(h->ntiles, kMaxGrid);
    return DG_OK;
}

char *carve_tables(dg_solver *h, char *p)
{
    h->Dtab = p;
    p += round_up(sizeof(double) * kMaxNP1 * kMaxNP1);
    h->wtab = reinterpret_cast<double *>(p);
    p += round_up(sizeof(double) * kMaxNP1);
    h->partial = reinterpret_cast<double *>(p);
    p += round_up(sizeof(double) * 8 * kReduceBlocks);
    h->ftab = reinterpret_cast<uint32_t *>(p);
    p += round_up(kFaceTableBytes);
    return p;
}

char *carve_rk_arrays(dg_solver *h, char *p, bool rk6)
{
    h->A = p;  p += h->lay.array;
    h->Ya = p; p += h->lay.array;
    h->Yb = p; p += h->lay.array;
    if (rk6)
        for (int i = 0; i < 5; ++i, p += h->lay.array) h->kx[i] = p;
    return p;
}

int upload_tables(dg_solver *h)
{
    // operator tables in the state precision (D) and FP64 (w)
    unsigned char dbuf[sizeof(double) * kMaxNP1 * kMaxNP1];
    const int nd = h->n1 * h->n1;
    if (h->prec == DG_FP64) {
        std::memcpy(dbuf, h->D, sizeof(double) * nd);
    } else {
        float *f = reinterpret_cast<float *>(dbuf);
        for (int i = 0; i < nd; ++i) f[i] = (float)h->D[i];
    }
    const size_t dbytes = (h->prec == DG_FP64 ? 8 : 4) * (size_t)nd;
    // (host buffers on the stack: no heap allocation on this path)
    const size_t fbytes = 16 * (size_t)face_table_size(h->dim, h->N, h->epb, h->epy);
    if (fbytes > kFaceTableBytes) return fail(DG_ENOTSUP, "face table larger than reserved");
    uint32_t ftab[kFaceTableBytes / 4];
    build_face_table(h->dim, h->N, h->epb, h->epy, h->nvar, ftab);
    hipError_t e;
    if ((e = hipMemcpyAsync(h->Dtab, dbuf, dbytes, hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(h->ftab, ftab, fbytes, hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(h->wtab, h->w, sizeof(double) * h->n1, hipMemcpyHostToDevice, h->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return hip_fail(e, "operator upload");
    return DG_OK;
}

double *staging(dg_solver *h)
{
    // Ya and Yb are adjacent and together hold at least unknowns doubles
    return static_cast<double *>(h->Ya);
}

int convert(dg_solver *h, const void *src, int src_prec, void *dst, int dst_prec, bool to_internal)
{
    LayoutParams c;
    c.src = src;
    c.dst = dst;
    c.nodes = h->nodes;
    c.nvar = h->nvar;
    c.np = h->np;
    c.to_internal = to_internal ? 1 : 0;
    DG_HIP(launch_layout(dst_prec, src_prec, c, h->stream), "layout kernel launch");
    return DG_OK;
}

namespace {

int launch(dg_solver *h, const StageParams &p)
{
    DG_HIP(h->stage(p, std::min<int64_t>(p.ntiles, kMaxGrid), h->stream), "stage kernel launch");
    return DG_OK;
}

int step_rk34(dg_solver *h, int rk, double dt)
{
    for (int st = 0; st < stage_count(rk); ++st) {
        int rc = launch(h, stage_program(h, rk, st, dt, true));
        if (rc) return rc;
    }
    return DG_OK;
}

// 1-D RK3/RK4: temporally blocked launches of up to smax steps each
int step_ms(dg_solver *h, int rk, double dt, int64_t nsteps, const MsPlan &pl)
{
    MsLaunch L;
    std::memset(&L, 0, sizeof(L));
    // one workgroup updates the state in place; several ping-pong between
    // U and Ya and end in U
    const bool pp = pl.nwg > 1;
    L.solves = nullptr;
    L.D = h->Dtab;
    L.one = ms_solve(h, rk, dt, pl, pp);
    L.rk = rk;
    L.nwg = (uint32_t)pl.nwg;
    const MsFn fn = ms_fn(h->prec, h->eq, h->N);
    const MsSchedule sc = ms_schedule(nsteps, pl.smax, pp);
    for (int64_t i = 0; i < sc.launches(); ++i) {
        L.nsteps = sc.steps(i);
        DG_HIP(fn(L, h->stream), "multi-step kernel launch");
        L.flip ^= pp ? 1 : 0;
    }
    return DG_OK;
}

// Luther's RK6 (eq. RK6): Y_s = U + (sum_j num[s][j] k_j) / den[s].
struct Rk6Tableau {
    double num[7][7];
    double den[7];
    double bnum[7];
    double bden;
};

const Rk6Tableau &rk6_tableau()
{
    static const Rk6Tableau t = [] {
        Rk6Tableau r;
        std::memset(&r, 0, sizeof(r));
        const double q = std::sqrt(21.0);
        r.den[1] = 1;    r.num[1][0] = 1;
        r.den[2] = 8;    r.num[2][0] = 3; r.num[2][1] = 1;
        r.den[3] = 27;   r.num[3][0] = 8; r.num[3][1] = 2; r.num[3][2] = 8;
        r.den[4] = 392;
        r.num[4][0] = 3 * (3 * q - 7);   r.num[4][1] = -8 * (7 - q);
        r.num[4][2] = 48 * (7 - q);      r.num[4][3] = -3 * (21 - q);
        r.den[5] = 1960;
        r.num[5][0] = -5 * (231 + 51 * q); r.num[5][1] = -40 * (7 + q);
        r.num[5][2] = -320 * q;            r.num[5][3] = 3 * (21 + 121 * q);
        r.num[5][4] = 392 * (6 + q);
        r.den[6] = 180;
        r.num[6][0] = 15 * (22 + 7 * q);  r.num[6][1] = 120;
        r.num[6][2] = 40 * (7 * q - 5);   r.num[6][3] = -63 * (3 * q - 2);
        r.num[6][4] = -14 * (49 + 9 * q); r.num[6][5] = 70 * (7 - q);
        r.bden = 180;
        r.bnum[0] = 9; r.bnum[2] = 64; r.bnum[4] = 49; r.bnum[5] = 49; r.bnum[6] = 9;
        return r;
    }();
    return t;
}

// Luther's RK6 (eq. RK6), fused: stage s evaluates R = F(Y_s) once and writes
//   k_s = dt R                                               (s < 6)
//   Y_{s+1} = U + sum_{j<s} (num[s+1][j]/den[s+1]) k_j + (num[s+1][s] dt/den[s+1]) R
// and the last stage U <- U + sum_{j<6} (bnum_j/bden) k_j + (bnum_6 dt/bden) R.
// k_0..k_5 live in A, kx[0..4]; Y alternates between Ya and Yb.
int step_rk6(dg_solver *h, double dt)
{
    for (int s = 0; s < 7; ++s) {
        StageParams p;
        ExtraIn x;
        const int rc = rk6_stage(h, s, dt, p, x);
        if (rc) return rc;
        DG_HIP(stage_x_fn(h->prec, h->eq, h->dim, h->N)(p, x, h->grid, h->stream), "RK6 stage kernel launch");
    }
    return DG_OK;
}

}  // namespace

int ensure_rk6(dg_solver *h)
{
    if (h->kx[0]) return DG_OK;
    char *mem = nullptr;
    if (!h->own_ws) {
        if (h->ws_bytes < h->lay.rk6)
            return fail(DG_ENOMEM, "workspace too small for RK6 (see dg_workspace_bytes)");
        mem = h->ws + h->lay.base;
    } else {
        hipError_t e = hipMalloc((void **)&h->rk6_mem, 5 * h->lay.array);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->rk6_mem = nullptr;
            return fail(DG_ENOMEM, "cannot allocate the RK6 stage store");
        }
        mem = h->rk6_mem;
    }
    for (int i = 0; i < 5; ++i) h->kx[i] = mem + i * h->lay.array;
    return DG_OK;
}

// Stage s of Luther's RK6 (eq. RK6) as one fused stage-kernel launch:
// k_s = dt R(Y_s) (s < 6) and Y_{s+1} (or, at s = 6, the new U) =
// U + (sum_j num_{s+1,j} k_j) / den_{s+1}, the k's with nonzero weights as
// further inputs.
int rk6_stage(const dg_solver *h, int s, double dt, StageParams &p, ExtraIn &x)
{
    const Rk6Tableau &t = rk6_tableau();
    void *k[6] = {h->A, h->kx[0], h->kx[1], h->kx[2], h->kx[3], h->kx[4]};
    void *Y[2] = {h->Ya, h->Yb};
    p = base_params(h);
    p.yin = s == 0 ? h->U : Y[(s - 1) % 2];
    const double *num = s < 6 ? t.num[s + 1] : t.bnum;
    const double den = s < 6 ? t.den[s + 1] : t.bden;
    int o = 0;
    if (s < 6) {                                   // k_s = dt R
        set_out(p, 0, k[s], 0.0, 0.0, 0.0, dt);
        o = 1;
    }
    // the combination: U first, then the stored k's with nonzero weights
    const void *in_ptr[8];
    double in_w[8];
    int nin = 0;
    in_ptr[nin] = h->U;
    in_w[nin++] = 1.0;
    for (int j = 0; j < s && j < 6; ++j)
        if (num[j] != 0.0) {
            in_ptr[nin] = k[j];
            in_w[nin++] = num[j] / den;
        }
    if (nin > 2 + kMaxExtraIn) return fail(DG_ENOTSUP, "too many RK6 stage inputs");
    void *dst = s < 6 ? Y[s % 2] : h->U;
    (o == 0 ? p.out0 : p.out1) = dst;
    p.cy[o] = 0.0;
    p.cr[o] = num[s] * dt / den;
    p.nin = std::min(2, nin);
    p.in0 = in_ptr[0];
    p.c0[o] = in_w[0];
    if (nin > 1) {
        p.in1 = in_ptr[1];
        p.c1[o] = in_w[1];
    }
    std::memset(&x, 0, sizeof(x));
    for (int j = 2; j < nin; ++j) {
        x.in[x.n] = in_ptr[j];
        x.c[o][x.n] = in_w[j];
        ++x.n;
    }
    p.nout = o + 1;
    return DG_OK;
}

int enqueue_steps(dg_solver *h, int rk, double dt, int64_t nsteps)
{
    // by default a chunk per CU: the steps of a launch then run in one round
    // of workgroups (chunking never changes an element's arithmetic)
    const int64_t tcap = h->ms_chunk == 0 ? ms_spread(h->K[0], h->cus) : (h->ms_chunk < 0 ? 0 : h->ms_chunk);
    const MsPlan pl = ms_plan(h, rk, tcap);
    if (pl.ok) return step_ms(h, rk, dt, nsteps, pl);
    for (int64_t s = 0; s < nsteps; ++s) {
        const int rc = rk == DG_RK6 ? step_rk6(h, dt) : step_rk34(h, rk, dt);
        if (rc) return rc;
    }
    return DG_OK;
}

namespace {

int check_count(const dg_solver *h, int64_t count)
{
    if (count != h->unknowns)
        return fail(DG_EINVAL, "count must equal nvar * nodes = " + std::to_string(h->unknowns));
    return DG_OK;
}

// Reduction over the current state (mode 0: mass; mode 1: L2 against the
// FP64 reference already staged at uref_dev). Returns per-variable sums.
int reduce(dg_solver *h, int mode, const double *uref_dev, double *s0, double *s1)
{
    ReduceParams r;
    std::memset(&r, 0, sizeof(r));
    r.u = h->U;
    r.uref = uref_dev;
    r.partial = h->partial;
    r.w = h->wtab;
    double jac = 1.0;
    for (int d = 0; d < h->dim; ++d) jac *= 0.5 / (double)h->K[d];
    r.jac = jac;
    r.stride = h->nodes;
    r.nvar = h->nvar;
    r.n1 = h->n1;
    r.np = h->np;
    r.dim = h->dim;
    r.mode = mode;
    int64_t blocks = (h->nodes + kReduceThreads - 1) / kReduceThreads;
    blocks = std::min<int64_t>(std::max<int64_t>(blocks, 1), kReduceBlocks);
    DG_HIP(launch_reduce(h->prec, r, blocks, h->stream), "reduce kernel launch");
    std::vector<double> part(8 * blocks);
    DG_HIP(hipMemcpyAsync(part.data(), h->partial, sizeof(double) * 8 * blocks,
                          hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    DG_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    for (int v = 0; v < h->nvar; ++v) {
        double a = 0.0, b = 0.0;
        for (int64_t i = 0; i < blocks; ++i) {
            a += part[8 * i + v];
            b += part[8 * i + 4 + v];
        }
        s0[v] = a;
        if (s1) s1[v] = b;
    }
    return DG_OK;
}

// Stage an FP64 host reference on the device (in the Ya/Yb region, free
// between steps: Ya and Yb are adjacent and together hold >= unknowns doubles).
int stage_reference(dg_solver *h, const double *u_ref, double **dev)
{
    double *d = static_cast<double *>(h->Ya);
    DG_HIP(hipMemcpyAsync(d, u_ref, sizeof(double) * h->unknowns, hipMemcpyHostToDevice, h->stream),
           "hipMemcpyAsync");
    *dev = d;
    return DG_OK;
}

void free_solver(dg_solver *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->rk6_mem) (void)hipFree(h->rk6_mem);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // namespace
}  // namespace dg

extern "C" {

const char *dg_last_error(void) { return g_last_error.c_str(); }

int dg_workspace_bytes(int dim, int N, const int64_t *K, int equation, int precision, int rk,
                       size_t *bytes)
{
    double dummy[3] = {1.0, 1.0, 1.0};
    int rc = validate(dim, N, K, equation, dummy, precision);
    if (rc) return rc;
    if (rk != DG_RK3 && rk != DG_RK4 && rk != DG_RK6) return fail(DG_EINVAL, "rk must be 3, 4 or 6");
    if (!bytes) return fail(DG_EINVAL, "bytes is NULL");
    Layout L = layout_for(dim, N, K, equation, precision);
    *bytes = rk == DG_RK6 ? L.rk6 : L.base;
    return DG_OK;
}

int dg_create_ex(int dim, int N, const int64_t *K, int equation, const double *params,
                 int precision, void *hip_stream, void *device_workspace, size_t workspace_bytes,
                 dg_solver **out)
{
    if (!out) return fail(DG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(dim, N, K, equation, params, precision);
    if (rc) return rc;
    if (!stage_fn(precision, equation, dim, N))
        return fail(DG_ENOTSUP, "no stage kernel built for this configuration");

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(DG_EDEVICE, "no HIP device available");
    }

    dg_solver *h = new (std::nothrow) dg_solver();
    if (!h) return fail(DG_ENOMEM, "host allocation failed");
    if ((rc = setup_solver(h, dim, N, K, equation, params, precision))) {
        delete h;
        return rc;
    }
    e = hipGetDevice(&h->device);
    if (e != hipSuccess) { delete h; return hip_fail(e, "hipGetDevice"); }
    h->cus = device_cus(h->device);

    if (hip_stream) {
        h->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete h; return hip_fail(e, "hipStreamCreate"); }
        h->own_stream = true;
    }
    if (device_workspace) {
        if (workspace_bytes < h->lay.base) {
            free_solver(h);
            return fail(DG_ENOMEM, "workspace smaller than dg_workspace_bytes(rk=4)");
        }
        if ((reinterpret_cast<uintptr_t>(device_workspace) % kAlign) != 0) {
            free_solver(h);
            return fail(DG_EINVAL, "workspace must be 256-byte aligned");
        }
        h->ws = static_cast<char *>(device_workspace);
        h->ws_bytes = workspace_bytes;
    } else {
        e = hipMalloc((void **)&h->ws, h->lay.base);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->ws = nullptr;
            free_solver(h);
            return fail(DG_ENOMEM, "cannot allocate " + std::to_string(h->lay.base) + " device bytes");
        }
        h->own_ws = true;
        h->ws_bytes = h->lay.base;
    }
    char *arrays = carve_tables(h, h->ws);
    h->U = arrays;
    carve_rk_arrays(h, arrays + h->lay.array, false);
    if ((rc = upload_tables(h))) {
        free_solver(h);
        return rc;
    }
    *out = h;
    return DG_OK;
}

int dg_create(int dim, int N, const int64_t *K, int equation, const double *params, dg_solver **out)
{
    return dg_create_ex(dim, N, K, equation, params, DG_FP64, nullptr, nullptr, 0, out);
}

int dg_destroy(dg_solver *h)
{
    if (h && h->batch) (void)dg_batch_remove(h->batch, h);
    free_solver(h);
    return DG_OK;
}

int dg_sizes(const dg_solver *h, int *nvar, int64_t *nodes)
{
    if (!h) return fail(DG_EINVAL, "solver is NULL");
    if (nvar) *nvar = h->nvar;
    if (nodes) *nodes = h->nodes;
    return DG_OK;
}

int dg_get_axis_coords(const dg_solver *h, int axis, double *x, int64_t count)
{
    if (!h || !x) return fail(DG_EINVAL, "NULL argument");
    if (axis < 0 || axis >= h->dim) return fail(DG_EINVAL, "axis out of range");
    if (count != h->K[axis] * h->n1) return fail(DG_EINVAL, "count must be K[axis] * (N+1)");
    const double dx = 1.0 / (double)h->K[axis];
    for (int64_t e = 0; e < h->K[axis]; ++e)
        for (int i = 0; i < h->n1; ++i) x[e * h->n1 + i] = (double)e * dx + 0.5 * dx * (h->xi[i] + 1.0);
    return DG_OK;
}

int dg_get_coords(const dg_solver *h, double *xyz, int64_t count)
{
    if (!h || !xyz) return fail(DG_EINVAL, "NULL argument");
    if (count != (int64_t)h->dim * h->nodes) return fail(DG_EINVAL, "count must be dim * nodes");
    // per-axis coordinates, then the tensor product in the canonical order
    std::vector<double> ax[3];
    for (int d = 0; d < h->dim; ++d) {
        ax[d].resize(h->K[d] * h->n1);
        int rc = dg_get_axis_coords(h, d, ax[d].data(), (int64_t)ax[d].size());
        if (rc) return rc;
    }
    const int n1 = h->n1;
    int64_t node = 0;
    for (int64_t ez = 0; ez < h->K[2]; ++ez)
        for (int64_t ey = 0; ey < h->K[1]; ++ey)
            for (int64_t ex = 0; ex < h->K[0]; ++ex)
                for (int k = 0; k < (h->dim > 2 ? n1 : 1); ++k)
                    for (int j = 0; j < (h->dim > 1 ? n1 : 1); ++j)
                        for (int i = 0; i < n1; ++i, ++node) {
                            xyz[node] = ax[0][ex * n1 + i];
                            if (h->dim > 1) xyz[h->nodes + node] = ax[1][ey * n1 + j];
                            if (h->dim > 2) xyz[2 * h->nodes + node] = ax[2][ez * n1 + k];
                        }
    return DG_OK;
}

int dg_set_state(dg_solver *h, const double *u, int64_t count)
{
    if (!h || !u) return fail(DG_EINVAL, "NULL argument");
    if (h->batch) return fail(DG_ESTATE, "solver belongs to a batch");
    int rc = check_count(h, count);
    if (rc || (rc = select_device(h))) return rc;
    if (h->prec == DG_FP64 && h->nvar == 1) {
        DG_HIP(hipMemcpyAsync(h->U, u, sizeof(double) * count, hipMemcpyHostToDevice, h->stream),
               "hipMemcpyAsync");
    } else {
        // variable-major FP64 into the free RK arrays, then converted into U
        double *stage = staging(h);
        DG_HIP(hipMemcpyAsync(stage, u, sizeof(double) * count, hipMemcpyHostToDevice, h->stream),
               "hipMemcpyAsync");
        if ((rc = convert(h, stage, DG_FP64, h->U, h->prec, true))) return rc;
    }
    DG_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    h->has_state = true;
    return DG_OK;
}

int dg_set_state_device(dg_solver *h, const void *u_dev, int64_t count)
{
    if (!h || !u_dev) return fail(DG_EINVAL, "NULL argument");
    if (h->batch) return fail(DG_ESTATE, "solver belongs to a batch");
    int rc = check_count(h, count);
    if (rc || (rc = select_device(h))) return rc;
    if (h->prec == DG_FP64 && h->nvar == 1) {
        DG_HIP(hipMemcpyAsync(h->U, u_dev, sizeof(double) * count, hipMemcpyDeviceToDevice, h->stream),
               "hipMemcpyAsync");
    } else if ((rc = convert(h, u_dev, DG_FP64, h->U, h->prec, true))) {
        return rc;
    }
    h->has_state = true;
    return DG_OK;
}

int dg_step(dg_solver *h, int rk, double dt, int64_t nsteps)
{
    if (!h) return fail(DG_EINVAL, "solver is NULL");
    if (rk != DG_RK3 && rk != DG_RK4 && rk != DG_RK6) return fail(DG_EINVAL, "rk must be 3, 4 or 6");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(DG_EINVAL, "dt must be finite and > 0");
    if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if (h->batch) return fail(DG_ESTATE, "solver belongs to a batch (use dg_batch_run)");
    if (nsteps == 0) return DG_OK;
    int rc = select_device(h);
    if (rc) return rc;
    if (rk == DG_RK6 && (rc = ensure_rk6(h))) return rc;
    return enqueue_steps(h, rk, dt, nsteps);
}

int dg_get_state(dg_solver *h, double *u, int64_t count)
{
    if (!h || !u) return fail(DG_EINVAL, "NULL argument");
    int rc = check_count(h, count);
    if (rc || (rc = select_device(h))) return rc;
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if ((rc = batch_order_member(h))) return rc;
    const void *src = h->U;
    if (!(h->prec == DG_FP64 && h->nvar == 1)) {
        // converted to variable-major FP64 in the free RK arrays first
        double *stage = staging(h);
        if ((rc = convert(h, h->U, h->prec, stage, DG_FP64, false))) return rc;
        src = stage;
    }
    DG_HIP(hipMemcpyAsync(u, src, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    DG_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return DG_OK;
}

int dg_get_state_device(dg_solver *h, void *u_dev, int64_t count)
{
    if (!h || !u_dev) return fail(DG_EINVAL, "NULL argument");
    int rc = check_count(h, count);
    if (rc || (rc = select_device(h))) return rc;
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if ((rc = batch_order_member(h))) return rc;
    if (h->prec == DG_FP64 && h->nvar == 1) {
        DG_HIP(hipMemcpyAsync(u_dev, h->U, sizeof(double) * count, hipMemcpyDeviceToDevice, h->stream),
               "hipMemcpyAsync");
    } else if ((rc = convert(h, h->U, h->prec, u_dev, DG_FP64, false))) {
        return rc;
    }
    // later batch work (which rewrites U and the conversion's staging) waits
    return batch_after_member(h);
}

int dg_l2_error_vars(dg_solver *h, const double *u_ref, int64_t count, double *sq_err, double *sq_ref)
{
    if (!h || !u_ref || !sq_err || !sq_ref) return fail(DG_EINVAL, "NULL argument");
    int rc = check_count(h, count);
    if (rc || (rc = select_device(h))) return rc;
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if ((rc = batch_order_member(h))) return rc;
    double *dref = nullptr;
    if ((rc = stage_reference(h, u_ref, &dref))) return rc;
    return reduce(h, 1, dref, sq_err, sq_ref);
}

int dg_l2_error(dg_solver *h, const double *u_ref, int64_t count, double *abs_err, double *rel_err)
{
    double se[4] = {0, 0, 0, 0}, sr[4] = {0, 0, 0, 0};
    int rc = dg_l2_error_vars(h, u_ref, count, se, sr);
    if (rc) return rc;
    double a = 0.0, b = 0.0;
    for (int v = 0; v < h->nvar; ++v) {
        a += se[v];
        b += sr[v];
    }
    a = std::sqrt(a);
    if (abs_err) *abs_err = a;
    if (rel_err) *rel_err = b > 0.0 ? a / std::sqrt(b) : HUGE_VAL;
    return DG_OK;
}

int dg_mass(dg_solver *h, double *mass)
{
    if (!h || !mass) return fail(DG_EINVAL, "NULL argument");
    int rc = select_device(h);
    if (rc) return rc;
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if ((rc = batch_order_member(h))) return rc;
    return reduce(h, 0, nullptr, mass, nullptr);
}

int dg_synchronize(dg_solver *h)
{
    if (!h) return fail(DG_EINVAL, "solver is NULL");
    int rc = select_device(h);
    if (rc || (rc = batch_order_member(h))) return rc;
    DG_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return DG_OK;
}

int dg_autotune(dg_solver *h, int rk, double dt, int trial_steps)
{
    if (!h) return fail(DG_EINVAL, "solver is NULL");
    if (rk != DG_RK3 && rk != DG_RK4 && rk != DG_RK6) return fail(DG_EINVAL, "rk must be 3, 4 or 6");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(DG_EINVAL, "dt must be finite and > 0");
    if (trial_steps < 1 || trial_steps > 1000) return fail(DG_EINVAL, "trial_steps must be in 1..1000");
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if (h->batch) return fail(DG_ESTATE, "solver belongs to a batch");
    // the tuner keeps a copy of the state: its own allocation for a
    // library-owned workspace, else the space after the scheme's arrays in
    // the caller's workspace
    const size_t used = rk == DG_RK6 ? h->lay.rk6 : h->lay.base;
    if (!h->own_ws && h->ws_bytes < used + h->lay.array)
        return fail(DG_ENOTSUP, "autotuning with an external workspace needs one state array more than "
                                "dg_workspace_bytes(rk) for its copy of the state");
    int rc = select_device(h);
    if (rc) return rc;
    if (rk == DG_RK6 && (rc = ensure_rk6(h))) return rc;

    // Launch configurations (tile order, 1-D halo bound and chunk length,
    // z-slab, x-block, z-march length), searched in stages: 3-D, first tile
    // order x x-block (one-layer units), then the z-slab, then the z-march
    // length (RK3/RK4 only: the RK6 kernel runs one layer per tile); 2-D, the
    // tile order; 1-D chunked meshes, the elements per workgroup (a chunk per
    // CU, two per CU, the halo-bound plan) x the halo bound. Each stage keeps
    // the fastest of its candidates (the defaults are among them). Every
    // candidate is timed for trial_steps steps from a saved copy of U (after
    // one warm-up step), then U is restored.
    struct Cfg { int plain, ms_div; int64_t slab, xblk, zlen, chunk; };
    const Cfg keep = {h->plain_order, h->ms_div, h->slab, h->xblk, h->zlen, h->ms_chunk};
    std::vector<std::vector<Cfg>> stages;
    const MsPlan pl = ms_plan(h, rk);
    if (pl.ok) {
        if (!pl.whole) {
            std::vector<Cfg> st;
            // elements per workgroup (a chunk per CU, two per CU, the halo-bound
            // plan) x steps per launch (the halo bound)
            for (int64_t ch : {int64_t(0), ms_spread(h->K[0], 2 * h->cus), int64_t(-1)})
                for (int dv : {6, 10, 16, 24, 40}) st.push_back({h->plain_order, dv, h->slab, h->xblk, h->zlen, ch});
            stages.push_back(st);
        }
    } else if (h->dim == 3) {
        std::vector<int64_t> xbs{h->tiles_x};          // the whole row, then halvings down to 2 tiles
        for (int64_t xb = h->tiles_x; xb % 2 == 0 && xb / 2 >= 2; xb /= 2) xbs.push_back(xb / 2);
        std::vector<Cfg> s1;
        for (int plain = 0; plain <= 1; ++plain)
            for (int64_t xb : xbs) s1.push_back({plain, h->ms_div, 1, xb, 1, h->ms_chunk});
        stages.push_back(s1);
        stages.push_back({});                          // z-slabs: filled from the stage-1 winner
        if (rk != DG_RK6) stages.push_back({});        // z-march lengths: filled likewise
    } else if (h->dim == 2) {
        stages.push_back({{0, h->ms_div, h->slab, h->xblk, h->zlen, h->ms_chunk},
                          {1, h->ms_div, h->slab, h->xblk, h->zlen, h->ms_chunk}});
    }
    if (stages.empty()) {
        h->tuned = 1;
        return DG_OK;
    }
    void *save = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipSuccess;
    if (h->own_ws) {
        e = hipMalloc(&save, h->lay.array);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(DG_ENOMEM, "cannot allocate the autotuning copy of the state");
        }
    } else {
        save = h->ws + used;
    }
    rc = DG_OK;
    auto apply = [h](const Cfg &c) {
        h->plain_order = c.plain;
        h->ms_div = c.ms_div;
        h->slab = c.slab;
        h->xblk = c.xblk;
        h->zlen = c.zlen;
        h->ms_chunk = c.chunk;
    };
    // time one candidate; U is restored afterwards
    auto time_cfg = [&](const Cfg &c, float &ms_t) {
        apply(c);
        rc = dg_step(h, rk, dt, 1);                                   // warm-up
        if (rc) return;
        e = hipMemcpyAsync(h->U, save, h->lay.array, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
        if (e != hipSuccess) return;
        rc = dg_step(h, rk, dt, trial_steps);
        if (rc) return;
        e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms_t, e0, e1);
        if (e == hipSuccess) e = hipMemcpyAsync(h->U, save, h->lay.array, hipMemcpyDeviceToDevice, h->stream);
    };
    e = hipMemcpyAsync(save, h->U, h->lay.array, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    Cfg best = keep;
    float best_ms = -1.0f;
    for (size_t si = 0; si < stages.size() && e == hipSuccess && rc == DG_OK; ++si) {
        std::vector<Cfg> cand = stages[si];
        if (h->dim == 3 && !pl.ok && si == 1) {
            for (int64_t sl = 2; sl <= h->K[2]; sl *= 2)
                if (h->K[2] % sl == 0) cand.push_back({best.plain, best.ms_div, sl, best.xblk, 1, best.chunk});
        } else if (h->dim == 3 && !pl.ok && si == 2) {
            for (int64_t zl : {2, 4, 8, 16}) {
                if (zl > h->K[2]) break;
                const int64_t nz = (h->K[2] + zl - 1) / zl;
                cand.push_back({best.plain, best.ms_div, nz % best.slab == 0 ? best.slab : 1, best.xblk, zl, best.chunk});
            }
        }
        for (const Cfg &c : cand) {
            float ms_t = 0.0f;
            time_cfg(c, ms_t);
            if (e != hipSuccess || rc != DG_OK) break;
            if (best_ms < 0.0f || ms_t < best_ms) {
                best_ms = ms_t;
                best = c;
            }
        }
    }
    if (e == hipSuccess && rc == DG_OK) e = hipStreamSynchronize(h->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (h->own_ws) (void)hipFree(save);
    apply((e == hipSuccess && rc == DG_OK) ? best : keep);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotuning");
    h->tuned = 1;
    return DG_OK;
}

int dg_launch_config(const dg_solver *h, int64_t *cfg, int n)
{
    if (!h || !cfg || n < 0) return fail(DG_EINVAL, "NULL argument or n < 0");
    const int64_t v[kLaunchCfg] = {h->plain_order, h->slab, h->ms_div, h->tuned, h->xblk, h->zlen, h->ms_chunk};
    for (int i = 0; i < n && i < kLaunchCfg; ++i) cfg[i] = v[i];
    for (int i = kLaunchCfg; i < n; ++i) cfg[i] = 0;
    return DG_OK;
}

int dg_set_launch_config(dg_solver *h, const int64_t *cfg, int n)
{
    if (!h || !cfg) return fail(DG_EINVAL, "NULL argument");
    if (n != kLaunchCfg) return fail(DG_EINVAL, "n must be 7");
    if (h->batch) return fail(DG_ESTATE, "solver belongs to a batch");
    const int64_t plain = cfg[0], slab = cfg[1], ms_div = cfg[2], xblk = cfg[4], zlen = cfg[5], chunk = cfg[6];
    if (plain != 0 && plain != 1) return fail(DG_EINVAL, "cfg[0] (tile order) must be 0 or 1");
    if (ms_div < 1 || ms_div > 1024) return fail(DG_EINVAL, "cfg[2] (halo-bound divisor) must be in 1..1024");
    if (chunk < -1 || chunk > (int64_t(1) << 30))
        return fail(DG_EINVAL, "cfg[6] (1-D chunk request) must be -1, 0 or an element count up to 2^30");
    if (h->dim == 3) {
        if (zlen < 1 || zlen > h->K[2]) return fail(DG_EINVAL, "cfg[5] (z-march length) must be in 1..K[2]");
        const int64_t nz = (h->K[2] + zlen - 1) / zlen;
        if (slab < 1 || nz % slab != 0)
            return fail(DG_EINVAL, "cfg[1] (z-slab) must divide the number of z-units ceil(K[2] / cfg[5])");
        if (xblk < 1 || h->tiles_x % xblk != 0)
            return fail(DG_EINVAL, "cfg[4] (x-block) must divide the number of x-tiles");
    } else if (slab != h->slab || xblk != h->xblk || zlen != h->zlen) {
        return fail(DG_EINVAL, "z-slab, x-block and z-march length apply to 3-D meshes only "
                               "(pass the values in use)");
    }
    h->plain_order = (int)plain;
    h->slab = slab;
    h->ms_div = (int)ms_div;
    h->xblk = xblk;
    h->zlen = zlen;
    h->ms_chunk = chunk;
    h->tuned = 0;
    return DG_OK;
}

void *dg_stream(const dg_solver *h)
{
    if (!h) return nullptr;
    // a member's stream is handed out ordered after the batch work so far
    if (h->batch && (select_device(h) != DG_OK || batch_order_member(const_cast<dg_solver *>(h)) != DG_OK))
        return nullptr;
    return static_cast<void *>(h->stream);
}

}  // extern "C"
