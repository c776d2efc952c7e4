// dg_host.hpp -- host-only declarations of the runtime (not part of the ABI):
// the solver object behind the opaque dg_solver handle, workspace layout,
// error helpers and the fused-stage programs shared by single-solve stepping
// and batched stepping.
#pragma once

#include <string>

#include "../../include/dg.h"
#include "dg_internal.hpp"
#include "dg_msplan.hpp"

namespace dg {

constexpr size_t kAlign = 256;
constexpr int64_t kReduceBlocks = 1024;
constexpr size_t kFaceTableBytes = 16384;

// LGL nodes xi[N+1], weights w[N+1] and D[(N+1)^2] (row-major, D[i*(N+1)+j]).
void lgl_operator(int N, double *xi, double *w, double *D);

// Face-point descriptor table of a workgroup tile (4 uint32 per face point).
int face_table_size(int dim, int N, int epb, int epy);
// nv: variables (values per element in the state arrays = nv * (N+1)^dim).
void build_face_table(int dim, int N, int epb, int epy, int nv, uint32_t *tab);

// Device workspace of one solver: tables, then the RK arrays.
struct Layout {
    size_t tables = 0;      // D (state precision), w (FP64), reduction partials, face table
    size_t array = 0;       // one state array
    size_t base = 0;        // tables + 4 arrays (RK3/RK4)
    size_t rk6 = 0;         // base + 5 more arrays (RK6 k-store)
};

// Record msg as the calling thread's last error and return code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
size_t round_up(size_t x);

#define DG_HIP(call, what)                                     \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ::dg::hip_fail(e_, what); \
    } while (0)

}  // namespace dg

// entries of a launch configuration (dg_launch_config / dg_set_launch_config)
constexpr int kLaunchCfg = 7;

struct dg_solver {
    int dim = 0, N = 0, eq = 0, prec = 0, nvar = 0, n1 = 0, np = 0;
    int64_t K[3] = {1, 1, 1};
    int64_t nodes = 0, unknowns = 0;
    double par[3] = {0, 0, 0};
    double xi[dg::kMaxNP1], w[dg::kMaxNP1], D[dg::kMaxNP1 * dg::kMaxNP1];
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    dg::Layout lay;
    void *Dtab = nullptr;
    double *wtab = nullptr;
    uint32_t *ftab = nullptr;
    double *partial = nullptr;
    void *U = nullptr, *A = nullptr, *Ya = nullptr, *Yb = nullptr;
    void *kx[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // RK6 k3..k7
    char *rk6_mem = nullptr;        // library-owned RK6 extension
    bool has_state = false;
    dg::StageFn stage = nullptr;
    int epb = 0, epy = 1;
    int64_t tiles_x = 0, tiles_y = 1, slab = 1, xblk = 1, ntiles = 0, grid = 0;
    // launch configuration (dg_autotune may change it; results do not depend
    // on it): tile order 0 XCD-contiguous / 1 plain; 1-D steps per launch
    // follow from the halo bound capacity / (ms_div * stages)
    int plain_order = 0;
    int ms_div = 10;
    // 1-D chunk request: 0 one chunk per CU, -1 none (the halo-bound plan),
    // k > 0 k owned elements per workgroup
    int64_t ms_chunk = 0;
    int cus = 256;                  // compute units of the device
    int64_t zlen = 1;               // 3-D: layers per z-marching unit (1 = one layer per tile)
    int tuned = 0;
    dg_batch *batch = nullptr;      // batch this solver belongs to, if any
};

namespace dg {

int select_device(const dg_solver *h);
// Argument checks shared by every entry point that describes a mesh.
int validate(int dim, int N, const int64_t *K, int eq, const double *params, int prec);
Layout layout_for(int dim, int N, const int64_t *K, int eq, int prec);
// Host-side description of a solve (mesh, operator, tiles, default launch
// configuration); no device call.
int setup_solver(dg_solver *h, int dim, int N, const int64_t *K, int equation, const double *params,
                 int precision);
// Point the table fields of h into device memory at p; returns the first
// byte after the tables (the start of the state arrays).
char *carve_tables(dg_solver *h, char *p);
// Point A, Ya, Yb (and the RK6 store when rk6) at consecutive state-sized
// arrays from p; returns the first byte after them.
char *carve_rk_arrays(dg_solver *h, char *p, bool rk6);
// Upload D, w and the face-point table to h's table fields on h's stream,
// and wait for them.
int upload_tables(dg_solver *h);
// Device staging area of at least unknowns doubles (the RK arrays Ya, Yb,
// free between steps).
double *staging(dg_solver *h);
// Convert a state array between the ABI's variable-major layout and the
// device's element-interleaved layout (to_internal: src variable-major), with
// precisions src_prec -> dst_prec, on h's stream.
int convert(dg_solver *h, const void *src, int src_prec, void *dst, int dst_prec, bool to_internal);
// Enqueue nsteps steps of scheme rk on h's stream (arguments already checked,
// device selected, RK6 storage in place).
int enqueue_steps(dg_solver *h, int rk, double dt, int64_t nsteps);
// Launch parameters common to every stage of h (mesh, operator, tiles).
// zmarch: for the single-solve RK3/RK4 stage kernel, whose 3-D classes run
// units of h->zlen layers; otherwise one layer per tile.
StageParams base_params(const dg_solver *h, bool zmarch = false);
// Number of fused stages of scheme rk (3, 4 or 7 for RK6).
int stage_count(int rk);
// Parameters of fused stage s of the RK3/RK4 schedule with step dt.
StageParams stage_program(const dg_solver *h, int rk, int s, double dt, bool zmarch = false);

// Batch members: before h's state is read on h's stream, that stream waits
// for the batch work enqueued so far; after an asynchronous read, the batch
// stream waits for the read (no-ops for a solver outside a batch).
int batch_order_member(dg_solver *h);
int batch_after_member(dg_solver *h);
// The RK6 stage store (kx) of h: in h's workspace, or allocated by the library
// for a library-owned workspace.
int ensure_rk6(dg_solver *h);
// Stage s (0..6) of the RK6 schedule as stage parameters and further inputs.
int rk6_stage(const dg_solver *h, int s, double dt, StageParams &p, ExtraIn &x);
// 1-D multi-step plan of h for scheme rk (ms_plan_for, after checking that
// the kernel exists and its stage program is the host's); tcap as there.
MsPlan ms_plan(const dg_solver *h, int rk, int64_t tcap = 0);
// compute units of a device (256 if the runtime does not say)
int device_cus(int device);
// Stage program of scheme rk as array indices (0 U, 1 A, 2 Ya, 3 Yb).
MsProgram ms_program(const dg_solver *h, int rk);
// whether a stage program is the multi-step kernel's kMsProgRk3/kMsProgRk4
bool ms_program_matches(const MsProgram &g, int rk);
// Per-solve multi-step parameters (coefficients for step dt).
// pingpong: the solve's launches alternate between U and Ya (V = Ya), else
// update U in place (V = U; only for a mesh held by one workgroup)
MsSolve ms_solve(const dg_solver *h, int rk, double dt, const MsPlan &pl, bool pingpong);


}  // namespace dg
