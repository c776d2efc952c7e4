// dg_batch.cpp -- batched stepping: many solvers advanced together, one
// launch per RK stage per kernel class (precision, equation, dim, N, scheme).
//
// Per class the batch keeps, on the device: the StageParams of every active
// member for every stage of its scheme (built by the same stage programs as
// dg_step, so a member's arithmetic is exactly what dg_step would run), and a
// virtual-tile -> member map. A tick is one RK step of every active member;
// dg_batch_run enqueues as many ticks as the shortest remaining member allows,
// optionally replaying a hipGraph of one tick. Descriptors are rebuilt only
// when the set of active members changes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "dg_host.hpp"

using namespace dg;

namespace {

// A graph of one tick (the per-stage launches of the 2-D/3-D classes) is
// captured once per membership, for the first run of at least this many
// ticks; shorter runs launch directly, since capture and instantiation cost
// more than a few direct launches. 1-D classes are advanced by the
// temporally blocked kernel, up to smax steps per launch.
constexpr int64_t kGraphMinTicks = 4;
// Groups run on up to kLanes streams at once: the batch stream and kLanes - 1
// side streams forked from it and joined back within every run (the GPU has
// four hardware queues per process).
constexpr int kLanes = 4;

struct Member {
    dg_solver *h;
    int rk;
    double dt;
    int64_t remaining;
};

struct Group {
    int prec = 0, eq = 0, dim = 0, N = 0, rk = 0, stages = 0;
    BatchFn fn = nullptr;
    BatchXFn fnx = nullptr;        // RK6: fused stages with further inputs
    int nin[8] = {};               // RK inputs of each stage (same for every member)
    // 1-D classes step with the temporally blocked kernel: per member an
    // MsSolve (header, at off_params) and its workgroups; up to smax steps
    // per launch
    bool ms = false;
    MsFn msfn = nullptr;
    int smax = 0;
    int64_t tcap = 0;              // owned elements per workgroup asked for (0: the plan's own)
    bool pp = false;               // members ping-pong between U and Ya (some has several workgroups)
    bool buf = true;
    std::vector<int> idx;          // member indices
    uint32_t ntiles = 0;
    size_t off_params = 0, off_solve = 0, off_base = 0, off_extra = 0;
    const void *D = nullptr;
    const uint32_t *ftab = nullptr;
    int64_t grid = 0;
    int lane = 0;                  // stream the group's launches go to
};

}  // namespace

struct dg_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int flags = 0;
    std::vector<Member> members;
    std::vector<Group> groups;
    bool dirty = true;
    char *dbuf = nullptr;
    size_t dbuf_cap = 0;
    // descriptors are staged in pinned host memory, two slots used in turn:
    // a slot is rewritten once the copy out of it (stream-ordered behind the
    // ticks enqueued before it) has run, so a rebuild never waits for the
    // whole stream
    char *pin[2] = {nullptr, nullptr};
    size_t pin_cap[2] = {0, 0};
    hipEvent_t pin_ev[2] = {nullptr, nullptr};
    bool pin_used[2] = {false, false};
    int pin_slot = 0;
    hipEvent_t done = nullptr;
    hipStream_t side[kLanes - 1] = {};
    hipEvent_t fork = nullptr, join[kLanes - 1] = {};
    int lanes = 1;                 // lanes the current groups use
    // per lane, the captured tick of its stage-kernel groups
    hipGraph_t graph[kLanes] = {};
    hipGraphExec_t gexec[kLanes] = {};
    // graphs replaced while launches of them may still be queued on the
    // stream: destroyed once the event recorded after their last launch has
    // completed
    struct Retired {
        hipGraphExec_t exec;
        hipGraph_t graph;
        hipEvent_t after;
    };
    std::vector<Retired> retired;
};

namespace {

int member_index(const dg_batch *b, const dg_solver *h)
{
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i].h == h) return (int)i;
    return -1;
}

// Destroy the retired graphs whose launches have all run (all of them when
// wait is set: the caller has synchronized the stream).
void reap_graphs(dg_batch *b, bool wait)
{
    size_t keep = 0;
    for (size_t i = 0; i < b->retired.size(); ++i) {
        dg_batch::Retired &r = b->retired[i];
        const hipError_t q = wait ? hipSuccess : hipEventQuery(r.after);
        if (q == hipSuccess) {
            (void)hipGraphExecDestroy(r.exec);
            if (r.graph) (void)hipGraphDestroy(r.graph);
            (void)hipEventDestroy(r.after);
        } else {
            if (q != hipErrorNotReady) (void)hipGetLastError();
            b->retired[keep++] = r;
        }
    }
    b->retired.resize(keep);
}

// Stop using the captured tick graphs. Launches of them may still be queued
// (the side streams' work is joined into the batch stream), so they are
// retired behind an event rather than destroyed (their kernel arguments must
// outlive those launches).
void drop_graph(dg_batch *b)
{
    for (int k = 0; k < kLanes; ++k) {
        if (b->gexec[k]) {
            hipEvent_t ev = nullptr;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
                hipEventRecord(ev, b->stream) == hipSuccess) {
                b->retired.push_back({b->gexec[k], b->graph[k], ev});
            } else {
                // no event: wait for the stream, then the graph is free
                (void)hipGetLastError();
                if (ev) (void)hipEventDestroy(ev);
                (void)hipStreamSynchronize(b->stream);
                (void)hipGraphExecDestroy(b->gexec[k]);
                if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
            }
        } else if (b->graph[k]) {
            (void)hipGraphDestroy(b->graph[k]);
        }
        b->gexec[k] = nullptr;
        b->graph[k] = nullptr;
    }
    reap_graphs(b, false);
}

hipStream_t lane_stream(const dg_batch *b, int k) { return k == 0 ? b->stream : b->side[k - 1]; }

// Spread the groups over the lanes, largest estimated work first, each to the
// least loaded lane; create the side streams and events on first use.
int assign_lanes(dg_batch *b)
{
    const int ng = (int)b->groups.size();
    std::vector<int> order(ng);
    std::vector<double> cost(ng);
    for (int i = 0; i < ng; ++i) {
        const Group &g = b->groups[i];
        order[i] = i;
        // a multi-step launch advances up to smax steps, a stage launch one stage
        cost[i] = (double)g.ntiles * (g.ms ? 2.0 * g.stages : (double)g.stages);
    }
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    b->lanes = std::max(1, std::min(kLanes, ng));
    double load[kLanes] = {};
    for (int i : order) {
        int best = 0;
        for (int k = 1; k < b->lanes; ++k)
            if (load[k] < load[best]) best = k;
        b->groups[i].lane = best;
        load[best] += cost[i];
    }
    for (int k = 1; k < b->lanes; ++k) {
        if (!b->side[k - 1])
            DG_HIP(hipStreamCreateWithFlags(&b->side[k - 1], hipStreamNonBlocking), "hipStreamCreate");
        if (!b->join[k - 1]) DG_HIP(hipEventCreateWithFlags(&b->join[k - 1], hipEventDisableTiming), "hipEventCreate");
    }
    if (b->lanes > 1 && !b->fork) DG_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate");
    return DG_OK;
}

// Group the active members by class and upload their stage descriptors.
int rebuild(dg_batch *b)
{
    drop_graph(b);
    b->groups.clear();
    b->lanes = 1;
    std::map<std::tuple<int, int, int, int, int>, int> key;
    for (size_t i = 0; i < b->members.size(); ++i) {
        const Member &m = b->members[i];
        if (m.remaining <= 0) continue;
        const dg_solver *h = m.h;
        auto k = std::make_tuple(h->prec, h->eq, h->dim, h->N, m.rk);
        auto it = key.find(k);
        if (it == key.end()) {
            Group g;
            g.prec = h->prec; g.eq = h->eq; g.dim = h->dim; g.N = h->N; g.rk = m.rk;
            g.stages = stage_count(m.rk);
            g.fn = batch_fn(h->prec, h->eq, h->dim, h->N);
            if (!g.fn) return fail(DG_ENOTSUP, "no batched kernel for this class");
            if (m.rk == DG_RK6) {
                g.fnx = batch_x_fn(h->prec, h->eq, h->dim, h->N);
                if (!g.fnx) return fail(DG_ENOTSUP, "no batched RK6 kernel for this class");
            }
            for (int s = 0; s < g.stages; ++s) {
                if (m.rk != DG_RK6) {
                    g.nin[s] = stage_program(h, m.rk, s, m.dt).nin;
                    continue;
                }
                StageParams p;
                ExtraIn x;
                const int rc = rk6_stage(h, s, m.dt, p, x);
                if (rc) return rc;
                g.nin[s] = p.nin;
            }
            if (ms_plan(h, m.rk).ok) {
                g.ms = true;
                g.msfn = ms_fn(h->prec, h->eq, h->N);
                g.smax = kMsWholeSteps;
            }
            g.D = h->Dtab;
            g.ftab = h->ftab;
            key[k] = (int)b->groups.size();
            b->groups.push_back(g);
            it = key.find(k);
        }
        b->groups[it->second].idx.push_back((int)i);
    }
    // device layout per group [params: stages x n][tile_solve: ntiles][tile_base: n+1];
    // the host stages params and tile_base, a fill kernel writes tile_solve.
    // header: per group params and tile_base (staged on the host, one copy);
    // after it the tile_solve arrays (written on the device).
    size_t header = 0;
    for (Group &g : b->groups) {
        const size_t n = g.idx.size();
        if (g.ms) {
            // a group of chunked meshes with fewer workgroups than the GPU
            // has CUs is cut into smaller chunks, about one per CU
            int64_t wgs = 0, chunked = 0;
            const int cus = b->members[g.idx[0]].h->cus;
            for (int i : g.idx) {
                const MsPlan pl = ms_plan(b->members[i].h, b->members[i].rk);
                if (!pl.ok) return fail(DG_ENOTSUP, "no multi-step plan for a 1-D member");
                wgs += pl.nwg;
                if (!pl.whole) chunked += b->members[i].h->K[0];
            }
            g.tcap = (chunked > 0 && wgs < cus) ? ms_spread(chunked, cus) : 0;
        }
        uint64_t tiles = 0;
        for (int i : g.idx) {
            const dg_solver *h = b->members[i].h;
            if (g.ms) {
                const MsPlan pl = ms_plan(h, b->members[i].rk, g.tcap);
                if (!pl.ok) return fail(DG_ENOTSUP, "no multi-step plan for a 1-D member");
                tiles += (uint64_t)pl.nwg;
                g.smax = std::min(g.smax, pl.smax);
                g.pp = g.pp || pl.nwg > 1;
                continue;
            }
            tiles += (uint64_t)h->ntiles;
            const int64_t bytes = h->nodes * h->nvar * (h->prec == DG_FP64 ? 8 : 4);
            if (bytes >= (int64_t(1) << 31)) g.buf = false;
        }
        if (tiles >= (uint64_t(1) << 32)) return fail(DG_ENOTSUP, "batch too large for one launch");
        g.ntiles = (uint32_t)tiles;
        g.off_params = header;
        header = round_up(header + (g.ms ? sizeof(MsSolve) * n : sizeof(StageParams) * n * g.stages));
        g.off_extra = header;
        if (g.fnx) header = round_up(header + sizeof(ExtraIn) * n * g.stages);
        g.off_base = header;
        header = round_up(header + sizeof(uint32_t) * (n + 1));
        g.grid = std::min<int64_t>((int64_t)tiles, kMaxGrid);
    }
    if (header == 0) return DG_OK;
    int rc = assign_lanes(b);
    if (rc) return rc;
    size_t total = header;
    for (Group &g : b->groups) {
        g.off_solve = total;
        total = round_up(total + sizeof(uint32_t) * g.ntiles);
    }
    // the staging slot: wait for the copy that last read it, grow it if needed
    const int slot = b->pin_slot;
    if (b->pin_used[slot]) DG_HIP(hipEventSynchronize(b->pin_ev[slot]), "hipEventSynchronize");
    if (header > b->pin_cap[slot]) {
        const size_t cap = std::max(header, 2 * b->pin_cap[slot]);     // grow geometrically
        if (b->pin[slot]) (void)hipHostFree(b->pin[slot]);
        b->pin[slot] = nullptr;
        b->pin_cap[slot] = 0;
        hipError_t e = hipHostMalloc((void **)&b->pin[slot], cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b->pin[slot] = nullptr;
            return fail(DG_ENOMEM, "cannot allocate pinned batch staging");
        }
        b->pin_cap[slot] = cap;
    }
    char *staging = b->pin[slot];
    for (Group &g : b->groups) {
        const size_t n = g.idx.size();
        StageParams *par = reinterpret_cast<StageParams *>(staging + g.off_params);
        uint32_t *base = reinterpret_cast<uint32_t *>(staging + g.off_base);
        uint32_t t0 = 0;
        for (size_t j = 0; j < n; ++j) {
            const Member &m = b->members[g.idx[j]];
            base[j] = t0;
            if (g.ms) {
                const MsPlan pl = ms_plan(m.h, m.rk, g.tcap);
                reinterpret_cast<MsSolve *>(par)[j] = ms_solve(m.h, m.rk, m.dt, pl, g.pp);
                t0 += (uint32_t)pl.nwg;
                continue;
            }
            if (g.fnx) {
                ExtraIn *ext = reinterpret_cast<ExtraIn *>(staging + g.off_extra);
                for (int s = 0; s < g.stages; ++s) {
                    const int rc = rk6_stage(m.h, s, m.dt, par[s * n + j], ext[s * n + j]);
                    if (rc) return rc;
                }
            } else {
                for (int s = 0; s < g.stages; ++s) par[s * n + j] = stage_program(m.h, m.rk, s, m.dt);
            }
            t0 += (uint32_t)m.h->ntiles;
        }
        base[n] = t0;
    }
    if (total > b->dbuf_cap) {
        DG_HIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        if (b->dbuf) (void)hipFree(b->dbuf);
        total = std::max(total, 2 * b->dbuf_cap);     // grow geometrically
        b->dbuf = nullptr;
        b->dbuf_cap = 0;
        hipError_t e = hipMalloc((void **)&b->dbuf, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b->dbuf = nullptr;
            return fail(DG_ENOMEM, "cannot allocate batch descriptors");
        }
        b->dbuf_cap = total;
    }
    // stream-ordered after the ticks already enqueued, which still read the
    // previous descriptors
    DG_HIP(hipMemcpyAsync(b->dbuf, staging, header, hipMemcpyHostToDevice, b->stream), "hipMemcpyAsync");
    if (!b->pin_ev[slot]) DG_HIP(hipEventCreateWithFlags(&b->pin_ev[slot], hipEventDisableTiming), "hipEventCreate");
    DG_HIP(hipEventRecord(b->pin_ev[slot], b->stream), "hipEventRecord");
    b->pin_used[slot] = true;
    b->pin_slot = slot ^ 1;
    for (const Group &g : b->groups)
        DG_HIP(launch_fill_tile_map(reinterpret_cast<const uint32_t *>(b->dbuf + g.off_base),
                                    (uint32_t)g.idx.size(),
                                    reinterpret_cast<uint32_t *>(b->dbuf + g.off_solve), b->stream),
               "tile map launch");
    return DG_OK;
}

// One RK step of the stage-kernel groups on lane k, enqueued on stream st.
int launch_tick(dg_batch *b, int k, hipStream_t st)
{
    int smax = 0;
    for (const Group &g : b->groups) smax = std::max(smax, g.stages);
    for (int s = 0; s < smax; ++s)
        for (const Group &g : b->groups) {
            if (g.ms || g.lane != k || s >= g.stages) continue;
            const uint32_t n = (uint32_t)g.idx.size();
            BatchLaunch L;
            L.params = reinterpret_cast<const StageParams *>(b->dbuf + g.off_params) + (size_t)s * n;
            L.tile_solve = reinterpret_cast<const uint32_t *>(b->dbuf + g.off_solve);
            L.tile_base = reinterpret_cast<const uint32_t *>(b->dbuf + g.off_base);
            L.D = g.D;
            L.ftab = g.ftab;
            L.ntiles = g.ntiles;
            L.xq = g.ntiles / kXcds;
            L.xr = g.ntiles % kXcds;
            L.nsolves = n;
            L.extra = nullptr;
            if (g.fnx) {
                L.extra = reinterpret_cast<const ExtraIn *>(b->dbuf + g.off_extra) + (size_t)s * n;
                DG_HIP(g.fnx(L, g.buf, g.grid, st), "batched RK6 stage kernel launch");
            } else {
                DG_HIP(g.fn(L, g.buf, g.nin[s], g.grid, st), "batched stage kernel launch");
            }
        }
    return DG_OK;
}

// Member streams wait for the batch work enqueued so far.
// The batch work enqueued so far ends at `done`; a member's stream waits for it
// when the member is read (batch_order_member), not after every run, so a run
// costs O(1) stream operations however many members the batch has.
int publish(dg_batch *b)
{
    DG_HIP(hipEventRecord(b->done, b->stream), "hipEventRecord");
    return DG_OK;
}

}  // namespace

namespace dg {

int batch_order_member(dg_solver *h)
{
    dg_batch *b = h->batch;
    if (b && h->stream != b->stream) DG_HIP(hipStreamWaitEvent(h->stream, b->done, 0), "hipStreamWaitEvent");
    return DG_OK;
}

int batch_after_member(dg_solver *h)
{
    dg_batch *b = h->batch;
    if (!b || h->stream == b->stream) return DG_OK;
    hipEvent_t ev;
    DG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hipError_t e = hipEventRecord(ev, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(e, "stream ordering");
    return DG_OK;
}

}  // namespace dg

extern "C" {

int dg_batch_create(void *hip_stream, int flags, dg_batch **out)
{
    if (!out) return fail(DG_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~DG_BATCH_GRAPH) return fail(DG_EINVAL, "unknown batch flags");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(DG_EDEVICE, "no HIP device available");
    }
    dg_batch *b = new (std::nothrow) dg_batch();
    if (!b) return fail(DG_ENOMEM, "host allocation failed");
    b->flags = flags;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) {
        if (hip_stream) {
            b->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
            b->own_stream = e == hipSuccess;
        }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return hip_fail(e, "batch setup");
    }
    *out = b;
    return DG_OK;
}

int dg_batch_destroy(dg_batch *b)
{
    if (!b) return DG_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (Member &m : b->members) m.h->batch = nullptr;
    drop_graph(b);
    reap_graphs(b, true);
    if (b->dbuf) (void)hipFree(b->dbuf);
    for (int i = 0; i < 2; ++i) {
        if (b->pin[i]) (void)hipHostFree(b->pin[i]);
        if (b->pin_ev[i]) (void)hipEventDestroy(b->pin_ev[i]);
    }
    if (b->done) (void)hipEventDestroy(b->done);
    for (int k = 0; k < kLanes - 1; ++k) {
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return DG_OK;
}

int dg_batch_add(dg_batch *b, dg_solver *h, int rk, double dt, int64_t nsteps)
{
    if (!b || !h) return fail(DG_EINVAL, "NULL argument");
    if (rk != DG_RK3 && rk != DG_RK4 && rk != DG_RK6) return fail(DG_EINVAL, "rk must be DG_RK3, DG_RK4 or DG_RK6");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(DG_EINVAL, "dt must be finite and > 0");
    if (nsteps < 1) return fail(DG_EINVAL, "nsteps must be >= 1");
    if (!h->has_state) return fail(DG_ESTATE, "dg_set_state has not been called");
    if (h->batch) return fail(DG_ESTATE, "solver already belongs to a batch");
    if (h->device != b->device) return fail(DG_EINVAL, "solver is on another device");
    int rc = select_device(h);
    if (rc) return rc;
    if (rk == DG_RK6 && (rc = ensure_rk6(h))) return rc;
    // the batch's work on h follows everything already enqueued on h's stream
    if (h->stream != b->stream) {
        hipEvent_t ev;
        DG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
        hipError_t e = hipEventRecord(ev, h->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess) return hip_fail(e, "stream ordering");
    }
    b->members.push_back(Member{h, rk, dt, nsteps});
    h->batch = b;
    b->dirty = true;
    return DG_OK;
}

int dg_batch_remove(dg_batch *b, dg_solver *h)
{
    if (!b || !h) return fail(DG_EINVAL, "NULL argument");
    const int i = member_index(b, h);
    if (i < 0) return fail(DG_EINVAL, "solver is not a member of this batch");
    int rc = publish(b);
    if (rc || (rc = batch_order_member(h))) return rc;
    const bool active = b->members[i].remaining > 0;
    b->members.erase(b->members.begin() + i);
    h->batch = nullptr;
    if (active) b->dirty = true;
    return DG_OK;
}

int dg_batch_run(dg_batch *b, int64_t max_steps, int64_t *steps_done)
{
    if (!b) return fail(DG_EINVAL, "batch is NULL");
    if (max_steps < 0) return fail(DG_EINVAL, "max_steps must be >= 0");
    if (steps_done) *steps_done = 0;
    DG_HIP(hipSetDevice(b->device), "hipSetDevice");
    int64_t steps = max_steps;
    bool any = false;
    for (const Member &m : b->members)
        if (m.remaining > 0) {
            steps = std::min(steps, m.remaining);
            any = true;
        }
    if (!any || steps == 0) return DG_OK;
    int rc;
    if (b->dirty) {
        if ((rc = rebuild(b))) return rc;
        b->dirty = false;
    }
    bool ticked[kLanes] = {};
    for (const Group &g : b->groups)
        if (!g.ms) ticked[g.lane] = true;
    // capture the lanes' tick graphs before any work is forked
    bool captured = false;
    for (int k = 0; k < kLanes; ++k) captured = captured || b->gexec[k];
    const bool graph = (b->flags & DG_BATCH_GRAPH) && (captured || steps >= kGraphMinTicks);
    for (int k = 0; graph && k < b->lanes; ++k) {
        if (!ticked[k] || b->gexec[k]) continue;
        const hipStream_t st = lane_stream(b, k);
        DG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        rc = launch_tick(b, k, st);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph[k] = g;
        e = hipGraphInstantiate(&b->gexec[k], b->graph[k], nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_fail(e, "hipGraphInstantiate");
        }
    }
    // fork: the side lanes start after everything enqueued on the batch stream
    if (b->lanes > 1) {
        DG_HIP(hipEventRecord(b->fork, b->stream), "hipEventRecord");
        for (int k = 1; k < b->lanes; ++k) DG_HIP(hipStreamWaitEvent(b->side[k - 1], b->fork, 0), "hipStreamWaitEvent");
    }
    // join: the batch stream continues after every lane's work (also when a
    // launch failed part way)
    auto join = [&]() -> int {
        for (int k = 1; k < b->lanes; ++k) {
            DG_HIP(hipEventRecord(b->join[k - 1], b->side[k - 1]), "hipEventRecord");
            DG_HIP(hipStreamWaitEvent(b->stream, b->join[k - 1], 0), "hipStreamWaitEvent");
        }
        return DG_OK;
    };
    for (const Group &g : b->groups) {
        if (!g.ms) continue;
        MsLaunch L;
        std::memset(&L, 0, sizeof(L));
        L.solves = reinterpret_cast<const MsSolve *>(b->dbuf + g.off_params);
        L.wg_solve = reinterpret_cast<const uint32_t *>(b->dbuf + g.off_solve);
        L.wg_base = reinterpret_cast<const uint32_t *>(b->dbuf + g.off_base);
        L.D = g.D;
        L.rk = g.rk;
        L.nwg = g.ntiles;
        const MsSchedule sc = ms_schedule(steps, g.smax, g.pp);
        for (int64_t i = 0; i < sc.launches(); ++i) {
            L.nsteps = sc.steps(i);
            const hipError_t e = g.msfn(L, lane_stream(b, g.lane));
            if (e != hipSuccess) {
                (void)join();
                return hip_fail(e, "batched multi-step kernel launch");
            }
            L.flip ^= g.pp ? 1 : 0;
        }
    }
    for (int k = 0; k < b->lanes; ++k) {
        if (!ticked[k]) continue;
        const hipStream_t st = lane_stream(b, k);
        for (int64_t t = 0; t < steps; ++t) {
            if (graph) {
                const hipError_t e = hipGraphLaunch(b->gexec[k], st);
                rc = e == hipSuccess ? DG_OK : hip_fail(e, "hipGraphLaunch");
            } else {
                rc = launch_tick(b, k, st);
            }
            if (rc) {
                (void)join();
                return rc;
            }
        }
    }
    if ((rc = join())) return rc;
    for (Member &m : b->members)
        if (m.remaining > 0) {
            m.remaining -= steps;
            if (m.remaining == 0) b->dirty = true;
        }
    if ((rc = publish(b))) return rc;
    if (steps_done) *steps_done = steps;
    return DG_OK;
}

int dg_batch_remaining(const dg_batch *b, const dg_solver *h, int64_t *remaining)
{
    if (!b || !h || !remaining) return fail(DG_EINVAL, "NULL argument");
    const int i = member_index(b, h);
    if (i < 0) return fail(DG_EINVAL, "solver is not a member of this batch");
    *remaining = std::max<int64_t>(b->members[i].remaining, 0);
    return DG_OK;
}

int dg_batch_size(const dg_batch *b, int *members, int *active)
{
    if (!b) return fail(DG_EINVAL, "batch is NULL");
    int a = 0;
    for (const Member &m : b->members) a += m.remaining > 0;
    if (members) *members = (int)b->members.size();
    if (active) *active = a;
    return DG_OK;
}

int dg_batch_synchronize(dg_batch *b)
{
    if (!b) return fail(DG_EINVAL, "batch is NULL");
    DG_HIP(hipSetDevice(b->device), "hipSetDevice");
    DG_HIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return DG_OK;
}

}  // extern "C"
