// dg_msplan.hpp -- the arithmetic of the temporally blocked 1-D plan and of its
// launch schedule, free of any runtime dependency (the CPU tests compile it
// with g++ and check its invariants).
#pragma once

#include <algorithm>
#include <cstdint>

namespace dg {

// Whole mode: one workgroup holds the whole periodic mesh and runs up to
// kMsWholeSteps steps per launch, when the mesh fits the workgroup's LDS with
// at most kMsWholeNodes nodes. Chunked mode: T owned elements per workgroup
// and at most smax steps per launch; the halo, stages * smax elements per
// side, is at most capacity / ms_div and at most K (the kernel wraps a halo
// around the periodic mesh once at most), and T + 2 * halo fits the
// capacity. tcap > 0 asks for T = tcap (a chunk per CU), with smax lowered as
// far as the halos then need to fit; a tcap that cannot fit is ignored.
constexpr int kMsWholeSteps = 4096;
constexpr int64_t kMsWholeNodes = 512;

struct MsPlan {
    bool ok = false;
    int whole = 0;
    int smax = 0;
    int64_t T = 0;
    int64_t nwg = 0;
};

inline MsPlan ms_plan_for(int64_t K, int n1, int64_t cap, int64_t stages, int64_t ms_div, int64_t tcap)
{
    MsPlan pl;
    if (K < 1 || n1 < 2 || cap < 1 || stages < 1 || ms_div < 1) return pl;
    if (K <= cap && K * n1 <= kMsWholeNodes) {
        pl.whole = 1;
        pl.smax = kMsWholeSteps;
        pl.T = K;
        pl.nwg = 1;
        pl.ok = true;
        return pl;
    }
    int64_t smax = std::max<int64_t>(1, std::min(cap / (ms_div * stages), K / stages));
    int64_t T;
    if (tcap > 0 && tcap + 2 * stages <= cap) {
        T = tcap;
        smax = std::max<int64_t>(1, std::min(smax, (cap - tcap) / (2 * stages)));
    } else {
        smax = std::max<int64_t>(1, std::min(smax, (cap - 1) / (2 * stages)));
        T = cap - 2 * stages * smax;
    }
    if (T < 1 || stages * smax > K) return pl;
    pl.smax = (int)smax;
    pl.T = T;
    pl.nwg = (K + T - 1) / T;
    if (pl.nwg > (int64_t(1) << 31)) return MsPlan();
    pl.ok = true;
    return pl;
}

// Launches for nsteps steps at most smax per launch. With ping-pong arrays
// (even) the count is made even so that the state ends in U: the steps are
// spread evenly over one more launch, or, when every launch already runs a
// single step, a final copy launch (0 steps) is added.
struct MsSchedule {
    int64_t count = 0;               // launches that step
    int64_t base = 0, extra = 0;     // launch i runs base + (i < extra) steps
    bool copy = false;               // a trailing 0-step launch
    int64_t launches() const { return count + (copy ? 1 : 0); }
    int steps(int64_t i) const { return i < count ? int(base + (i < extra ? 1 : 0)) : 0; }
};

inline MsSchedule ms_schedule(int64_t nsteps, int smax, bool even)
{
    MsSchedule s;
    if (nsteps < 1 || smax < 1) return s;
    s.count = (nsteps + smax - 1) / smax;
    if (even && (s.count & 1)) {
        if (nsteps > s.count)
            ++s.count;
        else
            s.copy = true;
    }
    s.base = nsteps / s.count;
    s.extra = nsteps % s.count;
    return s;
}

// the owned elements per workgroup that spread `elements` over `cus` CUs
inline int64_t ms_spread(int64_t elements, int cus) { return (elements + cus - 1) / cus; }

}  // namespace dg
