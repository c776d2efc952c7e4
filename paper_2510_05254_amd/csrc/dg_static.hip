// dg_static.hip -- dg_step_static: Runge-Kutta stepping of a device state the
// caller holds, with no solver handle and no device allocation, for callers
// that cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The work memory of dg_step -- the operator tables (D, w, face-point
// descriptors), the Runge-Kutta work arrays and, for more than one
// variable, the element-interleaved copy of the state -- comes from `scratch`, a
// fixed file-scope device array. Each GPU the library runs on holds its own
// copy until the process ends. In host code `scratch` names a host-side
// stand-in, so its device address is looked up once per device (with that
// device current) and kept; only that address is handed to kernels and copies.
// The kernels and stage schedules are those of dg_step, so the results are
// bitwise those of a solver created with dg_create_ex on the same arguments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/dg.h"
#include "dg_host.hpp"

namespace dg {
namespace {

constexpr size_t kStaticScratch = size_t(DG_STATIC_SCRATCH_BYTES);
static_assert(kStaticScratch % kAlign == 0, "scratch size must be a multiple of the alignment");

static __device__ __align__(256) unsigned char scratch[DG_STATIC_SCRATCH_BYTES];

// Per device: the scratch array's device address, and which operator tables
// (dim, N, equation, precision) it holds now, so a run of calls of one kernel
// class uploads them once.
constexpr int kMaxDevices = 64;
struct DeviceScratch {
    char *ptr = nullptr;
    int table_key = -1;
};
std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

int table_key(int dim, int N, int eq, int prec) { return dim + 4 * (N + 16 * (eq + 2 * prec)); }

// The device address of `scratch` on the current device (looked up once).
int scratch_on(int device, char **ptr)
{
    DeviceScratch &d = g_dev[device];
    if (!d.ptr) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(DG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        d.ptr = static_cast<char *>(p);
    }
    *ptr = d.ptr;
    return DG_OK;
}

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" int dg_step_static(int dim, int N, const int64_t *K, int equation, const double *params,
                              int precision, void *hip_stream, void *u_dev, int64_t count, int rk,
                              double dt, int64_t nsteps)
{
    int rc = validate(dim, N, K, equation, params, precision);
    if (rc) return rc;
    if (!u_dev) return fail(DG_EINVAL, "u_dev is NULL");
    if (rk != DG_RK3 && rk != DG_RK4 && rk != DG_RK6) return fail(DG_EINVAL, "rk must be 3, 4 or 6");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(DG_EINVAL, "dt must be finite and > 0");
    if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
    const size_t rsize = precision == DG_FP64 ? sizeof(double) : sizeof(float);
    if (reinterpret_cast<uintptr_t>(u_dev) % rsize != 0)
        return fail(DG_EINVAL, "u_dev must be aligned to its element size");

    dg_solver h;              // host description only; the memory is the caller's and scratch
    if ((rc = setup_solver(&h, dim, N, K, equation, params, precision))) return rc;
    if (count != h.unknowns)
        return fail(DG_EINVAL, "count must equal nvar * nodes = " + std::to_string(h.unknowns));
    // the device layout interleaves an element's variables: with more than
    // one variable the state is converted into a scratch array and back
    const bool conv = h.nvar > 1;
    const size_t need = h.lay.tables + ((rk == DG_RK6 ? 8 : 3) + (conv ? 1 : 0)) * h.lay.array;
    if (need > kStaticScratch)
        return fail(DG_ENOMEM, "dg_step_static: this problem needs " + std::to_string(need) +
                                   " bytes of work memory; the static scratch holds " +
                                   std::to_string(kStaticScratch) + " (DG_STATIC_SCRATCH_BYTES)");
    if (nsteps == 0) return DG_OK;

    hipError_t e = hipGetDevice(&h.device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (h.device < 0 || h.device >= kMaxDevices) return fail(DG_EDEVICE, "device ordinal out of range");
    h.cus = device_cus(h.device);
    h.stream = static_cast<hipStream_t>(hip_stream);

    std::lock_guard<std::mutex> lock(g_mu);
    char *base = nullptr;
    if ((rc = scratch_on(h.device, &base))) return rc;
    char *arrays = carve_tables(&h, base);
    if (conv) {
        h.U = arrays;
        arrays += h.lay.array;
    } else {
        h.U = u_dev;
    }
    carve_rk_arrays(&h, arrays, rk == DG_RK6);
    const int key = table_key(dim, N, equation, precision);
    if (g_dev[h.device].table_key != key) {
        g_dev[h.device].table_key = -1;
        if ((rc = upload_tables(&h))) return rc;
        g_dev[h.device].table_key = key;
    }
    h.has_state = true;
    if (conv && (rc = convert(&h, u_dev, precision, h.U, precision, true))) return rc;
    if ((rc = enqueue_steps(&h, rk, dt, nsteps))) return rc;
    if (conv && (rc = convert(&h, h.U, precision, u_dev, precision, false))) return rc;
    return DG_OK;
}
