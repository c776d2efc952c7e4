// dg_probe.hip -- streaming bandwidth reference for measurement (no part of
// the method): out_o[i] = sum_j in_j[i] + o over 16-byte elements, with the
// read:write mix of a fused stage. One thread per 16-byte element, coalesced
// b128 loads and stores, no LDS, no reuse: the rate it reaches is what plain
// streaming of the same bytes achieves on this GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dg.h"
#include "dg_host.hpp"

namespace dg {
namespace {

struct ProbeArgs {
    const double2 *in[3];
    double2 *out[2];
    int64_t n;   // 16-byte elements per array
};

template <int NIN, int NOUT>
__global__ void __launch_bounds__(256) probe_kernel(const ProbeArgs a)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= a.n) return;
    double2 s = a.in[0][i];
#pragma unroll
    for (int j = 1; j < NIN; ++j) {
        const double2 t = a.in[j][i];
        s.x += t.x;
        s.y += t.y;
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) a.out[o][i] = double2{s.x + o, s.y + o};
}

template <int NIN>
hipError_t launch_nout(const ProbeArgs &a, int nout, hipStream_t s)
{
    const dim3 g((unsigned)((a.n + 255) / 256)), b(256);
    if (nout == 1) hipLaunchKernelGGL((probe_kernel<NIN, 1>), g, b, 0, s, a);
    else hipLaunchKernelGGL((probe_kernel<NIN, 2>), g, b, 0, s, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace dg

extern "C" int dg_bandwidth_probe(void *hip_stream, const void *const *in, int nin, void *const *out,
                                  int nout, int64_t bytes)
{
    using namespace dg;
    if (nin < 1 || nin > 3 || nout < 1 || nout > 2) return fail(DG_EINVAL, "nin must be 1..3, nout 1..2");
    if (!in || !out) return fail(DG_EINVAL, "NULL argument");
    if (bytes < 16 || bytes % 16 != 0 || bytes / 16 > (int64_t(1) << 38))
        return fail(DG_EINVAL, "bytes must be a positive multiple of 16");
    ProbeArgs a{};
    for (int j = 0; j < nin; ++j) {
        if (!in[j] || reinterpret_cast<uintptr_t>(in[j]) % 16) return fail(DG_EINVAL, "input not 16-byte aligned");
        a.in[j] = static_cast<const double2 *>(in[j]);
    }
    for (int o = 0; o < nout; ++o) {
        if (!out[o] || reinterpret_cast<uintptr_t>(out[o]) % 16) return fail(DG_EINVAL, "output not 16-byte aligned");
        a.out[o] = static_cast<double2 *>(out[o]);
    }
    a.n = bytes / 16;
    if ((a.n + 255) / 256 > 0x7fffffff) return fail(DG_EINVAL, "arrays too large");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    switch (nin) {
    case 1: e = launch_nout<1>(a, nout, s); break;
    case 2: e = launch_nout<2>(a, nout, s); break;
    default: e = launch_nout<3>(a, nout, s); break;
    }
    DG_HIP(e, "probe kernel launch");
    return DG_OK;
}
