"""Host logic of the temporally blocked 1-D kernel's plan and launch schedule
(csrc/dg_msplan.hpp), compiled here with g++ and checked exhaustively over
small and large meshes, capacities, halo-bound divisors and requested chunk
sizes:
* whole mode only for meshes that fit; chunked plans have T >= 1, smax >= 1,
  T + 2 * stages * smax <= capacity (the chunk and its halos fit the LDS) and
  stages * smax <= K (the kernel wraps a halo around the mesh once at most);
* the chunks tile [0, K): every element is owned by exactly one workgroup, and
  every global element a workgroup loads (owned range plus halos, wrapped
  once) lies in [0, K);
* a schedule runs exactly nsteps steps in launches of 1..smax steps (plus a
  final 0-step copy launch only when asked for an even count that cannot be
  had otherwise), and an even count when asked.
Test infrastructure only; no GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2510_05254_amd", "csrc", "dg_msplan.hpp")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "dg_msplan.hpp"
using namespace dg;
static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails++ < 10) { printf("FAIL %s: ", #c); printf(__VA_ARGS__); printf("\n"); } } } while (0)
int main() {
    const int64_t Ks[] = {1, 2, 7, 16, 57, 63, 64, 100, 129, 255, 256, 257, 700, 1500, 5000, 20000, 57023, 65536, 1000003};
    const int64_t caps[] = {64, 113, 256, 282, 350, 508, 1017, 3412};
    const int64_t divs[] = {1, 2, 3, 6, 10, 24, 40, 1024};
    int plans = 0, scheds = 0;
    for (int64_t K : Ks) for (int n1 = 2; n1 <= 9; ++n1) for (int64_t cap : caps)
    for (int64_t stages = 3; stages <= 4; ++stages) for (int64_t div : divs)
    for (int64_t tcap : {int64_t(0), ms_spread(K, 256), ms_spread(K, 128), int64_t(1), cap}) {
        const MsPlan p = ms_plan_for(K, n1, cap, stages, div, tcap);
        ++plans;
        CHECK(p.ok, "K=%lld n1=%d cap=%lld", (long long)K, n1, (long long)cap);
        if (!p.ok) continue;
        if (p.whole) {
            CHECK(K <= cap && K * n1 <= kMsWholeNodes && p.T == K && p.nwg == 1, "whole K=%lld", (long long)K);
            continue;
        }
        const int64_t H = stages * p.smax;
        CHECK(p.T >= 1 && p.smax >= 1, "T=%lld smax=%d", (long long)p.T, p.smax);
        CHECK(p.T + 2 * H <= cap, "fit K=%lld cap=%lld T=%lld H=%lld", (long long)K, (long long)cap, (long long)p.T, (long long)H);
        CHECK(H <= K, "halo K=%lld H=%lld", (long long)K, (long long)H);
        CHECK(p.smax <= cap / (div * stages) || p.smax == 1, "bound smax=%d", p.smax);
        CHECK(p.nwg == (K + p.T - 1) / p.T, "nwg");
        // the kernel's chunk: own0 = c T, town = min(T, K - own0), loads
        // [own0 - h, own0 + town + h) for any launch halo h <= H, wrapped once
        std::vector<int> owned(K, 0);
        for (int64_t c = 0; c < p.nwg; ++c) {
            const int64_t own0 = c * p.T, town = std::min(p.T, K - own0);
            CHECK(town >= 1, "empty chunk c=%lld", (long long)c);
            for (int64_t e = own0; e < own0 + town; ++e) owned[e]++;
            for (int64_t g : {own0 - H, own0 + town + H - 1}) {
                int64_t w = g;
                if (w < 0) w += K;
                if (w >= K) w -= K;
                CHECK(w >= 0 && w < K, "load K=%lld g=%lld", (long long)K, (long long)g);
            }
        }
        for (int64_t e = 0; e < K; ++e) CHECK(owned[e] == 1, "owned e=%lld", (long long)e);
    }
    for (int64_t n = 1; n <= 200; ++n) for (int smax = 1; smax <= 40; ++smax) for (int even = 0; even <= 1; ++even) {
        const MsSchedule s = ms_schedule(n, smax, even);
        ++scheds;
        int64_t tot = 0;
        for (int64_t i = 0; i < s.launches(); ++i) {
            const int st = s.steps(i);
            tot += st;
            if (i < s.count) CHECK(st >= 1 && st <= smax, "steps n=%lld smax=%d i=%lld st=%d", (long long)n, smax, (long long)i, st);
            else CHECK(st == 0, "copy launch");
        }
        CHECK(tot == n, "total n=%lld smax=%d", (long long)n, smax);
        if (even) CHECK(s.launches() % 2 == 0, "even n=%lld smax=%d", (long long)n, smax);
        CHECK(!s.copy || (even && s.count == n), "copy only when unavoidable");
        CHECK(s.count >= (n + smax - 1) / smax, "count");
    }
    printf("plans %d schedules %d fails %d\n", plans, scheds, fails);
    return fails != 0;
}
"""


def test_ms_plan_and_schedule_invariants(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    shutil.copy(HDR, tmp_path / "dg_msplan.hpp")
    (tmp_path / "drv.cpp").write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(tmp_path / "drv.cpp")], check=True,
                   capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "fails 0" in r.stdout
