"""The work partition of a force call (plan_rule, nb6_plan.h) on the CPU: a
g++-built driver checks, over a grid of chip sizes, hints, cluster and block
sizes, the invariants the force kernels' grids and j-ranges rely on."""
import shutil
import subprocess

import pytest

from paper_1205_1222_amd import build

# The host logic runs under AddressSanitizer and UBSan: any invalid access,
# leak or undefined operation ends the driver with a report.
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", "-g"]

DRIVER = r"""
#include "nb6_plan.h"
#include <cmath>
#include <cstdio>
#include <vector>

static int fails = 0;
#define CHECK(cond, ...) do { if (!(cond)) { if (fails++ < 20) { \
    std::printf("FAIL %s: ", #cond); std::printf(__VA_ARGS__); std::printf("\n"); } } } while (0)

int main() {
    const std::vector<int> cus = {256, 304, 80, 8};
    const std::vector<std::vector<int>> hints = {   // ipl, jl, slice
        {0, 0, 0}, {1, 0, 0}, {2, 0, 0}, {0, 16, 0}, {0, 64, 0}, {0, 3, 0},
        {0, 0, 1}, {0, 0, 7}, {0, 0, 40}, {2, 0, 9}};
    const std::vector<int64_t> ns = {1, 2, 31, 32, 33, 255, 256, 257, 1000, 1024, 2048, 2049,
                                     8192, 8193, 16383, 16384, 131072, 131073, 1048576,
                                     2097155};
    const std::vector<int64_t> nis = {1, 2, 63, 64, 65, 128, 129, 256, 257, 1000, 4096,
                                      131072, 1048576};
    long cases = 0;
    for (int cu : cus)
    for (auto& h : hints)
    for (int64_t n : ns)
    for (int64_t ni : nis) {
        if (ni > 4 * n) continue;
        for (int ipl_arg : {0, 1, 2}) {
            const nb6::PlanInputs in{cu, h[0], h[1], h[2]};
            const nb6::Plan p = nb6::plan_rule(in, n, ni, ipl_arg);
            ++cases;
            const int want_ipl = ipl_arg > 0 ? ipl_arg : h[0] > 0 ? h[0] : 1;
            CHECK(p.ipl == want_ipl, "n %lld ni %lld", (long long)n, (long long)ni);
            CHECK(p.jl_shift >= 0 && p.jl_shift <= 6, "shift %d", p.jl_shift);
            CHECK(p.jl_shift == 0 || p.ipl == 1, "lanes with two i per lane");
            if (p.ipl == 1 && h[1] == 0) {
                // up to 1024 i take 8 to 32 lanes when one lane per i would
                // give fewer than 8 waves per CU at 256-j slices
                const bool thin = ((ni + 63) / 64) * std::max<int64_t>(1, (n + 255) / 256) <
                                  8 * (int64_t)cu;
                const bool mid = ni > 256 && ni <= 1024 && thin;
                const int want = ni <= 64 ? 6 : ni <= 128 ? 4 : ni <= 256 ? 3 : mid ? -1 : 0;
                if (want >= 0)
                    CHECK(p.jl_shift == want, "ni %lld shift %d", (long long)ni, p.jl_shift);
                else  // fewer lanes for the larger clusters
                    CHECK(p.jl_shift == (n <= 2048 ? 5 : n <= 8192 ? 4 : 3),
                          "mid lanes: n %lld ni %lld shift %d", (long long)n, (long long)ni,
                          p.jl_shift);
                // and then at most one slice per 256 j, about 4096 waves
                const int64_t g = (ni + (64 >> p.jl_shift) - 1) / (64 >> p.jl_shift);
                if (mid && h[2] <= 0)
                    CHECK((int64_t)p.nslices <= std::max<int64_t>(1, (n + 255) / 256) &&
                          (int64_t)p.nslices * g <= 4096 &&
                          (p.nslices >= 8 || (int64_t)p.nslices == std::max<int64_t>(1, std::min<int64_t>(
                              4096 / g, (n + 255) / 256))),
                          "mid lanes: n %lld ni %lld S %d len %d", (long long)n, (long long)ni,
                          p.nslices, p.slice_len);
            }
            if (p.ipl == 1 && h[1] > 0) CHECK((1 << p.jl_shift) >= h[1], "jl hint");
            const int64_t g = nb6::plan_group_size(p.ipl, p.jl_shift);
            const int64_t groups = (ni + g - 1) / g;
            CHECK(p.wpb >= 1 && p.wpb <= 4 && p.wpb <= groups, "wpb %d groups %lld", p.wpb,
                  (long long)groups);
            CHECK(p.slice_len >= nb6::kPlanTile && p.slice_len % nb6::kPlanTile == 0,
                  "slice_len %d", p.slice_len);
            CHECK(p.nslices >= 1 && p.nslices <= 65535, "nslices %d", p.nslices);
            // every j is in some slice
            CHECK((int64_t)p.nslices * p.slice_len >= n, "n %lld S %d len %d", (long long)n,
                  p.nslices, p.slice_len);
            const bool xcd = h[2] <= 0 && p.nslices >= 8 && p.nslices % 8 == 0;
            // without the XCD split no slice is empty
            if (!xcd) CHECK((int64_t)(p.nslices - 1) * p.slice_len < n,
                            "empty slice: n %lld S %d len %d", (long long)n, p.nslices,
                            p.slice_len);
            // the XCD split keeps a multiple of 8 whenever it applies
            if (h[2] <= 0 && p.nslices >= 8) CHECK(p.nslices % 8 == 0, "S %d", p.nslices);
            // more slices than one per 256 j: plans of one lane per i only,
            // whose 256-j slices would give fewer than 8 waves per CU, and at
            // most sqrt(1.5 n) of them
            if (h[2] <= 0 && (int64_t)p.nslices * 256 > n + 255)
                CHECK(p.jl_shift == 0 && (double)p.nslices <= std::sqrt(1.5 * (double)n) &&
                      groups * std::max<int64_t>(1, (n + 255) / 256) < 8 * (int64_t)cu,
                      "short slices: n %lld ni %lld S %d", (long long)n, (long long)ni,
                      p.nslices);
            // a forced slice count is kept within one slice per 256 j
            if (h[2] > 0) CHECK(p.nslices <= std::max<int64_t>(1, (n + 255) / 256) &&
                                p.nslices <= h[2], "forced S %d", p.nslices);
        }
    }
    std::printf("%ld cases, %d failures\n", cases, fails);
    return fails ? 1 : 0;
}
"""


def test_plan_invariants(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "plan_driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "plan_driver"
    r = subprocess.run([gxx, *SANITIZE, "-O1", "-std=c++17", "-I", build.CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:]
