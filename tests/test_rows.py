"""Host side of neighbour-list copies (nb6_rows.h) on the CPU: row offsets
from counts (negative counts hold nothing, counts past cap hold cap), and a
pack / unpack round trip, large enough to run on several host threads, that
moves exactly the valid entries of every row and leaves the rest alone."""
import shutil
import subprocess

import pytest

from paper_1205_1222_amd import build

# The host logic runs under AddressSanitizer and UBSan: any invalid access,
# leak or undefined operation ends the driver with a report.
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", "-g"]

DRIVER = r"""
#include "nb6_rows.h"
#include <cstdio>
#include <random>

int main() {
    int fails = 0;
    {   // offsets
        const int32_t count[6] = {0, 3, -1, 70, 64, 5};
        const auto off = nb6::row_offsets(count, 6, 64);
        const int64_t want[7] = {0, 0, 3, 3, 67, 131, 136};
        for (int k = 0; k < 7; ++k)
            if (off[k] != want[k]) { std::printf("offset %d: %lld\n", k, (long long)off[k]); ++fails; }
    }
    for (int n : {1, 1000, 300000}) {   // round trip; the last one is threaded
        const int cap = 64;
        std::mt19937 rng(n);
        std::vector<int32_t> count(n), rows((size_t)n * cap), back((size_t)n * cap, -7);
        for (int q = 0; q < n; ++q) {
            count[q] = (int32_t)(rng() % 90) - 5;   // some negative, some past cap
            for (int k = 0; k < cap; ++k) rows[(size_t)q * cap + k] = (int32_t)(q * 131 + k);
        }
        const auto off = nb6::row_offsets(count.data(), n, cap);
        std::vector<int32_t> packed((size_t)off[n] + 1, -9);
        nb6::pack_rows_host(off, n, cap, rows.data(), packed.data());
        if (packed[off[n]] != -9) { std::printf("pack wrote past the end\n"); ++fails; }
        nb6::unpack_rows_host(off, n, cap, packed.data(), back.data());
        for (int q = 0; q < n; ++q) {
            const int k_valid = std::min(std::max(count[q], 0), cap);
            for (int k = 0; k < cap; ++k) {
                const int32_t got = back[(size_t)q * cap + k];
                const int32_t want = k < k_valid ? rows[(size_t)q * cap + k] : -7;
                if (got != want) {
                    if (fails++ < 10) std::printf("n %d row %d entry %d: %d\n", n, q, k, got);
                }
            }
        }
    }
    std::printf(fails ? "failed\n" : "ok\n");
    return fails ? 1 : 0;
}
"""


def test_row_offsets_and_round_trip(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "rows_driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "rows_driver"
    r = subprocess.run([gxx, *SANITIZE, "-O1", "-std=c++17", "-pthread", "-I", build.CSRC, str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:]
