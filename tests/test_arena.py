"""The serving queue's scratch arena (first fit, coalescing on free), on the
CPU: a small C++ driver, built with g++ against the library's header, checks
it step by step against a byte-level model over random alloc/free
sequences."""
import os
import shutil
import subprocess

import pytest

from paper_1205_1222_amd import build

# The host logic runs under AddressSanitizer and UBSan: any invalid access,
# leak or undefined operation ends the driver with a report.
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", "-g"]

DRIVER = r"""
#include "nb6_arena.h"
#include <cstdio>
#include <random>
#include <vector>

// maximal free runs of the model, in offset order
static std::vector<std::pair<size_t, size_t>> runs(const std::vector<char>& used) {
    std::vector<std::pair<size_t, size_t>> r;
    size_t k = 0;
    while (k < used.size()) {
        if (used[k]) { ++k; continue; }
        size_t e = k;
        while (e < used.size() && !used[e]) ++e;
        r.push_back({k, e - k});
        k = e;
    }
    return r;
}

int main() {
    const size_t size = 4096;
    nb6::OffsetArena a;
    a.reset(size);
    std::vector<char> used(size, 0);
    std::vector<std::pair<size_t, size_t>> live;
    std::mt19937_64 rng(12051222);
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || rng() % 100 < 55;
        if (do_alloc) {
            const size_t bytes = 1 + rng() % (rng() % 8 == 0 ? 1024 : 96);
            size_t expect = size;  // first fit in the model
            for (auto& fr : runs(used))
                if (fr.second >= bytes) { expect = fr.first; break; }
            size_t off = 0;
            const bool ok = a.alloc(bytes, &off);
            if (ok != (expect != size)) { std::printf("fit mismatch at %d\n", step); return 1; }
            if (ok) {
                if (off != expect) { std::printf("not first fit at %d\n", step); return 1; }
                for (size_t k = off; k < off + bytes; ++k) used[k] = 1;
                live.push_back({off, bytes});
            }
        } else {
            const size_t pick = rng() % live.size();
            const auto blk = live[pick];
            live.erase(live.begin() + pick);
            a.free(blk.first, blk.second);
            for (size_t k = blk.first; k < blk.first + blk.second; ++k) used[k] = 0;
        }
        size_t in_use = 0;
        for (char u : used) in_use += u;
        if (a.used() != in_use) { std::printf("used mismatch at %d\n", step); return 1; }
        if (a.free_blocks() != runs(used).size()) {
            std::printf("not coalesced at %d\n", step); return 1;
        }
    }
    for (auto& blk : live) a.free(blk.first, blk.second);
    if (a.used() != 0 || a.free_blocks() != 1) { std::printf("leak at the end\n"); return 1; }
    std::printf("ok\n");
    return 0;
}
"""


def test_arena_first_fit_and_coalescing(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "arena_driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "arena_driver"
    r = subprocess.run([gxx, *SANITIZE, "-O1", "-std=c++17", "-I", build.CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
