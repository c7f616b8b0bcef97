// nb6_plan.h -- the work partition of a force call: i-particles per lane,
// lanes per i-particle, j-slices and their length, from the block size, the
// cluster size, the chip's compute units and the context's hints.  Host-only
// (no HIP types), so the CPU tests check its invariants directly; the force
// kernels, the finalize and the serving queue all take their grids from it.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace nb6 {

struct Plan {
    int ipl, jl_shift, wpb, nslices, slice_len;
};

// What the rule reads from a context.
struct PlanInputs {
    int num_cu;      // compute units of the GPU
    int ipl_hint;    // 0: choose; 1 or 2 i-particles per lane
    int jl_hint;     // 0: choose; lanes that share one i-particle
    int slice_hint;  // 0: choose; >0: that many j-slices
};

// j-particles per tile of the candidate bound: slice lengths are multiples
// of it (the force kernels' VTILE).
constexpr int kPlanTile = 32;

// i-particles of one work item: 64 per wave at one per lane, times the
// i-particles per lane, divided by the lanes that share one.
inline int plan_group_size(int ipl, int jl_shift) { return (64 * ipl) >> jl_shift; }

inline Plan plan_rule(const PlanInputs& in, int64_t n, int64_t ni, int ipl) {
    Plan p;
    // One i per lane unless asked for two: the one-i kernel holds at most 80
    // VGPRs against about 110, hence more waves per SIMD, and measured faster at every
    // block size from 512 to 2^20 active particles (at N = 2^17 and 2^20).
    p.ipl = ipl > 0 ? ipl : in.ipl_hint > 0 ? in.ipl_hint : 1;
    // Slices are at least 256 j-particles long (but see the short slices
    // below), and give each lane at least 32 of them (16 for the smallest
    // lanes plans, below).
    auto max_slices = [&](int sh, int per_lane = 32) {
        const int64_t len = std::max<int64_t>(256, (int64_t)per_lane << sh);
        return std::max<int64_t>(1, (n + len - 1) / len);
    };
    auto groups_of = [&](int sh) {
        const int g = plan_group_size(p.ipl, sh);
        return (ni + g - 1) / g;
    };
    // Lanes per i.  A block of at most 256 is latency-bound, not
    // throughput-bound: its i share the lanes of a wavefront (64 lanes per i
    // up to 64 i, then 16 and 8, whose workgroups share the j-records
    // through LDS: at N = 131072, N_i = 128 took 34.5 us per call with 16
    // lanes on 128 slices against 36.5 with 32 on 64, and N_i = 160, 200,
    // 256 took 40.0-40.9, 44.4-44.7, 45.0-45.2 us with 8 lanes on 128 slices
    // against 41.9-44.1, 44.5-47.7, 48.8-50.8 with 16), with slices sized to
    // balance the force kernel's dependent j-loads (slice_len / lanes / 4
    // per lane) against the finalize kernel's dependent partial loads
    // (slices / 32).
    int sh = 0;
    bool lanes_plan = false, mid_lanes = false;
    if (p.ipl == 1) {
        if (in.jl_hint > 0) {
            while ((1 << sh) < in.jl_hint) ++sh;
        } else if (ni <= 256) {
            sh = ni <= 64 ? 6 : ni <= 128 ? 4 : 3;
            lanes_plan = true;
        } else if (ni <= 1024 && groups_of(0) * max_slices(0) < (int64_t)in.num_cu * 8) {
            // A block of up to 1024 in a cluster too small for one lane per
            // i to fill the chip at 256-j slices (the short slices below)
            // takes lanes per i, on slices of at least 256 j and about 4096
            // waves: the power of 2 nearest 1024 / sqrt(N) lanes, 8 to 32
            // (measured best at N = 1024, 4096, 16384 for N_i = 300, 512,
            // 1024: 32, 16, 8 lanes; in one sweep, C1, N = N_i = 1024: 18.6
            // us per call with one lane per i, 15.3 with 32 lanes on 4
            // slices; C2, N_i = 1024 of N = 16384: 36.0 and 31.9 with 8
            // lanes on 32 slices).
            const double best = 1024.0 / std::sqrt((double)n);
            sh = std::min(5, std::max(3, (int)std::lround(std::log2(best))));
            mid_lanes = true;
        }
    }
    p.jl_shift = sh;
    const int64_t groups = groups_of(sh);
    p.wpb = (int)std::min<int64_t>(4, groups);
    // About 64 waves per SIMD over the launch, and slices of at most 16384
    // j: many rounds at the kernel's occupancy, so the last round's
    // imbalance is a small part (measured optimum at N_i = 2^12 .. 2^20).
    const int64_t target = (int64_t)in.num_cu * 4 * 64;
    int64_t s = in.slice_hint > 0 ? in.slice_hint
                                  : std::max((target + groups - 1) / groups, (n + 16383) / 16384);
    if (lanes_plan && in.slice_hint <= 0) {
        // measured optimum about sqrt(1.5 n / lanes), taken to a power of 2;
        // twice that for at most 8 groups (a few hundred waves, each one's
        // chain of j-loads the launch's duration), down to 16 j per lane: at
        // N = 131072 and 64 lanes, N_i = 1, 2, 4, 8 took 14.8, 15.5, 17.2,
        // 18.9 us per call at 128 slices against 16.1, 16.7, 18.0, 19.6 at
        // 64; from 16 on the two were the same
        const double best = std::sqrt(1.5 * (double)n / (double)(1 << sh));
        s = (int64_t)1 << (int)std::lround(std::log2(std::max(1.0, best)));
        if (groups <= 8) s *= 2;
    }
    if (mid_lanes && in.slice_hint <= 0) s = std::max<int64_t>(1, 4096 / groups);
    // A one-lane-per-i call whose 256-j slices give fewer than 8 waves per
    // CU leaves the chip idle, and each wavefront's chain of dependent
    // j-loads is then the launch's duration (N = N_i = 1024: 4 slices, 64
    // waves).  Such calls may take up to sqrt(1.5 N) slices (the power of 2
    // below it, as for the lanes), down to one tile of j each: measured 85 ->
    // 37 us per call at N = N_i = 1024 and 68 -> 55 us at N = 16384, N_i =
    // 1024.  Calls that already fill the chip keep 256-j slices: shorter
    // ones only add work items, which costs the serving queue's fused
    // batches throughput (measured on the C4 trace: 872 Gint/s at
    // saturation with short slices wherever the root allowed them, 991 with
    // this bound).
    int64_t cap = lanes_plan && groups <= 8 ? max_slices(sh, 16)
                : mid_lanes                  ? max_slices(sh, 8)
                                             : max_slices(sh);
    if (sh == 0 && groups * cap < (int64_t)in.num_cu * 8) {
        const double root = std::sqrt(1.5 * (double)n);
        const int64_t lim = (int64_t)1 << (int)std::floor(std::log2(std::max(1.0, root)));
        cap = std::max(cap, std::min<int64_t>(lim, (n + kPlanTile - 1) / kPlanTile));
    }
    s = std::max<int64_t>(1, std::min<int64_t>(s, in.slice_hint > 0 ? (n + 255) / 256 : cap));
    s = std::min<int64_t>(s, 65535);
    // a multiple of 8 lets the force kernel keep each slice on one XCD; the
    // count is kept even when rounding the length up to whole tiles leaves
    // the last slices empty (their partials are zero)
    const bool xcd_split = in.slice_hint <= 0 && s >= 8;
    if (xcd_split) s = s / 8 * 8;
    int64_t len = (n + s - 1) / s;
    len = (len + kPlanTile - 1) / kPlanTile * kPlanTile;
    p.slice_len = (int)len;
    p.nslices = xcd_split ? (int)s : (int)((n + len - 1) / len);
    return p;
}

}  // namespace nb6
