// nb6_rows.h -- host side of neighbour-list copies: rows of a [n][cap] list
// array hold min(count, cap) valid entries each; large copies move only
// those, packed back to back, and place them on up to 8 host threads.
// Host-only, so the CPU tests exercise it directly.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <thread>
#include <vector>

namespace nb6 {

// body(q0, q1) over the rows [0, n) on up to 8 host threads (one per 2^18
// entries moved).
template <typename F>
void for_rows(int n, int64_t entries, F body) {
    const int nt = (int)std::min<int64_t>(8, std::max<int64_t>(1, entries >> 18));
    std::vector<std::thread> helpers;
    for (int t = 1; t < nt; ++t)
        helpers.emplace_back(body, (int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt));
    body(0, (int)((int64_t)n / nt));
    for (auto& h : helpers) h.join();
}

// Row offsets of lists holding min(count, cap) entries per row (a negative
// count, the mark of an invalid row, holds none).
inline std::vector<int64_t> row_offsets(const int32_t* count, int n, int cap) {
    std::vector<int64_t> off((size_t)n + 1);
    off[0] = 0;
    for (int q = 0; q < n; ++q) off[q + 1] = off[q] + std::min(std::max(count[q], 0), cap);
    return off;
}

// Row-major [n][cap] rows to a packed array (row q at off[q]), and back.
inline void pack_rows_host(const std::vector<int64_t>& off, int n, int cap,
                           const int32_t* rows, int32_t* packed) {
    for_rows(n, off[n], [&](int q0, int q1) {
        for (int q = q0; q < q1; ++q) {
            const int32_t* r = rows + (size_t)q * cap;
            std::copy(r, r + (off[q + 1] - off[q]), packed + off[q]);
        }
    });
}
inline void unpack_rows_host(const std::vector<int64_t>& off, int n, int cap,
                             const int32_t* packed, int32_t* rows) {
    for_rows(n, off[n], [&](int q0, int q1) {
        for (int q = q0; q < q1; ++q)
            std::copy(packed + off[q], packed + off[q + 1], rows + (size_t)q * cap);
    });
}

}  // namespace nb6
