// nb6_arena.h -- first-fit allocation of offsets within one region, with
// free blocks coalesced on release.  The serving queue carves every admitted
// request's device scratch from one arena of the context's HBM budget with
// it; it holds no device memory itself, so the CPU tests exercise it alone.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace nb6 {

class OffsetArena {
  public:
    void reset(size_t size) {
        size_ = size;
        used_ = 0;
        free_.clear();
        if (size) free_[0] = size;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t free_blocks() const { return free_.size(); }
    // The lowest-offset free block that holds `bytes`; false when none does.
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    // Return [off, off + bytes), merging it with free neighbours.
    void free(size_t off, size_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
};

}  // namespace nb6
