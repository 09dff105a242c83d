// gom_arena.h -- host-side bookkeeping of the serving loop, kept free of HIP so that it can be
// unit-tested on a machine without a GPU:
//  * ArenaBlocks: first-fit sub-allocation of a caller-owned device arena in 256-byte units,
//    with frees that coalesce with both neighbours;
//  * drop_retired: removes the jobs a pass has retired from the active list, whatever way the
//    pass ends (normal return, error return or exception).
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace gom {

inline size_t arena_align(size_t x) { return (x + 255) & ~size_t(255); }

class ArenaBlocks {
public:
    explicit ArenaBlocks(size_t bytes = 0) { reset(bytes); }

    void reset(size_t bytes) {
        free_.clear();
        total_ = bytes & ~size_t(255);
        if (total_) free_[0] = total_;
    }

    size_t total() const { return total_; }

    size_t free_bytes() const {
        size_t t = 0;
        for (const auto &kv : free_) t += kv.second;
        return t;
    }

    size_t largest_free() const {
        size_t t = 0;
        for (const auto &kv : free_) t = std::max(t, kv.second);
        return t;
    }

    size_t free_blocks() const { return free_.size(); }

    // First fit: the lowest-offset free block that holds `need` (rounded up to 256 bytes).
    bool alloc(size_t need, size_t *off) {
        need = arena_align(need ? need : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need, at = it->first + need;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }

    // Return [off, off + size) (size rounded as in alloc); merges with adjacent free blocks.
    void release(size_t off, size_t size) {
        size = arena_align(size ? size : 1);
        auto it = free_.emplace(off, size).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    size_t total_ = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
};

// On destruction, erases every job whose `retired` flag is set, keeping the others in order.
template <class Job>
struct RetiredSweep {
    std::vector<Job> &jobs;
    ~RetiredSweep() {
        jobs.erase(std::remove_if(jobs.begin(), jobs.end(),
                                  [](const Job &j) { return j.retired; }),
                   jobs.end());
    }
};

}  // namespace gom
