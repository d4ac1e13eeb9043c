// First-fit allocator over an address range [0, size): the server hands out
// its HBM budget with it, so admitting a request never calls hipMalloc.
// Host-only code (no HIP), shared with a CPU test.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace pa {

inline uint64_t round256(uint64_t x) { return (x + 255) & ~255ull; }

// Sizes are rounded up to 256 bytes; frees coalesce with their neighbours.
class Arena {
public:
    explicit Arena(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t bytes, uint64_t* off)
    {
        bytes = round256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = round256(bytes);
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
    uint64_t peak() const { return peak_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0, peak_ = 0;
};

}  // namespace pa
