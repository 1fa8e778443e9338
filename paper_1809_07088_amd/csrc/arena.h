// Device-arena bookkeeping of the serving runtime (host only, plain C++): first-fit
// sub-allocation of byte ranges in 256-byte granules from one pre-allocated region,
// with coalescing of neighbouring free ranges.  It hands out offsets, never memory.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace dsx {

class Arena {
    // Offsets are multiples of 256; a range is released with the size it was allocated
    // with.  Not thread safe (the server holds its lock).
public:
    static size_t round(size_t n) { return (n + 255) & ~size_t(255); }
    void init(size_t n) { size_ = n; used_ = peak_ = 0; free_.clear(); free_[0] = n; }
    bool alloc(size_t n, size_t* off)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, next = it->first + n;
            free_.erase(it);
            if (rest) free_[next] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
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
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }

private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length of each free range
};

}  // namespace dsx
