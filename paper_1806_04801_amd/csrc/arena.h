// First-fit arena allocator of the serving runtime (host logic only: it
// hands out offsets into one device allocation; no HIP calls).
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <unordered_map>

namespace hsma {

// First-fit allocator over [0, cap) with coalescing of free neighbours.
class Arena {
   public:
    explicit Arena(size_t cap) : cap_(cap) { free_[0] = cap; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                sizes_[*off] = bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off) {
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        size_t bytes = s->second;
        sizes_.erase(s);
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
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t cap() const { return cap_; }

   private:
    size_t cap_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
    std::unordered_map<size_t, size_t> sizes_;
};

}  // namespace hsma
