// Best-fit allocator of offsets in [0, size), 256-byte granularity, for
// arenas of device or pinned host memory (host bookkeeping only).
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace tofh {

class Arena {
   public:
    void reset(size_t size) {
        holes_.clear();
        if (size) holes_[0] = size;
    }
    bool alloc(size_t bytes, size_t& off) {
        bytes = round(bytes);
        auto best = holes_.end();
        for (auto it = holes_.begin(); it != holes_.end(); ++it)
            if (it->second >= bytes && (best == holes_.end() || it->second < best->second)) best = it;
        if (best == holes_.end()) return false;
        off = best->first;
        const size_t rest = best->second - bytes;
        holes_.erase(best);
        if (rest) holes_[off + bytes] = rest;
        return true;
    }
    void free(size_t off, size_t bytes) {
        bytes = round(bytes);
        auto it = holes_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != holes_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            holes_.erase(nx);
        }
        if (it != holes_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                holes_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& h : holes_) m = std::max(m, h.second);
        return m;
    }

   private:
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    std::map<size_t, size_t> holes_;
};

}  // namespace tofh
