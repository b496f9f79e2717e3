// First-fit allocator over a byte range (offsets only, no device calls):
// the served form carves workspaces and results out of the caller's device
// buffer with it.  Blocks are 256-byte aligned; freed blocks coalesce with
// their free neighbours.  Not thread-safe: the server holds its lock.
#pragma once
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace hp {

class RangeAlloc {
  public:
    static constexpr size_t ALIGN = 256;
    static constexpr size_t NONE = ~size_t(0);

    explicit RangeAlloc(size_t bytes = 0) { reset(bytes); }

    void reset(size_t bytes) {
        free_.clear();
        used_.clear();
        cap_ = bytes / ALIGN * ALIGN;
        in_use_ = peak_ = 0;
        if (cap_) free_[0] = cap_;
    }

    static size_t round(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

    // Offset of a new block of n bytes (n == 0 takes one unit), or NONE.
    size_t alloc(size_t n) {
        const size_t need = round(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            used_[off] = need;
            in_use_ += need;
            if (in_use_ > peak_) peak_ = in_use_;
            return off;
        }
        return NONE;
    }

    // Returns false for an offset that is not the start of a live block.
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t len = u->second;
        used_.erase(u);
        in_use_ -= len;
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }

    // Would a block of n bytes fit right now / with everything released?
    bool fits_now(size_t n) const {
        const size_t need = round(n ? n : 1);
        for (auto &kv : free_)
            if (kv.second >= need) return true;
        return false;
    }
    bool fits_empty(size_t n) const { return round(n ? n : 1) <= cap_; }

    size_t capacity() const { return cap_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    size_t blocks() const { return used_.size(); }
    size_t free_ranges() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;   // offset -> length
    size_t cap_ = 0, in_use_ = 0, peak_ = 0;
};

}  // namespace hp
