// First-fit allocator over a caller-owned byte range (offsets only, no device
// calls), used by the request server to admit work by its HBM footprint.
// Header-only and free of HIP so that it is testable on the host.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <vector>

namespace gpk {

class Arena {
  public:
    static constexpr size_t kAlign = 256;

    explicit Arena(size_t bytes = 0) { reset(bytes); }

    void reset(size_t bytes)
    {
        size_ = bytes / kAlign * kAlign;
        free_.clear();
        if (size_ > 0) free_.push_back({0, size_});
        used_ = 0;
    }

    static size_t round(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // Returns true and the offset of a block of at least n bytes, or false
    // when no free block is large enough.
    bool alloc(size_t n, size_t &off)
    {
        n = round(n == 0 ? 1 : n);
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].len >= n) {
                off = free_[i].off;
                free_[i].off += n;
                free_[i].len -= n;
                if (free_[i].len == 0) free_.erase(free_.begin() + (long)i);
                used_ += n;
                return true;
            }
        }
        return false;
    }

    // Returns a block obtained from alloc(n) (same n).  Neighbouring free
    // blocks are merged.
    void release(size_t off, size_t n)
    {
        n = round(n == 0 ? 1 : n);
        Block blk{off, n};
        auto it = std::lower_bound(free_.begin(), free_.end(), blk,
                                   [](const Block &a, const Block &b) { return a.off < b.off; });
        it = free_.insert(it, blk);
        // merge with the next block, then with the previous one
        auto nx = it + 1;
        if (nx != free_.end() && it->off + it->len == nx->off) {
            it->len += nx->len;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = it - 1;
            if (pv->off + pv->len == it->off) {
                pv->len += it->len;
                free_.erase(it);
            }
        }
        used_ -= n;
    }

    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const Block &b : free_) m = std::max(m, b.len);
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

  private:
    struct Block {
        size_t off, len;
    };
    std::vector<Block> free_;   // sorted by offset, never adjacent
    size_t size_ = 0, used_ = 0;
};

}  // namespace gpk
