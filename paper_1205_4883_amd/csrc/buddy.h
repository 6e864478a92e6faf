// Buddy allocator used by the serving loop for its device bitmap pool and
// its pinned host arena (host code only; no HIP).
#pragma once

#include <algorithm>
#include <cstdint>
#include <iterator>
#include <map>
#include <set>

namespace sv {

// A buddy allocator over one region of `bytes` (host or device memory that
// the owner allocates): power-of-two blocks from 4 KiB up to max_block.  The
// region is cut into aligned root blocks, largest first (as many of the
// largest size as fit, then the binary digits of the rest), so every byte is
// usable; a freed block merges with its free buddy up to its root's size.
// Not thread-safe: guarded by the server mutex.
class Buddy {
  public:
    static constexpr int kMinOrder = 12;
    static int order_for(uint64_t bytes)
    {
        int o = kMinOrder;
        while ((uint64_t(1) << o) < bytes)
            ++o;
        return o;
    }
    // Returns the usable size (0 if bytes is below one minimum block).
    uint64_t init(uint64_t bytes, uint64_t max_block)
    {
        top_ = order_for(max_block);
        while (top_ > kMinOrder && (uint64_t(1) << top_) > bytes)
            --top_;
        uint64_t off = 0;
        const uint64_t top_bytes = uint64_t(1) << top_;
        while (bytes - off >= top_bytes) {
            roots_[off] = top_;
            free_[top_].insert(off);
            off += top_bytes;
        }
        for (int o = top_ - 1; o >= kMinOrder; --o) {  // the binary digits of the rest
            if (bytes - off >= (uint64_t(1) << o)) {
                roots_[off] = o;
                free_[o].insert(off);
                off += uint64_t(1) << o;
            }
        }
        size_ = off;
        return size_;
    }
    uint64_t size() const { return size_; }
    uint64_t max_block() const { return size_ ? uint64_t(1) << top_ : 0; }
    uint64_t used() const { return used_; }
    bool alloc(uint64_t bytes, uint64_t *off, int *order)
    {
        const int o = order_for(bytes);
        if (o > top_)
            return false;
        int k = o;
        while (k <= top_ && free_[k].empty())
            ++k;
        if (k > top_)
            return false;
        const uint64_t at = *free_[k].begin();
        free_[k].erase(free_[k].begin());
        while (k > o) {
            --k;
            free_[k].insert(at + (uint64_t(1) << k));
        }
        used_ += uint64_t(1) << o;
        *off = at;
        *order = o;
        return true;
    }
    void free(uint64_t off, int o)
    {
        used_ -= uint64_t(1) << o;
        auto root = std::prev(roots_.upper_bound(off));
        const int root_order = root->second;
        while (o < root_order) {
            const uint64_t buddy = off ^ (uint64_t(1) << o);
            auto it = free_[o].find(buddy);
            if (it == free_[o].end())
                break;
            free_[o].erase(it);
            off = std::min(off, buddy);
            ++o;
        }
        free_[o].insert(off);
    }

  private:
    int top_ = kMinOrder;
    uint64_t size_ = 0, used_ = 0;
    std::map<uint64_t, int> roots_;  // root block offset -> order
    std::set<uint64_t> free_[64];
};

}  // namespace sv
