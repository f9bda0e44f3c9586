// Arena sub-allocator: every device workspace of a context is carved out of
// one caller-provided block of HBM, so the hot path never calls hipMalloc.
// First fit over an address-ordered free list, 256-byte alignment, adjacent
// free blocks merged on release.  Pure host logic (offsets only), thread-safe.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>

namespace sparkcl {

class Arena {
  public:
    static constexpr uint64_t kAlign = 256;
    static constexpr uint64_t kFail = ~0ull;

    void reset(uint64_t bytes)
    {
        std::lock_guard<std::mutex> g(mu_);
        size_ = bytes / kAlign * kAlign;
        free_.clear();
        used_.clear();
        in_use_ = 0;
        peak_ = 0;
        if (size_)
            free_[0] = size_;
    }

    // Offset of a block of at least `bytes` (rounded up to kAlign), or kFail.
    uint64_t alloc(uint64_t bytes)
    {
        if (bytes == 0)
            bytes = 1;
        if (bytes > size_)
            return kFail;
        const uint64_t need = (bytes + kAlign - 1) / kAlign * kAlign;
        std::lock_guard<std::mutex> g(mu_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need)
                continue;
            const uint64_t off = it->first;
            const uint64_t rest = it->second - need;
            free_.erase(it);
            if (rest)
                free_[off + need] = rest;
            used_[off] = need;
            in_use_ += need;
            if (in_use_ > peak_)
                peak_ = in_use_;
            return off;
        }
        return kFail;
    }

    // Returns false for an offset that is not a live allocation.
    bool release(uint64_t off)
    {
        std::lock_guard<std::mutex> g(mu_);
        auto u = used_.find(off);
        if (u == used_.end())
            return false;
        uint64_t len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }

    uint64_t size() const { return size_; }
    uint64_t in_use() const
    {
        std::lock_guard<std::mutex> g(mu_);
        return in_use_;
    }
    uint64_t peak() const
    {
        std::lock_guard<std::mutex> g(mu_);
        return peak_;
    }
    uint64_t largest_free() const
    {
        std::lock_guard<std::mutex> g(mu_);
        uint64_t m = 0;
        for (auto &f : free_)
            m = f.second > m ? f.second : m;
        return m;
    }
    size_t live_blocks() const
    {
        std::lock_guard<std::mutex> g(mu_);
        return used_.size();
    }
    size_t free_blocks() const
    {
        std::lock_guard<std::mutex> g(mu_);
        return free_.size();
    }

  private:
    mutable std::mutex mu_;
    uint64_t size_ = 0, in_use_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_; // offset -> length
    std::map<uint64_t, uint64_t> used_; // offset -> length
};

} // namespace sparkcl
