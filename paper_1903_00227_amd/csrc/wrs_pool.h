// wrs_pool.h -- first-fit allocator over one region (host code only).
//
// The request server carves its whole HBM budget, one device allocation, with
// this allocator: sizes round up to 256 bytes, a request takes the free range
// with the lowest offset that holds it, and a released range merges with free
// neighbours.  It never touches the memory it manages, so it can be exercised
// on any address range.  The lengths of the free ranges are kept in a sorted
// multiset beside them, so a request that no range holds fails at once
// instead of scanning every range (a server retrying after evictions makes
// many such requests when the budget is fragmented).
#ifndef WRS_POOL_H
#define WRS_POOL_H

#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <set>

namespace wrs {

class FirstFit {
   public:
    // Manage [base, base + bytes), bytes rounded down to a multiple of 256.
    void reset(void* base, size_t bytes) {
        base_ = (char*)base;
        size_ = bytes & ~(size_t)255;
        used_ = peak_ = 0;
        free_.clear();
        lens_.clear();
        if (size_) put(0, size_);
    }
    void* alloc(size_t bytes) {
        bytes = round(bytes);
        if (lens_.empty() || *lens_.rbegin() < bytes) return nullptr;  // no range holds it
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, sz = it->second;
                take(it);
                if (sz > bytes) put(off + bytes, sz - bytes);
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return base_ + off;
            }
        }
        return nullptr;
    }
    // Give back a range that alloc(bytes) returned (nullptr is ignored).
    void release(void* p, size_t bytes) {
        if (!p) return;
        bytes = round(bytes);
        const size_t off = (size_t)((char*)p - base_);
        used_ -= bytes;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = take(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                const size_t at = pv->first, len = pv->second + bytes;
                take(pv);
                put(at, len);
                return;
            }
        }
        put(off, bytes);
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }
    size_t free_ranges() const { return free_.size(); }
    // The length index holds exactly the free ranges' lengths (a check for tests).
    bool index_consistent() const {
        std::multiset<size_t> l;
        for (const auto& kv : free_) l.insert(kv.second);
        return l == lens_;
    }
    void* base() const { return base_; }

   private:
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    // free range [off, off + len) in, or out, of both indexes
    void put(size_t off, size_t len) {
        free_[off] = len;
        lens_.insert(len);
    }
    std::map<size_t, size_t>::iterator take(std::map<size_t, size_t>::iterator it) {
        lens_.erase(lens_.find(it->second));
        return free_.erase(it);
    }
    char* base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length of each free range
    std::multiset<size_t> lens_;     // the lengths of those ranges
};

}  // namespace wrs

#endif
