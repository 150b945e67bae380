// wrs_pool.h -- first-fit allocator over one region (host code only).
//
// The request server carves its whole HBM budget, one device allocation, with
// this allocator: sizes round up to 256 bytes, a request takes the free range
// with the lowest offset that holds it, and a released range merges with free
// neighbours.  It never touches the memory it manages, so it can be exercised
// on any address range.
#ifndef WRS_POOL_H
#define WRS_POOL_H

#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace wrs {

class FirstFit {
   public:
    // Manage [base, base + bytes), bytes rounded down to a multiple of 256.
    void reset(void* base, size_t bytes) {
        base_ = (char*)base;
        size_ = bytes & ~(size_t)255;
        used_ = peak_ = 0;
        free_.clear();
        if (size_) free_[0] = size_;
    }
    void* alloc(size_t bytes) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
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
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }
    size_t free_ranges() const { return free_.size(); }
    void* base() const { return base_; }

   private:
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    char* base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length of each free range
};

}  // namespace wrs

#endif
