// Sub-allocator of a caller-provided device region (plain C++, no HIP
// calls: the addresses are only handed out and taken back here).
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <mutex>
#include <vector>

namespace lv {

// Backing store of a context's device memory.  Without a region every block
// comes from hipMalloc.  With a caller-provided region [base, base + bytes)
// blocks are carved from it (best fit over a free list in address order,
// neighbours coalesced on release) and nothing else is allocated: a request
// that does not fit gives ENOMEM.  Thread-safe; never holds its lock while
// taking a pool's.
struct Pool;
struct Arena {
    static constexpr size_t kAlign = 256;
    std::mutex mu;
    char *base = nullptr;
    size_t bytes = 0;
    std::map<size_t, size_t> free_;   // offset -> length, in address order
    std::map<size_t, size_t> used_;   // offset -> length
    size_t in_use = 0, high = 0;
    std::vector<Pool *> pools;        // caching pools drawing from the region

    Arena(void *b, size_t n) {
        const uintptr_t a = (uintptr_t)b;
        const uintptr_t al = (a + kAlign - 1) / kAlign * kAlign;
        const size_t skip = (size_t)(al - a);
        base = (char *)al;
        bytes = n > skip ? (n - skip) / kAlign * kAlign : 0;
        if (bytes) free_[0] = bytes;
    }
    // nullptr when no free range holds len bytes
    void *get(size_t len) {
        len = (len + kAlign - 1) / kAlign * kAlign;
        std::lock_guard<std::mutex> lk(mu);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= len && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return nullptr;
        const size_t off = best->first, have = best->second;
        free_.erase(best);
        if (have > len) free_[off + len] = have - len;
        used_[off] = len;
        in_use += len;
        if (in_use > high) high = in_use;
        return base + off;
    }
    void put(void *p) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = used_.find((size_t)((char *)p - base));
        if (it == used_.end()) return;
        size_t off = it->first, len = it->second;
        used_.erase(it);
        in_use -= len;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        free_[off] = len;
    }
    void attach(Pool *p) {
        std::lock_guard<std::mutex> lk(mu);
        pools.push_back(p);
    }
    void detach(Pool *p) {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < pools.size(); ++i)
            if (pools[i] == p) {
                pools.erase(pools.begin() + (ptrdiff_t)i);
                break;
            }
    }
    // Returns the cached blocks of every attached pool but `self` to the region.
    void reclaim(Pool *self);
};

}  // namespace lv
