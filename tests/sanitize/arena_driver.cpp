// Random allocation sequences against the device-region sub-allocator
// (lv::Arena) on a host buffer, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_cpu.py.  Checks that
// live blocks never overlap and stay inside the region, that every block is
// aligned, that the accounting (in use, high-water mark) is exact, and that
// releasing everything coalesces the region back into one free range.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "arena.hpp"

static int fail(const char *what) {
    std::printf("FAIL: %s\n", what);
    return 1;
}

int main() {
    const size_t region = (size_t)64 << 20;
    std::vector<unsigned char> host(region + 300);
    // a misaligned start: the arena aligns it up and drops the remainder
    lv::Arena a(host.data() + 3, region + 200);
    if (a.bytes % lv::Arena::kAlign || a.bytes > region + 200 || (uintptr_t)a.base % lv::Arena::kAlign)
        return fail("region alignment");
    struct Blk {
        char *p;
        size_t len;
        unsigned char tag;
    };
    std::vector<Blk> live;
    std::mt19937_64 rng(12345);
    size_t expect = 0, high = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool alloc = live.empty() || (rng() % 100) < 55;
        if (alloc) {
            const int cls = (int)(rng() % 4);
            size_t len = cls == 0 ? 1 + rng() % 512 : cls == 1 ? 1 + rng() % 65536
                         : cls == 2 ? 1 + rng() % (1 << 20) : 1 + rng() % (6 << 20);
            char *p = (char *)a.get(len);
            const size_t rounded = (len + lv::Arena::kAlign - 1) / lv::Arena::kAlign * lv::Arena::kAlign;
            if (!p) {
                if (a.in_use + rounded <= a.bytes && a.free_.size() == 1) return fail("refused a fitting request");
                continue;
            }
            if ((uintptr_t)p % lv::Arena::kAlign) return fail("unaligned block");
            if (p < a.base || p + rounded > a.base + a.bytes) return fail("block outside the region");
            const unsigned char tag = (unsigned char)(step & 0xff);
            std::memset(p, tag, len);   // ASan flags any write outside the host buffer
            live.push_back({p, len, tag});
            expect += rounded;
            if (expect > high) high = expect;
        } else {
            const size_t k = rng() % live.size();
            const Blk b = live[k];
            for (size_t i = 0; i < b.len; i += 997)
                if ((unsigned char)b.p[i] != b.tag) return fail("block overwritten by another block");
            a.put(b.p);
            live[k] = live.back();
            live.pop_back();
            expect -= (b.len + lv::Arena::kAlign - 1) / lv::Arena::kAlign * lv::Arena::kAlign;
        }
        if (a.in_use != expect) return fail("in-use accounting");
        if (a.high != high) return fail("high-water accounting");
    }
    for (const Blk &b : live) a.put(b.p);
    a.put(a.base + 12345);   // an address never handed out is ignored
    if (a.in_use != 0 || !a.used_.empty()) return fail("blocks left after releasing all");
    if (a.free_.size() != 1 || a.free_.begin()->first != 0 || a.free_.begin()->second != a.bytes)
        return fail("free ranges not coalesced");
    if (a.get(a.bytes) != a.base || a.get(1) != nullptr) return fail("whole-region request");
    std::printf("arena ok: high water %zu of %zu bytes\n", high, a.bytes);
    return 0;
}
