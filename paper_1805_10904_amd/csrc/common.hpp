// Internal definitions shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "arena.hpp"
#include "louvain.h"

namespace lv {

typedef __int128 i128;
typedef unsigned __int128 u128;

// ---------------------------------------------------------------- errors --

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e != hipSuccess) {
        char buf[512];
        snprintf(buf, sizeof buf, "%s failed at %s:%d: %s", what, file, line, hipGetErrorString(e));
        throw Error(e == hipErrorOutOfMemory ? LOUVAIN_ENOMEM : LOUVAIN_EDEVICE, buf);
    }
}
#define LV_HIP(call) ::lv::hip_check((call), #call, __FILE__, __LINE__)
#define LV_LAUNCHED(name) ::lv::hip_check(hipGetLastError(), name, __FILE__, __LINE__)

inline void require(bool ok, int code, const std::string &msg) {
    if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------- device memory --

// Caching device allocator of one stream (a context's, or a request-loop
// worker's).  Blocks are rounded to size classes (powers of two up to 1 MiB,
// multiples of 2 MiB above) and kept for reuse until the pool dies.  All
// users of a pool enqueue on its one stream, so a block handed back while
// kernels still use it is only reused by work ordered after them; a block
// goes back to the backing store only after a device-wide wait.  The lock
// lets another thread release a block (the request loop's plain worker
// releases requests ingested by the batched workers).
struct Pool {
    std::mutex mu;
    std::shared_ptr<Arena> arena;   // nullptr: hipMalloc / hipFree
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> live_;
    size_t cached = 0, in_use = 0;
    // fault injection: when > 0, the fault_at-th allocation request of this
    // pool (counted from when it was set) fails with ENOMEM, once
    long fault_at = 0, requests = 0;

    explicit Pool(std::shared_ptr<Arena> a = nullptr) : arena(std::move(a)) {
        if (arena) arena->attach(this);
    }
    Pool(const Pool &) = delete;
    Pool &operator=(const Pool &) = delete;

    static size_t round(size_t b) {
        if (b <= 512) return 512;
        if (b <= (1u << 20)) {
            size_t r = 512;
            while (r < b) r <<= 1;
            return r;
        }
        const size_t g = (size_t)2 << 20;
        return (b + g - 1) / g * g;
    }
    void *raw_get(size_t r) {
        if (arena) return arena->get(r);
        void *p = nullptr;
        if (hipMalloc(&p, r) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void raw_put(void *p) {
        if (arena) arena->put(p); else (void)hipFree(p);
    }
    void *get(size_t bytes) {
        const size_t r = round(bytes);
        {
            std::lock_guard<std::mutex> lk(mu);
            if (fault_at > 0 && ++requests == fault_at) {
                fault_at = 0;
                throw Error(LOUVAIN_ENOMEM, "injected failure of device allocation request " +
                                                std::to_string(requests) + " (LOUVAIN_FAULT_ALLOC_AT)");
            }
            auto it = free_.find(r);
            if (it != free_.end()) {
                void *p = it->second;
                free_.erase(it);
                cached -= r;
                live_[p] = r;
                in_use += r;
                return p;
            }
        }
        void *p = raw_get(r);
        if (!p) {
            trim();
            p = raw_get(r);
        }
        if (!p && arena) {
            arena->reclaim(this);
            p = raw_get(r);
        }
        if (!p)
            throw Error(LOUVAIN_ENOMEM, "device allocation of " + std::to_string(r) + " bytes failed" +
                                            (arena ? " (the caller's pool is exhausted)" : ""));
        std::lock_guard<std::mutex> lk(mu);
        live_[p] = r;
        in_use += r;
        return p;
    }
    void put(void *p) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = live_.find(p);
        if (it == live_.end()) return;
        free_.emplace(it->second, p);
        cached += it->second;
        in_use -= it->second;
        live_.erase(it);
    }
    // Release every cached block to the backing store (waits for the device first).
    void trim() {
        std::lock_guard<std::mutex> lk(mu);
        if (free_.empty()) return;
        (void)hipDeviceSynchronize();
        for (auto &kv : free_) raw_put(kv.second);
        free_.clear();
        cached = 0;
    }
    ~Pool() {
        (void)hipDeviceSynchronize();
        for (auto &kv : free_) raw_put(kv.second);
        for (auto &kv : live_) raw_put(kv.first);
        if (arena) arena->detach(this);
    }
};

inline void Arena::reclaim(Pool *self) {
    std::vector<Pool *> ps;
    {
        std::lock_guard<std::mutex> lk(mu);
        ps = pools;
    }
    for (Pool *p : ps)
        if (p != self) p->trim();
}

// The pool of the context whose call is running on this thread (set at the
// C ABI boundary); nullptr means plain hipMalloc / hipFree.
Pool *&current_pool();

// Owning device allocation from the current pool (or hipMalloc).
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    Pool *pool = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), pool(o.pool) { o.p = nullptr; o.n = 0; o.pool = nullptr; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; pool = o.pool;
            o.p = nullptr; o.n = 0; o.pool = nullptr;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        const size_t bytes = (count ? count : 1) * sizeof(T);
        pool = current_pool();
        if (pool) {
            p = (T *)pool->get(bytes);
        } else {
            hipError_t e = hipMalloc((void **)&p, bytes);
            if (e != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw Error(LOUVAIN_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
            }
        }
        n = count;
    }
    // grow-only reallocation (contents are not preserved)
    void reserve(size_t count) { if (count > n || !p) alloc(count); }
    void release() {
        if (p) {
            if (pool) pool->put(p); else (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        pool = nullptr;
    }
    T *get() const { return p; }
};

// ------------------------------------------------------------ diagnostics --

// A named range around host-side phases (a level's sweeps, its
// contraction, a batched step), visible to profilers that trace roctx
// markers (rocprofv3 --marker-trace); free when none is attached.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// LOUVAIN_LOG set to a non-empty value other than 0: per-level progress on
// stderr (read once per process).
inline bool log_on() {
    static const bool on = [] {
        const char *e = getenv("LOUVAIN_LOG");
        return e && *e && !(e[0] == '0' && e[1] == 0);
    }();
    return on;
}

// -------------------------------------------------------------- timing --

// Groups of kernels for per-level time accounting.
enum TimerGroup { TG_INGEST = 0, TG_LEVEL, TG_SWEEP, TG_CONTRACT, TG_OTHER };

// Optional per-launch device timing with HIP events (run statistics).
struct Timer {
    bool on = false;
    std::string only;   // non-empty: record only launches of this name
    hipStream_t stream = nullptr;
    struct Rec {
        std::string name;
        int group;
        hipEvent_t a, b;
        double bytes;   // algorithmic HBM bytes of the launch
        bool launched = false;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    hipEvent_t next_event() {
        if (used == pool.size()) {
            hipEvent_t e;
            LV_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    // Opens the record of one launch when timing is on (with a filter, only
    // for the filtered name); returns its index, or -1.  The launch fills
    // the record's events.
    int begin(int group, const char *name, const char *suffix, double bytes) {
        if (!on) return -1;
        std::string full = std::string(name) + (suffix ? suffix : "");
        if (!only.empty() && full != only) return -1;
        Rec r{std::move(full), group, next_event(), next_event(), bytes, false};
        recs.push_back(std::move(r));
        return (int)recs.size() - 1;
    }
    void reset() { recs.clear(); used = 0; }
    ~Timer() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Scope of one timed launch.  When the launch is recorded, its two events
// are filled by the kernel dispatch itself (hipExtLaunchKernel), so they
// bracket the kernel's execution and add no packets to the stream; a scope
// with several launches spans from the first kernel's start to the last
// one's end.
struct TimedLaunch {
    Timer *t;
    int id;
    bool started = false;
    TimedLaunch(Timer *t_, int group, const char *name, double bytes, const char *suffix = nullptr)
        : t(t_), id(t_ ? t_->begin(group, name, suffix, bytes) : -1) {}
    template <typename... KArgs, typename... Args>
    void launch(void (*k)(KArgs...), dim3 grid, dim3 block, uint32_t shm, hipStream_t s, Args... args) {
        hipEvent_t a = nullptr, b = nullptr;
        if (id >= 0) {
            b = t->recs[id].b;
            if (!started) a = t->recs[id].a;
            started = true;
            t->recs[id].launched = true;
        }
        static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
        std::tuple<std::decay_t<KArgs>...> tup{static_cast<std::decay_t<KArgs>>(args)...};
        void *argv[sizeof...(KArgs) + 1];
        std::apply([&argv](auto &...x) {
            int i = 0;
            ((argv[i++] = (void *)&x), ...);
        }, tup);
        LV_HIP(hipExtLaunchKernel((const void *)k, grid, block, argv, shm, s, a, b, 0));
    }
};

// Type names as they appear in demangled kernel names.
template <typename T> inline const char *type_name();
template <> inline const char *type_name<int32_t>() { return "int"; }
template <> inline const char *type_name<int64_t>() { return "long"; }
template <> inline const char *type_name<__int128>() { return "__int128"; }

// ------------------------------------------------------------- device helpers --

constexpr int32_t kEmpty = -1;  // empty hash slot (labels are >= 0)

// Fibonacci hashing of a label to a power-of-two table of 2^bits slots.
__device__ __forceinline__ uint32_t hash_pow2(int32_t key, int bits) {
    return ((uint32_t)key * 0x9E3779B1u) >> (32 - bits);
}
// Hash of a label into a table of any size (multiply-shift range reduction).
__device__ __forceinline__ uint64_t hash_range(int32_t key, uint64_t size) {
    uint32_t h = (uint32_t)key * 0x9E3779B1u;
    h ^= h >> 16;
    return ((uint64_t)h * size) >> 32;
}

// 128-bit value split in two 64-bit words for shuffles and stores.
__host__ __device__ __forceinline__ i128 make_i128(uint64_t lo, int64_t hi) {
    return (i128)(((u128)(uint64_t)hi << 64) | (u128)lo);
}

template <typename T>
__device__ __forceinline__ T shfl_xor_any(T v, int mask);
template <>
__device__ __forceinline__ int64_t shfl_xor_any<int64_t>(int64_t v, int mask) {
    return __shfl_xor(v, mask);
}
template <>
__device__ __forceinline__ i128 shfl_xor_any<i128>(i128 v, int mask) {
    uint64_t lo = (uint64_t)v;
    int64_t hi = (int64_t)(v >> 64);
    lo = (uint64_t)__shfl_xor((long long)lo, mask);
    hi = __shfl_xor((long long)hi, mask);
    return make_i128(lo, hi);
}

// Scores: exact integer s(C) = TW*e - delta*deg.  With TW <= floor(sqrt(2^63-1))
// every product and difference fits in int64 (all of e, delta, deg lie in
// [0, TW]); otherwise 128-bit arithmetic is used.
constexpr int64_t kTwFastMax = 3037000499LL;

__device__ __forceinline__ i128 mul_wide(int64_t a, int64_t b) {
    // a, b >= 0: one 64x64 -> 128 unsigned product
    uint64_t ua = (uint64_t)a, ub = (uint64_t)b;
    return make_i128(ua * ub, (int64_t)__umul64hi(ua, ub));
}
template <typename S>
__device__ __forceinline__ S score_mul(int64_t a, int64_t b);
template <>
__device__ __forceinline__ int64_t score_mul<int64_t>(int64_t a, int64_t b) { return a * b; }
template <>
__device__ __forceinline__ i128 score_mul<i128>(int64_t a, int64_t b) { return mul_wide(a, b); }

// Candidate order: larger score first, then smaller label; label < 0 = none.
template <typename S>
__device__ __forceinline__ bool better(S s, int32_t l, S bs, int32_t bl) {
    return l >= 0 && (bl < 0 || s > bs || (s == bs && l < bl));
}

inline unsigned grid_for(int64_t items, int per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace lv
