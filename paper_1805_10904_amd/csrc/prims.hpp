// Device-wide primitives: scans, fills, CSR ingest and row sums.
#pragma once

#include "common.hpp"

namespace lv {

// Temporary device allocation for the duration of a host scope: from the
// current context's pool (stream-ordered reuse), else hipMallocAsync.
struct TempBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    Pool *pool = nullptr;
    TempBuf(size_t bytes, hipStream_t stream) : s(stream), pool(current_pool()) {
        if (pool) {
            p = pool->get(bytes ? bytes : 16);
            return;
        }
        hipError_t e = hipMallocAsync(&p, bytes ? bytes : 16, stream);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw Error(LOUVAIN_ENOMEM, "temporary device allocation of " + std::to_string(bytes) + " bytes failed");
        }
    }
    TempBuf() = default;
    TempBuf(const TempBuf &) = delete;
    TempBuf &operator=(const TempBuf &) = delete;
    TempBuf(TempBuf &&o) noexcept : p(o.p), s(o.s), pool(o.pool) { o.p = nullptr; }
    TempBuf &operator=(TempBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            s = o.s;
            pool = o.pool;
            o.p = nullptr;
        }
        return *this;
    }
    ~TempBuf() { release(); }
    void release() {
        if (!p) return;
        if (pool) pool->put(p); else (void)hipFreeAsync(p, s);
        p = nullptr;
    }
    template <typename T> T *as() const { return (T *)p; }
};

// Device values the host needs, read in one round trip: each add() queues
// a device range (4-byte words) and returns where it will land in pinned
// host memory; fetch() (issue() then wait()) gathers every queued range with
// one small kernel that writes straight into that memory, then waits for it
// once.  The pinned block (kReadbackWords words) comes from a process-wide
// free list; its last word is a completion flag the kernel stores after the
// values, which the host polls for a while before it falls back to the
// event (a blocking wait adds its wake-up time to every round trip).
class Readback {
  public:
    static constexpr int kMaxRanges = 24;
    static constexpr int kReadbackWords = 1024;
    static constexpr int kFlagWord = kReadbackWords - 2;   // values use the words below it
    explicit Readback(hipStream_t s);
    ~Readback();
    Readback(const Readback &) = delete;
    Readback &operator=(const Readback &) = delete;
    template <typename T> T *add(const T *src, int64_t count = 1) {
        static_assert(sizeof(T) % 4 == 0, "whole 4-byte words");
        return (T *)add_words(src, count * (int64_t)(sizeof(T) / 4));
    }
    void issue();   // launch the gather of the queued ranges
    void wait();    // wait for the gather (then the values are in place); later work may still run
    void fetch() {
        issue();
        wait();
    }

  private:
    void *add_words(const void *src, int64_t words);
    hipStream_t s_;
    uint32_t *host_ = nullptr, *dev_ = nullptr;
    hipEvent_t ev_ = nullptr;   // recorded after the gather
    int device_ = 0;            // device current at construction (the stream's)
    bool pending_ = false;      // issued and not waited for
    bool flagged_ = false;      // the issued gather stores epoch_ in the flag word
    uint32_t epoch_ = 0;
    int n_ = 0;
    int used_ = 0;
    const uint32_t *src_[kMaxRanges];
    int off_[kMaxRanges], len_[kMaxRanges];
};

// Two extra streams of the current device, and the events that fork work
// from a main stream onto them and join it back, leased from a per-device
// free list so that repeated runs reuse them (default priority, like every
// stream here).
class SideStreams {
  public:
    SideStreams();
    ~SideStreams();
    SideStreams(const SideStreams &) = delete;
    SideStreams &operator=(const SideStreams &) = delete;
    hipStream_t operator[](int k) const { return set_->s[k]; }
    void fork(hipStream_t main);   // the side streams wait for the work enqueued on main so far
    void join(hipStream_t main);   // main waits for the work enqueued on the side streams so far

  private:
    struct Set {
        int device;
        hipStream_t s[2];
        hipEvent_t fork, join[2];
    };
    Set *set_ = nullptr;
};

// out[i] = sum_{k<i} in[k] for i in [0, m); *total_dev (optional, device)
// receives the sum of all m values.  in and out may alias.  TI, TO are
// int32_t or int64_t; sums are formed in TO.
template <typename TI, typename TO>
void scan_exclusive(const TI *in, TO *out, int64_t m, TO *total_dev, hipStream_t s, Timer *t);

template <typename T>
void fill(T *p, T v, int64_t m, hipStream_t s);

void iota_i32(int32_t *p, int64_t m, hipStream_t s);

// Reduction of per-block 128-bit partials (lo, hi word pairs) into one value at out[0..1].
void sum_i128_partials(const uint64_t *partials, int64_t count, uint64_t *out, hipStream_t s);

// CSR ingest (a1).  Validates row_ptr, columns (in range, strictly
// ascending per row) and weights (>= 1); computes delta (int64[n]) and
// TW.  Optionally checks symmetry.  Throws Error(EINVAL / EOVERFLOW).
template <typename W>
void ingest_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const W *w,
                int64_t *delta, int64_t *tw_host, bool check_symmetry, hipStream_t s, Timer *t);

// Device helper: largest r in [lo, hi] with row_ptr[r] <= e (the row holding entry e).
__device__ __forceinline__ int64_t row_of_entry(const int64_t *__restrict__ row_ptr, int64_t lo,
                                                int64_t hi, int64_t e) {
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same search over a block's slice of row_ptr staged in LDS: s_rp[i] =
// row_ptr[rlo + i] for i <= hi; returns the index i (row rlo + i).
__device__ __forceinline__ int row_of_entry_lds(const int64_t *s_rp, int hi, int64_t e) {
    int lo = 0;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rp[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Entry-parallel kernels find each entry's row in LDS: row_ptr[rlo .. rhi + 1]
// of the workgroup's rows is staged into s_rp (kRowStage words) when it fits
// (a workgroup's entries span at most kEntriesPerBlock non-empty rows; long
// runs of empty rows do not fit and keep the search in memory, which the
// caller does when this returns false).  rhi + 1 <= n, so every word read
// exists.  Ends with a workgroup barrier; all threads must call it.
constexpr int kRowStage = 256 * 8 + 2;
__device__ __forceinline__ bool stage_rows(const int64_t *__restrict__ row_ptr, int64_t rlo, int64_t rhi,
                                           int64_t *s_rp) {
    const bool fits = rhi - rlo + 2 <= kRowStage;
    if (fits)
        for (int64_t i = threadIdx.x; i <= rhi - rlo + 1; i += blockDim.x) s_rp[i] = row_ptr[rlo + i];
    __syncthreads();
    return fits;
}

// Largest r in [0, n) with a[r] <= x, for a nondecreasing with a[0] <= x,
// searched by all 64 lanes of a converged wavefront (each round probes 64
// positions at once, so about log64(n) dependent loads); every lane gets r.
__device__ __forceinline__ int64_t wave_find_le(const int64_t *__restrict__ a, int64_t n, int64_t x) {
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t step = (hi - lo + 64) / 64;
        const int64_t p = lo + (int64_t)lane * step;
        const bool ok = p <= hi && a[p] <= x;
        const unsigned long long m = __ballot(ok);
        const int last = 63 - __clzll(m);
        lo = lo + (int64_t)last * step;
        const int64_t top = lo + step - 1;
        hi = top < hi ? top : hi;
    }
    return lo;
}

// The rows holding the first and last entry of an entry-parallel block,
// found by the block's first wavefront and shared through LDS.
__device__ __forceinline__ void block_row_range(const int64_t *__restrict__ row_ptr, int64_t n, int64_t nnz,
                                                int64_t base, int64_t per_block, int64_t *srange) {
    if (threadIdx.x < 64) {
        int64_t last = base + per_block - 1;
        if (last > nnz - 1) last = nnz - 1;
        const int64_t r0 = wave_find_le(row_ptr, n, base);
        const int64_t r1 = wave_find_le(row_ptr, n, last);
        if (threadIdx.x == 0) {
            srange[0] = r0;
            srange[1] = r1;
        }
    }
    __syncthreads();
}

// Adds v to out[r] for lanes holding consecutive entries of nondecreasing
// rows r (segmented inclusive scan over the wavefront, one atomic per
// row segment).  Lanes with valid == false must form the wave's tail.
__device__ __forceinline__ void seg_add_wave(int64_t *out, int64_t r, int64_t v, bool valid) {
    const int lane = threadIdx.x & 63;
    int64_t x = valid ? v : 0;
    int64_t rr = valid ? r : -1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t xo = __shfl_up(x, off);
        int64_t ro = __shfl_up(rr, off);
        if (lane >= off && ro == rr) x += xo;
    }
    int64_t rn = __shfl_down(rr, 1);
    bool last = lane == 63 || rn != rr;
    if (valid && last && x != 0) atomicAdd((unsigned long long *)&out[rr], (unsigned long long)x);
}

// Entry-parallel tiling: a 256-thread block covers kEntriesPerBlock consecutive
// CSR entries, item k of thread t is entry base + k*256 + t.
constexpr int kEntryItems = 8;
constexpr int kEntriesPerBlock = 256 * kEntryItems;
static_assert(kRowStage == kEntriesPerBlock + 2, "row_ptr slice of one entry-parallel workgroup");

}  // namespace lv
