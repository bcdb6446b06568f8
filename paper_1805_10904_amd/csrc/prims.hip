// Device-wide primitives: scans, fills, CSR ingest (validation, delta, TW)
// and row sums.
#include "prims.hpp"

#include <atomic>
#include <chrono>
#include <mutex>
#include <vector>

namespace lv {

Pool *&current_pool() {
    static thread_local Pool *p = nullptr;
    return p;
}

// ------------------------------------------------------------------ fills --

template <typename T>
__global__ void k_fill(T *p, T v, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
void fill(T *p, T v, int64_t m, hipStream_t s) {
    if (m <= 0) return;
    unsigned g = grid_for(m, 256);
    if (g > 65536) g = 65536;
    k_fill<T><<<g, 256, 0, s>>>(p, v, m);
    LV_LAUNCHED("k_fill");
}
template void fill<int32_t>(int32_t *, int32_t, int64_t, hipStream_t);
template void fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);
template void fill<uint64_t>(uint64_t *, uint64_t, int64_t, hipStream_t);

__global__ void k_iota(int32_t *p, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

void iota_i32(int32_t *p, int64_t m, hipStream_t s) {
    if (m <= 0) return;
    unsigned g = grid_for(m, 256);
    if (g > 65536) g = 65536;
    k_iota<<<g, 256, 0, s>>>(p, m);
    LV_LAUNCHED("k_iota");
}

// ------------------------------------------------------------ block scans --

// Exclusive scan across a 256-thread block; `total` gets the block sum.
template <typename T>
__device__ __forceinline__ T block_excl_scan_256(T v, T &total) {
    __shared__ T wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    T woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        T sw = wsum[w];
        if (w < wid) woff += sw;
        tot += sw;
    }
    __syncthreads();
    total = tot;
    return woff + x - v;
}

template <typename T>
__device__ __forceinline__ T block_sum_256(T v) {
    T tot;
    (void)block_excl_scan_256<T>(v, tot);
    return tot;
}

constexpr int kScanItems = 8;
constexpr int kScanTile = 256 * kScanItems;

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_scan_reduce(const TI *__restrict__ in, int64_t m,
                                                     TO *__restrict__ block_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    TO s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * 256 + threadIdx.x;
        if (i < m) s += (TO)in[i];
    }
    s = block_sum_256<TO>(s);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s;
}

// Down-sweep of one tile: out = exclusive prefix + the tile's offset.  The
// last block writes the grand total to *total (if non-null).  With sums,
// block_off holds the blocks' sums and every block adds up those before its
// own (at most kScanFlat of them), so a mid-size scan takes two launches.
constexpr int kScanFlat = 4096;

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_scan_down(const TI *in, TO *out, int64_t m,
                                                   const TO *__restrict__ block_off, TO *total, int sums) {
    __shared__ TO tile[kScanTile];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    TO off = 0;
    if (block_off && sums) {
        TO p = 0;
        for (int b = t; b < (int)blockIdx.x; b += 256) p += block_off[b];
        off = block_sum_256<TO>(p);
    } else if (block_off) {
        off = block_off[blockIdx.x];
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * 256 + t;
        tile[k * 256 + t] = i < m ? (TO)in[i] : (TO)0;
    }
    __syncthreads();
    TO loc[kScanItems];
    TO sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = tile[t * kScanItems + k];
        sum += loc[k];
    }
    TO tot;
    TO run = block_excl_scan_256<TO>(sum, tot);
    run += off;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        tile[t * kScanItems + k] = run;
        run += loc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * 256 + t;
        if (i < m) out[i] = tile[k * 256 + t];
    }
    if (total && t == 0 && blockIdx.x == gridDim.x - 1) *total = off + tot;
}

template <typename TI, typename TO>
void scan_exclusive(const TI *in, TO *out, int64_t m, TO *total_dev, hipStream_t s, Timer *t) {
    if (m <= 0) {
        if (total_dev) fill<TO>(total_dev, (TO)0, 1, s);
        return;
    }
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        TimedLaunch tl(t, TG_OTHER, "k_scan_down", (double)m * (sizeof(TI) + sizeof(TO)));
        tl.launch(k_scan_down<TI, TO>, 1, 256, 0, s, in, out, m, nullptr, total_dev, 0);
        LV_LAUNCHED("k_scan_down");
        return;
    }
    TempBuf bs((size_t)nb * sizeof(TO), s);
    {
        TimedLaunch tl(t, TG_OTHER, "k_scan_reduce", (double)m * sizeof(TI));
        tl.launch(k_scan_reduce<TI, TO>, (unsigned)nb, 256, 0, s, in, m, bs.as<TO>());
        LV_LAUNCHED("k_scan_reduce");
    }
    const int sums = nb <= kScanFlat ? 1 : 0;   // else the block sums are scanned first
    if (!sums) scan_exclusive<TO, TO>(bs.as<TO>(), bs.as<TO>(), nb, (TO *)nullptr, s, t);
    {
        TimedLaunch tl(t, TG_OTHER, "k_scan_down", (double)m * (sizeof(TI) + sizeof(TO)));
        tl.launch(k_scan_down<TI, TO>, (unsigned)nb, 256, 0, s, in, out, m, bs.as<TO>(), total_dev, sums);
        LV_LAUNCHED("k_scan_down");
    }
}
template void scan_exclusive<int32_t, int32_t>(const int32_t *, int32_t *, int64_t, int32_t *, hipStream_t, Timer *);
template void scan_exclusive<int32_t, int64_t>(const int32_t *, int64_t *, int64_t, int64_t *, hipStream_t, Timer *);
template void scan_exclusive<int64_t, int64_t>(const int64_t *, int64_t *, int64_t, int64_t *, hipStream_t, Timer *);

// ------------------------------------------------------------ 128-bit sums --

__global__ __launch_bounds__(256) void k_sum_i128(const uint64_t *__restrict__ partials, int64_t count,
                                                  uint64_t *out) {
    __shared__ uint64_t slo[256];
    __shared__ int64_t shi[256];
    i128 s = 0;
    for (int64_t i = threadIdx.x; i < count; i += 256)
        s += make_i128(partials[2 * i], (int64_t)partials[2 * i + 1]);
    slo[threadIdx.x] = (uint64_t)s;
    shi[threadIdx.x] = (int64_t)(s >> 64);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            i128 a = make_i128(slo[threadIdx.x], shi[threadIdx.x]);
            i128 b = make_i128(slo[threadIdx.x + w], shi[threadIdx.x + w]);
            a += b;
            slo[threadIdx.x] = (uint64_t)a;
            shi[threadIdx.x] = (int64_t)(a >> 64);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = slo[0];
        out[1] = (uint64_t)shi[0];
    }
}

void sum_i128_partials(const uint64_t *partials, int64_t count, uint64_t *out, hipStream_t s) {
    k_sum_i128<<<1, 256, 0, s>>>(partials, count, out);
    LV_LAUNCHED("k_sum_i128");
}

// Block-wide 128-bit sum of one value per thread, written as a (lo, hi) pair.
__device__ __forceinline__ void block_store_i128_sum(i128 v, uint64_t *dst) {
    __shared__ uint64_t slo[4];
    __shared__ int64_t shi[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += shfl_xor_any<i128>(v, off);
    if (lane == 0) {
        slo[wid] = (uint64_t)v;
        shi[wid] = (int64_t)(v >> 64);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        i128 s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += make_i128(slo[w], shi[w]);
        dst[0] = (uint64_t)s;
        dst[1] = (uint64_t)(int64_t)(s >> 64);
    }
}

// ------------------------------------------------------------------ ingest --

enum { BAD_ROWPTR = 1, BAD_COL = 2, BAD_WEIGHT = 4, BAD_ORDER = 8, BAD_SYMMETRY = 16 };

__global__ void k_check_rowptr(const int64_t *__restrict__ rp, int64_t n, int64_t nnz, int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t v = rp[i];
    bool ok = v >= 0 && v <= nnz;
    if (i == 0) ok = ok && v == 0;
    if (i == n) ok = ok && v == nnz;
    if (i < n) ok = ok && rp[i + 1] >= v;
    if (!ok) atomicOr(bad, BAD_ROWPTR);
}

template <typename W>
__global__ __launch_bounds__(256) void k_ingest_entries(const int64_t *__restrict__ rp, int64_t n,
                                                        int64_t nnz, const int32_t *__restrict__ col,
                                                        const W *__restrict__ w, int64_t *delta,
                                                        uint64_t *tw_partials, int *bad, int check_sym) {
    __shared__ int64_t srange[2];
    __shared__ int64_t s_rp[kRowStage];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kEntriesPerBlock;
    block_row_range(rp, n, nnz, base, kEntriesPerBlock, srange);
    const int64_t rlo = srange[0], rhi = srange[1];
    const bool staged = stage_rows(rp, rlo, rhi, s_rp);
    int errs = 0;
    i128 tw = 0;
#pragma unroll 1
    for (int k = 0; k < kEntryItems; ++k) {
        const int64_t e = base + k * 256 + t;
        const bool valid = e < nnz;
        int64_t r = 0, wv = 0;
        if (valid) {
            int64_t r_end;   // row_ptr[r + 1]
            if (staged) {
                const int i = row_of_entry_lds(s_rp, (int)(rhi - rlo), e);
                r = rlo + i;
                r_end = s_rp[i + 1];
            } else {
                r = row_of_entry(rp, rlo, rhi, e);
                r_end = rp[r + 1];
            }
            const int32_t j = col[e];
            const int64_t x = (int64_t)w[e];
            if (j < 0 || (int64_t)j >= n) errs |= BAD_COL;
            if (x < 1) errs |= BAD_WEIGHT;
            if (e + 1 < r_end && col[e + 1] <= j) errs |= BAD_ORDER;
            wv = x;
            tw += (i128)x;
            if (check_sym && j >= 0 && (int64_t)j < n) {
                int64_t lo = rp[j], hi = rp[j + 1] - 1;
                bool found = false;
                while (lo <= hi) {
                    int64_t mid = (lo + hi) >> 1;
                    int32_t cm = col[mid];
                    if (cm == (int32_t)r) { found = (int64_t)w[mid] == x; break; }
                    if (cm < (int32_t)r) lo = mid + 1; else hi = mid - 1;
                }
                if (!found) errs |= BAD_SYMMETRY;
            }
        }
        seg_add_wave(delta, r, wv, valid && !(errs & BAD_COL));
    }
    if (errs) atomicOr(bad, errs);
    block_store_i128_sum(tw, tw_partials + 2 * blockIdx.x);
}

template <typename W>
void ingest_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const W *w,
                int64_t *delta, int64_t *tw_host, bool check_symmetry, hipStream_t s, Timer *t) {
    // scratch: [0, 4) error bits, [16, 32) the 128-bit total weight
    TempBuf badb(32, s);
    int *bad = badb.as<int>();
    uint64_t *tw2 = (uint64_t *)((char *)badb.p + 16);
    LV_HIP(hipMemsetAsync(badb.p, 0, 32, s));
    fill<int64_t>(delta, 0, n, s);
    {
        TimedLaunch tl(t, TG_INGEST, "k_check_rowptr", (double)(n + 1) * 8);
        tl.launch(k_check_rowptr, grid_for(n + 1, 256), 256, 0, s, row_ptr, n, nnz, bad);
        LV_LAUNCHED("k_check_rowptr");
    }
    Readback rb(s);
    const int *hb0 = rb.add(bad);
    rb.fetch();
    int hbad = *hb0;
    require(hbad == 0, LOUVAIN_EINVAL, "row_ptr is malformed (must start at 0, be nondecreasing and end at nnz)");
    uint64_t hw[2] = {0, 0};
    if (nnz > 0) {
        const int64_t nb = (nnz + kEntriesPerBlock - 1) / kEntriesPerBlock;
        TempBuf parts((size_t)nb * 2 * sizeof(uint64_t), s);
        {
            TimedLaunch tl(t, TG_INGEST, "k_ingest_entries", (double)nnz * (4 + sizeof(W)) + (double)n * 16, type_name<W>());
            tl.launch(k_ingest_entries<W>, (unsigned)nb, 256, 0, s, row_ptr, n, nnz, col, w, delta,
                      parts.as<uint64_t>(), bad, check_symmetry ? 1 : 0);
            LV_LAUNCHED("k_ingest_entries");
        }
        sum_i128_partials(parts.as<uint64_t>(), nb, tw2, s);
        const int *hb1 = rb.add(bad);
        const uint64_t *hw1 = rb.add(tw2, 2);
        rb.fetch();
        hbad = *hb1;
        hw[0] = hw1[0];
        hw[1] = hw1[1];
    }
    require(!(hbad & BAD_COL), LOUVAIN_EINVAL, "column index out of range [0, n)");
    require(!(hbad & BAD_WEIGHT), LOUVAIN_EINVAL, "edge weight < 1 (weights must be positive integers)");
    require(!(hbad & BAD_ORDER), LOUVAIN_EINVAL, "columns must be strictly ascending inside each row (no multi-edges)");
    require(!(hbad & BAD_SYMMETRY), LOUVAIN_EINVAL, "graph is not symmetric (A_ij != A_ji)");
    i128 tw = make_i128(hw[0], (int64_t)hw[1]);
    require(tw < ((i128)1 << 62), LOUVAIN_EOVERFLOW, "total weight 2W must be below 2^62");
    *tw_host = (int64_t)tw;
}
template void ingest_csr<int32_t>(int64_t, int64_t, const int64_t *, const int32_t *, const int32_t *,
                                  int64_t *, int64_t *, bool, hipStream_t, Timer *);
template void ingest_csr<int64_t>(int64_t, int64_t, const int64_t *, const int32_t *, const int64_t *,
                                  int64_t *, int64_t *, bool, hipStream_t, Timer *);

// ------------------------------------------------------------- read-back --

namespace {

struct GatherRanges {
    const uint32_t *src[Readback::kMaxRanges];
    int off[Readback::kMaxRanges], len[Readback::kMaxRanges];
    int n;
};

// Copies the ranges, then (every thread's stores made visible to the host
// first) stores the epoch in the flag word.
__global__ __launch_bounds__(256) void k_readback(GatherRanges r, uint32_t *dst, uint32_t epoch) {
    for (int k = 0; k < r.n; ++k)
        for (int i = threadIdx.x; i < r.len[k]; i += 256) dst[r.off[k] + i] = r.src[k][i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(dst + Readback::kFlagWord, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

std::atomic<uint32_t> g_rb_epoch{0};

std::mutex g_rb_mu;
struct RbBlock {
    uint32_t *host;
    hipEvent_t ev;   // belongs to the device it was created on
    int device;
};
std::vector<RbBlock> g_rb_free;

}  // namespace

Readback::Readback(hipStream_t s) : s_(s) {
    LV_HIP(hipGetDevice(&device_));
    {
        std::lock_guard<std::mutex> lk(g_rb_mu);
        for (size_t k = g_rb_free.size(); k-- > 0;)
            if (g_rb_free[k].device == device_) {
                host_ = g_rb_free[k].host;
                ev_ = g_rb_free[k].ev;
                g_rb_free.erase(g_rb_free.begin() + (std::ptrdiff_t)k);
                break;
            }
    }
    if (!host_) {
        LV_HIP(hipHostMalloc((void **)&host_, kReadbackWords * sizeof(uint32_t), hipHostMallocCoherent));
        LV_HIP(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
    }
    LV_HIP(hipHostGetDevicePointer((void **)&dev_, host_, 0));
}

Readback::~Readback() {
    // a gather still in flight writes into the block: let it land first
    if (pending_) (void)hipEventSynchronize(ev_);
    std::lock_guard<std::mutex> lk(g_rb_mu);
    g_rb_free.push_back(RbBlock{host_, ev_, device_});
}

void *Readback::add_words(const void *src, int64_t words) {
    require(n_ < kMaxRanges && used_ + words <= kFlagWord, LOUVAIN_EDEVICE, "read-back block is full");
    src_[n_] = (const uint32_t *)src;
    off_[n_] = used_;
    len_[n_] = (int)words;
    ++n_;
    void *at = host_ + used_;
    used_ += (int)((words + 1) & ~(int64_t)1);   // keep 8-byte alignment
    return at;
}

void Readback::issue() {
    if (n_ > 0) {
        GatherRanges r;
        for (int k = 0; k < n_; ++k) {
            r.src[k] = src_[k];
            r.off[k] = off_[k];
            r.len[k] = len_[k];
        }
        r.n = n_;
        epoch_ = g_rb_epoch.fetch_add(1, std::memory_order_relaxed) + 1;
        if (epoch_ == 0) epoch_ = g_rb_epoch.fetch_add(1, std::memory_order_relaxed) + 1;   // 0: never stored
        k_readback<<<1, 256, 0, s_>>>(r, dev_, epoch_);
        LV_LAUNCHED("k_readback");
        flagged_ = true;
    }
    n_ = 0;
    LV_HIP(hipEventRecord(ev_, s_));
    pending_ = true;
}

// Waits for the gather only: work enqueued after issue() keeps running.
// Polls the flag word for up to kSpinUs, then waits on the event, which
// also reports a failed stream (whose gather never runs).
void Readback::wait() {
    constexpr int64_t kSpinUs = 2000;
    if (!pending_) issue();
    bool seen = false;
    if (flagged_) {
        const uint32_t *flag = host_ + kFlagWord;
        const auto t0 = std::chrono::steady_clock::now();
        for (int k = 0;; ++k) {
            if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == epoch_) {
                seen = true;
                break;
            }
            if ((k & 255) == 255 && std::chrono::duration_cast<std::chrono::microseconds>(
                                        std::chrono::steady_clock::now() - t0).count() > kSpinUs)
                break;
        }
    }
    if (!seen) LV_HIP(hipEventSynchronize(ev_));
    pending_ = false;
    flagged_ = false;
}

// ---------------------------------------------------------- side streams --

namespace {
std::mutex g_side_mu;
std::vector<void *> g_side_free;
}  // namespace

SideStreams::SideStreams() {
    int dev = 0;
    LV_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        for (size_t k = 0; k < g_side_free.size(); ++k) {
            Set *x = (Set *)g_side_free[k];
            if (x->device == dev) {
                set_ = x;
                g_side_free.erase(g_side_free.begin() + (std::ptrdiff_t)k);
                break;
            }
        }
    }
    if (set_) return;
    Set *x = new Set();
    x->device = dev;
    for (int k = 0; k < 2; ++k) LV_HIP(hipStreamCreateWithFlags(&x->s[k], hipStreamNonBlocking));
    LV_HIP(hipEventCreateWithFlags(&x->fork, hipEventDisableTiming));
    for (int k = 0; k < 2; ++k) LV_HIP(hipEventCreateWithFlags(&x->join[k], hipEventDisableTiming));
    set_ = x;
}

SideStreams::~SideStreams() {
    if (!set_) return;
    std::lock_guard<std::mutex> lk(g_side_mu);
    g_side_free.push_back(set_);
}

void SideStreams::fork(hipStream_t main) {
    LV_HIP(hipEventRecord(set_->fork, main));
    for (int k = 0; k < 2; ++k) LV_HIP(hipStreamWaitEvent(set_->s[k], set_->fork, 0));
}

void SideStreams::join(hipStream_t main) {
    for (int k = 0; k < 2; ++k) {
        LV_HIP(hipEventRecord(set_->join[k], set_->s[k]));
        LV_HIP(hipStreamWaitEvent(main, set_->join[k], 0));
    }
}

}  // namespace lv
