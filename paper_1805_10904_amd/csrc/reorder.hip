// Level-0 vertex order by row length (gather locality; the paper suggests
// placing vertices of equal or similar degree next to each other).  Vertices
// are renumbered in descending order of their row-length class
// floor(log2(len)), keeping the given order within a class (empty rows
// last), and the CSR is rebuilt in that order with remapped columns.  The
// method's results do not change: every vertex starts in a community
// labelled with its given ID, and the scores, ties, singlet rule,
// renumbering and contraction compare and key labels, never positions.
#include "driver.hpp"
#include "prims.hpp"

namespace lv {
namespace {

constexpr int kSplitThreads = 1024;               // vertices per multi-split workgroup
constexpr int kSplitWaves = kSplitThreads / 64;
constexpr int kClasses = 33;                      // 0..31: 31 - floor(log2(len)); 32: empty rows
constexpr int kPermChunk = 2048;                  // entries per row-copy workgroup

__device__ __forceinline__ int len_class(int64_t len) {
    return len == 0 ? kClasses - 1 : 31 - (63 - __clzll((unsigned long long)len));
}

// counts[c * nb + b] = vertices of class c in workgroup b's range.
__global__ __launch_bounds__(kSplitThreads) void k_class_hist(const int64_t *__restrict__ rp, int64_t n,
                                                             int64_t nb, int64_t *counts) {
    __shared__ int cnt[kClasses];
    const int t = threadIdx.x;
    if (t < kClasses) cnt[t] = 0;
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * kSplitThreads + t;
    if (v < n) atomicAdd(&cnt[len_class(rp[v + 1] - rp[v])], 1);
    __syncthreads();
    if (t < kClasses) counts[(int64_t)t * nb + blockIdx.x] = cnt[t];
}

// Stable scatter: a vertex's new position is its class's offset for its
// workgroup plus the vertices of its class before it in the workgroup
// (earlier waves, then earlier lanes of its wave).
__global__ __launch_bounds__(kSplitThreads) void k_class_scatter(const int64_t *__restrict__ rp, int64_t n, int64_t nb,
                                                                const int64_t *__restrict__ off, int32_t *order,
                                                                int32_t *pos) {
    __shared__ int wc[kSplitWaves][kClasses];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t v = (int64_t)blockIdx.x * kSplitThreads + t;
    const int c = v < n ? len_class(rp[v + 1] - rp[v]) : kClasses;   // kClasses: no vertex
    const unsigned long long below = (1ull << lane) - 1ull;
    int rank = 0;
    for (int k = 0; k < kClasses; ++k) {
        const unsigned long long m = __ballot(c == k);
        if (c == k) rank = __popcll(m & below);
        if (lane == 0) wc[wave][k] = __popcll(m);
    }
    __syncthreads();
    if (c < kClasses) {
        int64_t dst = off[(int64_t)c * nb + blockIdx.x] + rank;
        for (int w = 0; w < wave; ++w) dst += wc[w][c];
        order[dst] = (int32_t)v;
        pos[v] = (int32_t)dst;
    }
}

__global__ void k_perm_len(const int64_t *__restrict__ rp, const int64_t *__restrict__ delta,
                           const int32_t *__restrict__ order, int64_t n, int64_t *len_out, int64_t *delta_out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t i = order[p];
    len_out[p] = rp[i + 1] - rp[i];
    delta_out[p] = delta[i];
}

// Entries [k0, k0 + kPermChunk) of the new CSR: the rows overlapping the
// chunk (at most kPermChunk of them, none empty: empty rows come last) are
// staged in LDS with their source row starts; each entry finds its row by
// binary search there, then copies its weight and remaps its column.
template <typename W>
__global__ __launch_bounds__(256) void k_perm_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   const W *__restrict__ w, const int32_t *__restrict__ order,
                                                   const int32_t *__restrict__ pos, const int64_t *__restrict__ rp2,
                                                   int64_t n, int64_t nnz, int32_t *col2, W *w2) {
    __shared__ int64_t s_rp[kPermChunk + 1];
    __shared__ int64_t s_src[kPermChunk + 1];
    __shared__ int64_t s_p0;
    __shared__ int s_rows;
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * kPermChunk;
    const int64_t k1 = min(k0 + kPermChunk, nnz);
    if (t == 0) {
        // last row starting at or before k0, and last row starting before k1
        int64_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (rp2[mid] <= k0) lo = mid; else hi = mid;
        }
        int64_t lo1 = lo, hi1 = n;
        while (hi1 - lo1 > 1) {
            const int64_t mid = (lo1 + hi1) >> 1;
            if (rp2[mid] < k1) lo1 = mid; else hi1 = mid;
        }
        s_p0 = lo;
        s_rows = (int)(lo1 - lo + 1);
    }
    __syncthreads();
    const int64_t p0 = s_p0;
    const int rows = s_rows;
    for (int r = t; r <= rows; r += 256) {
        s_rp[r] = rp2[p0 + r];
        s_src[r] = r < rows ? rp[order[p0 + r]] : 0;
    }
    __syncthreads();
    for (int64_t k = k0 + t; k < k1; k += 256) {
        int lo = 0, hi = rows;   // s_rp[lo] <= k < s_rp[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_rp[mid] <= k) lo = mid; else hi = mid;
        }
        const int64_t src = s_src[lo] + (k - s_rp[lo]);
        col2[k] = pos[col[src]];
        w2[k] = w[src];
    }
}

}  // namespace

bool reorder_applies(const GraphView &g, const Tuning &tn) {
    if (tn.reorder == 2 || g.n < 2) return false;
    if (tn.reorder == 1) return true;
    return g.tw >= kCompactTwMax && g.n >= ((int64_t)1 << 20);
}

GraphView ReorderedGraph::build(const GraphView &g, hipStream_t s, Timer *t) {
    const int64_t n = g.n, nnz = g.nnz;
    const int64_t nb = (n + kSplitThreads - 1) / kSplitThreads;
    order.alloc((size_t)n);
    pos.alloc((size_t)n);
    rp.alloc((size_t)n + 1);
    col.alloc((size_t)nnz);
    delta.alloc((size_t)n);
    if (g.wbytes == 4) w32.alloc((size_t)nnz); else w64.alloc((size_t)nnz);
    {
        TempBuf counts((size_t)(2 * kClasses * nb) * sizeof(int64_t), s);
        int64_t *cnt = counts.as<int64_t>();
        int64_t *off = cnt + kClasses * nb;
        TimedLaunch tl(t, TG_LEVEL, "k_class_split", (double)n * 24);
        tl.launch(k_class_hist, (unsigned)nb, kSplitThreads, 0, s, g.row_ptr, n, nb, cnt);
        LV_LAUNCHED("k_class_hist");
        scan_exclusive<int64_t, int64_t>(cnt, off, kClasses * nb, (int64_t *)nullptr, s, t);
        tl.launch(k_class_scatter, (unsigned)nb, kSplitThreads, 0, s, g.row_ptr, n, nb, (const int64_t *)off,
                  order.p, pos.p);
        LV_LAUNCHED("k_class_scatter");
    }
    {
        TempBuf len((size_t)n * sizeof(int64_t), s);
        TimedLaunch tl(t, TG_LEVEL, "k_perm_len", (double)n * 36);
        tl.launch(k_perm_len, grid_for(n, 256), 256, 0, s, g.row_ptr, g.delta, (const int32_t *)order.p, n,
                  len.as<int64_t>(), delta.p);
        LV_LAUNCHED("k_perm_len");
        scan_exclusive<int64_t, int64_t>(len.as<int64_t>(), rp.p, n, rp.p + n, s, t);
    }
    if (nnz > 0) {
        const int64_t chunks = (nnz + kPermChunk - 1) / kPermChunk;
        TimedLaunch tl(t, TG_LEVEL, "k_perm_rows", (double)nnz * (12 + 2 * g.wbytes));
        if (g.wbytes == 4)
            tl.launch(k_perm_rows<int32_t>, (unsigned)chunks, 256, 0, s, g.row_ptr, g.col, (const int32_t *)g.w,
                      (const int32_t *)order.p, (const int32_t *)pos.p, (const int64_t *)rp.p, n, nnz, col.p, w32.p);
        else
            tl.launch(k_perm_rows<int64_t>, (unsigned)chunks, 256, 0, s, g.row_ptr, g.col, (const int64_t *)g.w,
                      (const int32_t *)order.p, (const int32_t *)pos.p, (const int64_t *)rp.p, n, nnz, col.p, w64.p);
        LV_LAUNCHED("k_perm_rows");
    }
    GraphView v = g;
    v.row_ptr = rp.p;
    v.col = col.p;
    v.w = g.wbytes == 4 ? (const void *)w32.p : (const void *)w64.p;
    v.delta = delta.p;
    return v;
}

}  // namespace lv
