// Renumbering and graph rebuilding (paper Section 5.1, "Renumbering nodes"
// and "Inducing new graph"), and modularity (eq. 3) of a labelling.
//
// Renumbering: presence flags per label -> exclusive scan -> rank.
// Contraction: every CSR entry (i, j, w) becomes the key (a, b) =
// (new(i), new(j)) with weight w; an LSD radix sort on the packed key
// brings equal pairs together in (a, b) order, a segmented reduction sums
// their weights, and the row pointers come from a binary search per row
// over the sorted unique keys.
#include "contract.hpp"
#include "prims.hpp"

namespace lv {

// -------------------------------------------------------------- renumber --

__global__ void k_mark(const int32_t *__restrict__ labels, int64_t n, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[labels[i]] = 1;
}

__global__ void k_relabel(const int32_t *__restrict__ labels, const int32_t *__restrict__ map, int64_t n,
                          int32_t *newlab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) newlab[i] = map[labels[i]];
}

__global__ void k_mark_kept(const int32_t *__restrict__ labels, const int32_t *__restrict__ gid,
                            const int32_t *__restrict__ keep, int64_t n, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && keep[gid[i]]) flags[labels[i]] = 1;
}

__global__ void k_gather_offsets(const int32_t *__restrict__ map, const int64_t *__restrict__ loff, int64_t nslots,
                                 int64_t *newoff) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s <= nslots) newoff[s] = map[loff[s]];
}

__global__ void k_relabel_kept(const int32_t *__restrict__ labels, const int32_t *__restrict__ map,
                               const int32_t *__restrict__ gid, const int32_t *__restrict__ keep, int64_t n,
                               int32_t *newlab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) newlab[i] = keep[gid[i]] ? map[labels[i]] : -1;
}

__global__ void k_compose(int32_t *fin, int64_t n0, const int32_t *__restrict__ newlab) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n0) fin[v] = newlab[fin[v]];
}

void Contractor::reserve(int64_t n, int64_t nnz) {
    if (n > cap_n_) {
        flags_.alloc((size_t)n + 1);
        cap_n_ = n;
    }
    if (nnz > cap_nnz_) {
        for (auto &k : key_) k.alloc((size_t)nnz);
        for (auto &v : val_) v.alloc((size_t)nnz);
        head_.alloc((size_t)nnz);
        uid_.alloc((size_t)nnz + 1);
        cap_nnz_ = nnz;
    }
}

int64_t Contractor::renumber(const int32_t *labels, int64_t n, int32_t *newlab) {
    if (n == 0) return 0;
    int32_t *flags = flags_.p;
    fill<int32_t>(flags, 0, n, s_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_mark", (double)n * 8);
        k_mark<<<grid_for(n, 256), 256, 0, s_>>>(labels, n, flags);
        LV_LAUNCHED("k_mark");
    }
    scan_exclusive<int32_t, int32_t>(flags, flags, n, flags + n, s_, t_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_relabel", (double)n * 12);
        k_relabel<<<grid_for(n, 256), 256, 0, s_>>>(labels, flags, n, newlab);
        LV_LAUNCHED("k_relabel");
    }
    int32_t k = 0;
    LV_HIP(hipMemcpyAsync(&k, flags + n, sizeof k, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));
    return k;
}

int64_t Contractor::renumber_kept(const int32_t *labels, int64_t n, const int32_t *gid, const int32_t *keep,
                                  const int64_t *loff, int64_t nslots, int32_t *newlab, int64_t *newoff) {
    if (n == 0) return 0;
    int32_t *flags = flags_.p;
    fill<int32_t>(flags, 0, n, s_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_mark_kept", (double)n * 12);
        k_mark_kept<<<grid_for(n, 256), 256, 0, s_>>>(labels, gid, keep, n, flags);
        LV_LAUNCHED("k_mark_kept");
    }
    scan_exclusive<int32_t, int32_t>(flags, flags, n, flags + n, s_, t_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_relabel_kept", (double)n * 16);
        k_relabel_kept<<<grid_for(n, 256), 256, 0, s_>>>(labels, flags, gid, keep, n, newlab);
        LV_LAUNCHED("k_relabel_kept");
    }
    // a kept graph's labels lie in its own vertex range, so the count of
    // present labels below loff[s] is the first new ID of graph s
    k_gather_offsets<<<grid_for(nslots + 1, 256), 256, 0, s_>>>(flags, loff, nslots, newoff);
    LV_LAUNCHED("k_gather_offsets");
    int32_t k = 0;
    LV_HIP(hipMemcpyAsync(&k, flags + n, sizeof k, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));
    return k;
}

void Contractor::compose(int32_t *final_labels, int64_t n0, const int32_t *newlab) {
    if (n0 == 0) return;
    TimedLaunch tl(t_, TG_CONTRACT, "k_compose", (double)n0 * 12);
    k_compose<<<grid_for(n0, 256), 256, 0, s_>>>(final_labels, n0, newlab);
    LV_LAUNCHED("k_compose");
}

// ----------------------------------------------------------- contraction --

template <typename W>
__global__ __launch_bounds__(256) void k_contract_keys(const int64_t *__restrict__ rp, int64_t n, int64_t nnz,
                                                       const int32_t *__restrict__ col, const W *__restrict__ w,
                                                       const int32_t *__restrict__ newlab, int bits,
                                                       uint64_t *keys, int64_t *vals) {
    __shared__ int64_t srange[2];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kEntriesPerBlock;
    block_row_range(rp, n, nnz, base, kEntriesPerBlock, srange);
    const int64_t rlo = srange[0], rhi = srange[1];
#pragma unroll 1
    for (int k = 0; k < kEntryItems; ++k) {
        const int64_t e = base + k * 256 + t;
        if (e >= nnz) break;
        const int64_t r = row_of_entry(rp, rlo, rhi, e);
        const int32_t na = newlab[r];
        if (na < 0) {
            keys[e] = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1);   // dropped: sorts last
            vals[e] = 0;
            continue;
        }
        const uint64_t a = (uint32_t)na, b = (uint32_t)newlab[col[e]];
        keys[e] = (a << bits) | b;
        vals[e] = (int64_t)w[e];
    }
}

constexpr int kRadixItems = 16;
constexpr int kRadixTile = 256 * kRadixItems;

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t m, int shift,
                                                    int32_t *hist, int64_t nblocks) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t e = base + k * 256 + threadIdx.x;
        if (e < m) atomicAdd(&h[(keys[e] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one 8-bit digit: the block's keys keep their order
// inside each digit (items visited in index order: k, then wave, then lane).
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const int64_t *__restrict__ vin, uint64_t *kout,
                                                       int64_t *vout, int64_t m, int shift,
                                                       const int64_t *__restrict__ offs, int64_t nblocks) {
    __shared__ int64_t s_base[256];
    __shared__ int32_t s_run[256];
    __shared__ int32_t s_wc[4][256];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    s_base[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    s_run[t] = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) s_wc[w][t] = 0;
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t e = base + k * 256 + t;
        const bool valid = e < m;
        uint64_t key = 0;
        int64_t val = 0;
        if (valid) {
            key = kin[e];
            val = vin[e];
        }
        const int d = (int)((key >> shift) & 255);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long mb = __ballot(bit);
            peers &= bit ? mb : ~mb;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) s_wc[wid][d] = __popcll(peers);
        __syncthreads();
        {
            int run = s_run[t];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int c = s_wc[w][t];
                s_wc[w][t] = run;
                run += c;
            }
            s_run[t] = run;
        }
        __syncthreads();
        if (valid) {
            const int64_t pos = s_base[d] + s_wc[wid][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 4; ++w) s_wc[w][t] = 0;
        __syncthreads();
    }
}

__global__ void k_heads(const uint64_t *__restrict__ keys, int64_t m, int32_t *head) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) head[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

// Sum the weights of equal keys into w_out[uid] and write the column and
// key of every unique entry.
__global__ __launch_bounds__(256) void k_reduce_by_key(const uint64_t *__restrict__ keys,
                                                       const int64_t *__restrict__ vals,
                                                       const int32_t *__restrict__ head,
                                                       const int64_t *__restrict__ uid, int64_t m, int bits,
                                                       int32_t *col_out, int64_t *w_out, uint64_t *ukey) {
    const int64_t base = (int64_t)blockIdx.x * kEntriesPerBlock;
    const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
#pragma unroll 1
    for (int k = 0; k < kEntryItems; ++k) {
        const int64_t e = base + k * 256 + threadIdx.x;
        const bool valid = e < m;
        int64_t u = 0, v = 0;
        if (valid) {
            // uid is the exclusive count of heads: a head's own segment index,
            // one past it for the entries that follow the head
            const int32_t h = head[e];
            u = uid[e] + h - 1;
            v = vals[e];
            if (h) {
                const uint64_t key = keys[e];
                col_out[u] = (int32_t)(key & mask);
                ukey[u] = key;
            }
        }
        seg_add_wave(w_out, u, v, valid);
    }
}

// row_ptr[a] = first unique entry whose row is >= a.
__global__ void k_rowptr(const uint64_t *__restrict__ ukey, int64_t m, int bits, int64_t n_new, int64_t *rp) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a > n_new) return;
    const uint64_t target = (uint64_t)a << bits;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ukey[mid] < target) lo = mid + 1; else hi = mid;
    }
    rp[a] = lo;
}

static int bits_for(int64_t k) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < k) ++b;
    return b;
}

int64_t Contractor::contract(const GraphView &g, const int32_t *newlab, int64_t n_new, int64_t *rp_out,
                             int32_t *col_out, int64_t *w_out) {
    const int64_t m = g.nnz;
    if (m == 0) {
        fill<int64_t>(rp_out, 0, n_new + 1, s_);
        return 0;
    }
    const int bits = bits_for(n_new + 1);   // leaves the all-ones key free for dropped entries
    const int64_t eb = (m + kEntriesPerBlock - 1) / kEntriesPerBlock;
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_contract_keys", (double)m * (4 + g.wbytes + 4 + 16) + (double)g.n * 12, g.wbytes == 4 ? "<int>" : "<long>");
        if (g.wbytes == 4)
            k_contract_keys<int32_t><<<(unsigned)eb, 256, 0, s_>>>(g.row_ptr, g.n, m, g.col, (const int32_t *)g.w,
                                                                   newlab, bits, key_[0].p, val_[0].p);
        else
            k_contract_keys<int64_t><<<(unsigned)eb, 256, 0, s_>>>(g.row_ptr, g.n, m, g.col, (const int64_t *)g.w,
                                                                   newlab, bits, key_[0].p, val_[0].p);
        LV_LAUNCHED("k_contract_keys");
    }
    // LSD radix sort of (key, weight) on the 2*bits key bits
    const int key_bits = 2 * bits;
    const int64_t rb = (m + kRadixTile - 1) / kRadixTile;
    TempBuf hist((size_t)256 * rb * sizeof(int32_t), s_);
    TempBuf offs((size_t)256 * rb * sizeof(int64_t), s_);
    int src = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        {
            TimedLaunch tl(t_, TG_CONTRACT, "k_radix_hist", (double)m * 8);
            k_radix_hist<<<(unsigned)rb, 256, 0, s_>>>(key_[src].p, m, shift, hist.as<int32_t>(), rb);
            LV_LAUNCHED("k_radix_hist");
        }
        scan_exclusive<int32_t, int64_t>(hist.as<int32_t>(), offs.as<int64_t>(), 256 * rb, (int64_t *)nullptr,
                                         s_, t_);
        {
            TimedLaunch tl(t_, TG_CONTRACT, "k_radix_scatter", (double)m * 32);
            k_radix_scatter<<<(unsigned)rb, 256, 0, s_>>>(key_[src].p, val_[src].p, key_[1 - src].p,
                                                          val_[1 - src].p, m, shift, offs.as<int64_t>(), rb);
            LV_LAUNCHED("k_radix_scatter");
        }
        src = 1 - src;
    }
    const uint64_t *keys = key_[src].p;
    const int64_t *vals = val_[src].p;
    uint64_t *ukey = key_[1 - src].p;
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_heads", (double)m * 12);
        k_heads<<<grid_for(m, 256), 256, 0, s_>>>(keys, m, head_.p);
        LV_LAUNCHED("k_heads");
    }
    scan_exclusive<int32_t, int64_t>(head_.p, uid_.p, m, uid_.p + m, s_, t_);
    int64_t m_new = 0;
    uint64_t last_key = 0;
    LV_HIP(hipMemcpyAsync(&m_new, uid_.p + m, sizeof m_new, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipMemcpyAsync(&last_key, keys + (m - 1), sizeof last_key, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));
    const uint64_t dropped_key = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1);
    const int64_t m_keep = last_key == dropped_key ? m_new - 1 : m_new;
    fill<int64_t>(w_out, 0, m_new, s_);   // the dropped segment (if any) is the last one
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_reduce_by_key", (double)m * 28 + (double)m_new * 20);
        k_reduce_by_key<<<(unsigned)eb, 256, 0, s_>>>(keys, vals, head_.p, uid_.p, m, bits, col_out, w_out, ukey);
        LV_LAUNCHED("k_reduce_by_key");
    }
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_rowptr", (double)(n_new + 1) * 8);
        k_rowptr<<<grid_for(n_new + 1, 256), 256, 0, s_>>>(ukey, m_keep, bits, n_new, rp_out);
        LV_LAUNCHED("k_rowptr");
    }
    return m_keep;
}

// ----------------------------------------------------------- modularity --

template <typename W>
__global__ __launch_bounds__(256) void k_inner_weight(const int64_t *__restrict__ rp, int64_t n, int64_t nnz,
                                                      const int32_t *__restrict__ col, const W *__restrict__ w,
                                                      const int32_t *__restrict__ lab, unsigned long long *acc) {
    __shared__ int64_t srange[2];
    __shared__ unsigned long long s_acc;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kEntriesPerBlock;
    if (t == 0) {
        s_acc = 0;
    }
    block_row_range(rp, n, nnz, base, kEntriesPerBlock, srange);
    const int64_t rlo = srange[0], rhi = srange[1];
    unsigned long long s = 0;
#pragma unroll 1
    for (int k = 0; k < kEntryItems; ++k) {
        const int64_t e = base + k * 256 + t;
        if (e >= nnz) break;
        const int64_t r = row_of_entry(rp, rlo, rhi, e);
        if (lab[r] == lab[col[e]]) s += (unsigned long long)w[e];
    }
    if (s) atomicAdd(&s_acc, s);
    __syncthreads();
    if (t == 0 && s_acc) atomicAdd(acc, s_acc);
}

__global__ void k_label_degrees(const int32_t *__restrict__ lab, const int64_t *__restrict__ delta, int64_t n,
                                int64_t *deg) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) atomicAdd((unsigned long long *)&deg[lab[v]], (unsigned long long)delta[v]);
}

__global__ __launch_bounds__(256) void k_sq_partials(const int64_t *__restrict__ deg, int64_t n, uint64_t *part) {
    __shared__ uint64_t slo[256];
    __shared__ int64_t shi[256];
    i128 s = 0;
    const int64_t base = (int64_t)blockIdx.x * 2048;
    for (int k = 0; k < 8; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v < n) s += mul_wide(deg[v], deg[v]);
    }
    slo[threadIdx.x] = (uint64_t)s;
    shi[threadIdx.x] = (int64_t)(s >> 64);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            i128 x = make_i128(slo[threadIdx.x], shi[threadIdx.x]) + make_i128(slo[threadIdx.x + w], shi[threadIdx.x + w]);
            slo[threadIdx.x] = (uint64_t)x;
            shi[threadIdx.x] = (int64_t)(x >> 64);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = slo[0];
        part[2 * blockIdx.x + 1] = (uint64_t)shi[0];
    }
}

i128 modularity_int(const GraphView &g, const int32_t *labels, hipStream_t s, Timer *t) {
    if (g.n == 0 || g.tw == 0) return 0;
    const int64_t nb = (g.n + 2047) / 2048;
    TempBuf deg((size_t)g.n * sizeof(int64_t), s);
    TempBuf part((size_t)(2 * nb + 4) * sizeof(uint64_t), s);
    uint64_t *acc = part.as<uint64_t>() + 2 * nb;      // I
    uint64_t *tot = acc + 2;                           // sum deg^2
    fill<int64_t>(deg.as<int64_t>(), 0, g.n, s);
    fill<uint64_t>(acc, 0, 1, s);
    TimedLaunch tl(t, TG_OTHER, "modularity", (double)g.nnz * 16 + (double)g.n * 24);
    k_label_degrees<<<grid_for(g.n, 256), 256, 0, s>>>(labels, g.delta, g.n, deg.as<int64_t>());
    LV_LAUNCHED("k_label_degrees");
    if (g.nnz > 0) {
        const int64_t eb = (g.nnz + kEntriesPerBlock - 1) / kEntriesPerBlock;
        if (g.wbytes == 4)
            k_inner_weight<int32_t><<<(unsigned)eb, 256, 0, s>>>(g.row_ptr, g.n, g.nnz, g.col, (const int32_t *)g.w,
                                                                 labels, (unsigned long long *)acc);
        else
            k_inner_weight<int64_t><<<(unsigned)eb, 256, 0, s>>>(g.row_ptr, g.n, g.nnz, g.col, (const int64_t *)g.w,
                                                                 labels, (unsigned long long *)acc);
        LV_LAUNCHED("k_inner_weight");
    }
    k_sq_partials<<<(unsigned)nb, 256, 0, s>>>(deg.as<int64_t>(), g.n, part.as<uint64_t>());
    LV_LAUNCHED("k_sq_partials");
    sum_i128_partials(part.as<uint64_t>(), nb, tot, s);
    uint64_t h[4];
    LV_HIP(hipMemcpyAsync(h, acc, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LV_HIP(hipStreamSynchronize(s));
    const i128 I = (i128)h[0];
    const i128 S = (i128)(((u128)h[3] << 64) | (u128)h[2]);
    return (i128)g.tw * I - S;
}

}  // namespace lv
