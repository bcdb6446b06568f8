// Renumbering and graph rebuilding (paper Section 5.1, "Renumbering nodes"
// and "Inducing new graph"), and modularity (eq. 3) of a labelling.
//
// Renumbering: presence flags per label -> exclusive scan -> rank.
// Contraction: every CSR entry (i, j, w) becomes (new(i), new(j), w); the
// entries are grouped by new(i), equal new(j) within a group are summed and
// the groups sorted by new(j) (segmented contraction below), which gives the
// contracted CSR with ascending columns.
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
        seg_off_.alloc((size_t)n + 1);
        seg_cur_.alloc((size_t)n + 1);
        seg_start_.alloc((size_t)n + 1);
        seg_m_.alloc((size_t)n + 1);
        cap_n_ = n;
    }
    if (nnz > cap_nnz_) {
        for (auto &k : key_) k.alloc((size_t)nnz);
        for (auto &v : val_) v.alloc((size_t)nnz);
        head_.alloc((size_t)nnz);
        uid_.alloc((size_t)nnz + 1);
        tcol_.alloc((size_t)nnz);
        tw_.alloc((size_t)nnz);
        cap_nnz_ = nnz;
    }
}

int64_t Contractor::renumber(const int32_t *labels, int64_t n, int32_t *newlab) {
    if (n == 0) return 0;
    int32_t *flags = flags_.p;
    fill<int32_t>(flags, 0, n, s_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_mark", (double)n * 8);
        tl.launch(k_mark, grid_for(n, 256), 256, 0, s_, labels, n, flags);
        LV_LAUNCHED("k_mark");
    }
    scan_exclusive<int32_t, int32_t>(flags, flags, n, flags + n, s_, t_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_relabel", (double)n * 12);
        tl.launch(k_relabel, grid_for(n, 256), 256, 0, s_, labels, flags, n, newlab);
        LV_LAUNCHED("k_relabel");
    }
    Readback rb(s_);
    const int32_t *k = rb.add(flags + n);
    rb.fetch();
    return *k;
}

int64_t Contractor::renumber_kept(const int32_t *labels, int64_t n, const int32_t *gid, const int32_t *keep,
                                  const int64_t *loff, int64_t nslots, int32_t *newlab, int64_t *newoff) {
    if (n == 0) return 0;
    int32_t *flags = flags_.p;
    fill<int32_t>(flags, 0, n, s_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_mark_kept", (double)n * 12);
        tl.launch(k_mark_kept, grid_for(n, 256), 256, 0, s_, labels, gid, keep, n, flags);
        LV_LAUNCHED("k_mark_kept");
    }
    scan_exclusive<int32_t, int32_t>(flags, flags, n, flags + n, s_, t_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_relabel_kept", (double)n * 16);
        tl.launch(k_relabel_kept, grid_for(n, 256), 256, 0, s_, labels, flags, gid, keep, n, newlab);
        LV_LAUNCHED("k_relabel_kept");
    }
    // a kept graph's labels lie in its own vertex range, so the count of
    // present labels below loff[s] is the first new ID of graph s
    k_gather_offsets<<<grid_for(nslots + 1, 256), 256, 0, s_>>>(flags, loff, nslots, newoff);
    LV_LAUNCHED("k_gather_offsets");
    Readback rb(s_);
    const int32_t *k = rb.add(flags + n);
    rb.fetch();
    return *k;
}

void Contractor::compose(int32_t *final_labels, int64_t n0, const int32_t *newlab) {
    if (n0 == 0) return;
    TimedLaunch tl(t_, TG_CONTRACT, "k_compose", (double)n0 * 12);
    tl.launch(k_compose, grid_for(n0, 256), 256, 0, s_, final_labels, n0, newlab);
    LV_LAUNCHED("k_compose");
}

// ----------------------------------------------------------- contraction --

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

// Stable scatter of one 8-bit digit of a tile of kRadixTile items.  Wave w
// ranks the tile's items [w * 1024, (w + 1) * 1024) in rounds of 64
// consecutive items: lanes with equal digits find each other by ballots,
// and the group's first lane takes the wave's running count of that digit
// from LDS, so every item's rank among the wave's items of its digit keeps
// index order.  The tile is then laid out in digit order in LDS (digit
// offsets of the tile, then of the wave), and thread t writes positions t,
// t + 256, ... of that layout: consecutive threads write consecutive
// entries of one digit's output run, so the global writes coalesce.  Keys
// and values pass through the same LDS buffer one after the other.
constexpr int kRadixWaveItems = kRadixTile / 4;

__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const int64_t *__restrict__ vin, uint64_t *kout,
                                                       int64_t *vout, int64_t m, int shift,
                                                       const int64_t *__restrict__ offs, int64_t nblocks) {
    __shared__ int64_t s_base[256];        // output position of the tile's first item of digit d
    __shared__ int32_t s_cnt[4][256];      // wave w's items of digit d, then their offset in the digit's run
    __shared__ int32_t s_off[256];         // first position of digit d in the tile's digit-ordered layout
    __shared__ int32_t s_wsum[4];
    __shared__ uint64_t s_stage[kRadixTile];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    s_base[t] = offs[(int64_t)t * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < 4; ++w) s_cnt[w][t] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kRadixTile;
    const int64_t base = tile0 + (int64_t)wid * kRadixWaveItems;
    const int tile_count = (int)(m - tile0 < kRadixTile ? m - tile0 : kRadixTile);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t key[kRadixItems];
    int64_t val[kRadixItems];
    int32_t rank[kRadixItems];
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t e = base + k * 64 + lane;
        key[k] = 0;
        val[k] = 0;
        if (e < m) {
            key[k] = kin[e];
            val[k] = vin[e];
        }
    }
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const bool valid = base + k * 64 + lane < m;
        const int d = (int)((key[k] >> shift) & 255);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long mb = __ballot(bit);
            peers &= bit ? mb : ~mb;
        }
        const int before = __popcll(peers & lt);
        int run = 0;
        if (valid && before == 0) {   // the group's first lane: the wave's count of digit d so far
            run = s_cnt[wid][d];
            s_cnt[wid][d] = run + __popcll(peers);
        }
        const int leader = valid ? __ffsll((long long)peers) - 1 : lane;
        run = __shfl(run, leader);
        rank[k] = run + before;
    }
    __syncthreads();
    // digit t: the waves' offsets inside the tile's run of t, and the run's start
    int total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int c = s_cnt[w][t];
        s_cnt[w][t] = total;
        total += c;
    }
    int x = total;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wsum[wid] = x;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wid; ++w) wbase += s_wsum[w];
    s_off[t] = wbase + x - total;
    __syncthreads();
    int32_t lpos[kRadixItems];
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        lpos[k] = -1;
        if (base + k * 64 + lane < m) {
            const int d = (int)((key[k] >> shift) & 255);
            lpos[k] = s_off[d] + s_cnt[wid][d] + rank[k];
            s_stage[lpos[k]] = key[k];
        }
    }
    __syncthreads();
    int64_t gpos[kRadixItems];
#pragma unroll
    for (int j = 0; j < kRadixItems; ++j) {
        const int p = j * 256 + t;
        gpos[j] = -1;
        if (p < tile_count) {
            const uint64_t kk = s_stage[p];
            const int d = (int)((kk >> shift) & 255);
            gpos[j] = s_base[d] + (p - s_off[d]);
            kout[gpos[j]] = kk;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k)
        if (lpos[k] >= 0) s_stage[lpos[k]] = (uint64_t)val[k];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRadixItems; ++j)
        if (gpos[j] >= 0) vout[gpos[j]] = (int64_t)s_stage[j * 256 + t];
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
                if (col_out) col_out[u] = (int32_t)(key & mask);
                ukey[u] = key;
            }
        }
        seg_add_wave(w_out, u, v, valid);
    }
}

static int bits_for(int64_t k) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < k) ++b;
    return b;
}

// ------------------------------------------------- segmented contraction --
//
// 1. every kept vertex's row gets a place in its community's segment of a
//    grouped entry array (segment sizes: per-community sums of row lengths;
//    places: one LDS-aggregated cursor add per workgroup and community);
// 2. entries are copied there with their new column (community of the
//    neighbour) and weight;
// 3. workgroups take 1,024 grouped entries each, sum equal (segment, column)
//    pairs in an LDS hash table and sort the distinct pairs (bitonic, in
//    LDS): a segment that lies inside one chunk is final and written back in
//    place; the pairs of segments spread over several chunks are merged by a
//    radix sort and a segmented sum;
// 4. row pointers are the scan of the distinct counts, and a last pass packs
//    the segments into the output CSR.

constexpr int kSegTile = 2048;    // vertices per workgroup in the grouping kernels (a community spread over
                                  // the level takes one atomic per tile: larger tiles, fewer on its address)
constexpr int kSegBits = 12;      // their LDS tables: 2^12 slots for at most 2,048 keys
constexpr int kChunk = 1024;      // grouped entries per aggregation workgroup (nominal)
constexpr int kChunkSeg = 512;    // segments of at most this many entries never cross a chunk boundary
constexpr int kChunkLen = kChunk + kChunkSeg;   // longest chunk
constexpr int kChunkBits = 11;    // its LDS hash table: 2^11 slots (load < 0.75)
constexpr unsigned long long kNoKey = ~0ull;

__device__ __forceinline__ int lds_slot(int32_t *key, int32_t k) {
    constexpr uint32_t mask = (1u << kSegBits) - 1;
    uint32_t h = ((uint32_t)k * 0x9E3779B1u) >> (32 - kSegBits);
    while (true) {
        const int32_t prev = atomicCAS(&key[h], kEmpty, k);   // claims, or returns the slot's key
        if (prev == kEmpty || prev == k) return (int)h;
        h = (h + 1) & mask;
    }
}

// cnt[a] += row length of every kept vertex of community a.
// Entries per community segment; with dsum, also the weighted degree of
// every super-vertex (delta'_a = sum of delta_i over its members: the row
// sums of the contracted graph, whose entry (a, b) sums A_ij over i in a,
// j in b).
__global__ __launch_bounds__(256) void k_seg_count(const int64_t *__restrict__ rp, const int32_t *__restrict__ newlab,
                                                   int64_t n, unsigned long long *cnt,
                                                   const int64_t *__restrict__ delta, unsigned long long *dsum) {
    constexpr int T = 1 << kSegBits;
    __shared__ int32_t s_key[T];
    __shared__ unsigned long long s_sum[T], s_del[T];
    for (int x = threadIdx.x; x < T; x += 256) {
        s_key[x] = kEmpty;
        s_sum[x] = 0;
        s_del[x] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSegTile;
#pragma unroll
    for (int k = 0; k < kSegTile / 256; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v >= n) continue;
        const int32_t a = newlab[v];
        const int64_t d = rp[v + 1] - rp[v];
        if (a < 0 || d == 0) continue;
        const int slot = lds_slot(s_key, a);
        atomicAdd(&s_sum[slot], (unsigned long long)d);
        if (dsum) atomicAdd(&s_del[slot], (unsigned long long)delta[v]);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < T; x += 256)
        if (s_key[x] != kEmpty) {
            atomicAdd(&cnt[s_key[x]], s_sum[x]);
            if (dsum) atomicAdd(&dsum[s_key[x]], s_del[x]);
        }
}

// start[v] = place of vertex v's row in its community's segment.
__global__ __launch_bounds__(256) void k_seg_start(const int64_t *__restrict__ rp, const int32_t *__restrict__ newlab,
                                                   int64_t n, const int64_t *__restrict__ off,
                                                   unsigned long long *cursor, int64_t *start) {
    constexpr int T = 1 << kSegBits;
    constexpr int K = kSegTile / 256;
    __shared__ int32_t s_key[T];
    __shared__ unsigned long long s_sum[T];
    for (int x = threadIdx.x; x < T; x += 256) {
        s_key[x] = kEmpty;
        s_sum[x] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSegTile;
    int slot[K];
    unsigned long long local[K];
    int32_t lab[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        slot[k] = -1;
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v >= n) continue;
        lab[k] = newlab[v];
        const int64_t d = rp[v + 1] - rp[v];
        if (lab[k] < 0 || d == 0) continue;
        slot[k] = lds_slot(s_key, lab[k]);
        local[k] = atomicAdd(&s_sum[slot[k]], (unsigned long long)d);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < T; x += 256)   // the workgroup's share of each community's segment
        if (s_key[x] != kEmpty) s_sum[x] = atomicAdd(&cursor[s_key[x]], s_sum[x]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (slot[k] < 0) continue;
        const int64_t v = base + k * 256 + threadIdx.x;
        start[v] = off[lab[k]] + (int64_t)(s_sum[slot[k]] + local[k]);
    }
}

template <typename W>
__global__ __launch_bounds__(256) void k_seg_scatter(const int64_t *__restrict__ rp, int64_t n, int64_t nnz,
                                                     const int32_t *__restrict__ col, const W *__restrict__ w,
                                                     const int32_t *__restrict__ newlab,
                                                     const int64_t *__restrict__ start, int32_t *tcol, int64_t *tw) {
    __shared__ int64_t srange[2];
    __shared__ int64_t s_rp[kRowStage];
    const int64_t base = (int64_t)blockIdx.x * kEntriesPerBlock;
    block_row_range(rp, n, nnz, base, kEntriesPerBlock, srange);
    const int64_t rlo = srange[0], rhi = srange[1];
    const bool staged = stage_rows(rp, rlo, rhi, s_rp);
#pragma unroll 1
    for (int k = 0; k < kEntryItems; ++k) {
        const int64_t e = base + k * 256 + threadIdx.x;
        if (e >= nnz) break;
        int64_t r, r0;   // the entry's row and its first entry
        if (staged) {
            const int i = row_of_entry_lds(s_rp, (int)(rhi - rlo), e);
            r = rlo + i;
            r0 = s_rp[i];
        } else {
            r = row_of_entry(rp, rlo, rhi, e);
            r0 = rp[r];
        }
        const int32_t a = newlab[r];
        if (a < 0) continue;
        const int64_t dst = start[r] + (e - r0);
        tcol[dst] = newlab[col[e]];
        tw[dst] = (int64_t)w[e];
    }
}

// Inclusive max-scan of s[0, kChunkLen) in place (256 threads, R items each).
__device__ __forceinline__ void block_max_scan_chunk(int32_t *s, int32_t *s_wave) {
    constexpr int R = kChunkLen / 256;
    static_assert(kChunkLen % 256 == 0, "scan tiling");
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    int32_t v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = s[R * t + i];
#pragma unroll
    for (int i = 1; i < R; ++i) v[i] = v[i] > v[i - 1] ? v[i] : v[i - 1];
    int32_t x = v[R - 1];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off);
        if (lane >= off && y > x) x = y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    int32_t before = __shfl_up(x, 1);
    if (lane == 0) before = INT32_MIN;
    for (int w2 = 0; w2 < wid; ++w2) before = s_wave[w2] > before ? s_wave[w2] : before;
#pragma unroll
    for (int i = 0; i < R; ++i) s[R * t + i] = v[i] > before ? v[i] : before;
    __syncthreads();
}

// Start of chunk b: b * kChunk moved back to the start of the segment
// holding it when that segment has at most kChunkSeg entries, so such a
// segment never crosses a chunk boundary and its pairs are always final in
// its chunk (longer segments are aggregated by the middle tier and the
// pieces, or, in the exported contraction, merged).  Starts increase with b
// and a chunk has fewer than kChunkLen entries.  Called by one full
// wavefront.
__device__ __forceinline__ int64_t chunk_start(const int64_t *__restrict__ off, int64_t k, int64_t m_raw, int64_t b) {
    const int64_t x = b * kChunk;
    if (x <= 0) return 0;
    if (x >= m_raw) return m_raw;
    const int64_t s = wave_find_le(off, k, x);   // segment holding entry x
    const int64_t st = off[s];
    return off[s + 1] - st <= kChunkSeg ? st : x;
}

// Shared first half of the chunk kernels: the chunk's first and last
// segment (slo, shi), the local segment of every entry (s_mark) and the sum
// of every (local segment, column) pair in the LDS hash table s_hk / s_hv.
// Chunks cut the space of coff (segment starts of the entries the chunks
// aggregate: off itself, or the short segments' entries only, where every
// other segment is empty); entry x of a chunk is then entry
// off[sg] + (cb + x - coff[sg]) of the grouped arrays.
__device__ __forceinline__ void chunk_aggregate(const int64_t *__restrict__ coff, const int64_t *__restrict__ off,
                                                int64_t k, int64_t cb, int len,
                                                const int32_t *__restrict__ tcol, const int64_t *__restrict__ tw,
                                                unsigned long long *s_hk, long long *s_hv, int32_t *s_mark,
                                                int32_t *s_wave, int64_t *s_range) {
    constexpr int T = 1 << kChunkBits;
    constexpr uint32_t mask = T - 1;
    const int t = threadIdx.x;
    for (int x = t; x < T; x += 256) {
        s_hk[x] = kNoKey;
        s_hv[x] = 0;
    }
    for (int x = t; x < kChunkLen; x += 256) s_mark[x] = -1;
    if (t < 64) {   // segments of the chunk's first and last entry (64-way search)
        const int64_t a0 = wave_find_le(coff, k, cb);
        const int64_t a1 = wave_find_le(coff, k, cb + len - 1);
        if (t == 0) {
            s_range[0] = a0;
            s_range[1] = a1;
        }
    }
    __syncthreads();
    const int64_t slo = s_range[0], shi = s_range[1];
    if (shi - slo <= kChunkLen) {
        // segment of every entry: markers at segment starts, then a max-scan
        for (int64_t sg = slo + 1 + t; sg <= shi; sg += 256) atomicMax(&s_mark[coff[sg] - cb], (int32_t)(sg - slo));
        if (t == 0) s_mark[0] = 0;   // markers never land on position 0
        __syncthreads();
        block_max_scan_chunk(s_mark, s_wave);
    } else {
        // the chunk spans many empty segments (communities without entries):
        // the last segment starting at or before each entry, by binary search
        for (int x = t; x < len; x += 256) {
            int64_t lo = slo, hi = shi;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (coff[mid] <= cb + x) lo = mid; else hi = mid - 1;
            }
            s_mark[x] = (int32_t)(lo - slo);
        }
        __syncthreads();
    }
    for (int x = t; x < len; x += 256) {
        const int32_t ls = s_mark[x];
        const int64_t e = off[slo + ls] + (cb + x - coff[slo + ls]);
        const unsigned long long key = ((unsigned long long)(uint32_t)ls << 32) | (uint32_t)tcol[e];
        const long long val = (long long)tw[e];
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - kChunkBits));
        while (true) {
            const unsigned long long prev = atomicCAS(&s_hk[h], kNoKey, key);   // claims, or returns the key
            if (prev == kNoKey || prev == key) break;
            h = (h + 1) & mask;
        }
        atomicAdd((unsigned long long *)&s_hv[h], (unsigned long long)val);
    }
    __syncthreads();
}

// Levels inside a run: the order of a row's columns does not matter to the
// method (sweeps and contraction depend on each row's multiset of columns
// and weights only), so distinct pairs are placed in table order, each
// segment's through its own LDS counter, without sorting.
__global__ __launch_bounds__(256) void k_seg_chunk_any(const int64_t *__restrict__ coff, const int64_t *__restrict__ off,
                                                       int64_t k, int64_t m_raw, int32_t *tcol, int64_t *tw,
                                                       int64_t *mcount, uint64_t *pkey, int64_t *pval,
                                                       unsigned long long *pcount, int bits) {
    constexpr int T = 1 << kChunkBits;
    __shared__ unsigned long long s_hk[T];
    __shared__ long long s_hv[T];
    __shared__ int32_t s_mark[kChunkLen];
    __shared__ int32_t s_cnt[kChunkLen];   // pairs per segment, at the segment's first position
    __shared__ int32_t s_cur[kChunkLen];
    __shared__ int32_t s_wave[4];
    __shared__ int64_t s_range[2];
    __shared__ int64_t s_bounds[2];
    __shared__ unsigned long long s_pbase;
    const int t = threadIdx.x;
    if (t < 64) {
        const int64_t b0 = chunk_start(coff, k, m_raw, blockIdx.x);
        const int64_t b1 = chunk_start(coff, k, m_raw, (int64_t)blockIdx.x + 1);
        if (t == 0) {
            s_bounds[0] = b0;
            s_bounds[1] = b1;
        }
    }
    for (int x = t; x < kChunkLen; x += 256) {
        s_cnt[x] = 0;
        s_cur[x] = 0;
    }
    __syncthreads();
    const int64_t cb = s_bounds[0], ce = s_bounds[1];
    const int len = (int)(ce - cb);
    if (len <= 0) return;   // uniform: every segment around here was taken by a neighbour
    chunk_aggregate(coff, off, k, cb, len, tcol, tw, s_hk, s_hv, s_mark, s_wave, s_range);
    const int64_t slo = s_range[0], shi = s_range[1];
    const bool first_spans = coff[slo] < cb;
    const bool last_spans = coff[shi + 1] > ce;
    const uint32_t last_local = (uint32_t)(shi - slo);
    for (int x = t; x < T; x += 256) {
        const unsigned long long key = s_hk[x];
        if (key == kNoKey) continue;
        const uint32_t ls = (uint32_t)(key >> 32);
        const int p = ls == 0 ? 0 : (int)(coff[slo + ls] - cb);
        atomicAdd(&s_cnt[p], 1);
    }
    __syncthreads();
    const int p_last = last_local == 0 ? 0 : (int)(coff[shi] - cb);
    if (t == 0) {
        int np = 0;
        if (last_local == 0) {
            if (first_spans || last_spans) np = s_cnt[0];
        } else {
            if (first_spans) np += s_cnt[0];
            if (last_spans) np += s_cnt[p_last];
        }
        s_pbase = np ? atomicAdd(pcount, (unsigned long long)np) : 0;
    }
    __syncthreads();
    const unsigned long long pbase = s_pbase;
    const int first_n = (first_spans && last_local != 0) ? s_cnt[0] : 0;
    for (int x = t; x < T; x += 256) {
        const unsigned long long key = s_hk[x];
        if (key == kNoKey) continue;
        const uint32_t ls = (uint32_t)(key >> 32);
        const int64_t sg = slo + ls;
        const int p = ls == 0 ? 0 : (int)(coff[sg] - cb);
        const int pos = atomicAdd(&s_cur[p], 1);
        const int32_t c = (int32_t)(uint32_t)key;
        const long long val = s_hv[x];
        if (ls == 0 && first_spans) {
            pkey[pbase + pos] = ((uint64_t)sg << bits) | (uint32_t)c;
            pval[pbase + pos] = val;
        } else if (ls == last_local && last_spans) {
            pkey[pbase + first_n + pos] = ((uint64_t)sg << bits) | (uint32_t)c;
            pval[pbase + first_n + pos] = val;
        } else {
            tcol[off[sg] + pos] = c;
            tw[off[sg] + pos] = val;
        }
    }
    // counts of the segments that end here
    for (int p = t; p < len; p += 256) {
        const int32_t n_p = s_cnt[p];
        if (n_p == 0) continue;
        const uint32_t ls = (uint32_t)s_mark[p];
        if ((ls == 0 && first_spans) || (ls == last_local && last_spans)) continue;
        mcount[slo + ls] = n_p;
    }
}

// Segments longer than kMidMax entries (the communities with the most
// member entries) are cut into pieces of kPiece entries, one 1,024-thread
// workgroup each with a 2^13-slot LDS table keyed by column.  A segment of
// one piece whose columns all found a slot and that has at most direct_max
// distinct columns (the next level's longest row swept from LDS) writes its
// pairs in place (table order) and its count.  Otherwise the piece's pairs
// (and any pair that found no slot) join the partial pairs that are sorted
// and merged, like those of segments crossing a chunk boundary: the longer
// rows are swept through HBM hub tables at the next level, whose LDS
// pre-aggregation gains from ascending columns.
constexpr int kPiece = 16384;
constexpr int kPieceBits = 13;
constexpr int kPieceProbe = 32;
constexpr int kPieceThreads = 1024;
// Segments of kChunkSeg + 1 .. kMidMax entries take one 256-thread
// workgroup each with a 2^12-slot table (a quarter of the long pieces' LDS,
// so three workgroups share a CU instead of one): their distinct columns
// always fit the table's claimable 3/4.
constexpr int kMidMax = 2730;
constexpr int kMidBits = 12;
constexpr int kMidThreads = 256;

// Pieces of every segment longer than kMidMax (0 otherwise), a flag for
// every segment of kChunkSeg + 1 .. kMidMax entries, and the entries of
// every segment the chunks aggregate (0 for the others); tot[0] / tot[1]
// receive the entry counts of the first two kinds.
__global__ __launch_bounds__(256) void k_big_pieces(const int64_t *__restrict__ off, int64_t k, int64_t *pieces,
                                                    int64_t *mids, int64_t *shorts, unsigned long long *tot,
                                                    int64_t piece) {
    __shared__ unsigned long long s_tot[4][2];
    unsigned long long big = 0, mid = 0;
    for (int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x; a < k; a += (int64_t)gridDim.x * 256) {
        const int64_t sz = off[a + 1] - off[a];
        pieces[a] = sz > kMidMax ? (sz + piece - 1) / piece : 0;
        mids[a] = sz > kChunkSeg && sz <= kMidMax ? 1 : 0;
        shorts[a] = sz <= kChunkSeg ? sz : 0;
        if (sz > kMidMax) big += (unsigned long long)sz;
        else if (sz > kChunkSeg) mid += (unsigned long long)sz;
    }
    // one atomic per workgroup and total (the grid is at most a few
    // thousand workgroups)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        big += __shfl_xor(big, o);
        mid += __shfl_xor(mid, o);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_tot[wid][0] = big;
        s_tot[wid][1] = mid;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const unsigned long long x = s_tot[0][threadIdx.x] + s_tot[1][threadIdx.x] + s_tot[2][threadIdx.x] +
                                     s_tot[3][threadIdx.x];
        if (x) atomicAdd(&tot[threadIdx.x], x);
    }
}

// One workgroup per piece of PIECE entries (THREADS threads, a table of
// 2^TBITS slots); poff: exclusive scan of the pieces of every segment (k + 1).
template <int THREADS, int TBITS, int PIECE>
__global__ __launch_bounds__(THREADS) void k_big_piece(const int64_t *__restrict__ off, int64_t k,
                                                       const int64_t *__restrict__ poff, int32_t *tcol,
                                                       int64_t *tw, int64_t *mcount, uint64_t *pkey,
                                                       int64_t *pval, unsigned long long *pcount, int bits,
                                                       int64_t direct_max) {
    constexpr int T = 1 << TBITS;
    constexpr int Q = T / THREADS;
    __shared__ int32_t s_k[T];
    __shared__ long long s_v[T];
    __shared__ int64_t s_seg, s_idx;
    __shared__ int s_n, s_over, s_used;
    __shared__ unsigned long long s_base, s_obase;
    const int t = threadIdx.x;
    for (int x = t; x < T; x += THREADS) {
        s_k[x] = kEmpty;
        s_v[x] = 0;
    }
    if (t < 64) {
        const int64_t a = wave_find_le(poff, k, (int64_t)blockIdx.x);   // the segment holding this piece
        if (t == 0) {
            s_seg = a;
            s_idx = (int64_t)blockIdx.x - poff[a];
            s_n = 0;
            s_over = 0;
            s_used = 0;
        }
    }
    __syncthreads();
    const int64_t a = s_seg;
    const int64_t lo = off[a] + s_idx * PIECE;
    const int64_t end = off[a + 1] < lo + PIECE ? off[a + 1] : lo + PIECE;
    // New columns claim slots only while the table is at most 3/4 full, so
    // probes stay short; a column that finds neither its slot nor room is
    // an overflow pair (marked here, written after one reservation).
    constexpr int kClaimMax = 3 * T / 4;
    uint32_t over = 0;   // entry q of this thread overflowed
    int n_over = 0;
    static_assert(PIECE / THREADS <= 32, "one mask bit per entry of a thread");
    for (int q = 0; lo + t + (int64_t)q * THREADS < end; ++q) {
        const int64_t e = lo + t + (int64_t)q * THREADS;
        const int32_t c = tcol[e];
        const int64_t w = tw[e];
        uint32_t h = ((uint32_t)c * 0x9E3779B1u) >> (32 - TBITS);
        bool placed = false;
        for (int p = 0; p < kPieceProbe; ++p) {
            const int32_t cur = s_k[h];
            if (cur == c) {
                placed = true;
                break;
            }
            if (cur == kEmpty) {
                if (s_used >= kClaimMax) break;
                const int32_t prev = atomicCAS(&s_k[h], kEmpty, c);
                if (prev == kEmpty) atomicAdd(&s_used, 1);
                if (prev == kEmpty || prev == c) {
                    placed = true;
                    break;
                }
            }
            h = (h + 1) & (T - 1);
        }
        if (placed) {
            atomicAdd((unsigned long long *)&s_v[h], (unsigned long long)w);
        } else {
            over |= 1u << q;
            ++n_over;
        }
    }
    const int my_over = n_over ? atomicAdd(&s_over, n_over) : 0;
    __syncthreads();
    if (t == 0 && s_over) s_obase = atomicAdd(pcount, (unsigned long long)s_over);
    __syncthreads();
    if (n_over) {
        unsigned long long qpos = s_obase + (unsigned long long)my_over;
        for (int q = 0; over; ++q, over >>= 1) {
            if (!(over & 1u)) continue;
            const int64_t e = lo + t + (int64_t)q * THREADS;
            pkey[qpos] = ((uint64_t)a << bits) | (uint32_t)tcol[e];
            pval[qpos] = tw[e];
            ++qpos;
        }
    }
    int pos[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int x = t + q * THREADS;
        pos[q] = s_k[x] != kEmpty ? atomicAdd(&s_n, 1) : -1;
    }
    __syncthreads();
    const bool direct = poff[a + 1] - poff[a] == 1 && s_over == 0 && s_n <= direct_max;
    if (direct) {
        // the whole segment was read above; its pairs go in place
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (pos[q] < 0) continue;
            const int x = t + q * THREADS;
            tcol[off[a] + pos[q]] = s_k[x];
            tw[off[a] + pos[q]] = s_v[x];
        }
        if (t == 0) mcount[a] = s_n;
        return;
    }
    if (t == 0) s_base = atomicAdd(pcount, (unsigned long long)s_n);
    __syncthreads();
    const unsigned long long base = s_base;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (pos[q] < 0) continue;
        const int x = t + q * THREADS;
        pkey[base + pos[q]] = ((uint64_t)a << bits) | (uint32_t)s_k[x];
        pval[base + pos[q]] = s_v[x];
    }
}

// As k_big_piece with a table of single words, (column + 1) << shift | the
// weight sum, when every column + 1 fits the 64 - shift high bits and every
// weight sum (at most 2W) the low ones: half the LDS per slot, so a piece of
// kPieceW entries gets a 16,384-slot table (128 KB) whose claimable 3/4
// hold every column of a piece even when all are distinct, and the middle
// tier's 4,096-slot table takes 32 KB.  A claim is one compare-and-swap of
// the whole word; an add to a claimed slot never carries into the column.
constexpr int kPieceW = 12288;
constexpr int kPieceWBits = 14;

template <int THREADS, int TBITS, int PIECE>
__global__ __launch_bounds__(THREADS) void k_piece_word(const int64_t *__restrict__ off, int64_t k,
                                                        const int64_t *__restrict__ poff, int32_t *tcol,
                                                        int64_t *tw, int64_t *mcount, uint64_t *pkey,
                                                        int64_t *pval, unsigned long long *pcount, int bits,
                                                        int64_t direct_max, int shift) {
    constexpr int T = 1 << TBITS;
    constexpr int Q = T / THREADS;
    __shared__ unsigned long long s_t[T];
    __shared__ int64_t s_seg, s_idx;
    __shared__ int s_n, s_over, s_used;
    __shared__ unsigned long long s_base, s_obase;
    const int t = threadIdx.x;
    for (int x = t; x < T; x += THREADS) s_t[x] = 0;
    if (t < 64) {
        const int64_t a = wave_find_le(poff, k, (int64_t)blockIdx.x);   // the segment holding this piece
        if (t == 0) {
            s_seg = a;
            s_idx = (int64_t)blockIdx.x - poff[a];
            s_n = 0;
            s_over = 0;
            s_used = 0;
        }
    }
    __syncthreads();
    const int64_t a = s_seg;
    const int64_t lo = off[a] + s_idx * PIECE;
    const int64_t end = off[a + 1] < lo + PIECE ? off[a + 1] : lo + PIECE;
    const unsigned long long tmask = ~0ull << shift;
    constexpr int kClaimMax = 3 * T / 4;
    uint32_t over = 0;   // entry q of this thread overflowed
    int n_over = 0;
    static_assert(PIECE / THREADS <= 32, "one mask bit per entry of a thread");
    for (int q = 0; lo + t + (int64_t)q * THREADS < end; ++q) {
        const int64_t e = lo + t + (int64_t)q * THREADS;
        const int32_t c = tcol[e];
        const unsigned long long w = (unsigned long long)tw[e];
        const unsigned long long tag = (unsigned long long)(uint32_t)(c + 1) << shift;
        uint32_t h = ((uint32_t)c * 0x9E3779B1u) >> (32 - TBITS);
        bool placed = false;
        for (int p = 0; p < kPieceProbe; ++p) {
            const unsigned long long cur = ((volatile unsigned long long *)s_t)[h];
            if ((cur & tmask) == tag) {
                atomicAdd(&s_t[h], w);
                placed = true;
                break;
            }
            if (cur == 0) {
                if (s_used >= kClaimMax) break;
                const unsigned long long prev = atomicCAS(&s_t[h], 0ull, tag | w);
                if (prev == 0) {
                    atomicAdd(&s_used, 1);
                    placed = true;
                    break;
                }
                if ((prev & tmask) == tag) {
                    atomicAdd(&s_t[h], w);
                    placed = true;
                    break;
                }
            }
            h = (h + 1) & (T - 1);
        }
        if (!placed) {
            over |= 1u << q;
            ++n_over;
        }
    }
    const int my_over = n_over ? atomicAdd(&s_over, n_over) : 0;
    __syncthreads();
    if (t == 0 && s_over) s_obase = atomicAdd(pcount, (unsigned long long)s_over);
    __syncthreads();
    if (n_over) {
        unsigned long long qpos = s_obase + (unsigned long long)my_over;
        for (int q = 0; over; ++q, over >>= 1) {
            if (!(over & 1u)) continue;
            const int64_t e = lo + t + (int64_t)q * THREADS;
            pkey[qpos] = ((uint64_t)a << bits) | (uint32_t)tcol[e];
            pval[qpos] = tw[e];
            ++qpos;
        }
    }
    int pos[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int x = t + q * THREADS;
        pos[q] = s_t[x] != 0 ? atomicAdd(&s_n, 1) : -1;
    }
    __syncthreads();
    const bool direct = poff[a + 1] - poff[a] == 1 && s_over == 0 && s_n <= direct_max;
    unsigned long long base = 0;
    if (!direct) {
        if (t == 0) s_base = atomicAdd(pcount, (unsigned long long)s_n);
        __syncthreads();
        base = s_base;
    } else if (t == 0) {
        mcount[a] = s_n;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (pos[q] < 0) continue;
        const unsigned long long wd = s_t[t + q * THREADS];
        const int32_t c = (int32_t)(wd >> shift) - 1;
        const int64_t w = (int64_t)(wd & ~tmask);
        if (direct) {
            // the whole segment was read above; its pairs go in place
            tcol[off[a] + pos[q]] = c;
            tw[off[a] + pos[q]] = w;
        } else {
            pkey[base + pos[q]] = ((uint64_t)a << bits) | (uint32_t)c;
            pval[base + pos[q]] = w;
        }
    }
}

// The exported contraction: as k_seg_chunk_any, but the distinct pairs of
// a chunk are sorted (bitonic, in LDS) so that every row's columns ascend.
__global__ __launch_bounds__(256) void k_seg_chunk(const int64_t *__restrict__ off, int64_t k, int64_t m_raw,
                                                   int32_t *tcol, int64_t *tw, int64_t *mcount, uint64_t *pkey,
                                                   int64_t *pval, unsigned long long *pcount, int bits) {
    constexpr int T = 1 << kChunkBits;
    __shared__ unsigned long long s_hk[T];
    __shared__ long long s_hv[T];
    __shared__ unsigned long long s_sk[2 * kChunk];   // sorted pairs (padded to a power of two)
    __shared__ long long s_sv[2 * kChunk];
    __shared__ int32_t s_mark[kChunkLen];
    static_assert(kChunkLen <= 2 * kChunk, "a chunk's distinct pairs fit the sort buffer");
    __shared__ int32_t s_wave[4];
    __shared__ int s_nd;
    __shared__ int64_t s_range[2];
    __shared__ int64_t s_bounds[2];
    __shared__ unsigned long long s_pbase;
    const int t = threadIdx.x;
    if (t < 64) {
        const int64_t b0 = chunk_start(off, k, m_raw, blockIdx.x);
        const int64_t b1 = chunk_start(off, k, m_raw, (int64_t)blockIdx.x + 1);
        if (t == 0) {
            s_bounds[0] = b0;
            s_bounds[1] = b1;
            s_nd = 0;
            s_pbase = 0;
        }
    }
    __syncthreads();
    const int64_t cb = s_bounds[0], ce = s_bounds[1];
    const int len = (int)(ce - cb);
    if (len <= 0) return;
    chunk_aggregate(off, off, k, cb, len, tcol, tw, s_hk, s_hv, s_mark, s_wave, s_range);
    const int64_t slo = s_range[0], shi = s_range[1];
    {   // compaction of the occupied slots: one LDS atomic per wavefront and round
        const int lane = t & 63;
        const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        for (int x0 = 0; x0 < T; x0 += 256) {
            const int x = x0 + t;
            const bool occ = s_hk[x] != kNoKey;
            const unsigned long long msk = __ballot(occ);
            int base = 0;
            if (lane == 0 && msk) base = atomicAdd(&s_nd, (int)__popcll(msk));
            base = __shfl(base, 0);
            if (occ) {
                const int i = base + (int)__popcll(msk & lt);
                s_sk[i] = s_hk[x];
                s_sv[i] = s_hv[x];
            }
        }
    }
    __syncthreads();
    const int nd = s_nd;
    int P = 1;
    while (P < nd) P <<= 1;
    for (int x = nd + t; x < P; x += 256) s_sk[x] = kNoKey;
    __syncthreads();
    // bitonic sort of (key, value) pairs, keys ascending
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = t; q < P / 2; q += 256) {
                const int i = 2 * q - (q & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const unsigned long long a = s_sk[i], b = s_sk[j];
                if ((a > b) == up) {
                    s_sk[i] = b;
                    s_sk[j] = a;
                    const long long va = s_sv[i];
                    s_sv[i] = s_sv[j];
                    s_sv[j] = va;
                }
            }
            __syncthreads();
        }
    }
    // the first and the last segment may continue in other chunks
    const bool first_spans = off[slo] < cb;
    const bool last_spans = off[shi + 1] > ce;
    const uint32_t last_local = (uint32_t)(shi - slo);
    int n_first = 0, n_last = 0;
    if (first_spans || last_spans) {
        // entries of the first segment form a prefix, those of the last a suffix
        int lo = 0, hi = nd;   // first index with local segment > 0
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((s_sk[mid] >> 32) > 0) hi = mid; else lo = mid + 1;
        }
        n_first = lo;
        lo = 0;
        hi = nd;                // first index of the last segment
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((uint32_t)(s_sk[mid] >> 32) >= last_local) hi = mid; else lo = mid + 1;
        }
        n_last = nd - lo;
        if (t == 0) {
            int np = 0;
            if (first_spans) np += n_first;
            if (last_spans && !(first_spans && last_local == 0)) np += n_last;
            s_pbase = np ? atomicAdd(pcount, (unsigned long long)np) : 0;
        }
    }
    __syncthreads();
    const unsigned long long pbase = s_pbase;
    for (int i = t; i < nd; i += 256) {
        const unsigned long long key = s_sk[i];
        const uint32_t sl = (uint32_t)(key >> 32);
        const int64_t sg = slo + sl;
        const int32_t c = (int32_t)(uint32_t)key;
        const long long val = s_sv[i];
        const bool spans = (sl == 0 && first_spans) || (sl == last_local && last_spans);
        if (spans) {
            const int64_t r = (sl == 0 && first_spans) ? i : (first_spans ? n_first : 0) + (i - (nd - n_last));
            pkey[pbase + r] = ((uint64_t)sg << bits) | (uint32_t)c;
            pval[pbase + r] = val;
            continue;
        }
        // first index of this segment in the sorted pairs
        int lo = 0, hi = i;
        const unsigned long long lb = (unsigned long long)sl << 32;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_sk[mid] < lb) lo = mid + 1; else hi = mid;
        }
        const int64_t pos = i - lo;
        tcol[off[sg] + pos] = c;
        tw[off[sg] + pos] = val;
        if (i + 1 == nd || (uint32_t)(s_sk[i + 1] >> 32) != sl) mcount[sg] = pos + 1;
    }
}

// Merged pairs of segments spread over several chunks: write them to their
// segments in key order and record the counts.
__global__ void k_seg_merge_write(const uint64_t *__restrict__ ukey, const int64_t *__restrict__ usum,
                                  const int64_t *__restrict__ u_n_dev, int bits, const int64_t *__restrict__ off,
                                  int32_t *tcol, int64_t *tw, int64_t *mcount) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t u_n = *u_n_dev;
    if (u >= u_n) return;
    const uint64_t key = ukey[u];
    const int64_t sg = (int64_t)(key >> bits);
    const uint64_t lb = (uint64_t)sg << bits;
    int64_t lo = 0, hi = u;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ukey[mid] < lb) lo = mid + 1; else hi = mid;
    }
    const int64_t pos = u - lo;
    tcol[off[sg] + pos] = (int32_t)(key & ((1ull << bits) - 1));
    tw[off[sg] + pos] = usum[u];
    if (u + 1 == u_n || (int64_t)(ukey[u + 1] >> bits) != sg) mcount[sg] = pos + 1;
}

// Output CSR: entry u of row a comes from its segment's u - rp[a]-th pair.
// The entry count m_new = rp[n_new] is read on the device; the grid covers
// an upper bound of it.  WO: output weight type (int32 only where every
// weight is known to be below 2^31).
template <typename WO>
__global__ __launch_bounds__(256) void k_seg_pack(const int64_t *__restrict__ rp, int64_t n_new,
                                                  const int64_t *__restrict__ off, const int32_t *__restrict__ tcol,
                                                  const int64_t *__restrict__ tw, int32_t *col_out, WO *w_out) {
    __shared__ int64_t srange[2];
    const int64_t base = (int64_t)blockIdx.x * kEntriesPerBlock;
    const int64_t m_new = rp[n_new];
    if (base >= m_new) return;   // uniform over the workgroup
    block_row_range(rp, n_new, m_new, base, kEntriesPerBlock, srange);
    const int64_t rlo = srange[0], rhi = srange[1];
    __shared__ int64_t s_rp[kRowStage];
    const bool staged = stage_rows(rp, rlo, rhi, s_rp);
#pragma unroll 1
    for (int k = 0; k < kEntryItems; ++k) {
        const int64_t u = base + k * 256 + threadIdx.x;
        if (u >= m_new) break;
        int64_t a, a0;   // the entry's row and its first entry
        if (staged) {
            const int i = row_of_entry_lds(s_rp, (int)(rhi - rlo), u);
            a = rlo + i;
            a0 = s_rp[i];
        } else {
            a = row_of_entry(rp, rlo, rhi, u);
            a0 = rp[a];
        }
        const int64_t src = off[a] + (u - a0);
        col_out[u] = tcol[src];
        w_out[u] = (WO)tw[src];
    }
}

const int64_t *Contractor::sort_sum(int64_t m, int key_bits, const uint64_t **ukeys, const int64_t **usums) {
    const int64_t rb = (m + kRadixTile - 1) / kRadixTile;
    TempBuf hist((size_t)256 * rb * sizeof(int32_t), s_);
    TempBuf offs((size_t)256 * rb * sizeof(int64_t), s_);
    int src = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        {
            TimedLaunch tl(t_, TG_CONTRACT, "k_radix_hist", (double)m * 8);
            tl.launch(k_radix_hist, (unsigned)rb, 256, 0, s_, key_[src].p, m, shift, hist.as<int32_t>(), rb);
            LV_LAUNCHED("k_radix_hist");
        }
        scan_exclusive<int32_t, int64_t>(hist.as<int32_t>(), offs.as<int64_t>(), 256 * rb, (int64_t *)nullptr,
                                         s_, t_);
        {
            TimedLaunch tl(t_, TG_CONTRACT, "k_radix_scatter", (double)m * 32);
            tl.launch(k_radix_scatter, (unsigned)rb, 256, 0, s_, key_[src].p, val_[src].p, key_[1 - src].p,
                      val_[1 - src].p, m, shift, offs.as<int64_t>(), rb);
            LV_LAUNCHED("k_radix_scatter");
        }
        src = 1 - src;
    }
    const uint64_t *keys = key_[src].p;
    const int64_t *vals = val_[src].p;
    uint64_t *ukey = key_[1 - src].p;
    int64_t *usum = val_[1 - src].p;
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_heads", (double)m * 12);
        tl.launch(k_heads, grid_for(m, 256), 256, 0, s_, keys, m, head_.p);
        LV_LAUNCHED("k_heads");
    }
    scan_exclusive<int32_t, int64_t>(head_.p, uid_.p, m, uid_.p + m, s_, t_);
    fill<int64_t>(usum, 0, m, s_);   // the distinct-key count (uid_[m]) is at most m
    {
        const int64_t eb = (m + kEntriesPerBlock - 1) / kEntriesPerBlock;
        TimedLaunch tl(t_, TG_CONTRACT, "k_reduce_by_key", (double)m * 44);
        tl.launch(k_reduce_by_key, (unsigned)eb, 256, 0, s_, keys, vals, head_.p, uid_.p, m, 64, nullptr, usum, ukey);
        LV_LAUNCHED("k_reduce_by_key");
    }
    *ukeys = ukey;
    *usums = usum;
    return uid_.p + m;
}

int64_t Contractor::contract(const GraphView &g, const int32_t *newlab, int64_t n_new, int64_t *rp_out,
                             int32_t *col_out, void *w_out, int wout_bytes, int64_t *delta_out, bool sorted,
                             int64_t direct_max) {
    require(wout_bytes == 4 || wout_bytes == 8, LOUVAIN_EDEVICE, "contracted weights are 4 or 8 bytes");
    if (delta_out) fill<int64_t>(delta_out, 0, n_new, s_);
    if (n_new == 0) {
        fill<int64_t>(rp_out, 0, 1, s_);
        return 0;
    }
    if (g.nnz == 0) {
        fill<int64_t>(rp_out, 0, n_new + 1, s_);
        return 0;
    }
    const int64_t n = g.n, k = n_new;
    int64_t *cnt = seg_off_.p;            // k + 1: raw counts, then (scanned) segment offsets
    int64_t *off = seg_off_.p;
    unsigned long long *cursor = (unsigned long long *)seg_cur_.p;
    fill<int64_t>(cnt, 0, k + 1, s_);
    fill<int64_t>(seg_cur_.p, 0, k, s_);
    const unsigned vb = (unsigned)((n + kSegTile - 1) / kSegTile);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_seg_count", (double)n * (delta_out ? 28 : 20));
        tl.launch(k_seg_count, vb, 256, 0, s_, g.row_ptr, newlab, n, (unsigned long long *)cnt, g.delta,
                  (unsigned long long *)delta_out);
        LV_LAUNCHED("k_seg_count");
    }
    scan_exclusive<int64_t, int64_t>(cnt, off, k, off + k, s_, t_);
    {
        TimedLaunch tl(t_, TG_CONTRACT, "k_seg_start", (double)n * 28);
        tl.launch(k_seg_start, vb, 256, 0, s_, g.row_ptr, newlab, n, off, cursor, seg_start_.p);
        LV_LAUNCHED("k_seg_start");
    }
    // unsorted contraction: pieces of the segments longer than kMidMax, and
    // the segments of kChunkSeg + 1 .. kMidMax entries
    TempBuf pieces(sorted ? 16 : (size_t)(3 * (k + 1) + 2) * sizeof(int64_t), s_);
    int64_t *poff = pieces.as<int64_t>();
    int64_t *moff = poff + (k + 1);
    int64_t *soff = moff + (k + 1);   // chunk space: the short segments' entries only
    unsigned long long *ptot = (unsigned long long *)(soff + (k + 1));
    // single-word piece tables when column + 1 and a weight sum (<= 2W) fit 64 bits together
    int pshift = 64 - bits_for(k + 1);
    if (pshift > 62 || (uint64_t)g.tw >= (1ull << pshift)) pshift = 0;
    const int64_t piece = pshift ? kPieceW : kPiece;
    if (!sorted) {
        fill<uint64_t>((uint64_t *)ptot, 0, 2, s_);
        TimedLaunch tl(t_, TG_CONTRACT, "k_big_pieces", (double)k * 32);
        const unsigned pb = grid_for(k, 256) < 2048u ? grid_for(k, 256) : 2048u;
        tl.launch(k_big_pieces, pb, 256, 0, s_, off, k, poff, moff, soff, ptot, piece);
        LV_LAUNCHED("k_big_pieces");
        scan_exclusive<int64_t, int64_t>(poff, poff, k, poff + k, s_, t_);
        scan_exclusive<int64_t, int64_t>(moff, moff, k, moff + k, s_, t_);
        scan_exclusive<int64_t, int64_t>(soff, soff, k, soff + k, s_, t_);
    }
    Readback rb(s_);
    const int64_t *mr = rb.add(off + k);
    const int64_t *npc = sorted ? nullptr : rb.add(poff + k);
    const int64_t *nmid = sorted ? nullptr : rb.add(moff + k);
    const unsigned long long *ntot = sorted ? nullptr : rb.add(ptot, 2);
    rb.issue();   // read while the scatter runs
    {
        const int64_t eb = (g.nnz + kEntriesPerBlock - 1) / kEntriesPerBlock;
        TimedLaunch tl(t_, TG_CONTRACT, "k_seg_scatter", (double)g.nnz * (4 + g.wbytes + 4 + 12) + (double)n * 12,
                       g.wbytes == 4 ? "<int>" : "<long>");
        if (g.wbytes == 4)
            tl.launch(k_seg_scatter<int32_t>, (unsigned)eb, 256, 0, s_, g.row_ptr, n, g.nnz, g.col,
                      (const int32_t *)g.w, newlab, seg_start_.p, tcol_.p, tw_.p);
        else
            tl.launch(k_seg_scatter<int64_t>, (unsigned)eb, 256, 0, s_, g.row_ptr, n, g.nnz, g.col,
                      (const int64_t *)g.w, newlab, seg_start_.p, tcol_.p, tw_.p);
        LV_LAUNCHED("k_seg_scatter");
    }
    rb.wait();
    const int64_t m_raw = *mr;
    int64_t *mcount = seg_m_.p;           // k + 1
    fill<int64_t>(mcount, 0, k + 1, s_);
    if (m_raw == 0) {
        fill<int64_t>(rp_out, 0, k + 1, s_);
        return 0;
    }
    const int bits = bits_for(k + 1);
    TempBuf pc(sizeof(unsigned long long), s_);
    fill<uint64_t>(pc.as<uint64_t>(), 0, 1, s_);
    // entries the chunks aggregate: all of them in the exported contraction,
    // else those of segments of at most kChunkSeg entries
    const int64_t m_chunks = sorted ? m_raw : m_raw - (int64_t)ntot[0] - (int64_t)ntot[1];
    if (m_chunks > 0) {
        const int64_t cb = (m_chunks + kChunk - 1) / kChunk;
        TimedLaunch tl(t_, TG_CONTRACT, sorted ? "k_seg_chunk" : "k_seg_chunk_any", (double)m_chunks * 24);
        if (sorted)
            tl.launch(k_seg_chunk, (unsigned)cb, 256, 0, s_, off, k, m_raw, tcol_.p, tw_.p, mcount, key_[0].p,
                      val_[0].p, pc.as<unsigned long long>(), bits);
        else
            tl.launch(k_seg_chunk_any, (unsigned)cb, 256, 0, s_, (const int64_t *)soff, off, k, m_chunks, tcol_.p,
                      tw_.p, mcount, key_[0].p, val_[0].p, pc.as<unsigned long long>(), bits);
        LV_LAUNCHED("k_seg_chunk");
    }
    const bool log = log_on();
    TempBuf pc_chunks(log ? sizeof(unsigned long long) : 8, s_);
    if (log)   // the pairs the chunks left to the sort
        LV_HIP(hipMemcpyAsync(pc_chunks.p, pc.p, sizeof(unsigned long long), hipMemcpyDeviceToDevice, s_));
    if (npc && *npc > 0) {
        // per entry: column and weight read, one pair (column, weight) written at most
        TimedLaunch tl(t_, TG_CONTRACT, "k_big_piece", (double)ntot[0] * 24);
        if (pshift)
            tl.launch(k_piece_word<kPieceThreads, kPieceWBits, kPieceW>, (unsigned)*npc, kPieceThreads, 0, s_, off,
                      k, (const int64_t *)poff, tcol_.p, tw_.p, mcount, key_[0].p, val_[0].p,
                      pc.as<unsigned long long>(), bits, direct_max, pshift);
        else
            tl.launch(k_big_piece<kPieceThreads, kPieceBits, kPiece>, (unsigned)*npc, kPieceThreads, 0, s_, off, k,
                      (const int64_t *)poff, tcol_.p, tw_.p, mcount, key_[0].p, val_[0].p,
                      pc.as<unsigned long long>(), bits, direct_max);
        LV_LAUNCHED("k_big_piece");
    }
    if (nmid && *nmid > 0) {
        TimedLaunch tl(t_, TG_CONTRACT, "k_mid_seg", (double)ntot[1] * 24);
        if (pshift)
            tl.launch(k_piece_word<kMidThreads, kMidBits, 4096>, (unsigned)*nmid, kMidThreads, 0, s_, off, k,
                      (const int64_t *)moff, tcol_.p, tw_.p, mcount, key_[0].p, val_[0].p,
                      pc.as<unsigned long long>(), bits, direct_max, pshift);
        else
            tl.launch(k_big_piece<kMidThreads, kMidBits, 4096>, (unsigned)*nmid, kMidThreads, 0, s_, off, k,
                      (const int64_t *)moff, tcol_.p, tw_.p, mcount, key_[0].p, val_[0].p,
                      pc.as<unsigned long long>(), bits, direct_max);
        LV_LAUNCHED("k_mid_seg");
    }
    const uint64_t *npp = rb.add(pc.as<uint64_t>());
    const uint64_t *npc0 = log ? rb.add(pc_chunks.as<uint64_t>()) : nullptr;
    rb.fetch();
    const uint64_t np = *npp;
    if (log)
        fprintf(stderr,
                "[louvain] contraction: n %lld -> %lld, entries %lld, pieces %lld (%llu entries), middle segments %lld "
                "(%llu entries), pairs merged by sorting %llu (%llu from chunks)\n",
                (long long)n, (long long)k, (long long)m_raw, (long long)(npc ? *npc : 0),
                (unsigned long long)(ntot ? ntot[0] : 0), (long long)(nmid ? *nmid : 0),
                (unsigned long long)(ntot ? ntot[1] : 0), (unsigned long long)np, (unsigned long long)*npc0);
    if (np > 0) {
        const uint64_t *ukey;
        const int64_t *usum;
        // the merged pair count stays on the device; np bounds the grid
        const int64_t *u_n = sort_sum((int64_t)np, 2 * bits, &ukey, &usum);
        TimedLaunch tl(t_, TG_CONTRACT, "k_seg_merge_write", (double)np * 28);
        tl.launch(k_seg_merge_write, grid_for((int64_t)np, 256), 256, 0, s_, ukey, usum, u_n, bits, off, tcol_.p,
                  tw_.p, mcount);
        LV_LAUNCHED("k_seg_merge_write");
    }
    scan_exclusive<int64_t, int64_t>(mcount, rp_out, k, rp_out + k, s_, t_);
    {
        // m_new <= m_raw: merging pairs only removes entries
        const int64_t eb = (m_raw + kEntriesPerBlock - 1) / kEntriesPerBlock;
        TimedLaunch tl(t_, TG_CONTRACT, "k_seg_pack", (double)m_raw * (24 + wout_bytes),
                       wout_bytes == 4 ? "<int>" : "<long>");
        if (wout_bytes == 4)
            tl.launch(k_seg_pack<int32_t>, (unsigned)eb, 256, 0, s_, rp_out, k, off, tcol_.p, tw_.p, col_out,
                      (int32_t *)w_out);
        else
            tl.launch(k_seg_pack<int64_t>, (unsigned)eb, 256, 0, s_, rp_out, k, off, tcol_.p, tw_.p, col_out,
                      (int64_t *)w_out);
        LV_LAUNCHED("k_seg_pack");
    }
    const int64_t *mn = rb.add(rp_out + k);
    rb.fetch();
    const int64_t m_new = *mn;
    return m_new;
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

size_t modularity_ws_bytes(int64_t n) {
    const int64_t nb = (n + 2047) / 2048;
    return (size_t)n * sizeof(int64_t) + (size_t)(2 * nb + 4) * sizeof(uint64_t);
}

i128 modularity_int(const GraphView &g, const int32_t *labels, hipStream_t s, Timer *t, void *ws) {
    if (g.n == 0 || g.tw == 0) return 0;
    const int64_t nb = (g.n + 2047) / 2048;
    TempBuf deg_buf, part_buf;
    int64_t *deg_p;
    uint64_t *part_p;
    if (ws) {
        // the caller's workspace: deg_C (n words), then the partial sums
        deg_p = (int64_t *)ws;
        part_p = (uint64_t *)(deg_p + g.n);
    } else {
        deg_buf = TempBuf((size_t)g.n * sizeof(int64_t), s);
        part_buf = TempBuf((size_t)(2 * nb + 4) * sizeof(uint64_t), s);
        deg_p = deg_buf.as<int64_t>();
        part_p = part_buf.as<uint64_t>();
    }
    uint64_t *acc = part_p + 2 * nb;      // I
    uint64_t *tot = acc + 2;              // sum deg^2
    fill<int64_t>(deg_p, 0, g.n, s);
    fill<uint64_t>(acc, 0, 1, s);
    TimedLaunch tl(t, TG_OTHER, "modularity", (double)g.nnz * 16 + (double)g.n * 24);
    tl.launch(k_label_degrees, grid_for(g.n, 256), 256, 0, s, labels, g.delta, g.n, deg_p);
    LV_LAUNCHED("k_label_degrees");
    if (g.nnz > 0) {
        const int64_t eb = (g.nnz + kEntriesPerBlock - 1) / kEntriesPerBlock;
        if (g.wbytes == 4)
            tl.launch(k_inner_weight<int32_t>, (unsigned)eb, 256, 0, s, g.row_ptr, g.n, g.nnz, g.col,
                      (const int32_t *)g.w, labels, (unsigned long long *)acc);
        else
            tl.launch(k_inner_weight<int64_t>, (unsigned)eb, 256, 0, s, g.row_ptr, g.n, g.nnz, g.col,
                      (const int64_t *)g.w, labels, (unsigned long long *)acc);
        LV_LAUNCHED("k_inner_weight");
    }
    tl.launch(k_sq_partials, (unsigned)nb, 256, 0, s, deg_p, g.n, part_p);
    LV_LAUNCHED("k_sq_partials");
    sum_i128_partials(part_p, nb, tot, s);
    uint64_t h[4];
    LV_HIP(hipMemcpyAsync(h, acc, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LV_HIP(hipStreamSynchronize(s));
    const i128 I = (i128)h[0];
    const i128 S = (i128)(((u128)h[3] << 64) | (u128)h[2]);
    return (i128)g.tw * I - S;
}

}  // namespace lv
