// Local-moving phase on the device (paper: Alg. 1 with eqs. 1-5 and the
// minimum-label heuristics of Section 3.1).
//
// One sweep pass over ring slot cur -> nxt:
//   k_qsum      sum_C deg_C^2 of the labelling read by the pass
//   k_sweep_*   per vertex: e_{i->C} for every neighbouring community C,
//               accumulated in an LDS hash table keyed by community label
//               (HBM tables for hubs), integer scores, argmax with the
//               minimum-label tie-break, the singlet rule, the new label,
//               and e_{i->c_i} (+ loop) summed into I for Q_int
//   k_commit    deg_C / size updates of the movers with integer atomics
//   k_finalize  Q_int = TW*I - sum deg_C^2 of the labelling read, and the
//               exact acceptance test of the previous sweep
// Every decision is integer arithmetic, so results do not depend on the
// order in which threads run.
#include "prims.hpp"
#include "sweep.hpp"

namespace lv {

struct SweepArgs {
    const int64_t *row_ptr;
    const int32_t *col;
    const void *w;
    const int32_t *c_cur;
    int32_t *c_nxt;
    const int64_t *delta;
    const int64_t *deg;
    const int32_t *size;
    int64_t tw;
    int singlet;
    PhaseState *st;
    int64_t *e_self;   // optional per-vertex e_{i->c_i} incl. loop
};

template <typename W>
__device__ __forceinline__ int64_t wload(const void *w, int64_t e) {
    return (int64_t)((const W *)w)[e];
}

// ------------------------------------------------------------ hash tables --

// Add weight w under label k in an LDS table of 2^BITS slots (open
// addressing, linear probing).  The table is never more than half full.
template <int BITS>
__device__ __forceinline__ void lds_insert(int32_t *key, unsigned long long *val, int32_t k, int64_t w) {
    constexpr uint32_t kMask = (1u << BITS) - 1;
    uint32_t h = hash_pow2(k, BITS);
    while (true) {
        int32_t cur = ((volatile int32_t *)key)[h];
        if (cur == k) {
            atomicAdd(&val[h], (unsigned long long)w);
            return;
        }
        if (cur == kEmpty) {
            int32_t prev = atomicCAS(&key[h], kEmpty, k);
            if (prev == kEmpty || prev == k) {
                atomicAdd(&val[h], (unsigned long long)w);
                return;
            }
        }
        h = (h + 1) & kMask;
    }
}

// Same in an HBM table of `size` slots.
__device__ __forceinline__ void hbm_insert(int32_t *key, unsigned long long *val, int64_t size, int32_t k,
                                           unsigned long long w) {
    uint64_t h = hash_range(k, (uint64_t)size);
    while (true) {
        int32_t prev = atomicCAS(&key[h], kEmpty, k);
        if (prev == kEmpty || prev == k) {
            atomicAdd(&val[h], w);
            return;
        }
        h = (h + 1 == (uint64_t)size) ? 0 : h + 1;
    }
}

// ------------------------------------------------------------- decisions --

// New community of vertex i given its best candidate (bs, bl) and
// e_{i->C(i)\{i}} = e_own (loops excluded): move iff the candidate's score
// beats the own community's strictly, unless both communities are
// singletons and the candidate's label is larger (singlet rule).
template <typename S>
__device__ __forceinline__ int32_t decide(const SweepArgs &a, int32_t i, int32_t ci, S bs, int32_t bl,
                                          int64_t e_own) {
    const int64_t di = a.delta[i];
    const S s_own = score_mul<S>(a.tw, e_own) - score_mul<S>(di, a.deg[ci] - di);
    if (bl >= 0 && bs > s_own) {
        if (a.singlet && a.size[ci] == 1 && a.size[bl] == 1 && bl > ci) return ci;
        return bl;
    }
    return ci;
}

// Reduction over the G lanes of a group (G <= 64, groups aligned in the wave).
template <int G, typename S>
__device__ __forceinline__ void group_reduce_wave(S &bs, int32_t &bl, int64_t &e_own, int64_t &loop) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        S os = shfl_xor_any<S>(bs, off);
        int32_t ol = __shfl_xor(bl, off);
        if (better<S>(os, ol, bs, bl)) {
            bs = os;
            bl = ol;
        }
        e_own += shfl_xor_any<int64_t>(e_own, off);
        loop += shfl_xor_any<int64_t>(loop, off);
    }
}

// Reduction over a whole 256-thread block; the result is valid in thread 0.
template <typename S>
__device__ __forceinline__ void group_reduce_block(S &bs, int32_t &bl, int64_t &e_own, int64_t &loop) {
    __shared__ S r_s[4];
    __shared__ int32_t r_l[4];
    __shared__ int64_t r_e[4], r_p[4];
    group_reduce_wave<64, S>(bs, bl, e_own, loop);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        r_s[wid] = bs;
        r_l[wid] = bl;
        r_e[wid] = e_own;
        r_p[wid] = loop;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            if (better<S>(r_s[w], r_l[w], bs, bl)) {
                bs = r_s[w];
                bl = r_l[w];
            }
            e_own += r_e[w];
            loop += r_p[w];
        }
    }
}

// ----------------------------------------------------- group sweep kernel --

// G lanes per vertex (G in {4, 16, 64}: several vertices per wavefront; G =
// 256: one workgroup per vertex).  Each group owns an LDS table of 2^BITS
// slots, at least twice the largest row of its bucket.
template <int G, int BITS, typename W, typename S>
__global__ __launch_bounds__(256) void k_sweep_group(SweepArgs a, const int32_t *__restrict__ list,
                                                     int64_t count) {
    constexpr int T = 1 << BITS;
    constexpr int NG = 256 / G;
    __shared__ int32_t s_key[NG * T];
    __shared__ unsigned long long s_val[NG * T];
    __shared__ unsigned long long s_I;
    if (a.st->done) return;
    const int tid = threadIdx.x;
    const int g = tid / G, lane = tid % G;
    int32_t *key = s_key + g * T;
    unsigned long long *val = s_val + g * T;
#pragma unroll
    for (int x = lane; x < T; x += G) {
        key[x] = kEmpty;
        val[x] = 0;
    }
    if (tid == 0) s_I = 0;
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * NG + g;
    const bool active = idx < count;
    int32_t i = 0, ci = 0;
    int64_t rs = 0, re = 0;
    if (active) {
        i = list[idx];
        rs = a.row_ptr[i];
        re = a.row_ptr[i + 1];
        ci = a.c_cur[i];
    }
    int64_t loop = 0;
    for (int64_t e = rs + lane; e < re; e += G) {
        const int32_t j = a.col[e];
        const int64_t w = wload<W>(a.w, e);
        if (j == i) {
            loop += w;
            continue;
        }
        lds_insert<BITS>(key, val, a.c_cur[j], w);
    }
    __syncthreads();
    S bs = 0;
    int32_t bl = -1;
    int64_t e_own = 0;
    if (active) {
        const int64_t di = a.delta[i];
#pragma unroll
        for (int x = lane; x < T; x += G) {
            const int32_t k = key[x];
            if (k == kEmpty) continue;
            const int64_t ev = (int64_t)val[x];
            if (k == ci) {
                e_own = ev;
                continue;
            }
            const S sc = score_mul<S>(a.tw, ev) - score_mul<S>(di, a.deg[k]);
            if (better<S>(sc, k, bs, bl)) {
                bs = sc;
                bl = k;
            }
        }
    }
    if constexpr (G <= 64)
        group_reduce_wave<G, S>(bs, bl, e_own, loop);
    else
        group_reduce_block<S>(bs, bl, e_own, loop);
    if (active && lane == 0) {
        a.c_nxt[i] = decide<S>(a, i, ci, bs, bl, e_own);
        const int64_t self = e_own + loop;
        if (a.e_self) a.e_self[i] = self;
        if (self) atomicAdd(&s_I, (unsigned long long)self);
    }
    __syncthreads();
    if (tid == 0 && s_I) atomicAdd(&a.st->acc_I, s_I);
}

// ------------------------------------------------------------- hub kernels --

// Hub metadata: 4 arrays of (hubs + 1) int64 laid out back to back.
struct HubMeta {
    const int32_t *v;        // hub vertices
    const int64_t *tab_off;  // first table slot of each hub
    const int64_t *chunk_off;// first accumulation block of each hub
    const int64_t *scan_off; // first scan block of each hub
    const int64_t *tab_size; // table slots of each hub (multiple of kHubScan, >= 2 * row length)
    int64_t hubs;
};

// Largest h in [0, hubs) with off[h] <= b.
__device__ __forceinline__ int64_t find_segment(const int64_t *off, int64_t hubs, int64_t b) {
    int64_t lo = 0, hi = hubs - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int kHubLdsBits = 11;  // 2048 slots for a chunk of kHubChunk = 1024 entries

// One workgroup per kHubChunk entries of a hub row: pre-aggregate e_{i->C}
// in LDS, then add each distinct community once into the hub's HBM table.
template <typename W>
__global__ __launch_bounds__(256) void k_hub_accum(SweepArgs a, HubMeta hm, int32_t *gkey,
                                                   unsigned long long *gval, unsigned long long *hub_loop) {
    constexpr int T = 1 << kHubLdsBits;
    __shared__ int32_t s_key[T];
    __shared__ unsigned long long s_val[T];
    __shared__ int64_t s_h;
    if (a.st->done) return;
    const int t = threadIdx.x;
    if (t == 0) s_h = find_segment(hm.chunk_off, hm.hubs, blockIdx.x);
    for (int x = t; x < T; x += 256) {
        s_key[x] = kEmpty;
        s_val[x] = 0;
    }
    __syncthreads();
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int64_t k = (int64_t)blockIdx.x - hm.chunk_off[h];
    const int64_t row_end = a.row_ptr[v + 1];
    const int64_t rs = a.row_ptr[v] + k * kHubChunk;
    const int64_t re = rs + kHubChunk < row_end ? rs + kHubChunk : row_end;
    for (int64_t e = rs + t; e < re; e += 256) {
        const int32_t j = a.col[e];
        const int64_t w = wload<W>(a.w, e);
        if (j == v) {
            atomicAdd(&hub_loop[h], (unsigned long long)w);
            continue;
        }
        lds_insert<kHubLdsBits>(s_key, s_val, a.c_cur[j], w);
    }
    __syncthreads();
    const int64_t base = hm.tab_off[h], size = hm.tab_size[h];
    for (int x = t; x < T; x += 256) {
        const int32_t key = s_key[x];
        if (key != kEmpty) hbm_insert(gkey + base, gval + base, size, key, s_val[x]);
    }
}

// One workgroup per kHubScan slots of a hub table: best candidate and own
// e over its slots (partial), clearing the slots for the next pass.
template <typename S>
__global__ __launch_bounds__(256) void k_hub_scan(SweepArgs a, HubMeta hm, int32_t *gkey,
                                                  unsigned long long *gval, uint64_t *part) {
    __shared__ int64_t s_h;
    if (a.st->done) return;
    const int t = threadIdx.x;
    if (t == 0) s_h = find_segment(hm.scan_off, hm.hubs, blockIdx.x);
    __syncthreads();
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int32_t ci = a.c_cur[v];
    const int64_t di = a.delta[v];
    const int64_t base = hm.tab_off[h] + ((int64_t)blockIdx.x - hm.scan_off[h]) * kHubScan;
    S bs = 0;
    int32_t bl = -1;
    int64_t e_own = 0, unused = 0;
#pragma unroll
    for (int q = 0; q < kHubScan / 256; ++q) {
        const int64_t x = base + q * 256 + t;
        const int32_t k = gkey[x];
        if (k == kEmpty) continue;
        const int64_t ev = (int64_t)gval[x];
        gkey[x] = kEmpty;
        gval[x] = 0;
        if (k == ci) {
            e_own += ev;
            continue;
        }
        const S sc = score_mul<S>(a.tw, ev) - score_mul<S>(di, a.deg[k]);
        if (better<S>(sc, k, bs, bl)) {
            bs = sc;
            bl = k;
        }
    }
    group_reduce_block<S>(bs, bl, e_own, unused);
    if (t == 0) {
        i128 w = (i128)bs;
        uint64_t *p = part + 4 * (int64_t)blockIdx.x;
        p[0] = (uint64_t)w;
        p[1] = (uint64_t)(int64_t)(w >> 64);
        p[2] = (uint64_t)(int64_t)bl;
        p[3] = (uint64_t)e_own;
    }
}

// One wavefront per hub: combine the scan partials and decide.
template <typename S>
__global__ __launch_bounds__(256) void k_hub_decide(SweepArgs a, HubMeta hm, const uint64_t *part,
                                                    unsigned long long *hub_loop) {
    if (a.st->done) return;
    const int lane = threadIdx.x & 63;
    const int64_t h = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (h >= hm.hubs) return;
    S bs = 0;
    int32_t bl = -1;
    int64_t e_own = 0, unused = 0;
    for (int64_t b = hm.scan_off[h] + lane; b < hm.scan_off[h + 1]; b += 64) {
        const uint64_t *p = part + 4 * b;
        const int32_t l = (int32_t)(int64_t)p[2];
        const S sc = (S)make_i128(p[0], (int64_t)p[1]);
        if (better<S>(sc, l, bs, bl)) {
            bs = sc;
            bl = l;
        }
        e_own += (int64_t)p[3];
    }
    group_reduce_wave<64, S>(bs, bl, e_own, unused);
    if (lane == 0) {
        const int32_t v = hm.v[h];
        const int32_t ci = a.c_cur[v];
        a.c_nxt[v] = decide<S>(a, v, ci, bs, bl, e_own);
        const int64_t self = e_own + (int64_t)hub_loop[h];
        hub_loop[h] = 0;
        if (a.e_self) a.e_self[v] = self;
        if (self) atomicAdd(&a.st->acc_I, (unsigned long long)self);
    }
}

// --------------------------------------------------- commit, Q, acceptance --

// Community degrees and sizes follow the movers (integer atomics, so the
// result does not depend on their order).
__global__ __launch_bounds__(256) void k_commit(const int32_t *__restrict__ c_cur, const int32_t *__restrict__ c_nxt,
                                                const int64_t *__restrict__ delta, int64_t *deg, int32_t *size,
                                                int64_t n, PhaseState *st) {
    __shared__ unsigned long long s_m;
    if (st->done) return;
    if (threadIdx.x == 0) s_m = 0;
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n) {
        const int32_t a = c_cur[v], b = c_nxt[v];
        if (a != b) {
            const int64_t d = delta[v];
            atomicAdd((unsigned long long *)&deg[b], (unsigned long long)d);
            atomicAdd((unsigned long long *)&deg[a], (unsigned long long)(-d));
            atomicAdd(&size[b], 1);
            atomicAdd(&size[a], -1);
            atomicAdd(&s_m, 1ull);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_m) atomicAdd(&st->moved, s_m);
}

constexpr int kQsumTile = 2048;

// Per-block partial sums of deg_C^2 (128-bit).
__global__ __launch_bounds__(256) void k_qsum(const int64_t *__restrict__ deg, int64_t n, uint64_t *part,
                                              const PhaseState *st) {
    __shared__ uint64_t slo[4];
    __shared__ int64_t shi[4];
    if (st->done) return;
    i128 s = 0;
    const int64_t base = (int64_t)blockIdx.x * kQsumTile;
#pragma unroll
    for (int k = 0; k < kQsumTile / 256; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v < n) {
            const int64_t d = deg[v];
            s += mul_wide(d, d);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += shfl_xor_any<i128>(s, off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        slo[wid] = (uint64_t)s;
        shi[wid] = (int64_t)(s >> 64);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        i128 t = 0;
        for (int w = 0; w < 4; ++w) t += make_i128(slo[w], shi[w]);
        part[2 * blockIdx.x] = (uint64_t)t;
        part[2 * blockIdx.x + 1] = (uint64_t)(int64_t)(t >> 64);
    }
}

// 128 x 64 -> 192-bit unsigned product as (hi, lo).
__device__ __forceinline__ void mul_u128_u64(u128 a, uint64_t b, uint64_t &hi, u128 &lo) {
    const u128 p0 = (u128)(uint64_t)a * b;
    const u128 p1 = (u128)(uint64_t)(a >> 64) * b;
    const u128 l = p0 + (p1 << 64);
    hi = (uint64_t)(p1 >> 64) + (l < p0 ? 1 : 0);
    lo = l;
}

// theta_den * (qn - qp) > theta_num * |qp|, exactly.
__device__ __forceinline__ bool relative_gain_passes(i128 qn, i128 qp, int64_t num, int64_t den) {
    if (qn <= qp) return false;
    const u128 gain = (u128)(qn - qp);
    const u128 mag = (u128)(qp < 0 ? -qp : qp);
    uint64_t lh, rh;
    u128 ll, rl;
    mul_u128_u64(gain, (uint64_t)den, lh, ll);
    mul_u128_u64(mag, (uint64_t)num, rh, rl);
    return lh > rh || (lh == rh && ll > rl);
}

// Q_int of the labelling the pass read (slot p-1) and the acceptance test of
// sweep p-1 against the last kept labelling.
__global__ __launch_bounds__(256) void k_finalize(PhaseState *st, const uint64_t *__restrict__ part,
                                                  int64_t nparts, int64_t tw, int64_t theta_num,
                                                  int64_t theta_den, int32_t max_sweeps, int32_t p) {
    __shared__ uint64_t slo[256];
    __shared__ int64_t shi[256];
    if (st->done) return;
    i128 s = 0;
    for (int64_t b = threadIdx.x; b < nparts; b += 256) s += make_i128(part[2 * b], (int64_t)part[2 * b + 1]);
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
    if (threadIdx.x != 0) return;
    const i128 S = make_i128(slo[0], shi[0]);
    const i128 q = mul_wide(tw, (int64_t)st->acc_I) - S;
    st->pass = p;
    st->q_last[0] = (uint64_t)q;
    st->q_last[1] = (uint64_t)(int64_t)(q >> 64);
    const i128 qref = make_i128(st->q_ref[0], (int64_t)st->q_ref[1]);
    bool keep = true;
    if (p == 1) {
        st->q_ref[0] = (uint64_t)q;
        st->q_ref[1] = (uint64_t)(int64_t)(q >> 64);
    } else if (relative_gain_passes(q, qref, theta_num, theta_den)) {
        st->q_ref[0] = (uint64_t)q;
        st->q_ref[1] = (uint64_t)(int64_t)(q >> 64);
        st->accepted += 1;
    } else {
        keep = false;
        st->done = 1;
        st->final_slot = (p - 2) % 3;
    }
    if (keep) {
        if (st->accepted >= max_sweeps) {
            st->done = 1;
            st->limit = 1;
            st->final_slot = (p - 1) % 3;
        } else if (st->moved == 0) {
            st->done = 1;   // the next sweep cannot change Q, so it would be discarded
            st->final_slot = (p - 1) % 3;
        }
    }
    st->acc_I = 0;
    st->moved = 0;
}

// ------------------------------------------------------------ level set-up --

__global__ void k_init_singletons(int32_t *c0, int32_t *c1, int32_t *c2, const int64_t *__restrict__ delta,
                                  int64_t *deg, int32_t *size, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    c0[v] = c1[v] = c2[v] = (int32_t)v;
    deg[v] = delta[v];
    size[v] = 1;
}

__global__ void k_init_labels(int32_t *c0, int32_t *c1, int32_t *c2, const int32_t *__restrict__ labels,
                              const int64_t *__restrict__ delta, int64_t *deg, int32_t *size, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = labels[v];
    c0[v] = c1[v] = c2[v] = l;
    atomicAdd((unsigned long long *)&deg[l], (unsigned long long)delta[v]);
    atomicAdd(&size[l], 1);
}

// ---------------------------------------------------------------- bucketing --

constexpr int kBucketTile = 2048;  // vertices per bucketing block (256 x 8)

__device__ __forceinline__ int bucket_of(int64_t d) {
    if (d <= 0) return -1;
#pragma unroll
    for (int b = 0; b < NBUCKET - 1; ++b)
        if (d <= kBucketMax[b]) return b;
    return B_HUB;
}

__global__ __launch_bounds__(256) void k_bucket_count(const int64_t *__restrict__ rp, int64_t n, int32_t *counts,
                                                      int64_t nblocks, unsigned long long *bucket_nnz) {
    __shared__ int cnt[NBUCKET];
    __shared__ unsigned long long ecnt[NBUCKET];
    if (threadIdx.x < NBUCKET) {
        cnt[threadIdx.x] = 0;
        ecnt[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBucketTile;
#pragma unroll
    for (int k = 0; k < kBucketTile / 256; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v < n) {
            const int64_t d = rp[v + 1] - rp[v];
            const int b = bucket_of(d);
            if (b >= 0) {
                atomicAdd(&cnt[b], 1);
                atomicAdd(&ecnt[b], (unsigned long long)d);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < NBUCKET) {
        counts[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
        if (ecnt[threadIdx.x]) atomicAdd(&bucket_nnz[threadIdx.x], ecnt[threadIdx.x]);
    }
}

// Stable scatter of the vertices into their bucket lists (ascending order
// inside each bucket).
__global__ __launch_bounds__(256) void k_bucket_scatter(const int64_t *__restrict__ rp, int64_t n,
                                                        const int32_t *__restrict__ offs, int64_t nblocks,
                                                        int32_t *list) {
    __shared__ int run[NBUCKET];
    __shared__ int wc[4][NBUCKET];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t < NBUCKET) run[t] = offs[t * nblocks + blockIdx.x];
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kBucketTile;
    for (int k = 0; k < kBucketTile / 256; ++k) {
        const int64_t v = base + k * 256 + t;
        const int b = v < n ? bucket_of(rp[v + 1] - rp[v]) : -1;
        int rank = 0;
#pragma unroll
        for (int bb = 0; bb < NBUCKET; ++bb) {
            const unsigned long long m = __ballot(b == bb);
            if (b == bb) rank = __popcll(m & lt);
            if (lane == 0) wc[wid][bb] = __popcll(m);
        }
        __syncthreads();
        if (b >= 0) {
            int pos = run[b] + rank;
            for (int w = 0; w < wid; ++w) pos += wc[w][b];
            list[pos] = (int32_t)v;
        }
        __syncthreads();
        if (t < NBUCKET) run[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        __syncthreads();
    }
}

__global__ void k_hub_sizes(const int64_t *__restrict__ rp, const int32_t *__restrict__ hubv, int64_t hubs,
                            int64_t *tab_off, int64_t *chunk_off, int64_t *scan_off, int64_t *tab_size) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= hubs) return;
    const int32_t v = hubv[h];
    const int64_t d = rp[v + 1] - rp[v];
    const int64_t T = (2 * d + kHubScan - 1) / kHubScan * kHubScan;
    tab_size[h] = T;
    tab_off[h] = T;
    chunk_off[h] = (d + kHubChunk - 1) / kHubChunk;
    scan_off[h] = T / kHubScan;
}

// ------------------------------------------------------------------- host --

void Sweeper::reserve(int64_t n, int64_t nnz) {
    if (n <= cap_n_ && nnz <= cap_nnz_) return;
    for (auto &c : c_) c.alloc((size_t)n);
    deg_.alloc((size_t)n);
    size_.alloc((size_t)n);
    list_.alloc((size_t)n);
    const int64_t nblk = (n + kBucketTile - 1) / kBucketTile;
    bcount_.alloc((size_t)(NBUCKET * nblk + 1));
    st_.alloc(1);
    qpart_.alloc((size_t)(2 * ((n + kQsumTile - 1) / kQsumTile) + 2));
    const int64_t max_hubs = nnz / (kBucketMax[NBUCKET - 2] + 1) + 1;
    hub_meta_.alloc((size_t)(4 * (max_hubs + 1)));
    hub_loop_.alloc((size_t)max_hubs);
    cap_n_ = n;
    cap_nnz_ = nnz;
}

void Sweeper::plan(const GraphView &g) {
    n_ = g.n;
    const int64_t nblk = (g.n + kBucketTile - 1) / kBucketTile;
    for (int b = 0; b <= NBUCKET; ++b) bstart_[b] = 0;
    hubs_ = hub_chunks_ = hub_scans_ = hub_slots_ = 0;
    qblocks_ = (g.n + kQsumTile - 1) / kQsumTile;
    if (g.n == 0) return;
    TempBuf bnnz(NBUCKET * sizeof(unsigned long long), s_);
    LV_HIP(hipMemsetAsync(bnnz.p, 0, NBUCKET * sizeof(unsigned long long), s_));
    int32_t *counts = bcount_.p;
    {
        TimedLaunch tl(t_, TG_LEVEL, "k_bucket_count", (double)g.n * 16);
        k_bucket_count<<<(unsigned)nblk, 256, 0, s_>>>(g.row_ptr, g.n, counts, nblk, bnnz.as<unsigned long long>());
        LV_LAUNCHED("k_bucket_count");
    }
    const int64_t m = NBUCKET * nblk;
    scan_exclusive<int32_t, int32_t>(counts, counts, m, counts + m, s_, t_);
    {
        TimedLaunch tl(t_, TG_LEVEL, "k_bucket_scatter", (double)g.n * 20);
        k_bucket_scatter<<<(unsigned)nblk, 256, 0, s_>>>(g.row_ptr, g.n, counts, nblk, list_.p);
        LV_LAUNCHED("k_bucket_scatter");
    }
    int32_t hs[NBUCKET + 1];
    for (int b = 0; b < NBUCKET; ++b)
        LV_HIP(hipMemcpyAsync(&hs[b], counts + (int64_t)b * nblk, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
    LV_HIP(hipMemcpyAsync(&hs[NBUCKET], counts + m, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
    unsigned long long hn[NBUCKET];
    LV_HIP(hipMemcpyAsync(hn, bnnz.p, sizeof hn, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));
    for (int b = 0; b <= NBUCKET; ++b) bstart_[b] = hs[b];
    for (int b = 0; b < NBUCKET; ++b) bucket_nnz_[b] = (int64_t)hn[b];
    hubs_ = bucket_count(B_HUB);
    if (hubs_ == 0) return;
    int64_t *tab_off = hub_meta_.p, *chunk_off = tab_off + (hubs_ + 1), *scan_off = chunk_off + (hubs_ + 1),
            *tab_size = scan_off + (hubs_ + 1);
    const int32_t *hubv = list_.p + bstart_[B_HUB];
    k_hub_sizes<<<grid_for(hubs_, 256), 256, 0, s_>>>(g.row_ptr, hubv, hubs_, tab_off, chunk_off, scan_off, tab_size);
    LV_LAUNCHED("k_hub_sizes");
    scan_exclusive<int64_t, int64_t>(tab_off, tab_off, hubs_, tab_off + hubs_, s_, t_);
    scan_exclusive<int64_t, int64_t>(chunk_off, chunk_off, hubs_, chunk_off + hubs_, s_, t_);
    scan_exclusive<int64_t, int64_t>(scan_off, scan_off, hubs_, scan_off + hubs_, s_, t_);
    int64_t tot[3];
    LV_HIP(hipMemcpyAsync(&tot[0], tab_off + hubs_, 8, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipMemcpyAsync(&tot[1], chunk_off + hubs_, 8, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipMemcpyAsync(&tot[2], scan_off + hubs_, 8, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));
    hub_slots_ = tot[0];
    hub_chunks_ = tot[1];
    hub_scans_ = tot[2];
    if (hub_slots_ > hub_slot_cap_) {
        hub_key_.alloc((size_t)hub_slots_);
        hub_val_.alloc((size_t)hub_slots_);
        hub_slot_cap_ = hub_slots_;
    }
    hub_part_.reserve((size_t)(4 * hub_scans_));
    fill<int32_t>(hub_key_.p, kEmpty, hub_slots_, s_);
    fill<uint64_t>((uint64_t *)hub_val_.p, 0, hub_slots_, s_);
    fill<uint64_t>((uint64_t *)hub_loop_.p, 0, hubs_, s_);
}

void Sweeper::init_singletons(const GraphView &g) {
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_LEVEL, "k_init_singletons", (double)g.n * 28);
        k_init_singletons<<<grid_for(g.n, 256), 256, 0, s_>>>(c_[0].p, c_[1].p, c_[2].p, g.delta, deg_.p, size_.p, g.n);
        LV_LAUNCHED("k_init_singletons");
    }
    LV_HIP(hipMemsetAsync(st_.p, 0, sizeof(PhaseState), s_));
}

void Sweeper::init_from_labels(const GraphView &g, const int32_t *labels) {
    fill<int64_t>(deg_.p, 0, g.n, s_);
    fill<int32_t>(size_.p, 0, g.n, s_);
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_LEVEL, "k_init_labels", (double)g.n * 28);
        k_init_labels<<<grid_for(g.n, 256), 256, 0, s_>>>(c_[0].p, c_[1].p, c_[2].p, labels, g.delta, deg_.p, size_.p, g.n);
        LV_LAUNCHED("k_init_labels");
    }
    LV_HIP(hipMemsetAsync(st_.p, 0, sizeof(PhaseState), s_));
}

template <typename W, typename S>
static void launch_pass(const SweepArgs &a, const int32_t *list, const int64_t *bstart,
                        const int64_t *bnnz, HubMeta hm, int64_t hub_chunks, int64_t hub_scans, int32_t *hkey,
                        unsigned long long *hval, unsigned long long *hloop, uint64_t *hpart, hipStream_t s,
                        Timer *t) {
    const std::string sfx = t ? std::string(type_name<W>()) + "," + type_name<S>() + ">" : std::string();
    const std::string wsfx = t ? std::string(type_name<W>()) + ">" : std::string();
    const std::string ssfx = t ? std::string(type_name<S>()) + ">" : std::string();
    const double eb = 8.0 + sizeof(W);   // col + weight + label gather per entry
    const double vb = 40.0;              // per evaluated vertex
    auto cnt = [&](int b) { return bstart[b + 1] - bstart[b]; };
    auto bytes = [&](int b) { return (double)cnt(b) * vb + (double)bnnz[b] * eb; };
    if (cnt(B_G4) > 0) {
        TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<4,4,", bytes(B_G4), sfx.c_str());
        k_sweep_group<4, 4, W, S><<<grid_for(cnt(B_G4), 64), 256, 0, s>>>(a, list + bstart[B_G4], cnt(B_G4));
        LV_LAUNCHED("k_sweep_group<4>");
    }
    if (cnt(B_G16) > 0) {
        TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<16,6,", bytes(B_G16), sfx.c_str());
        k_sweep_group<16, 6, W, S><<<grid_for(cnt(B_G16), 16), 256, 0, s>>>(a, list + bstart[B_G16], cnt(B_G16));
        LV_LAUNCHED("k_sweep_group<16>");
    }
    if (cnt(B_G64) > 0) {
        TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<64,8,", bytes(B_G64), sfx.c_str());
        k_sweep_group<64, 8, W, S><<<grid_for(cnt(B_G64), 4), 256, 0, s>>>(a, list + bstart[B_G64], cnt(B_G64));
        LV_LAUNCHED("k_sweep_group<64>");
    }
    if (cnt(B_BLOCK) > 0) {
        TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<256,11,", bytes(B_BLOCK), sfx.c_str());
        k_sweep_group<256, 11, W, S><<<(unsigned)cnt(B_BLOCK), 256, 0, s>>>(a, list + bstart[B_BLOCK], cnt(B_BLOCK));
        LV_LAUNCHED("k_sweep_group<256>");
    }
    if (hm.hubs > 0) {
        {
            TimedLaunch tl(t, TG_SWEEP, "k_hub_accum<", (double)bnnz[B_HUB] * eb, wsfx.c_str());
            k_hub_accum<W><<<(unsigned)hub_chunks, 256, 0, s>>>(a, hm, hkey, hval, hloop);
            LV_LAUNCHED("k_hub_accum");
        }
        {
            TimedLaunch tl(t, TG_SWEEP, "k_hub_scan<", (double)hub_scans * kHubScan * 24.0, ssfx.c_str());
            k_hub_scan<S><<<(unsigned)hub_scans, 256, 0, s>>>(a, hm, hkey, hval, hpart);
            LV_LAUNCHED("k_hub_scan");
        }
        {
            TimedLaunch tl(t, TG_SWEEP, "k_hub_decide<", (double)hm.hubs * vb + (double)hub_scans * 32.0, ssfx.c_str());
            k_hub_decide<S><<<grid_for(hm.hubs, 4), 256, 0, s>>>(a, hm, hpart, hloop);
            LV_LAUNCHED("k_hub_decide");
        }
    }
}

void Sweeper::pass(const GraphView &g, int p, const SweepParams &prm, int64_t *e_self_out) {
    const int cur = (p - 1) % 3, nxt = p % 3;
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_SWEEP, "k_qsum", (double)g.n * 8);
        k_qsum<<<(unsigned)qblocks_, 256, 0, s_>>>(deg_.p, g.n, qpart_.p, st_.p);
        LV_LAUNCHED("k_qsum");
    }
    SweepArgs a{g.row_ptr, g.col, g.w, c_[cur].p, c_[nxt].p, g.delta, deg_.p, size_.p,
                g.tw, prm.singlet, st_.p, e_self_out};
    int64_t *tab_off = hub_meta_.p;
    HubMeta hm{list_.p + bstart_[B_HUB], tab_off, tab_off + (hubs_ + 1), tab_off + 2 * (hubs_ + 1),
               tab_off + 3 * (hubs_ + 1), hubs_};
    const bool fast = g.tw <= kTwFastMax;
    if (g.wbytes == 4) {
        if (fast)
            launch_pass<int32_t, int64_t>(a, list_.p, bstart_, bucket_nnz_, hm, hub_chunks_, hub_scans_,
                                          hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_);
        else
            launch_pass<int32_t, i128>(a, list_.p, bstart_, bucket_nnz_, hm, hub_chunks_, hub_scans_,
                                       hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_);
    } else {
        if (fast)
            launch_pass<int64_t, int64_t>(a, list_.p, bstart_, bucket_nnz_, hm, hub_chunks_, hub_scans_,
                                          hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_);
        else
            launch_pass<int64_t, i128>(a, list_.p, bstart_, bucket_nnz_, hm, hub_chunks_, hub_scans_,
                                       hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_);
    }
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_SWEEP, "k_commit", (double)g.n * 8);
        k_commit<<<grid_for(g.n, 256), 256, 0, s_>>>(c_[cur].p, c_[nxt].p, g.delta, deg_.p, size_.p, g.n, st_.p);
        LV_LAUNCHED("k_commit");
    }
    {
        TimedLaunch tl(t_, TG_SWEEP, "k_finalize", 0.0);
        k_finalize<<<1, 256, 0, s_>>>(st_.p, qpart_.p, qblocks_, g.tw, prm.theta_num, prm.theta_den,
                                      prm.max_sweeps, p);
        LV_LAUNCHED("k_finalize");
    }
}

PhaseState Sweeper::read_state() {
    PhaseState h;
    LV_HIP(hipMemcpyAsync(&h, st_.p, sizeof h, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));
    return h;
}

}  // namespace lv
