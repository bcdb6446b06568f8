// Local-moving phase on the device (paper: Alg. 1 with eqs. 1-5 and the
// minimum-label heuristics of Section 3.1).
//
// One sweep pass over label ring slot cur -> nxt and degree state p-1 -> p:
//   k_qsum      sum_C deg_C^2 of the labelling read by the pass
//   k_sweep_*   per vertex: e_{i->C} for every neighbouring community C,
//               integer scores, argmax with the minimum-label tie-break, the
//               singlet rule, the new label, and e_{i->c_i} (+ loop) summed
//               into I for Q_int.  Rows of <= 8 entries: one thread per
//               vertex in registers; <= 512: packed workgroups with LDS hash
//               tables; <= 1024: one workgroup per vertex; longer rows: LDS
//               pre-aggregation into HBM hash tables.
//   k_commit    deg_C / size updates of the movers with integer atomics
//   k_finalize  Q_int = TW*I - sum deg_C^2 of the labelling read, and the
//               exact acceptance test of the previous sweep
// Every decision is integer arithmetic, so results do not depend on the
// order in which threads run.
#include <type_traits>

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
    const int64_t *deg;        // deg_C of the labelling read (read-only in the pass)
    const int32_t *size;
    int64_t tw;
    int singlet;
    PhaseState *st;
    int64_t *e_self;   // optional per-vertex e_{i->c_i} incl. loop
    int hub_shift;     // > 0: hub tables hold one word (label + 1) << hub_shift | e per slot
    int first;         // the labelling read is the singletons: score entries directly, no tables
    // Published words of the labelling read, one per vertex (nullptr: read
    // c_cur and deg): label c_j in the low pw_bits bits, deg of c_j in bits
    // pw_bits .. 62, bit 63 set iff c_j is a singleton.  Written at the start
    // of each pass when pw_bits + the bits of TW fit 63.
    const uint64_t *pw;
    int pw_bits;
    // the pass's sums (I, then the mover count) spread over kAccSlots
    // counters a 128-byte line apart: the kernels' thousands of workgroups
    // would otherwise queue their atomics on one address
    unsigned long long *acc;
};

__device__ __forceinline__ void acc_add(unsigned long long *acc, uint64_t slot, int field, unsigned long long x) {
    atomicAdd(&acc[(slot & (kAccSlots - 1)) * kAccStride + field], x);
}

__device__ __forceinline__ int32_t pw_label(uint64_t w, int bits) { return (int32_t)(w & ((1ull << bits) - 1)); }
__device__ __forceinline__ int64_t pw_deg(uint64_t w, int bits) { return (int64_t)((w << 1) >> (bits + 1)); }

// Community of neighbour j (and, with published words, its degree).
__device__ __forceinline__ int32_t nb_label(const SweepArgs &a, int32_t j, int64_t *deg) {
    if (a.pw) {
        const uint64_t w = a.pw[j];
        *deg = pw_deg(w, a.pw_bits);
        return pw_label(w, a.pw_bits);
    }
    *deg = -1;
    return a.c_cur[j];
}

template <typename W>
__device__ __forceinline__ int64_t wload(const void *w, int64_t e) {
    return (int64_t)((const W *)w)[e];
}

// ------------------------------------------------------------ hash tables --

// Add weight w under label k in an LDS table of 2^BITS slots (open
// addressing, linear probing).  The table is never more than half full.
template <int BITS>
__device__ __forceinline__ int lds_insert(int32_t *key, unsigned long long *val, int32_t k, int64_t w) {
    constexpr uint32_t kMask = (1u << BITS) - 1;
    uint32_t h = hash_pow2(k, BITS);
    while (true) {
        const int32_t prev = atomicCAS(&key[h], kEmpty, k);   // claims, or returns the slot's key
        if (prev == kEmpty || prev == k) {
            atomicAdd(&val[h], (unsigned long long)w);
            return (int)h;
        }
        h = (h + 1) & kMask;
    }
}

// Tables keyed by the neighbour's whole published word (label, deg_C and
// singleton flag, all functions of the label within a pass), so scoring
// reads deg_C from the key instead of gathering it.  No inserted word is
// all ones: that would be a singleton community holding all of 2W (deg_C
// needs every bit above the label, and the publish condition keeps 2W below
// that), whose only vertex is then nobody's neighbour but its own.
constexpr unsigned long long kEmptyWord = ~0ull;

template <int BITS>
__device__ __forceinline__ void lds_insert_word(unsigned long long *key, unsigned long long *val, uint64_t word,
                                                int32_t k, int64_t w) {
    constexpr uint32_t kMask = (1u << BITS) - 1;
    uint32_t h = hash_pow2(k, BITS);
    while (true) {
        const unsigned long long prev = atomicCAS(&key[h], kEmptyWord, (unsigned long long)word);
        if (prev == kEmptyWord || prev == word) {
            atomicAdd(&val[h], (unsigned long long)w);
            return;
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

// Insert or add x for a label into an HBM hub table of one word per slot,
// (label + 1) << shift | e, 0 = empty: used when every label + 1 fits the
// 64 - shift high bits and every e (at most 2W) the low shift bits, so the
// add never carries into the label.  The compare-and-swap comes first: on
// these levels nearly every label a hub's chunk inserts is new to the table
// (R-MAT scale 24, level 0: 98% of a hub row's neighbour labels are
// distinct), so a claim costs one memory-side atomic and no line fetch.
__device__ __forceinline__ void packed_insert(unsigned long long *tab, uint64_t size, int32_t label,
                                              unsigned long long x, int shift) {
    const unsigned long long tag = (unsigned long long)(uint32_t)(label + 1) << shift;
    const unsigned long long tmask = ~0ull << shift;
    uint64_t h = hash_range(label, size);
    while (true) {
        const unsigned long long prev = atomicCAS(&tab[h], 0ull, tag | x);
        if (prev == 0) return;
        if ((prev & tmask) == tag) {
            atomicAdd(&tab[h], x);
            return;
        }
        h = (h + 1 == size) ? 0 : h + 1;
    }
}

// Low bits of a single-word table slot, (label + 1) << shift | e, for a
// level of n vertices and total weight tw: label + 1 <= n needs the high
// 64 - shift bits and every e (at most tw) the low ones; 0 if they do not
// fit together.
static int word_shift(int64_t n, int64_t tw) {
    int tag_bits = 1;
    while (tag_bits < 32 && ((int64_t)1 << tag_bits) <= n) ++tag_bits;
    const int shift = 64 - tag_bits;
    return (shift < 63 && (uint64_t)tw < (1ull << shift)) ? shift : 0;
}

// LOUVAIN_HUB_BUCKET_SHRINK=s (1..4096, read once per process): hub bucket
// regions and tables s times smaller, so that tests reach the spills to the
// hub tables on small graphs.  Results do not depend on it.
static int hub_bucket_shrink() {
    static const int v = [] {
        const char *e = getenv("LOUVAIN_HUB_BUCKET_SHRINK");
        const int x = e ? atoi(e) : 1;
        return x >= 1 && x <= 4096 ? x : 1;
    }();
    return v;
}

// Label bits of the published words of a level of n vertices.
static int pw_label_bits(int64_t n) {
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
    return bits;
}

// Published words (label, deg_C, singleton flag) on levels with 128-bit
// scores, when the label bits and the bits of TW fit 63 together.
static bool publishes(const GraphView &g) {
    return g.tw > kTwFastMax && g.n > 0 &&
           pw_label_bits(g.n) + 64 - __builtin_clzll((unsigned long long)g.tw) <= 63;
}

int64_t lds_row_max(int64_t n, int64_t tw, const Tuning &tn) {
    if (tw < kCompactTwMax) return tn.block_max;
    return word_shift(n, tw) ? kBucketMax[B_WIDE] : kBucketMax[B_BLOCK];
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
// slots, at least twice the largest row of its bucket.  KW (levels with
// published words): slots are keyed by the neighbour's published word.
template <int G, int BITS, typename W, typename S, bool KW = false>
__global__ __launch_bounds__(256) void k_sweep_group(SweepArgs a, const int32_t *__restrict__ list,
                                                     int64_t count) {
    constexpr int T = 1 << BITS;
    constexpr int NG = 256 / G;
    using K = typename std::conditional<KW, unsigned long long, int32_t>::type;
    constexpr K kNone = KW ? (K)kEmptyWord : (K)kEmpty;
    __shared__ K s_key[NG * T];
    __shared__ unsigned long long s_val[NG * T];
    // candidates' deg_C beside their e in LDS (with published words), for
    // the small tables only: the larger ones key their slots by the whole
    // published word instead (8 bytes per slot more, not 12)
    constexpr bool DEG_LDS = !KW && NG * T <= 1024;
    __shared__ int64_t s_deg[DEG_LDS ? NG * T : 1];
    __shared__ unsigned long long s_I;
    if (a.st->done) return;
    const int tid = threadIdx.x;
    const int g = tid / G, lane = tid % G;
    K *key = s_key + g * T;
    unsigned long long *val = s_val + g * T;
    int64_t *tdeg = s_deg + (DEG_LDS ? g * T : 0);
    if (!a.first) {   // the first pass from singletons uses no table
#pragma unroll
        for (int x = lane; x < T; x += G) {
            key[x] = kNone;
            val[x] = 0;
        }
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
    S bs = 0;
    int32_t bl = -1;
    const int64_t di = active ? a.delta[i] : 0;
    // entries in rounds of U per lane: a round's loads and label gathers are
    // all issued before its inserts (from singletons: scored directly)
    constexpr int U = 4;
    for (int64_t e0 = rs + lane; e0 < re; e0 += (int64_t)U * G) {
        int32_t jq[U], lq[U];
        int64_t wq[U], dq[U];
        uint64_t uq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t e = e0 + (int64_t)q * G;
            jq[q] = -1;
            wq[q] = 0;
            if (e < re) {
                jq[q] = a.col[e];
                wq[q] = wload<W>(a.w, e);
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            lq[q] = -1;
            dq[q] = -1;
            uq[q] = 0;
            if (jq[q] >= 0 && jq[q] != i) {
                if constexpr (KW) {
                    uq[q] = a.pw[jq[q]];
                    lq[q] = pw_label(uq[q], a.pw_bits);
                    dq[q] = pw_deg(uq[q], a.pw_bits);
                } else {
                    lq[q] = nb_label(a, jq[q], &dq[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (jq[q] == i) loop += wq[q];
            if (lq[q] < 0) continue;
            if (a.first) {   // every neighbour is its own community
                const int64_t dg = dq[q] >= 0 ? dq[q] : a.deg[lq[q]];
                const S sc = score_mul<S>(a.tw, wq[q]) - score_mul<S>(di, dg);
                if (better<S>(sc, lq[q], bs, bl)) {
                    bs = sc;
                    bl = lq[q];
                }
            } else if constexpr (KW) {
                lds_insert_word<BITS>(key, val, uq[q], lq[q], wq[q]);
            } else {
                const int h = lds_insert<BITS>((int32_t *)key, val, lq[q], wq[q]);
                if (DEG_LDS && a.pw) tdeg[h] = dq[q];   // every inserter of a label writes the same degree
            }
        }
    }
    __syncthreads();
    int64_t e_own = 0;
    if (active && !a.first) {
#pragma unroll
        for (int x = lane; x < T; x += G) {
            const K kx = key[x];
            if (kx == kNone) continue;
            const int32_t k = KW ? pw_label((uint64_t)kx, a.pw_bits) : (int32_t)kx;
            const int64_t ev = (int64_t)val[x];
            if (k == ci) {
                e_own = ev;
                continue;
            }
            const int64_t dk = KW ? pw_deg((uint64_t)kx, a.pw_bits) : DEG_LDS && a.pw ? tdeg[x] : a.deg[k];
            const S sc = score_mul<S>(a.tw, ev) - score_mul<S>(di, dk);
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
    if (tid == 0 && s_I) acc_add(a.acc, blockIdx.x, 0, s_I);
}

// ---------------------------------------------------- thread-per-vertex kernel --

// One thread per vertex of row length <= MAXD: the row is held in registers,
// equal neighbour labels are merged by pairwise compares (fully unrolled),
// and every load of a vertex (entries, neighbour labels, candidate degrees)
// is independent of the others, so a wavefront keeps many in flight.  No
// LDS and no barriers.  64-bit scores.
template <int MAXD, typename W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_sweep_thread(SweepArgs a, const int32_t *__restrict__ list,
                                                      int64_t count) {
    if (a.st->done) return;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool active = k < count;
    int64_t self = 0;
    if (active) {
        const int32_t v = list[k];
        const int64_t rs = a.row_ptr[v];
        const int d = (int)(a.row_ptr[v + 1] - rs);
        const int32_t ci = a.c_cur[v];
        const int64_t di = a.delta[v];
        const int64_t deg_ci = a.deg[ci];
        const int32_t size_ci = a.size[ci];
        int32_t lab[MAXD];
        int64_t w[MAXD];
#pragma unroll
        for (int p = 0; p < MAXD; ++p) {
            lab[p] = -1;
            w[p] = 0;
            if (p < d) {
                lab[p] = a.col[rs + p];
                w[p] = wload<W>(a.w, rs + p);
            }
        }
        int64_t loop = 0;
#pragma unroll
        for (int p = 0; p < MAXD; ++p) {
            if (p < d) {
                if (lab[p] == v) {
                    loop += w[p];
                    lab[p] = -1;
                } else {
                    lab[p] = a.c_cur[lab[p]];
                }
            }
        }
        // merge equal labels into their first occurrence
        int64_t e_own = 0;
#pragma unroll
        for (int p = 0; p < MAXD; ++p) {
            if (lab[p] == ci && lab[p] >= 0) {
                e_own += w[p];
                lab[p] = -1;
            }
        }
#pragma unroll
        for (int p = 0; p < MAXD; ++p) {
#pragma unroll
            for (int q = p + 1; q < MAXD; ++q) {
                if (lab[p] >= 0 && lab[q] == lab[p]) {
                    w[p] += w[q];
                    lab[q] = -1;
                }
            }
        }
        int64_t dg[MAXD];
#pragma unroll
        for (int p = 0; p < MAXD; ++p) dg[p] = lab[p] >= 0 ? a.deg[lab[p]] : 0;
        int64_t bs = 0;
        int32_t bl = -1;
#pragma unroll
        for (int p = 0; p < MAXD; ++p) {
            if (lab[p] < 0) continue;
            const int64_t sc = a.tw * w[p] - di * dg[p];
            if (better<int64_t>(sc, lab[p], bs, bl)) {
                bs = sc;
                bl = lab[p];
            }
        }
        int32_t nxt = ci;
        if (bl >= 0 && bs > a.tw * e_own - di * (deg_ci - di)) {
            nxt = bl;
            if (a.singlet && size_ci == 1 && bl > ci && a.size[bl] == 1) nxt = ci;
        }
        a.c_nxt[v] = nxt;
        self = e_own + loop;
        if (a.e_self) a.e_self[v] = self;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) self += __shfl_xor(self, off);
    if ((threadIdx.x & 63) == 0 && self) acc_add(a.acc, (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6), 0, (unsigned long long)self);
}

// ------------------------------------------------------- packed sweep kernel --

__device__ __forceinline__ int pack_bits(int64_t d) { return pack_table_bits(d); }

// Largest k in [0, n) with a[k] <= x (a strictly increasing, a[0] <= x).
__device__ __forceinline__ int lds_find(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Add w under label k in the table of 2^bits slots at key/val (runtime
// size); the thread that claims a slot records the table's owner vertex.
__device__ __forceinline__ void lds_insert_rt(int32_t *key, unsigned long long *val, uint8_t *owner, int bits,
                                             int32_t k, int64_t w, int own) {
    const uint32_t mask = (1u << bits) - 1;
    uint32_t h = ((uint32_t)k * 0x9E3779B1u) >> (32 - bits);
    while (true) {
        const int32_t prev = atomicCAS(&key[h], kEmpty, k);   // claims, or returns the slot's key
        if (prev == kEmpty) owner[h] = (uint8_t)own;
        if (prev == kEmpty || prev == k) {
            atomicAdd(&val[h], (unsigned long long)w);
            return;
        }
        h = (h + 1) & mask;
    }
}

// Line position cost of a packed vertex.
__global__ void k_pack_cost(const int64_t *__restrict__ rp, const int32_t *__restrict__ list, int64_t m,
                            int32_t *cost) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int32_t v = list[k];
    const int c = 1 << pack_bits(rp[v + 1] - rp[v]);
    cost[k] = c > kPackMinCost ? c : kPackMinCost;
}

// first[b] = first packed vertex whose line position is >= b * kPackW
// (b in [0, nblocks]; first[nblocks] = m).
__global__ void k_pack_first(const int64_t *__restrict__ pos, int64_t m, int64_t nblocks, int64_t *first) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nblocks) return;
    const int64_t target = b * kPackW;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (pos[mid] < target) lo = mid + 1; else hi = mid;
    }
    first[b] = b == nblocks ? m : lo;
}

constexpr int kPackUnroll = 4;

// Many vertices per workgroup, edges spread over all threads (independent
// loads of kPackUnroll entries per thread in flight), per-vertex LDS tables,
// scores stored back into the table and reduced with LDS atomics on an
// order-preserving key (score with the sign bit flipped), ties broken by a
// second pass of atomicMin on the label.  64-bit scores only.
template <typename W>
__global__ __launch_bounds__(256) void k_sweep_pack(SweepArgs a, const int32_t *__restrict__ list,
                                                    const int64_t *__restrict__ pos,
                                                    const int64_t *__restrict__ first) {
    __shared__ int32_t s_key[kPackSlots];
    __shared__ unsigned long long s_val[kPackSlots];
    __shared__ uint8_t s_own[kPackSlots];
    __shared__ int32_t s_v[256], s_ci[256], s_toff[256], s_eoff[257];
    __shared__ int64_t s_rs[256], s_delta[256];
    __shared__ int32_t s_bits[256];
    __shared__ unsigned long long s_best[256], s_eown[256], s_loop[256];
    __shared__ int32_t s_bestl[256];
    __shared__ unsigned long long s_I;
    if (a.st->done) return;
    const int t = threadIdx.x;
    const int64_t lo_pos = (int64_t)blockIdx.x * kPackW;
    if (t == 0) s_I = 0;
    for (int x = t; x < kPackSlots; x += 256) {
        s_key[x] = kEmpty;
        s_val[x] = 0;
    }
    const int64_t k0 = first[blockIdx.x];
    const int nv = (int)(first[blockIdx.x + 1] - k0);
    // vertex descriptors (thread t owns vertex t)
    int32_t v = 0, ci = 0;
    int64_t d = 0, di = 0, deg_ci = 0;
    int32_t size_ci = 0;
    if (t < nv) {
        v = list[k0 + t];
        const int64_t rs = a.row_ptr[v];
        d = a.row_ptr[v + 1] - rs;
        ci = a.c_cur[v];
        di = a.delta[v];
        s_v[t] = v;
        s_ci[t] = ci;
        s_rs[t] = rs;
        s_delta[t] = di;
        s_toff[t] = (int32_t)(pos[k0 + t] - lo_pos);
        s_bits[t] = pack_bits(d);
        s_best[t] = 0;
        s_bestl[t] = 0x7fffffff;
        s_eown[t] = 0;
        s_loop[t] = 0;
    }
    {   // exclusive scan of row lengths -> edge offsets
        __shared__ int32_t wsum[4];
        const int lane = t & 63, wid = t >> 6;
        int32_t x = (int32_t)d;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (w < wid) before += wsum[w];
            total += wsum[w];
        }
        s_eoff[t] = before + x - (int32_t)d;
        if (t == 0) s_eoff[256] = total;
    }
    if (t < nv) {   // loads for the decision, issued early
        deg_ci = a.deg[ci];
        size_ci = a.size[ci];
    }
    __syncthreads();
    const int32_t E = s_eoff[256];
    // entries: kPackUnroll independent loads per thread in flight
    for (int32_t base = 0; base < E; base += 256 * kPackUnroll) {
        int kk[kPackUnroll];
        int64_t e[kPackUnroll];
        int32_t j[kPackUnroll], lab[kPackUnroll];
        int64_t w[kPackUnroll];
#pragma unroll
        for (int u = 0; u < kPackUnroll; ++u) {
            const int32_t x = base + u * 256 + t;
            kk[u] = -1;
            if (x < E) {
                kk[u] = lds_find(s_eoff, nv, x);
                e[u] = s_rs[kk[u]] + (x - s_eoff[kk[u]]);
            }
        }
#pragma unroll
        for (int u = 0; u < kPackUnroll; ++u) {
            if (kk[u] >= 0) {
                j[u] = a.col[e[u]];
                w[u] = wload<W>(a.w, e[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < kPackUnroll; ++u) {
            lab[u] = -1;
            if (kk[u] >= 0 && j[u] != s_v[kk[u]]) lab[u] = a.c_cur[j[u]];
        }
#pragma unroll
        for (int u = 0; u < kPackUnroll; ++u) {
            if (kk[u] < 0) continue;
            if (lab[u] < 0)
                atomicAdd(&s_loop[kk[u]], (unsigned long long)w[u]);
            else
                lds_insert_rt(s_key + s_toff[kk[u]], s_val + s_toff[kk[u]], s_own + s_toff[kk[u]], s_bits[kk[u]],
                              lab[u], w[u], kk[u]);
        }
    }
    __syncthreads();
    // scores: the own community is recorded and removed; every other
    // candidate's score key is stored in place of its weight.  Each thread
    // takes kPackSlots / 256 slots with all their deg_C gathers in flight.
    constexpr int SPT = kPackSlots / 256;
    const int32_t used = nv > 0 ? s_toff[nv - 1] + (1 << s_bits[nv - 1]) : 0;
    {
        int32_t key[SPT];
        int kv[SPT];
        int64_t ev[SPT], dg[SPT];
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int32_t x = q * 256 + t;
            key[q] = x < used ? s_key[x] : kEmpty;
            kv[q] = 0;
            ev[q] = 0;
            if (key[q] != kEmpty) {
                kv[q] = s_own[x];
                ev[q] = (int64_t)s_val[x];
            }
        }
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            dg[q] = 0;
            if (key[q] != kEmpty && key[q] != s_ci[kv[q]]) dg[q] = a.deg[key[q]];
        }
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            if (key[q] == kEmpty) continue;
            const int32_t x = q * 256 + t;
            if (key[q] == s_ci[kv[q]]) {
                s_eown[kv[q]] = (unsigned long long)ev[q];
                s_key[x] = kEmpty;
                continue;
            }
            const int64_t sc = a.tw * ev[q] - s_delta[kv[q]] * dg[q];
            const unsigned long long ok = (unsigned long long)sc ^ 0x8000000000000000ull;
            s_val[x] = ok;
            atomicMax(&s_best[kv[q]], ok);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int32_t x = q * 256 + t;
        if (x >= used) continue;
        const int32_t key = s_key[x];
        if (key == kEmpty) continue;
        const int kv = s_own[x];
        if (s_val[x] == s_best[kv]) atomicMin(&s_bestl[kv], key);
    }
    __syncthreads();
    if (t < nv) {
        const int64_t e_own = (int64_t)s_eown[t];
        const int64_t s_own = a.tw * e_own - di * (deg_ci - di);
        int32_t nxt = ci;
        if (s_best[t] != 0) {
            const int64_t bs = (int64_t)(s_best[t] ^ 0x8000000000000000ull);
            const int32_t bl = s_bestl[t];
            if (bs > s_own) {
                nxt = bl;
                if (a.singlet && size_ci == 1 && bl > ci && a.size[bl] == 1) nxt = ci;
            }
        }
        a.c_nxt[v] = nxt;
        const int64_t self = e_own + (int64_t)s_loop[t];
        if (a.e_self) a.e_self[v] = self;
        if (self) atomicAdd(&s_I, (unsigned long long)self);
    }
    __syncthreads();
    if (t == 0 && s_I) acc_add(a.acc, blockIdx.x, 0, s_I);
}

// ------------------------------------------------------------- hub kernels --

// Hub metadata: 4 arrays of (hubs + 1) int64 laid out back to back.
struct HubMeta {
    const int32_t *v;        // hub vertices
    const int64_t *tab_off;  // first table slot of each hub
    const int64_t *chunk_off;// first accumulation block of each hub
    const int64_t *scan_off; // first scan block of each hub
    const int64_t *tab_size; // table slots of each hub (multiple of kHubScan, >= 2 * row length)
    const int32_t *chunk_hub;// hub of each accumulation workgroup
    const int32_t *scan_hub; // hub of each scan workgroup
    int64_t hubs;
    const int64_t *bkt_off;  // first bucket of each hub (no buckets: the hub uses its table only)
    const int64_t *reg_off;  // first pair slot of each hub's bucket regions
    const int32_t *bkt_hub;  // hub of each bucket
    int shrink;              // bucket regions and tables divided by this (1; more only to test the spills)
};

// Hub rows on levels with published words and single-word tables are swept
// by partition.  Each accumulation workgroup sums its chunk in LDS, keyed by
// the neighbour's published word, then appends every distinct (word, e) to
// one of the hub's buckets, chosen by a hash of the label, with one cursor
// add per bucket and workgroup; one workgroup per bucket then sums its pairs
// in an LDS table and scores them (deg_C is in the key).  On R-MAT scale 24
// nearly every label a hub's chunk meets is new to it, so the table path
// cost one memory-side atomic per entry, most of the hubs' time.  The table
// stays the path of hubs with more than kBktMax buckets, and of a bucket
// whose pairs overflow its region or its LDS table: all that bucket's pairs
// then go to the table (the spill flag makes the scan read it), so a label
// is never split between a bucket and the table.

constexpr int kHubLdsBits = 11;  // 2048 slots for a chunk of kHubChunk = 1024 entries

// One workgroup per kHubChunk entries of a hub row: pre-aggregate e_{i->C}
// in LDS, then add each distinct community once into the hub's HBM table.
template <typename W, typename S>
__global__ __launch_bounds__(256) void k_hub_accum(SweepArgs a, HubMeta hm, int32_t *gkey,
                                                   unsigned long long *gval, unsigned long long *hub_loop,
                                                   uint64_t *part, uint64_t *bkey, uint64_t *bval,
                                                   unsigned int *bcur, unsigned int *spill) {
    constexpr int T = 1 << kHubLdsBits;
    // keyed by the neighbour's published word, or by its label without words
    __shared__ unsigned long long s_key[T];
    __shared__ unsigned long long s_val[T];
    __shared__ unsigned int s_cnt[kBktMax], s_base[kBktMax];
    __shared__ int64_t s_h;
    if (a.st->done) return;
    const int t = threadIdx.x;
    if (t == 0) s_h = hm.chunk_hub[blockIdx.x];
    if (!a.first)
        for (int x = t; x < T; x += 256) {
            s_key[x] = kEmptyWord;
            s_val[x] = 0;
        }
    __syncthreads();
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int64_t k = (int64_t)blockIdx.x - hm.chunk_off[h];
    const int64_t row_end = a.row_ptr[v + 1];
    const int64_t rs = a.row_ptr[v] + k * kHubChunk;
    const int64_t re = rs + kHubChunk < row_end ? rs + kHubChunk : row_end;
    // kHubChunk / 256 entries per lane: loads and label gathers first, then inserts
    constexpr int U = kHubChunk / 256;
    static_assert(kHubChunk % 256 == 0, "a chunk is whole rounds of the workgroup");
    int32_t jq[U], lq[U];
    int64_t wq[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int64_t e = rs + t + q * 256;
        jq[q] = -1;
        wq[q] = 0;
        if (e < re) {
            jq[q] = a.col[e];
            wq[q] = wload<W>(a.w, e);
        }
    }
    int64_t dq[U];
    uint64_t uq[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        lq[q] = -1;
        dq[q] = -1;
        uq[q] = 0;
        if (jq[q] >= 0 && jq[q] != v) {
            if (a.pw) {
                uq[q] = a.pw[jq[q]];
                lq[q] = pw_label(uq[q], a.pw_bits);
                dq[q] = pw_deg(uq[q], a.pw_bits);
            } else {
                lq[q] = nb_label(a, jq[q], &dq[q]);
                uq[q] = (uint32_t)lq[q];
            }
        }
    }
    int64_t loop = 0;
#pragma unroll
    for (int q = 0; q < U; ++q)
        if (jq[q] == v) loop += wq[q];
    if (loop) atomicAdd(&hub_loop[h], (unsigned long long)loop);
    if (a.first) {
        // singletons: every entry is its own candidate; the chunk's best goes
        // to its partial (decided over the hub's chunks), no tables
        const int64_t di = a.delta[v];
        S bs = 0;
        int32_t bl = -1;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (lq[q] < 0) continue;
            const S sc = score_mul<S>(a.tw, wq[q]) - score_mul<S>(di, dq[q] >= 0 ? dq[q] : a.deg[lq[q]]);
            if (better<S>(sc, lq[q], bs, bl)) {
                bs = sc;
                bl = lq[q];
            }
        }
        int64_t u0 = 0, u1 = 0;
        group_reduce_block<S>(bs, bl, u0, u1);
        if (t == 0) {
            const i128 w = (i128)bs;
            uint64_t *p = part + 4 * (int64_t)blockIdx.x;
            p[0] = (uint64_t)w;
            p[1] = (uint64_t)(int64_t)(w >> 64);
            p[2] = (uint64_t)(int64_t)bl;
            p[3] = 0;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
        if (lq[q] >= 0) lds_insert_word<kHubLdsBits>(s_key, s_val, uq[q], lq[q], wq[q]);
    __syncthreads();
    const int64_t base = hm.tab_off[h], size = hm.tab_size[h];
    const int64_t b0 = hm.bkt_off[h], P = hm.bkt_off[h + 1] - b0;
    auto label_of = [&](unsigned long long key) {
        return a.pw ? pw_label(key, a.pw_bits) : (int32_t)(uint32_t)key;
    };
    if (P == 0) {   // the hub's table
        for (int x = t; x < T; x += 256) {
            const unsigned long long key = s_key[x];
            if (key == kEmptyWord) continue;
            if (a.hub_shift)
                packed_insert(gval + base, (uint64_t)size, label_of(key), s_val[x], a.hub_shift);
            else
                hbm_insert(gkey + base, gval + base, size, label_of(key), s_val[x]);
        }
        return;
    }
    // buckets: every distinct pair's rank among the workgroup's pairs of its
    // bucket, then one cursor add per bucket
    for (int b = t; b < P; b += 256) s_cnt[b] = 0;
    __syncthreads();
    constexpr int Q = T / 256;
    int32_t bq[Q];
    uint32_t rq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const unsigned long long key = s_key[t + q * 256];
        bq[q] = -1;
        rq[q] = 0;
        if (key != kEmptyWord) {
            bq[q] = (int32_t)bkt_of(label_of(key), P);
            rq[q] = atomicAdd(&s_cnt[bq[q]], 1u);
        }
    }
    __syncthreads();
    for (int b = t; b < P; b += 256) s_base[b] = s_cnt[b] ? atomicAdd(&bcur[b0 + b], s_cnt[b]) : 0u;
    __syncthreads();
    const int64_t cap = bkt_cap(row_end - a.row_ptr[v], P, hm.shrink);
    bool over = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (bq[q] < 0) continue;
        const int x = t + q * 256;
        const int64_t pos = (int64_t)s_base[bq[q]] + rq[q];
        if (pos < cap) {
            const int64_t at = hm.reg_off[h] + (int64_t)bq[q] * cap + pos;
            bkey[at] = s_key[x];
            bval[at] = s_val[x];
        } else {   // the bucket's region is full: the bucket goes to the table
            packed_insert(gval + base, (uint64_t)size, label_of(s_key[x]), s_val[x], a.hub_shift);
            over = true;
        }
    }
    if (over) spill[h] = 1u;
}

// One workgroup per bucket of a hub: sum its pairs in LDS and score them
// (best candidate and own e as a partial for k_hub_decide), or, when its
// pairs overflowed its region or its table, add all of them to the hub's
// table instead.  Leaves the bucket's cursor at 0.
template <typename S>
__global__ __launch_bounds__(256) void k_hub_bucket(SweepArgs a, HubMeta hm, unsigned long long *gval,
                                                    const uint64_t *__restrict__ bkey,
                                                    const uint64_t *__restrict__ bval, unsigned int *bcur,
                                                    unsigned int *spill, uint64_t *bpart) {
    constexpr int T = 1 << kBktBits;
    __shared__ unsigned long long s_key[T], s_val[T];
    __shared__ int64_t s_h;
    __shared__ unsigned int s_n;
    __shared__ int s_used, s_over;
    if (a.st->done) return;
    const int t = threadIdx.x;
    const int64_t bk = blockIdx.x;
    if (t == 0) {
        s_h = hm.bkt_hub[bk];
        s_n = bcur[bk];
        s_used = 0;
        s_over = 0;
    }
    for (int x = t; x < T; x += 256) {
        s_key[x] = kEmptyWord;
        s_val[x] = 0;
    }
    __syncthreads();
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int64_t b0 = hm.bkt_off[h], P = hm.bkt_off[h + 1] - b0;
    const int64_t cap = bkt_cap(a.row_ptr[v + 1] - a.row_ptr[v], P, hm.shrink);
    const int64_t reg = hm.reg_off[h] + (bk - b0) * cap;
    const int claim = kBktClaim / hm.shrink > 0 ? kBktClaim / hm.shrink : 1;
    const int64_t n = s_n;
    bool spill_all = n > cap;
    if (!spill_all) {
        bool over = false;
        for (int64_t i = t; i < n; i += 256) {
            const uint64_t word = bkey[reg + i];
            const unsigned long long e = bval[reg + i];
            uint32_t x = hash_pow2(pw_label(word, a.pw_bits), kBktBits);
            while (true) {
                const unsigned long long cur = s_key[x];
                if (cur == word) {
                    atomicAdd(&s_val[x], e);
                    break;
                }
                if (cur == kEmptyWord) {
                    if (s_used >= claim) {
                        over = true;
                        break;
                    }
                    const unsigned long long prev = atomicCAS(&s_key[x], kEmptyWord, (unsigned long long)word);
                    if (prev == kEmptyWord) atomicAdd(&s_used, 1);
                    if (prev == kEmptyWord || prev == word) {
                        atomicAdd(&s_val[x], e);
                        break;
                    }
                }
                x = (x + 1) & (T - 1);
            }
        }
        if (over) s_over = 1;
        __syncthreads();
        spill_all = s_over != 0;
    }
    S bs = 0;
    int32_t bl = -1;
    int64_t e_own = 0, unused = 0;
    if (spill_all) {
        const int64_t m = n < cap ? n : cap;
        const int64_t base = hm.tab_off[h], size = hm.tab_size[h];
        for (int64_t i = t; i < m; i += 256)
            packed_insert(gval + base, (uint64_t)size, pw_label(bkey[reg + i], a.pw_bits), bval[reg + i],
                          a.hub_shift);
        if (t == 0) spill[h] = 1u;
    } else {
        const int32_t ci = a.c_cur[v];
        const int64_t di = a.delta[v];
        for (int x = t; x < T; x += 256) {
            const unsigned long long key = s_key[x];
            if (key == kEmptyWord) continue;
            const int32_t k = pw_label(key, a.pw_bits);
            const int64_t ev = (int64_t)s_val[x];
            if (k == ci) {
                e_own += ev;
                continue;
            }
            const S sc = score_mul<S>(a.tw, ev) - score_mul<S>(di, pw_deg(key, a.pw_bits));
            if (better<S>(sc, k, bs, bl)) {
                bs = sc;
                bl = k;
            }
        }
    }
    group_reduce_block<S>(bs, bl, e_own, unused);
    if (t == 0) {
        const i128 w = (i128)bs;
        uint64_t *p = bpart + 4 * bk;
        p[0] = (uint64_t)w;
        p[1] = (uint64_t)(int64_t)(w >> 64);
        p[2] = (uint64_t)(int64_t)bl;
        p[3] = (uint64_t)e_own;
        bcur[bk] = 0u;
    }
}

// One workgroup per kHubScan slots of a hub table: best candidate and own
// e over its slots (partial), clearing the slots for the next pass.
template <typename S>
__global__ __launch_bounds__(256) void k_hub_scan(SweepArgs a, HubMeta hm, int32_t *gkey,
                                                  unsigned long long *gval, uint64_t *part,
                                                  const unsigned int *spill) {
    __shared__ int64_t s_h;
    __shared__ int s_skip;
    if (a.st->done) return;
    const int t = threadIdx.x;
    if (t == 0) {
        s_h = hm.scan_hub[blockIdx.x];
        // a hub swept by buckets has nothing in its table unless one spilled
        s_skip = hm.bkt_off[s_h + 1] > hm.bkt_off[s_h] && spill[s_h] == 0u;
        if (s_skip) {
            uint64_t *p = part + 4 * (int64_t)blockIdx.x;
            p[0] = 0;
            p[1] = 0;
            p[2] = (uint64_t)(int64_t)-1;
            p[3] = 0;
        }
    }
    __syncthreads();
    if (s_skip) return;
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int32_t ci = a.c_cur[v];
    const int64_t di = a.delta[v];
    const int64_t base = hm.tab_off[h] + ((int64_t)blockIdx.x - hm.scan_off[h]) * kHubScan;
    S bs = 0;
    int32_t bl = -1;
    int64_t e_own = 0, unused = 0;
    const int shift = a.hub_shift;
#pragma unroll
    for (int q = 0; q < kHubScan / 256; ++q) {
        const int64_t x = base + q * 256 + t;
        int32_t k;
        int64_t ev;
        if (shift) {
            const unsigned long long wd = gval[x];
            if (wd == 0) continue;
            gval[x] = 0;
            k = (int32_t)(wd >> shift) - 1;
            ev = (int64_t)(wd & ~(~0ull << shift));
        } else {
            k = gkey[x];
            if (k == kEmpty) continue;
            ev = (int64_t)gval[x];
            gkey[x] = kEmpty;
            gval[x] = 0;
        }
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
                                                    unsigned long long *hub_loop, const uint64_t *bpart,
                                                    unsigned int *spill) {
    if (a.st->done) return;
    const int lane = threadIdx.x & 63;
    const int64_t h = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (h >= hm.hubs) return;
    S bs = 0;
    int32_t bl = -1;
    int64_t e_own = 0, unused = 0;
    // partials: one per scan workgroup, or one per chunk on the first pass
    // from singletons
    const int64_t *range = a.first ? hm.chunk_off : hm.scan_off;
    auto take = [&](const uint64_t *p) {
        const int32_t l = (int32_t)(int64_t)p[2];
        const S sc = (S)make_i128(p[0], (int64_t)p[1]);
        if (better<S>(sc, l, bs, bl)) {
            bs = sc;
            bl = l;
        }
        e_own += (int64_t)p[3];
    };
    for (int64_t b = range[h] + lane; b < range[h + 1]; b += 64) take(part + 4 * b);
    if (!a.first)   // and the buckets' partials
        for (int64_t b = hm.bkt_off[h] + lane; b < hm.bkt_off[h + 1]; b += 64) take(bpart + 4 * b);
    group_reduce_wave<64, S>(bs, bl, e_own, unused);
    if (lane == 0) {
        spill[h] = 0u;
        const int32_t v = hm.v[h];
        const int32_t ci = a.c_cur[v];
        a.c_nxt[v] = decide<S>(a, v, ci, bs, bl, e_own);
        const int64_t self = e_own + (int64_t)hub_loop[h];
        hub_loop[h] = 0;
        if (a.e_self) a.e_self[v] = self;
        if (self) acc_add(a.acc, (uint64_t)h, 0, (unsigned long long)self);
    }
}

// --------------------------------------------------- commit, Q, acceptance --

constexpr int kQsumTile = 2048;

// Community degrees and sizes follow the movers.  A workgroup takes
// kCommitTile vertices and sums its movers' updates per community in an LDS
// table first (a community that many of the tile's vertices join or leave,
// such as a hub's, then takes one global atomic per array instead of one per
// mover); an update that finds no slot within kGenCommitProbe probes goes to
// HBM directly.  Integer sums (modulo 2^64 for the degrees), so the result
// does not depend on their order.
constexpr int kCommitTile = 2048;
constexpr int kCommitBits = 12;       // 2 slots per vertex of the tile
constexpr int kGenCommitProbe = 32;

__device__ __forceinline__ bool gen_commit_insert(int32_t *key, unsigned long long *dsum, int *ssum, int32_t k,
                                                  unsigned long long d, int s) {
    constexpr uint32_t mask = (1u << kCommitBits) - 1;
    uint32_t h = ((uint32_t)k * 0x9E3779B1u) >> (32 - kCommitBits);
    for (int probe = 0; probe < kGenCommitProbe; ++probe) {
        const int32_t prev = atomicCAS(&key[h], kEmpty, k);   // claims, or returns the slot's key
        if (prev == kEmpty || prev == k) {
            atomicAdd(&dsum[h], d);
            atomicAdd(&ssum[h], s);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

__global__ __launch_bounds__(256) void k_commit(const int32_t *__restrict__ c_cur, const int32_t *__restrict__ c_nxt,
                                                const int64_t *__restrict__ delta, int64_t *deg, int32_t *size,
                                                int64_t n, PhaseState *st, unsigned long long *acc) {
    constexpr int T = 1 << kCommitBits;
    __shared__ int32_t s_key[T];
    __shared__ unsigned long long s_deg[T];
    __shared__ int s_size[T];
    __shared__ unsigned long long s_m;
    if (st->done) return;
    for (int x = threadIdx.x; x < T; x += 256) {
        s_key[x] = kEmpty;
        s_deg[x] = 0;
        s_size[x] = 0;
    }
    if (threadIdx.x == 0) s_m = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kCommitTile;
    unsigned long long moved = 0;
#pragma unroll 2
    for (int k = 0; k < kCommitTile / 256; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v >= n) break;
        const int32_t a = c_cur[v], b = c_nxt[v];
        if (a == b) continue;
        const unsigned long long d = (unsigned long long)delta[v];
        if (!gen_commit_insert(s_key, s_deg, s_size, b, d, 1)) {
            atomicAdd((unsigned long long *)&deg[b], d);
            atomicAdd(&size[b], 1);
        }
        if (!gen_commit_insert(s_key, s_deg, s_size, a, 0 - d, -1)) {
            atomicAdd((unsigned long long *)&deg[a], 0 - d);
            atomicAdd(&size[a], -1);
        }
        ++moved;
    }
    if (moved) atomicAdd(&s_m, moved);
    __syncthreads();
    for (int x = threadIdx.x; x < T; x += 256) {
        const int32_t key = s_key[x];
        if (key == kEmpty) continue;
        if (s_deg[x] != 0) atomicAdd((unsigned long long *)&deg[key], s_deg[x]);
        if (s_size[x] != 0) atomicAdd(&size[key], s_size[x]);
    }
    if (threadIdx.x == 0 && s_m) acc_add(acc, blockIdx.x, 1, s_m);
}

// Per-block partial sums of deg_C^2 (128-bit) of the labelling a pass reads;
// with pw, also every vertex's published word of that labelling.
__global__ __launch_bounds__(256) void k_qsum(const int64_t *__restrict__ deg, int64_t n, uint64_t *part,
                                              const PhaseState *st, const int32_t *__restrict__ c,
                                              const int32_t *__restrict__ size, uint64_t *pw, int pw_bits) {
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
            if (pw) {
                const int32_t cv = c[v];
                pw[v] = (uint64_t)(uint32_t)cv | ((uint64_t)deg[cv] << pw_bits) |
                        (size[cv] == 1 ? (1ull << 63) : 0ull);
            }
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
                                                  int64_t theta_den, int32_t max_sweeps, int32_t p,
                                                  unsigned long long *acc) {
    static_assert(kAccSlots == 256, "one slot of the pass's sums per thread");
    __shared__ uint64_t slo[256];
    __shared__ int64_t shi[256];
    __shared__ unsigned long long s_I[4], s_m[4];
    if (st->done) return;
    // the pass's I and mover count: one slot per thread, then cleared for the next pass
    unsigned long long vi = acc[threadIdx.x * kAccStride], vm = acc[threadIdx.x * kAccStride + 1];
    acc[threadIdx.x * kAccStride] = 0;
    acc[threadIdx.x * kAccStride + 1] = 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        vi += (unsigned long long)__shfl_xor((long long)vi, off);
        vm += (unsigned long long)__shfl_xor((long long)vm, off);
    }
    if ((threadIdx.x & 63) == 0) {
        s_I[threadIdx.x >> 6] = vi;
        s_m[threadIdx.x >> 6] = vm;
    }
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
    const unsigned long long acc_I = s_I[0] + s_I[1] + s_I[2] + s_I[3];
    const unsigned long long moved = s_m[0] + s_m[1] + s_m[2] + s_m[3];
    const i128 S = make_i128(slo[0], shi[0]);
    const i128 q = mul_wide(tw, (int64_t)acc_I) - S;
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
        } else if (moved == 0) {
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

// small_max: the longest row of the thread-per-vertex bucket; block_max: the
// longest row swept from an LDS table (the hub path takes longer ones).
__device__ __forceinline__ int bucket_of(int64_t d, int small_max, int64_t block_max) {
    if (d <= 0) return -1;
    if (d <= small_max) return B_T8;
    if (d > block_max) return B_HUB;
#pragma unroll
    for (int b = B_T16; b < B_WIDE; ++b)
        if (d <= kBucketMax[b]) return b;
    return B_WIDE;
}

// Bucket of vertex v, or -1 if it is not evaluated (empty row, or its graph's
// phase is over when gid and st are given).
__device__ __forceinline__ int bucket_of_vertex(const int64_t *__restrict__ rp, const int32_t *__restrict__ gid,
                                                const PhaseState *__restrict__ st, int64_t v, int64_t *deg,
                                                int small_max, int64_t block_max) {
    const int64_t d = rp[v + 1] - rp[v];
    *deg = d;
    if (gid && st[gid[v]].done) return -1;
    return bucket_of(d, small_max, block_max);
}

// Largest delta_i of a level: a grid of at most kDeltaMaxBlocks workgroups
// strides over the vertices, each reduces its maxima (wavefront, then LDS)
// and makes one atomic (one per wavefront queued about 30,000 atomics on the
// one address at 2^24 vertices).
constexpr int kDeltaMaxBlocks = 512;
__global__ __launch_bounds__(256) void k_delta_max(const int64_t *__restrict__ delta, int64_t n,
                                                   unsigned long long *out) {
    __shared__ unsigned long long s_m[4];
    unsigned long long m = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256)
        m = max(m, (unsigned long long)delta[v]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned long long)__shfl_xor((long long)m, off));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
        if (m) atomicMax(out, m);
    }
}

__global__ __launch_bounds__(256) void k_bucket_count(const int64_t *__restrict__ rp, int64_t n, int32_t *counts,
                                                      int64_t nblocks, unsigned long long *bucket_nnz,
                                                      const int32_t *__restrict__ gid,
                                                      const PhaseState *__restrict__ st, int small_max,
                                                      int64_t block_max) {
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
            int64_t d;
            const int b = bucket_of_vertex(rp, gid, st, v, &d, small_max, block_max);
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
                                                        int32_t *list, const int32_t *__restrict__ gid,
                                                        const PhaseState *__restrict__ st, int small_max,
                                                        int64_t block_max) {
    __shared__ int run[NBUCKET];
    __shared__ int wc[4][NBUCKET];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t < NBUCKET) run[t] = offs[t * nblocks + blockIdx.x];
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kBucketTile;
    for (int k = 0; k < kBucketTile / 256; ++k) {
        const int64_t v = base + k * 256 + t;
        int64_t d;
        const int b = v < n ? bucket_of_vertex(rp, gid, st, v, &d, small_max, block_max) : -1;
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

// hub_of[b] = h for every workgroup b in [off[h], off[h + 1]).
__global__ void k_hub_map(const int64_t *__restrict__ off, int64_t hubs, int32_t *hub_of) {
    const int64_t h = blockIdx.x;
    if (h >= hubs) return;
    for (int64_t b = off[h] + threadIdx.x; b < off[h + 1]; b += blockDim.x) hub_of[b] = (int32_t)h;
}

__global__ void k_hub_sizes(const int64_t *__restrict__ rp, const int32_t *__restrict__ hubv, int64_t hubs,
                            int64_t *tab_off, int64_t *chunk_off, int64_t *scan_off, int64_t *tab_size,
                            int64_t *bkt_off, int64_t *reg_off, int bucketed, int shrink) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= hubs) return;
    const int32_t v = hubv[h];
    const int64_t d = rp[v + 1] - rp[v];
    const int64_t T = (2 * d + kHubScan - 1) / kHubScan * kHubScan;
    tab_size[h] = T;
    tab_off[h] = T;
    chunk_off[h] = (d + kHubChunk - 1) / kHubChunk;
    scan_off[h] = T / kHubScan;
    const int64_t P = bucketed ? bkt_count(d) : 0;
    bkt_off[h] = P;
    reg_off[h] = P ? P * bkt_cap(d, P, shrink) : 0;
}

// ------------------------------------------------------------------- host --

void Sweeper::reserve(int64_t n, int64_t nnz) {
    if (n <= cap_n_ && nnz <= cap_nnz_) return;
    for (auto &c : c_) c.alloc((size_t)n);
    deg_.alloc((size_t)n);
    size_.alloc((size_t)n);
    ds_.alloc((size_t)n);
    vw_.alloc((size_t)n);
    es_.alloc((size_t)n);
    acc_.alloc((size_t)kAccSlots * kAccStride);   // general levels: the pass's sums, by slot
    fill<uint64_t>((uint64_t *)acc_.p, 0, (int64_t)kAccSlots * kAccStride, s_);
    active_.alloc(3);   // graphs still in their phase (by pass parity), commit arrivals
    fill<int32_t>((int32_t *)active_.p, 0, 3, s_);
    tw_one_.alloc(1);
    list_.alloc((size_t)n);
    const int64_t nblk = (n + kBucketTile - 1) / kBucketTile;
    bcount_.alloc((size_t)(NBUCKET * nblk + 1));
    st_.alloc(1);
    qpart_.alloc((size_t)(2 * ((n + kQsumTile - 1) / kQsumTile) + 2));
    // hubs are rows longer than the workgroup bucket's limit, at least
    // kPackMaxDeg + 1 entries whatever the tuning
    const int64_t max_hubs = nnz / (kPackMaxDeg + 1) + 1;
    hub_cap_ = max_hubs;
    hub_meta_.alloc((size_t)(6 * (max_hubs + 1)));
    pack_pos_.alloc((size_t)n + 1);
    hub_loop_.alloc((size_t)max_hubs);
    cap_n_ = n;
    cap_nnz_ = nnz;
}

void Sweeper::set_batch(int64_t ngraphs, const int32_t *gid, const int64_t *tw) {
    batch_ = true;
    ngraphs_ = ngraphs;
    gid_ = gid;
    tw_ = tw;
}

void Sweeper::plan(const GraphView &g) { plan_impl(g, false); }

void Sweeper::replan_active(const GraphView &g) { plan_impl(g, true); }

void Sweeper::plan_impl(const GraphView &g, bool active_only) {
    n_ = g.n;
    compact_ = batch_ || g.tw < kCompactTwMax;   // before anything that depends on the level's kind
    general_classes_ = false;
    score64_ = g.tw <= kTwFastMax;
    fill<uint64_t>((uint64_t *)acc_.p, 0, (int64_t)kAccSlots * kAccStride, s_);   // a phase starts from zero sums
    const int small_max = compact_ ? tuning_.small_max : (int)kBucketMax[B_T8];
    const int64_t block_max = compact_ ? tuning_.block_max : lds_row_max(g.n, g.tw, tuning_);
    const int32_t *skip_gid = active_only && batch_ ? gid_ : nullptr;
    const PhaseState *skip_st = active_only && batch_ ? st_.p : nullptr;
    if (!batch_) {
        ngraphs_ = 1;
        gid_ = nullptr;
        if (compact_) {
            LV_HIP(hipMemcpyAsync(tw_one_.p, &g.tw, sizeof(int64_t), hipMemcpyHostToDevice, s_));
            tw_ = tw_one_.p;
        }
    }
    if ((int64_t)st_.n < ngraphs_) st_.alloc((size_t)ngraphs_);
    const int64_t nblk = (g.n + kBucketTile - 1) / kBucketTile;
    for (int b = 0; b <= NBUCKET; ++b) bstart_[b] = 0;
    hubs_ = hub_chunks_ = hub_scans_ = hub_slots_ = hub_buckets_ = 0;
    pack_count_ = pack_blocks_ = 0;
    qblocks_ = (g.n + kQsumTile - 1) / kQsumTile;
    if (g.n == 0) return;
    TempBuf bnnz(NBUCKET * sizeof(unsigned long long), s_);
    LV_HIP(hipMemsetAsync(bnnz.p, 0, NBUCKET * sizeof(unsigned long long), s_));
    int32_t *counts = bcount_.p;
    {
        TimedLaunch tl(t_, TG_LEVEL, "k_bucket_count", (double)g.n * 16);
        tl.launch(k_bucket_count, (unsigned)nblk, 256, 0, s_, g.row_ptr, g.n, counts, nblk,
                  bnnz.as<unsigned long long>(), skip_gid, skip_st, small_max, block_max);
        LV_LAUNCHED("k_bucket_count");
    }
    const int64_t m = NBUCKET * nblk;
    scan_exclusive<int32_t, int32_t>(counts, counts, m, counts + m, s_, t_);
    {
        TimedLaunch tl(t_, TG_LEVEL, "k_bucket_scatter", (double)g.n * 20);
        tl.launch(k_bucket_scatter, (unsigned)nblk, 256, 0, s_, g.row_ptr, g.n, counts, nblk, list_.p, skip_gid,
                  skip_st, small_max, block_max);
        LV_LAUNCHED("k_bucket_scatter");
    }
    Readback rb(s_);
    const int32_t *hs[NBUCKET + 1];
    for (int b = 0; b < NBUCKET; ++b) hs[b] = rb.add(counts + (int64_t)b * nblk);
    hs[NBUCKET] = rb.add(counts + m);
    const unsigned long long *hn = rb.add(bnnz.as<unsigned long long>(), NBUCKET);
    // 64-bit scores whenever every product of a score fits: TW e and
    // delta_i deg_C are at most TW max_i delta_i (e_{i->C} <= delta_i and
    // deg_C <= TW), so TW max delta < 2^62 keeps scores and their
    // differences inside int64 (always so when TW <= kTwFastMax)
    const unsigned long long *hdmax = nullptr;
    if (!compact_ && g.tw > kTwFastMax) {
        dmax_.reserve(1);
        fill<uint64_t>((uint64_t *)dmax_.p, 0, 1, s_);
        const unsigned db = grid_for(g.n, 256) < (unsigned)kDeltaMaxBlocks ? grid_for(g.n, 256) : (unsigned)kDeltaMaxBlocks;
        k_delta_max<<<db, 256, 0, s_>>>(g.delta, g.n, dmax_.p);
        LV_LAUNCHED("k_delta_max");
        hdmax = rb.add(dmax_.p);
    }
    rb.fetch();
    score64_ = g.tw <= kTwFastMax || (hdmax && (i128)g.tw * (i128)*hdmax < ((i128)1 << 62));
    for (int b = 0; b <= NBUCKET; ++b) bstart_[b] = *hs[b];
    for (int b = 0; b < NBUCKET; ++b) bucket_nnz_[b] = (int64_t)hn[b];
    // line positions of the packed vertices (buckets B_T16 to B_MID, contiguous in the list)
    pack_count_ = bstart_[B_BLOCK] - bstart_[B_T16];
    if (compact_) {
        // every row swept from LDS (small_max + 1 .. block_max entries), by table size
        const int64_t nl = bstart_[B_HUB] - bstart_[B_T16];
        glist_.reserve((size_t)(nl > 0 ? nl : 1));
        ginfo_.reserve((size_t)(nl > 0 ? nl : 1));
        compact_classes(g.row_ptr, list_.p + bstart_[B_T16], nl, glist_.p, ginfo_.p, cstart_, cnnz_, s_, t_);
    } else if (g.tw > kTwFastMax) {
        // 128-bit scores: rows small_max + 1 .. block_max swept by table-size class
        const int64_t nl = bstart_[B_HUB] - bstart_[B_T16];
        glist_.reserve((size_t)(nl > 0 ? nl : 1));
        ginfo_.reserve((size_t)(nl > 0 ? nl : 1));
        compact_classes(g.row_ptr, list_.p + bstart_[B_T16], nl, glist_.p, ginfo_.p, cstart_, cnnz_, s_, t_);
        general_classes_ = true;
    } else if (pack_count_ > 0 && g.tw <= kTwFastMax) {
        TempBuf cost((size_t)pack_count_ * sizeof(int32_t), s_);
        k_pack_cost<<<grid_for(pack_count_, 256), 256, 0, s_>>>(g.row_ptr, list_.p + bstart_[B_T16], pack_count_,
                                                               cost.as<int32_t>());
        LV_LAUNCHED("k_pack_cost");
        scan_exclusive<int32_t, int64_t>(cost.as<int32_t>(), pack_pos_.p, pack_count_, pack_pos_.p + pack_count_,
                                         s_, t_);
        const int64_t *lp = rb.add(pack_pos_.p + pack_count_);
        rb.fetch();
        const int64_t line = *lp;
        pack_blocks_ = (line + kPackW - 1) / kPackW;
        pack_first_.reserve((size_t)pack_blocks_ + 1);
        k_pack_first<<<grid_for(pack_blocks_ + 1, 256), 256, 0, s_>>>(pack_pos_.p, pack_count_, pack_blocks_,
                                                                      pack_first_.p);
        LV_LAUNCHED("k_pack_first");
    }
    hubs_ = bucket_count(B_HUB);
    if (hubs_ == 0) return;
    require(hubs_ <= hub_cap_, LOUVAIN_EDEVICE, "hub count exceeds the reserved hub tables");
    int64_t *tab_off = hub_meta_.p, *chunk_off = tab_off + (hubs_ + 1), *scan_off = chunk_off + (hubs_ + 1),
            *tab_size = scan_off + (hubs_ + 1);
    int64_t *bkt_off = tab_size + (hubs_ + 1), *reg_off = bkt_off + (hubs_ + 1);
    const int32_t *hubv = list_.p + bstart_[B_HUB];
    // hubs are summed by buckets on compact levels and on general levels with
    // published words and single-word tables
    const int bucketed = compact_ || (publishes(g) && word_shift(g.n, g.tw) > 0) ? 1 : 0;
    k_hub_sizes<<<grid_for(hubs_, 256), 256, 0, s_>>>(g.row_ptr, hubv, hubs_, tab_off, chunk_off, scan_off, tab_size,
                                                      bkt_off, reg_off, bucketed, hub_bucket_shrink());
    LV_LAUNCHED("k_hub_sizes");
    scan_exclusive<int64_t, int64_t>(tab_off, tab_off, hubs_, tab_off + hubs_, s_, t_);
    scan_exclusive<int64_t, int64_t>(chunk_off, chunk_off, hubs_, chunk_off + hubs_, s_, t_);
    scan_exclusive<int64_t, int64_t>(scan_off, scan_off, hubs_, scan_off + hubs_, s_, t_);
    scan_exclusive<int64_t, int64_t>(bkt_off, bkt_off, hubs_, bkt_off + hubs_, s_, t_);
    scan_exclusive<int64_t, int64_t>(reg_off, reg_off, hubs_, reg_off + hubs_, s_, t_);
    const int64_t *tot[3] = {rb.add(tab_off + hubs_), rb.add(chunk_off + hubs_), rb.add(scan_off + hubs_)};
    const int64_t *btot[2] = {rb.add(bkt_off + hubs_), rb.add(reg_off + hubs_)};
    rb.fetch();
    hub_slots_ = *tot[0];
    hub_chunks_ = *tot[1];
    hub_scans_ = *tot[2];
    hub_buckets_ = *btot[0];
    if (hub_buckets_ > 0) {
        const int64_t pairs = *btot[1];
        bkt_key_.reserve((size_t)pairs);
        if (!compact_) bkt_val_.reserve((size_t)pairs);   // compact pairs are single words
        bkt_cur_.reserve((size_t)hub_buckets_);
        bkt_part_.reserve((size_t)(4 * hub_buckets_));
        hub_of_bkt_.reserve((size_t)hub_buckets_);
        fill<int32_t>((int32_t *)bkt_cur_.p, 0, hub_buckets_, s_);
        k_hub_map<<<(unsigned)hubs_, 256, 0, s_>>>(bkt_off, hubs_, hub_of_bkt_.p);
        LV_LAUNCHED("k_hub_map");
    }
    hub_spill_.reserve((size_t)hubs_);
    fill<int32_t>((int32_t *)hub_spill_.p, 0, hubs_, s_);
    if (hub_slots_ > hub_slot_cap_) {
        hub_key_.alloc((size_t)hub_slots_);
        hub_val_.alloc((size_t)hub_slots_);
        hub_slot_cap_ = hub_slots_;
    }
    hub_part_.reserve((size_t)(4 * hub_scans_));
    hub_of_chunk_.reserve((size_t)hub_chunks_);
    hub_of_scan_.reserve((size_t)hub_scans_);
    k_hub_map<<<(unsigned)hubs_, 256, 0, s_>>>(chunk_off, hubs_, hub_of_chunk_.p);
    LV_LAUNCHED("k_hub_map");
    k_hub_map<<<(unsigned)hubs_, 256, 0, s_>>>(scan_off, hubs_, hub_of_scan_.p);
    LV_LAUNCHED("k_hub_map");
    if (!compact_) fill<int32_t>(hub_key_.p, kEmpty, hub_slots_, s_);   // compact tables are one word per slot
    fill<uint64_t>((uint64_t *)hub_val_.p, 0, hub_slots_, s_);
    fill<uint64_t>((uint64_t *)hub_loop_.p, 0, hubs_, s_);
}

void Sweeper::init_singletons(const GraphView &g) {
    singleton_start_ = true;
    if (compact_) {
        compact_init_singletons(c_[0].p, c_[1].p, c_[2].p, g.delta, ds_.p, es_.p, g.n, s_);
        LV_HIP(hipMemsetAsync(st_.p, 0, sizeof(PhaseState) * (size_t)ngraphs_, s_));
        return;
    } else if (g.n > 0) {
        TimedLaunch tl(t_, TG_LEVEL, "k_init_singletons", (double)g.n * 28);
        tl.launch(k_init_singletons, grid_for(g.n, 256), 256, 0, s_, c_[0].p, c_[1].p, c_[2].p, g.delta, deg_.p,
                  size_.p, g.n);
        LV_LAUNCHED("k_init_singletons");
    }
    LV_HIP(hipMemsetAsync(st_.p, 0, sizeof(PhaseState), s_));
}

void Sweeper::init_singletons(const GraphView &g, const int32_t *ids) {
    init_from_labels(g, ids);
    singleton_start_ = true;   // a permutation: every community holds one vertex
}

void Sweeper::init_from_labels(const GraphView &g, const int32_t *labels) {
    singleton_start_ = false;
    if (compact_) {
        fill<uint64_t>(ds_.p, 0, g.n, s_);
        compact_init_labels(c_[0].p, c_[1].p, c_[2].p, labels, g.delta, ds_.p, es_.p, g.n, s_);
        LV_HIP(hipMemsetAsync(st_.p, 0, sizeof(PhaseState) * (size_t)ngraphs_, s_));
        return;
    }
    fill<int64_t>(deg_.p, 0, g.n, s_);
    fill<int32_t>(size_.p, 0, g.n, s_);
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_LEVEL, "k_init_labels", (double)g.n * 28);
        tl.launch(k_init_labels, grid_for(g.n, 256), 256, 0, s_, c_[0].p, c_[1].p, c_[2].p, labels, g.delta, deg_.p,
                  size_.p, g.n);
        LV_LAUNCHED("k_init_labels");
    }
    LV_HIP(hipMemsetAsync(st_.p, 0, sizeof(PhaseState), s_));
}

// Rows of up to kBucketMax[B_WIDE] entries on general levels: one
// 1,024-thread workgroup per vertex with an LDS table of 16,384 single-word
// slots, (label + 1) << shift | e (only launched when labels and weights fit
// 64 bits together), otherwise as k_sweep_group.
constexpr int kWideThreads = 1024;
constexpr int kWideBits = 14;
static_assert(kBucketMax[B_WIDE] <= 3 * 4 * kWideThreads, "a wide row is at most three rounds of its workgroup");

template <typename W, typename S>
__global__ __launch_bounds__(kWideThreads) void k_sweep_wide(SweepArgs a, const int32_t *__restrict__ list) {
    constexpr int T = kWideThreads, SL = 1 << kWideBits, SPL = SL / T, NW = T / 64;
    __shared__ unsigned long long tab[SL];
    __shared__ S r_s[NW];
    __shared__ int32_t r_l[NW];
    __shared__ int64_t s_eown, s_loop;
    if (a.st->done) return;
    const int t = threadIdx.x;
    if (!a.first)   // the first pass from singletons uses no table
#pragma unroll
        for (int q = 0; q < SPL; ++q) tab[t + q * T] = 0;
    if (t == 0) {
        s_eown = 0;
        s_loop = 0;
    }
    const int32_t i = list[blockIdx.x];
    const int64_t rs = a.row_ptr[i], re = a.row_ptr[i + 1];
    const int32_t ci = a.c_cur[i];
    const int shift = a.hub_shift;
    const unsigned long long tmask = ~0ull << shift;
    __syncthreads();
    const int64_t di = a.delta[i];
    S bs = 0;
    int32_t bl = -1;
    constexpr int U = 4;
    // With published words the lane that claims a slot scores it after the
    // inserts, with the candidate's deg_C from its word (no gather of deg_C):
    // the slot and the degree of every claim stay in registers (a row has at
    // most R rounds of U entries per lane).
    constexpr int R = (int)((kBucketMax[B_WIDE] + U * T - 1) / (U * T));
    int32_t hc[R * U];
    int64_t dc[R * U];
#pragma unroll
    for (int c = 0; c < R * U; ++c) hc[c] = -1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t e0 = rs + t + (int64_t)r * U * T;
        if (e0 >= re) break;
        int32_t jq[U], lq[U];
        int64_t wq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t e = e0 + (int64_t)q * T;
            jq[q] = -1;
            wq[q] = 0;
            if (e < re) {
                jq[q] = a.col[e];
                wq[q] = wload<W>(a.w, e);
            }
        }
        int64_t dq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            lq[q] = -1;
            dq[q] = -1;
            if (jq[q] >= 0 && jq[q] != i) lq[q] = nb_label(a, jq[q], &dq[q]);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (jq[q] == i) s_loop = wq[q];   // a row has at most one loop
            if (lq[q] < 0) continue;
            if (a.first) {   // every neighbour is its own community
                const S sc = score_mul<S>(a.tw, wq[q]) - score_mul<S>(di, dq[q] >= 0 ? dq[q] : a.deg[lq[q]]);
                if (better<S>(sc, lq[q], bs, bl)) {
                    bs = sc;
                    bl = lq[q];
                }
                continue;
            }
            const unsigned long long tag = (unsigned long long)(uint32_t)(lq[q] + 1) << shift;
            uint32_t h = ((uint32_t)lq[q] * 0x9E3779B1u) >> (32 - kWideBits);
            while (true) {
                const unsigned long long prev = atomicCAS(&tab[h], 0ull, tag | (unsigned long long)wq[q]);
                if (prev == 0) {
                    hc[r * U + q] = (int32_t)h;
                    dc[r * U + q] = dq[q];
                    break;
                }
                if ((prev & tmask) == tag) {
                    atomicAdd(&tab[h], (unsigned long long)wq[q]);
                    break;
                }
                h = (h + 1) & (SL - 1);
            }
        }
    }
    __syncthreads();
    if (!a.first && a.pw) {
#pragma unroll
        for (int c = 0; c < R * U; ++c) {
            if (hc[c] < 0) continue;
            const unsigned long long wd = tab[hc[c]];
            const int32_t k = (int32_t)(wd >> shift) - 1;
            const int64_t ev = (int64_t)(wd & ~tmask);
            if (k == ci) {
                s_eown = ev;
                continue;
            }
            const S sc = score_mul<S>(a.tw, ev) - score_mul<S>(di, dc[c]);
            if (better<S>(sc, k, bs, bl)) {
                bs = sc;
                bl = k;
            }
        }
    }
#pragma unroll 4
    for (int q = 0; q < SPL; ++q) {
        if (a.first || a.pw) break;
        const unsigned long long wd = tab[t + q * T];
        if (wd == 0) continue;
        const int32_t k = (int32_t)(wd >> shift) - 1;
        const int64_t ev = (int64_t)(wd & ~tmask);
        if (k == ci) {
            s_eown = ev;
            continue;
        }
        const S sc = score_mul<S>(a.tw, ev) - score_mul<S>(di, a.deg[k]);
        if (better<S>(sc, k, bs, bl)) {
            bs = sc;
            bl = k;
        }
    }
    int64_t u0 = 0, u1 = 0;
    group_reduce_wave<64, S>(bs, bl, u0, u1);
    const int wid = t >> 6;
    if ((t & 63) == 0) {
        r_s[wid] = bs;
        r_l[wid] = bl;
    }
    __syncthreads();
    if (t == 0) {
        for (int w2 = 1; w2 < NW; ++w2)
            if (better<S>(r_s[w2], r_l[w2], bs, bl)) {
                bs = r_s[w2];
                bl = r_l[w2];
            }
        a.c_nxt[i] = decide<S>(a, i, ci, bs, bl, s_eown);
        const int64_t self = s_eown + s_loop;
        if (a.e_self) a.e_self[i] = self;
        if (self) acc_add(a.acc, blockIdx.x, 0, (unsigned long long)self);
    }
}

// Rows swept from LDS on levels with 128-bit scores, sorted by table size
// (the classes of the compact levels: S = 16 << c slots for c < 6, then
// 2,048, 4,096 and 16,384): class c goes to k_sweep_group with 4 slots per
// lane (8 for c = 5), so a row's table and lane group fit its length.
struct ClassLists {
    const int32_t *list = nullptr;              // nullptr: sweep by degree buckets
    const int64_t *cstart = nullptr;            // kLdsClasses + 1 offsets into list
    const int64_t *cnnz = nullptr;              // entries of every class
};

// Buffers of the hubs swept by buckets.
struct HubBuckets {
    int64_t buckets;
    uint64_t *key, *val;   // pair regions
    unsigned int *cur;     // pairs appended to each bucket
    uint64_t *part;        // per bucket: score lo, score hi, label, e_own
    unsigned int *spill;   // per hub: some bucket went to the table
};

template <typename W, typename S>
static void launch_pass(const SweepArgs &a, const int32_t *list, const int64_t *bstart,
                        const int64_t *bnnz, const int64_t *pack_pos, const int64_t *pack_first,
                        int64_t pack_blocks, HubMeta hm, const HubBuckets &hb,
                        int64_t hub_chunks, int64_t hub_scans, int32_t *hkey, unsigned long long *hval,
                        unsigned long long *hloop, uint64_t *hpart, hipStream_t s, Timer *t,
                        const ClassLists &cl = ClassLists()) {
    const std::string sfx = t ? std::string(type_name<W>()) + "," + type_name<S>() + ">" : std::string();
    const std::string wsfx = t ? std::string(type_name<W>()) + ">" : std::string();
    const std::string ssfx = t ? std::string(type_name<S>()) + ">" : std::string();
    // per entry: column, weight and the neighbour's label (4 bytes) or published word (8)
    const double eb = (a.pw ? 12.0 : 8.0) + sizeof(W);
    const double vb = 40.0;              // per evaluated vertex
    auto cnt = [&](int b) { return bstart[b + 1] - bstart[b]; };
    auto bytes = [&](int b) { return (double)cnt(b) * vb + (double)bnnz[b] * eb; };
    if (cl.list) {
        if (cnt(B_T8) > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<4,4,", bytes(B_T8), sfx.c_str());
            tl.launch(k_sweep_group<4, 4, W, S>, grid_for(cnt(B_T8), 64), 256, 0, s, a, list + bstart[B_T8], cnt(B_T8));
            LV_LAUNCHED("k_sweep_group<4>");
        }
        auto ccount = [&](int c) { return cl.cstart[c + 1] - cl.cstart[c]; };
        auto cbytes = [&](int c) { return (double)ccount(c) * vb + (double)cl.cnnz[c] * eb; };
        auto group = [&](auto kernel, int c, int per_block, const char *name) {
            if (ccount(c) <= 0) return;
            TimedLaunch tl(t, TG_SWEEP, name, cbytes(c), sfx.c_str());
            tl.launch(kernel, grid_for(ccount(c), per_block), 256, 0, s, a, cl.list + cl.cstart[c], ccount(c));
            LV_LAUNCHED(name);
        };
        group(k_sweep_group<4, 4, W, S>, 0, 64, "k_sweep_group<4,4,");
        group(k_sweep_group<8, 5, W, S>, 1, 32, "k_sweep_group<8,5,");
        group(k_sweep_group<16, 6, W, S>, 2, 16, "k_sweep_group<16,6,");
        group(k_sweep_group<32, 7, W, S>, 3, 8, "k_sweep_group<32,7,");
        group(k_sweep_group<64, 8, W, S>, 4, 4, "k_sweep_group<64,8,");
        if (a.pw) {   // tables keyed by published words: no deg_C gathers when scoring
            group(k_sweep_group<64, 9, W, S, true>, 5, 4, "k_sweep_group<64,9,");
            group(k_sweep_group<256, 11, W, S, true>, 6, 1, "k_sweep_group<256,11,");
            group(k_sweep_group<256, 12, W, S, true>, 7, 1, "k_sweep_group<256,12,");
        } else {
            group(k_sweep_group<64, 9, W, S>, 5, 4, "k_sweep_group<64,9,");
            group(k_sweep_group<256, 11, W, S>, 6, 1, "k_sweep_group<256,11,");
            group(k_sweep_group<256, 12, W, S>, 7, 1, "k_sweep_group<256,12,");
        }
        const int c8 = kLdsClasses - 1;
        if (ccount(c8) > 0) {   // rows up to kBucketMax[B_WIDE]: only when a.hub_shift > 0
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_wide<", cbytes(c8), sfx.c_str());
            tl.launch(k_sweep_wide<W, S>, (unsigned)ccount(c8), kWideThreads, 0, s, a, cl.list + cl.cstart[c8]);
            LV_LAUNCHED("k_sweep_wide");
        }
    } else if constexpr (std::is_same<S, int64_t>::value) {
        if (cnt(B_T8) > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_thread<8,", bytes(B_T8), wsfx.c_str());
            tl.launch(k_sweep_thread<8, W>, grid_for(cnt(B_T8), 256), 256, 0, s, a, list + bstart[B_T8], cnt(B_T8));
            LV_LAUNCHED("k_sweep_thread<8>");
        }
        const int64_t np = bstart[B_BLOCK] - bstart[B_T16];
        if (np > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_pack<", bytes(B_T16) + bytes(B_G64) + bytes(B_MID), wsfx.c_str());
            tl.launch(k_sweep_pack<W>, (unsigned)pack_blocks, 256, 0, s, a, list + bstart[B_T16], pack_pos, pack_first);
            LV_LAUNCHED("k_sweep_pack");
        }
        if (cnt(B_BLOCK) > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<256,11,", bytes(B_BLOCK), sfx.c_str());
            tl.launch(k_sweep_group<256, 11, W, S>, (unsigned)cnt(B_BLOCK), 256, 0, s, a, list + bstart[B_BLOCK],
                      cnt(B_BLOCK));
            LV_LAUNCHED("k_sweep_group<256>");
        }
    } else {
        if (cnt(B_T8) > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<4,4,", bytes(B_T8), sfx.c_str());
            tl.launch(k_sweep_group<4, 4, W, S>, grid_for(cnt(B_T8), 64), 256, 0, s, a, list + bstart[B_T8], cnt(B_T8));
            LV_LAUNCHED("k_sweep_group<4>");
        }
        if (cnt(B_T16) > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<16,6,", bytes(B_T16), sfx.c_str());
            tl.launch(k_sweep_group<16, 6, W, S>, grid_for(cnt(B_T16), 16), 256, 0, s, a, list + bstart[B_T16],
                      cnt(B_T16));
            LV_LAUNCHED("k_sweep_group<16>");
        }
        if (cnt(B_G64) > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<64,8,", bytes(B_G64), sfx.c_str());
            tl.launch(k_sweep_group<64, 8, W, S>, grid_for(cnt(B_G64), 4), 256, 0, s, a, list + bstart[B_G64],
                      cnt(B_G64));
            LV_LAUNCHED("k_sweep_group<64>");
        }
        const int64_t nb = bstart[B_WIDE] - bstart[B_MID];
        if (nb > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_sweep_group<256,11,", bytes(B_MID) + bytes(B_BLOCK), sfx.c_str());
            tl.launch(k_sweep_group<256, 11, W, S>, (unsigned)nb, 256, 0, s, a, list + bstart[B_MID], nb);
            LV_LAUNCHED("k_sweep_group<256>");
        }
    }
    if (!cl.list && cnt(B_WIDE) > 0) {   // only bucketed when a.hub_shift > 0
        TimedLaunch tl(t, TG_SWEEP, "k_sweep_wide<", bytes(B_WIDE), sfx.c_str());
        tl.launch(k_sweep_wide<W, S>, (unsigned)cnt(B_WIDE), kWideThreads, 0, s, a, list + bstart[B_WIDE]);
        LV_LAUNCHED("k_sweep_wide");
    }
    if (hm.hubs > 0) {
        {
            TimedLaunch tl(t, TG_SWEEP, "k_hub_accum<", (double)bnnz[B_HUB] * eb, wsfx.c_str());
            tl.launch(k_hub_accum<W, S>, (unsigned)hub_chunks, 256, 0, s, a, hm, hkey, hval, hloop, hpart, hb.key,
                      hb.val, hb.cur, hb.spill);
            LV_LAUNCHED("k_hub_accum");
        }
        if (!a.first && hb.buckets > 0) {
            // per pair (at most one per hub entry): word and e read
            TimedLaunch tl(t, TG_SWEEP, "k_hub_bucket<", (double)bnnz[B_HUB] * 16.0, ssfx.c_str());
            tl.launch(k_hub_bucket<S>, (unsigned)hb.buckets, 256, 0, s, a, hm, hval, hb.key, hb.val, hb.cur, hb.spill,
                      hb.part);
            LV_LAUNCHED("k_hub_bucket");
        }
        if (!a.first) {
            TimedLaunch tl(t, TG_SWEEP, "k_hub_scan<", (double)hub_scans * kHubScan * 24.0, ssfx.c_str());
            tl.launch(k_hub_scan<S>, (unsigned)hub_scans, 256, 0, s, a, hm, hkey, hval, hpart, hb.spill);
            LV_LAUNCHED("k_hub_scan");
        }
        {
            TimedLaunch tl(t, TG_SWEEP, "k_hub_decide<", (double)hm.hubs * vb + (double)hub_scans * 32.0, ssfx.c_str());
            tl.launch(k_hub_decide<S>, grid_for(hm.hubs, 4), 256, 0, s, a, hm, hpart, hloop, hb.part, hb.spill);
            LV_LAUNCHED("k_hub_decide");
        }
    }
}

int64_t *Sweeper::deg() {
    if (compact_) compact_expand(ds_.p, es_.p, n_, deg_.p, size_.p, nullptr, s_);
    return deg_.p;
}

void Sweeper::e_self_out(int64_t *dst) {
    if (compact_) compact_expand(ds_.p, es_.p, n_, deg_.p, size_.p, dst, s_);
}

unsigned int Sweeper::active_after(int p) {
    Readback rb(s_);
    const unsigned int *h = rb.add(active_.p + (p & 1));
    rb.fetch();
    return *h;
}

void Sweeper::pass(const GraphView &g, int p, const SweepParams &prm, int64_t *e_self_out) {
    const int cur = (p - 1) % 3, nxt = p % 3;
    if (compact_) {
        CompactPass cp;
        cp.n = g.n;
        cp.list = list_.p;
        for (int b = 0; b <= NBUCKET; ++b) cp.bstart[b] = bstart_[b];
        for (int b = 0; b < NBUCKET; ++b) cp.bnnz[b] = bucket_nnz_[b];
        cp.pack_pos = pack_pos_.p;
        cp.pack_first = pack_first_.p;
        cp.pack_blocks = pack_blocks_;
        cp.glist = glist_.p;
        cp.ginfo = ginfo_.p;
        cp.small_max = tuning_.small_max;
        cp.group_slots = tuning_.group_slots;
        cp.group_vertices = tuning_.group_vertices;
        cp.group_tiles = tuning_.group_tiles;
        cp.first = singleton_start_ && p == 1 ? 1 : 0;
        cp.overlap = tuning_.overlap;
        for (int c = 0; c <= kLdsClasses; ++c) cp.cstart[c] = cstart_[c];
        for (int c = 0; c < kLdsClasses; ++c) cp.cnnz[c] = cnnz_[c];
        cp.hubs = hubs_;
        cp.hub_chunks = hub_chunks_;
        cp.hub_scans = hub_scans_;
        cp.tab_off = hub_meta_.p;
        cp.chunk_off = hub_meta_.p + (hubs_ + 1);
        cp.scan_off = hub_meta_.p + 2 * (hubs_ + 1);
        cp.tab_size = hub_meta_.p + 3 * (hubs_ + 1);
        cp.chunk_hub = hub_of_chunk_.p;
        cp.scan_hub = hub_of_scan_.p;
        cp.hkey = hub_key_.p;
        cp.hval = hub_val_.p;
        cp.hloop = hub_loop_.p;
        cp.hpart = hub_part_.p;
        cp.hub_buckets = hub_buckets_;
        cp.bkt_off = hub_meta_.p + 4 * (hubs_ + 1);
        cp.reg_off = hub_meta_.p + 5 * (hubs_ + 1);
        cp.bkt_hub = hub_of_bkt_.p;
        cp.shrink = hub_bucket_shrink();
        cp.bkey = (unsigned long long *)bkt_key_.p;
        cp.bcur = bkt_cur_.p;
        cp.bpart = bkt_part_.p;
        cp.spill = hub_spill_.p;
        CompactState cs;
        cs.c_cur = c_[cur].p;
        cs.c_nxt = c_[nxt].p;
        cs.ds = ds_.p;
        cs.vw = vw_.p;
        cs.es = es_.p;
        cs.gid = gid_;
        cs.tw = tw_;
        cs.st = st_.p;
        cs.active = active_.p;
        cs.ngraphs = ngraphs_;
        cs.slots = gid_ ? nullptr : acc_.p;
        if (tuning_.overlap && !side_) side_.reset(new SideStreams());
        cs.side = side_.get();
        compact_pass(g, cp, cs, p, prm, s_, t_);
        return;
    }
    const int pw_bits = pw_label_bits(g.n);
    const bool publish = publishes(g);
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_SWEEP, "k_qsum", (double)g.n * (publish ? 32 : 8));
        tl.launch(k_qsum, (unsigned)qblocks_, 256, 0, s_, deg_.p, g.n, qpart_.p, st_.p, (const int32_t *)c_[cur].p,
                  (const int32_t *)size_.p, publish ? vw_.p : (uint64_t *)nullptr, pw_bits);
        LV_LAUNCHED("k_qsum");
    }
    // hub and wide-row tables as single words when label + 1 and e (<= 2W)
    // fit 64 bits together
    const int hub_shift = word_shift(g.n, g.tw);
    SweepArgs a{g.row_ptr, g.col, g.w, c_[cur].p, c_[nxt].p, g.delta, deg_.p, size_.p,
                g.tw, prm.singlet, st_.p, e_self_out, hub_shift, singleton_start_ && p == 1 ? 1 : 0,
                publish ? vw_.p : nullptr, pw_bits, acc_.p};
    int64_t *tab_off = hub_meta_.p;
    HubMeta hm{list_.p + bstart_[B_HUB], tab_off, tab_off + (hubs_ + 1), tab_off + 2 * (hubs_ + 1),
               tab_off + 3 * (hubs_ + 1), hub_of_chunk_.p, hub_of_scan_.p, hubs_, tab_off + 4 * (hubs_ + 1),
               tab_off + 5 * (hubs_ + 1), hub_of_bkt_.p, hub_bucket_shrink()};
    HubBuckets hb{hub_buckets_, bkt_key_.p, bkt_val_.p, bkt_cur_.p, bkt_part_.p, hub_spill_.p};
    const bool fast = score64_;
    ClassLists cls;
    if (general_classes_) {
        cls.list = glist_.p;
        cls.cstart = cstart_;
        cls.cnnz = cnnz_;
    }
    if (g.wbytes == 4) {
        if (fast)
            launch_pass<int32_t, int64_t>(a, list_.p, bstart_, bucket_nnz_, pack_pos_.p, pack_first_.p, pack_blocks_, hm, hb, hub_chunks_, hub_scans_,
                                          hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_, cls);
        else
            launch_pass<int32_t, i128>(a, list_.p, bstart_, bucket_nnz_, pack_pos_.p, pack_first_.p, pack_blocks_, hm, hb, hub_chunks_, hub_scans_,
                                       hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_, cls);
    } else {
        if (fast)
            launch_pass<int64_t, int64_t>(a, list_.p, bstart_, bucket_nnz_, pack_pos_.p, pack_first_.p, pack_blocks_, hm, hb, hub_chunks_, hub_scans_,
                                          hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_, cls);
        else
            launch_pass<int64_t, i128>(a, list_.p, bstart_, bucket_nnz_, pack_pos_.p, pack_first_.p, pack_blocks_, hm, hb, hub_chunks_, hub_scans_,
                                       hub_key_.p, hub_val_.p, hub_loop_.p, hub_part_.p, s_, t_, cls);
    }
    if (g.n > 0) {
        TimedLaunch tl(t_, TG_SWEEP, "k_commit", (double)g.n * 8);
        tl.launch(k_commit, grid_for(g.n, kCommitTile), 256, 0, s_, c_[cur].p, c_[nxt].p, g.delta, deg_.p, size_.p,
                  g.n, st_.p, acc_.p);
        LV_LAUNCHED("k_commit");
    }
    {
        TimedLaunch tl(t_, TG_SWEEP, "k_finalize", 0.0);
        tl.launch(k_finalize, 1, 256, 0, s_, st_.p, qpart_.p, qblocks_, g.tw, prm.theta_num, prm.theta_den,
                  prm.max_sweeps, p, acc_.p);
        LV_LAUNCHED("k_finalize");
    }
}

PhaseState Sweeper::read_state() {
    Readback rb(s_);
    const PhaseState *h = rb.add(st_.p);
    rb.fetch();
    return *h;
}

}  // namespace lv
