// Local-moving sweeps for levels whose total weight TW = 2W is below 2^31
// (paper: Alg. 1, eqs. 1-5, minimum-label heuristics of Section 3.1), for
// one graph or for a batch of graphs laid out as one block-diagonal union
// (graph g owns a contiguous vertex range; every graph keeps its own TW,
// modularity, acceptance test and phase state, so each result equals a run
// on that graph alone).
//
// Below 2^31 every degree, community degree and e_{i->C} fits in 31 bits,
// which allows two compact words:
//   community word DS[C]   low 32 bits deg_C, high 32 bits size_C; a mover
//                          updates both halves with one 64-bit atomic;
//   published word VW[j]   low 32 bits the label c_j, bits 32..62 deg of
//                          community c_j, bit 63 set iff c_j is a singleton.
// Each pass first publishes VW from the labelling it reads, so a vertex
// gets a neighbour's community, that community's degree and its singleton
// flag with one 8-byte gather; scores need no further global loads.
// Scores TW*e - delta*deg stay below 2^62 (int64); sum_C deg_C^2 <= TW^2
// fits 64 bits.
//
// Pass kernels: k_cpt_publish (VW, sum deg^2 per graph) -> k_cpt_small /
// k_cpt_groups / k_cpt_group / hub kernels (new labels, e_{i->c_i} incl.
// loop per vertex)
// -> k_cpt_commit (movers' atomics, per-graph I and mover counts) ->
// k_cpt_finalize (per graph: Q_int and the acceptance test).
#include "prims.hpp"
#include "sweep.hpp"

namespace lv {
namespace {

constexpr uint64_t kSizeOne = 1ull << 32;

__device__ __forceinline__ uint64_t vw_make(int32_t c, uint64_t ds) {
    const uint32_t deg = (uint32_t)ds, sz = (uint32_t)(ds >> 32);
    return ((uint64_t)(deg | (sz == 1 ? 0x80000000u : 0u)) << 32) | (uint32_t)c;
}
__device__ __forceinline__ int32_t vw_label(uint64_t w) { return (int32_t)(uint32_t)w; }
__device__ __forceinline__ uint32_t hi_deg(uint32_t hi) { return hi & 0x7fffffffu; }
__device__ __forceinline__ bool hi_single(uint32_t hi) { return (hi >> 31) != 0; }

// Row start and length of a class-list entry in one word: start << 14 |
// length (rows swept from LDS have at most kCompactBlockMax < 2^14 entries).
__device__ __forceinline__ uint64_t row_info(int64_t rs, int64_t d) { return ((uint64_t)rs << 14) | (uint64_t)d; }
__device__ __forceinline__ int64_t info_start(uint64_t x) { return (int64_t)(x >> 14); }
__device__ __forceinline__ int64_t info_len(uint64_t x) { return (int64_t)(x & 16383u); }
static_assert(kCompactBlockMax < 16384, "row lengths swept from LDS fit 14 bits");

struct CArgs {
    const int64_t *row_ptr;
    const int32_t *col;
    const void *w;
    const int32_t *c_cur;
    int32_t *c_nxt;
    const int64_t *delta;
    const uint64_t *vw;      // published words of the labelling read
    const uint64_t *ds;      // community words of the labelling read (not written during the sweep)
    const int32_t *gid;      // graph of every vertex (nullptr: a single graph)
    const int64_t *tw;       // TW of every graph
    const PhaseState *st;    // phase state of every graph
    uint32_t *e_self;        // e_{i->c_i} incl. loop, written for every evaluated vertex
    int singlet;
    int first;   // the labelling read is the singletons: score entries directly, no tables
};

__device__ __forceinline__ int graph_of(const int32_t *gid, int64_t v) { return gid ? gid[v] : 0; }

// A single graph whose phase has ended: the pass (one of a batch of passes
// enqueued ahead of the host's check) has nothing to do.  Uniform over the
// grid, so kernels return at once, before any barrier.
__device__ __forceinline__ bool single_done(const int32_t *gid, const PhaseState *st) {
    return gid == nullptr && st[0].done;
}

template <typename W>
__device__ __forceinline__ uint32_t cw(const void *w, int64_t e) {
    return (uint32_t)((const W *)w)[e];   // weights are below TW < 2^31 here
}

// New label of a vertex: own word (ci, own_hi), best candidate (score bs,
// label bl, singleton flag bsingle), e_own = e_{i->C(i)\{i}}.
__device__ __forceinline__ int32_t cpt_decide(int singlet, int64_t tw, int32_t ci, uint32_t own_hi, int64_t di,
                                              int64_t e_own, bool has, int64_t bs, int32_t bl, bool bsingle) {
    if (!has) return ci;
    const int64_t s_own = tw * e_own - di * ((int64_t)hi_deg(own_hi) - di);
    if (bs <= s_own) return ci;
    if (singlet && hi_single(own_hi) && bsingle && bl > ci) return ci;
    return bl;
}

// Per-graph sums over a workgroup that covers the contiguous vertex range
// [lo, hi]: graphs are contiguous vertex ranges, so the range touches the
// graphs gid[lo] .. gid[hi]; up to kSpan of them are summed in LDS and
// flushed with one atomic each, wider spans fall back to per-lane atomics.
constexpr int kSpan = 64;

struct SpanSums {
    int g_lo, span;
};

__device__ __forceinline__ SpanSums span_begin(const int32_t *gid, int64_t lo, int64_t hi, int *s_glo, int *s_span,
                                               unsigned long long (*acc)[2]) {
    if (threadIdx.x == 0) {
        const int a = graph_of(gid, lo), b = graph_of(gid, hi);
        *s_glo = a;
        *s_span = b - a + 1;
    }
    if (threadIdx.x < kSpan) {
        acc[threadIdx.x][0] = 0;
        acc[threadIdx.x][1] = 0;
    }
    __syncthreads();
    return SpanSums{*s_glo, *s_span};
}

__device__ __forceinline__ void span_add(const SpanSums &sp, unsigned long long (*acc)[2], int k, int g,
                                         unsigned long long x, PhaseState *st, int field) {
    if (x == 0) return;
    if (sp.span <= kSpan) {
        atomicAdd(&acc[g - sp.g_lo][k], x);
    } else {
        unsigned long long *f = field == 0 ? &st[g].acc_I : field == 1 ? &st[g].moved : &st[g].s_acc;
        atomicAdd(f, x);
    }
}

__device__ __forceinline__ void span_flush(const SpanSums &sp, unsigned long long (*acc)[2], PhaseState *st,
                                           int field0, int field1, unsigned long long *slots) {
    __syncthreads();
    if (slots) {   // one graph: the workgroup's slot (fields 0, 1, 2 as in PhaseState)
        if (threadIdx.x == 0) {
            unsigned long long *sl = slots + (blockIdx.x & (kAccSlots - 1)) * kAccStride;
            if (field0 >= 0 && acc[0][0]) atomicAdd(sl + field0, acc[0][0]);
            if (field1 >= 0 && acc[0][1]) atomicAdd(sl + field1, acc[0][1]);
        }
        return;
    }
    if (sp.span <= kSpan && (int)threadIdx.x < sp.span) {
        const int g = sp.g_lo + threadIdx.x;
        const int fs[2] = {field0, field1};
        for (int k = 0; k < 2; ++k) {
            if (fs[k] < 0 || acc[threadIdx.x][k] == 0) continue;
            unsigned long long *f = fs[k] == 0 ? &st[g].acc_I : fs[k] == 1 ? &st[g].moved : &st[g].s_acc;
            atomicAdd(f, acc[threadIdx.x][k]);
        }
    }
}

// ----------------------------------------------------------------- set-up --

__global__ void k_cpt_init_singletons(int32_t *c0, int32_t *c1, int32_t *c2, const int64_t *__restrict__ delta,
                                      uint64_t *ds, uint32_t *es, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    c0[v] = c1[v] = c2[v] = (int32_t)v;
    ds[v] = kSizeOne | (uint64_t)delta[v];
    es[v] = 0;
}

__global__ void k_cpt_init_labels(int32_t *c0, int32_t *c1, int32_t *c2, const int32_t *__restrict__ labels,
                                  const int64_t *__restrict__ delta, uint64_t *ds, uint32_t *es, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = labels[v];
    c0[v] = c1[v] = c2[v] = l;
    es[v] = 0;
    atomicAdd((unsigned long long *)&ds[l], (unsigned long long)(kSizeOne + (uint64_t)delta[v]));
}

// Each vertex's label in its own graph's result slot (graphs of a batch end
// their phases at different passes).
__global__ void k_cpt_final_labels(const int32_t *__restrict__ c0, const int32_t *__restrict__ c1,
                                   const int32_t *__restrict__ c2, const int32_t *__restrict__ gid,
                                   const PhaseState *__restrict__ st, int64_t n, int32_t *out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int k = st[graph_of(gid, v)].final_slot;
    out[v] = k == 0 ? c0[v] : k == 1 ? c1[v] : c2[v];
}

__global__ void k_cpt_expand(const uint64_t *__restrict__ ds, const uint32_t *__restrict__ es, int64_t n,
                             int64_t *deg, int32_t *size, int64_t *e_self) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    deg[v] = (int64_t)(uint32_t)ds[v];
    size[v] = (int32_t)(ds[v] >> 32);
    if (e_self) e_self[v] = (int64_t)es[v];
}

// ---------------------------------------------------- publish + sum deg^2 --

// TILE vertices per workgroup (512..2048, see compact_tile)
template <int TILE>
__global__ __launch_bounds__(256) void k_cpt_publish(const uint64_t *__restrict__ ds, const int32_t *__restrict__ c,
                                                     uint64_t *vw, const int32_t *__restrict__ gid, PhaseState *st,
                                                     int64_t n, unsigned int *active_zero, unsigned long long *slots) {
    __shared__ unsigned long long acc[kSpan][2];
    __shared__ int s_glo, s_span;
    if (active_zero && blockIdx.x == 0 && threadIdx.x == 0) *active_zero = 0;
    if (single_done(gid, st)) return;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int64_t last = base + TILE - 1 < n - 1 ? base + TILE - 1 : n - 1;
    const SpanSums sp = span_begin(gid, base, last, &s_glo, &s_span, acc);
    // per-thread sums while consecutive vertices share a graph
    int gcur = -1;
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < TILE / 256; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v > last) continue;
        const int g = graph_of(gid, v);
        if (st[g].done) continue;
        if (g != gcur) {
            if (gcur >= 0) span_add(sp, acc, 1, gcur, sum, st, 2);
            gcur = g;
            sum = 0;
        }
        const uint64_t d = (uint32_t)ds[v];
        sum += d * d;
        const int32_t cv = c[v];
        vw[v] = vw_make(cv, ds[cv]);
    }
    if (gcur >= 0) span_add(sp, acc, 1, gcur, sum, st, 2);
    span_flush(sp, acc, st, -1, 2, slots);
}

// ------------------------------------------------------------- acceptance --

__device__ __forceinline__ void cpt_mul_u128_u64(u128 a, uint64_t b, uint64_t &hi, u128 &lo) {
    const u128 p0 = (u128)(uint64_t)a * b;
    const u128 p1 = (u128)(uint64_t)(a >> 64) * b;
    const u128 l = p0 + (p1 << 64);
    hi = (uint64_t)(p1 >> 64) + (l < p0 ? 1 : 0);
    lo = l;
}

// theta_den * (qn - qp) > theta_num * |qp|, exactly.
__device__ __forceinline__ bool cpt_gain_passes(i128 qn, i128 qp, int64_t num, int64_t den) {
    if (qn <= qp) return false;
    const u128 gain = (u128)(qn - qp);
    const u128 mag = (u128)(qp < 0 ? -qp : qp);
    uint64_t lh, rh;
    u128 ll, rl;
    cpt_mul_u128_u64(gain, (uint64_t)den, lh, ll);
    cpt_mul_u128_u64(mag, (uint64_t)num, rh, rl);
    return lh > rh || (lh == rh && ll > rl);
}

// Graph g: Q_int of the labelling the pass read (slot p-1) and the
// acceptance test of sweep p-1 against the last kept labelling.  acc_I and
// moved are read with agent-scope atomic loads: the commit's workgroups on
// other XCDs added to them in the same launch.
__device__ __forceinline__ void cpt_finalize_sums(PhaseState *st, const int64_t *__restrict__ tw, int64_t g,
                                                  unsigned long long acc_i, unsigned long long moved,
                                                  unsigned long long s_acc, int64_t theta_num, int64_t theta_den,
                                                  int32_t max_sweeps, int32_t p, unsigned int *active) {
    PhaseState &s = st[g];
    const i128 q = (i128)tw[g] * (i128)acc_i - (i128)s_acc;
    s.pass = p;
    s.q_last[0] = (uint64_t)q;
    s.q_last[1] = (uint64_t)(int64_t)(q >> 64);
    const i128 qref = make_i128(s.q_ref[0], (int64_t)s.q_ref[1]);
    bool keep = true;
    if (p == 1) {
        s.q_ref[0] = (uint64_t)q;
        s.q_ref[1] = (uint64_t)(int64_t)(q >> 64);
    } else if (cpt_gain_passes(q, qref, theta_num, theta_den)) {
        s.q_ref[0] = (uint64_t)q;
        s.q_ref[1] = (uint64_t)(int64_t)(q >> 64);
        s.accepted += 1;
    } else {
        keep = false;
        s.done = 1;
        s.final_slot = (p - 2) % 3;
    }
    if (keep) {
        if (s.accepted >= max_sweeps) {
            s.done = 1;
            s.limit = 1;
            s.final_slot = (p - 1) % 3;
        } else if (moved == 0) {
            s.done = 1;   // the next sweep cannot change Q, so it would be discarded
            s.final_slot = (p - 1) % 3;
        }
    }
    s.acc_I = 0;
    s.moved = 0;
    s.s_acc = 0;
    if (!s.done) atomicAdd(active, 1u);
}

__device__ __forceinline__ void cpt_finalize_graph(PhaseState *st, const int64_t *__restrict__ tw, int64_t g,
                                                   int64_t theta_num, int64_t theta_den, int32_t max_sweeps,
                                                   int32_t p, unsigned int *active) {
    PhaseState &s = st[g];
    if (s.done) return;
    const unsigned long long acc_i = __hip_atomic_load(&s.acc_I, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long moved = __hip_atomic_load(&s.moved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cpt_finalize_sums(st, tw, g, acc_i, moved, s.s_acc, theta_num, theta_den, max_sweeps, p, active);
}

// One graph's sums from its slots (called by all 256 threads of a
// workgroup): thread t reads slot t with agent-scope atomic loads (the
// commit's workgroups on other XCDs added to them in the same launch) and
// clears it for the next pass; thread 0 then runs the test.
__device__ __forceinline__ void cpt_finalize_slots(PhaseState *st, const int64_t *__restrict__ tw,
                                                   unsigned long long *slots, int64_t theta_num,
                                                   int64_t theta_den, int32_t max_sweeps, int32_t p,
                                                   unsigned int *active) {
    static_assert(kAccSlots == 256, "one slot per thread");
    __shared__ unsigned long long r[4][3];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    unsigned long long v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = __hip_atomic_load(slots + t * kAccStride + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        slots[t * kAccStride + k] = 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += (unsigned long long)__shfl_xor((long long)v[k], off);
        if (lane == 0) r[wid][k] = v[k];
    }
    __syncthreads();
    if (t != 0 || st[0].done) return;
    cpt_finalize_sums(st, tw, 0, r[0][0] + r[1][0] + r[2][0] + r[3][0], r[0][1] + r[1][1] + r[2][1] + r[3][1],
                      r[0][2] + r[1][2] + r[2][2] + r[3][2], theta_num, theta_den, max_sweeps, p, active);
}

// One thread per graph (passes over levels without vertices), or, for one
// graph with slots, one workgroup summing them.
__global__ void k_cpt_finalize(PhaseState *st, const int64_t *__restrict__ tw, int64_t ngraphs, int64_t theta_num,
                               int64_t theta_den, int32_t max_sweeps, int32_t p, unsigned int *active,
                               unsigned long long *slots) {
    if (slots) {
        cpt_finalize_slots(st, tw, slots, theta_num, theta_den, max_sweeps, p, active);
        return;
    }
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ngraphs) cpt_finalize_graph(st, tw, g, theta_num, theta_den, max_sweeps, p, active);
}

// ------------------------------------------------------------------ commit --

// Vertices per workgroup of the publish and commit kernels: 2,048 when the
// level has enough vertices for 1,024 such workgroups, down to 512 so that
// small levels (the later levels of a run, whose passes are many) still
// spread over the CUs instead of running a few long workgroups.
static int compact_tile(int64_t n) { return n >= ((int64_t)2048 << 10) ? 2048 : n >= ((int64_t)1024 << 10) ? 1024 : 512; }
constexpr int kCommitProbe = 32;   // probes before an update goes straight to HBM

// Add x to community k's pending update in the workgroup's LDS table of
// 2^BITS slots; false if no slot was found within kCommitProbe probes.
template <int BITS>
__device__ __forceinline__ bool commit_insert(int32_t *key, unsigned long long *val, int32_t k,
                                              unsigned long long x) {
    constexpr uint32_t mask = (1u << BITS) - 1;
    uint32_t h = ((uint32_t)k * 0x9E3779B1u) >> (32 - BITS);
    for (int probe = 0; probe < kCommitProbe; ++probe) {
        const int32_t prev = atomicCAS(&key[h], kEmpty, k);   // claims, or returns the slot's key
        if (prev == kEmpty || prev == k) {
            atomicAdd(&val[h], x);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

// Movers' community updates (size +-1, degree +-delta in one word) are
// summed per community in LDS first, so a community that many vertices of
// the tile join or leave takes one global atomic instead of one per mover;
// a tile of 2,048 vertices keeps the atomics on a large community's word to
// one per tile.  Updates that find no LDS slot (tiles where most vertices
// move between distinct communities) go to HBM directly.  The sums are
// integers modulo 2^64, so the result does not depend on the order.
// With `arrive` (a single graph of at most kFuseMaxN vertices), the last
// workgroup to finish (counted on `arrive`, which it leaves at 0) then runs
// the pass's acceptance test: no launch of its own.  Larger graphs and a
// batch's thousands of graphs keep their own launch (one thread per graph):
// the agent-scope release each workgroup needs before its arrival, and the
// arrivals on one counter, cost more than that launch once the grid is
// large (measured on a 2^20-vertex level: 64 us a commit fused, 43 us
// without the fence and the arrival).  A launch over a finished single
// graph returns in every workgroup.
constexpr int64_t kFuseMaxN = 1 << 16;
struct FinalizeArgs {
    const int64_t *tw;
    int64_t ngraphs, theta_num, theta_den;
    int32_t max_sweeps, p;
    unsigned int *active, *arrive;
    unsigned long long *slots;   // one graph: the pass's sums by slot
};

template <int TILE>
__global__ __launch_bounds__(256) void k_cpt_commit(const int32_t *__restrict__ c_cur, const int32_t *__restrict__ c_nxt,
                                                    const int64_t *__restrict__ delta, const uint32_t *__restrict__ es,
                                                    uint64_t *ds, const int32_t *__restrict__ gid, PhaseState *st,
                                                    int64_t n, FinalizeArgs fa) {
    if (single_done(gid, st)) return;
    constexpr int BITS = TILE == 2048 ? 12 : TILE == 1024 ? 11 : 10;   // two slots per vertex
    constexpr int T = 1 << BITS;
    __shared__ unsigned long long acc[kSpan][2];
    __shared__ int s_glo, s_span;
    __shared__ int32_t s_key[T];
    __shared__ unsigned long long s_val[T];
    for (int x = threadIdx.x; x < T; x += 256) {
        s_key[x] = kEmpty;
        s_val[x] = 0;
    }
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int64_t last = base + TILE - 1 < n - 1 ? base + TILE - 1 : n - 1;
    const SpanSums sp = span_begin(gid, base, last, &s_glo, &s_span, acc);
    // per-thread sums while consecutive vertices share a graph
    int gcur = -1;
    unsigned long long sum_e = 0, sum_m = 0;
#pragma unroll 2
    for (int k = 0; k < TILE / 256; ++k) {
        const int64_t v = base + k * 256 + threadIdx.x;
        if (v > last) continue;
        const int g = graph_of(gid, v);
        if (st[g].done) continue;
        if (g != gcur) {
            if (gcur >= 0) {
                span_add(sp, acc, 0, gcur, sum_e, st, 0);
                span_add(sp, acc, 1, gcur, sum_m, st, 1);
            }
            gcur = g;
            sum_e = 0;
            sum_m = 0;
        }
        const int32_t from = c_cur[v], to = c_nxt[v];
        if (from != to) {
            const uint64_t inc = kSizeOne + (uint64_t)delta[v];
            if (!commit_insert<BITS>(s_key, s_val, to, (unsigned long long)inc))
                atomicAdd((unsigned long long *)&ds[to], (unsigned long long)inc);
            if (!commit_insert<BITS>(s_key, s_val, from, (unsigned long long)(0 - inc)))
                atomicAdd((unsigned long long *)&ds[from], (unsigned long long)(0 - inc));
            sum_m += 1;
        }
        sum_e += es[v];
    }
    if (gcur >= 0) {
        span_add(sp, acc, 0, gcur, sum_e, st, 0);
        span_add(sp, acc, 1, gcur, sum_m, st, 1);
    }
    // the pass's sums go out first (after a barrier: the table is complete
    // too), so a workgroup's arrival waits for them and not for the degree
    // updates, which only the next pass reads
    span_flush(sp, acc, st, 0, 1, fa.slots);
    __shared__ int s_last;
    if (fa.arrive) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) s_last = atomicAdd(fa.arrive, 1u) == gridDim.x - 1;
    } else if (threadIdx.x == 0) {
        s_last = 0;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < T; x += 256) {
        const int32_t key = s_key[x];
        if (key != kEmpty && s_val[x] != 0) atomicAdd((unsigned long long *)&ds[key], s_val[x]);
    }
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (fa.slots)
        cpt_finalize_slots(st, fa.tw, fa.slots, fa.theta_num, fa.theta_den, fa.max_sweeps, fa.p, fa.active);
    else
        for (int64_t g = threadIdx.x; g < fa.ngraphs; g += 256)
            cpt_finalize_graph(st, fa.tw, g, fa.theta_num, fa.theta_den, fa.max_sweeps, fa.p, fa.active);
    if (threadIdx.x == 0) atomicExch(fa.arrive, 0u);
}

// ---------------------------------------------- rows of <= small_max entries --

// One thread per vertex in vertex-ID order (coalesced per-vertex accesses);
// threads whose row is empty or longer than small_max (<= 8) entries do nothing.  The row
// is held in registers and equal labels are merged by pairwise compares.
template <typename W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_cpt_small(CArgs a, int64_t n,
                                                                                          int small_max) {
    if (single_done(a.gid, a.st)) return;
    constexpr int MAXD = 8;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int64_t rs = a.row_ptr[v];
    const int d = (int)(a.row_ptr[v + 1] - rs);
    if (d < 1 || d > small_max) return;   // small_max <= MAXD
    const int g = graph_of(a.gid, v);
    if (a.st[g].done) return;
    const int64_t tw = a.tw[g];
    const uint64_t own = a.vw[v];
    const int32_t ci = vw_label(own);
    const uint32_t own_hi = (uint32_t)(own >> 32);
    const int64_t di = a.delta[v];
    int32_t lab[MAXD];
    uint32_t hi[MAXD], wt[MAXD];
#pragma unroll
    for (int p = 0; p < MAXD; ++p) {
        lab[p] = -1;
        wt[p] = 0;
        hi[p] = 0;
        if (p < d) {
            lab[p] = a.col[rs + p];
            wt[p] = cw<W>(a.w, rs + p);
        }
    }
    uint32_t loop = 0;
#pragma unroll
    for (int p = 0; p < MAXD; ++p) {
        if (p < d) {
            if (lab[p] == (int32_t)v) {
                loop += wt[p];
                lab[p] = -1;
            } else {
                const uint64_t nw = a.vw[lab[p]];
                lab[p] = vw_label(nw);
                hi[p] = (uint32_t)(nw >> 32);
            }
        }
    }
    uint32_t e_own = 0;
#pragma unroll
    for (int p = 0; p < MAXD; ++p) {
        if (lab[p] == ci) {
            e_own += wt[p];
            lab[p] = -1;
        }
    }
#pragma unroll
    for (int p = 0; p < MAXD; ++p) {
#pragma unroll
        for (int q = p + 1; q < MAXD; ++q) {
            if (lab[p] >= 0 && lab[q] == lab[p]) {
                wt[p] += wt[q];
                lab[q] = -1;
            }
        }
    }
    bool has = false;
    int64_t bs = 0;
    int32_t bl = 0;
    bool bsingle = false;
#pragma unroll
    for (int p = 0; p < MAXD; ++p) {
        if (lab[p] < 0) continue;
        const int64_t sc = tw * (int64_t)wt[p] - di * (int64_t)hi_deg(hi[p]);
        if (!has || sc > bs || (sc == bs && lab[p] < bl)) {
            has = true;
            bs = sc;
            bl = lab[p];
            bsingle = hi_single(hi[p]);
        }
    }
    a.c_nxt[v] = cpt_decide(a.singlet, tw, ci, own_hi, di, e_own, has, bs, bl, bsingle);
    a.e_self[v] = e_own + loop;
}

// ------------------------------------------------------ lane groups by size --

// Insert or add for a table of 2^bits slots: key, e_{i->C} (32-bit adds)
// and the community's published high word, stored once by the claimer.
__device__ __forceinline__ void grp_insert(int32_t *key, uint32_t *es, uint32_t *hs, int bits, int32_t k, uint32_t w,
                                           uint32_t hi) {
    const uint32_t mask = (1u << bits) - 1;
    uint32_t h = ((uint32_t)k * 0x9E3779B1u) >> (32 - bits);
    while (true) {
        // the compare-and-swap returns the slot's key whether or not it claims it
        const int32_t prev = atomicCAS(&key[h], kEmpty, k);
        if (prev == kEmpty) {
            hs[h] = hi;
            break;
        }
        if (prev == k) break;
        h = (h + 1) & mask;
    }
    atomicAdd(&es[h], w);
}

template <int X> struct Log2 { static constexpr int value = 1 + Log2<X / 2>::value; };
template <> struct Log2<1> { static constexpr int value = 0; };

// One step of the arg-max over a lane group: take the partner's candidate
// if its key is larger, or equal with a smaller label word (branch-free).
__device__ __forceinline__ void best_take(unsigned long long &bok, uint32_t &blf, uint32_t olo, uint32_t ohi,
                                          uint32_t olf) {
    const unsigned long long ook = ((unsigned long long)ohi << 32) | olo;
    const bool take = (ook > bok) | ((ook == bok) & (olf < blf));
    bok = take ? ook : bok;
    blf = take ? olf : blf;
}

template <int CTRL>
__device__ __forceinline__ void best_dpp(unsigned long long &bok, uint32_t &blf) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)bok, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(bok >> 32), CTRL, 0xF, 0xF, false);
    const uint32_t lf = (uint32_t)__builtin_amdgcn_mov_dpp((int)blf, CTRL, 0xF, 0xF, false);
    best_take(bok, blf, lo, hi, lf);
}

// Arg-max (largest key, then smallest label word) over every aligned group
// of G lanes of the wavefront (G a power of two, 2..64; uniform): after the
// quad steps every lane holds its quad's best, so the half-row and row
// mirrors pair whole quads and half-rows; a swizzle and a permute cover 16
// and 32.  Every lane ends with its group's best.
__device__ __forceinline__ void group_best(unsigned long long &bok, uint32_t &blf, int G) {
    if (G >= 2) best_dpp<0xB1>(bok, blf);    // quad_perm [1,0,3,2]
    if (G >= 4) best_dpp<0x4E>(bok, blf);    // quad_perm [2,3,0,1]
    if (G >= 8) best_dpp<0x141>(bok, blf);   // row_half_mirror
    if (G >= 16) best_dpp<0x140>(bok, blf);  // row_mirror
    if (G >= 32) {                           // lanes xor 16 inside each half-wavefront
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)bok, 0x401F);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(bok >> 32), 0x401F);
        const uint32_t lf = (uint32_t)__builtin_amdgcn_ds_swizzle((int)blf, 0x401F);
        best_take(bok, blf, lo, hi, lf);
    }
    if (G >= 64) {                           // lanes xor 32
        const int addr = (int)((__lane_id() ^ 32u) << 2);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)bok);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(bok >> 32));
        const uint32_t lf = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)blf);
        best_take(bok, blf, lo, hi, lf);
    }
}

// Rows sorted into table-size classes: a workgroup holds 256/G vertices of
// one class, each with an LDS table of S slots (S >= 1.5 d) and a group of G
// lanes (packed classes G = S/4; rows of up to 1,365 entries S = 2048 and of
// up to 2,730 entries S = 4096, G = 256).  Lane i of a group takes entries
// i, i + G, ... of its vertex's row, then scores slots i, i + G, ... (lanes
// read consecutive words, free of bank conflicts); the argmax (largest
// score, then smallest label) is a DPP / swizzle reduction inside each
// wavefront, with an LDS step across waves when the group spans several.
template <int S, int G, typename W>
__global__ __launch_bounds__(256) void k_cpt_group(CArgs a, const int32_t *__restrict__ list,
                                                   const uint64_t *__restrict__ info, int64_t count) {
    if (single_done(a.gid, a.st)) return;
    constexpr int NV = 256 / G;
    constexpr int SPL = S / G;
    constexpr int BITS = Log2<S>::value;
    constexpr int GW = G < 64 ? G : 64;   // lanes of a group inside one wave
    constexpr int WPG = G / GW;           // waves per group
    __shared__ int32_t s_key[NV * S];
    __shared__ uint32_t s_e[NV * S], s_hi[NV * S];
    __shared__ unsigned long long r_ok[4];
    __shared__ uint32_t r_lf[4], r_eo[4], r_lp[4];
    const int t = threadIdx.x;
    const int kv = t / G, li = t % G;
    int32_t *key = s_key + kv * S;
    uint32_t *es = s_e + kv * S, *hs = s_hi + kv * S;
    if (!a.first) {   // the first pass from singletons uses no table
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            key[li + q * G] = kEmpty;   // lane-consecutive words: no bank conflicts
            es[li + q * G] = 0;
        }
    }
    const int64_t k = (int64_t)blockIdx.x * NV + kv;
    bool live = false;
    int32_t v = 0;
    int g = 0;
    int64_t rs = 0, d = 0;
    if (k < count) {
        v = list[k];
        const uint64_t ri = info[k];
        g = graph_of(a.gid, v);
        live = !a.st[g].done;
        if (live) {
            rs = info_start(ri);
            d = info_len(ri);
        }
    }
    int32_t ci = -1;
    uint32_t own_hi = 0;
    int64_t di = 0, tw = 0;
    if (live) {
        const uint64_t own = a.vw[v];
        ci = vw_label(own);
        own_hi = (uint32_t)(own >> 32);
        di = a.delta[v];
        tw = a.tw[g];
    }
    __syncthreads();
    // Entries in rounds of U per lane: a round's loads and gathers are all
    // issued before its inserts (from singletons: scored directly, no table).
    constexpr int U = 4;
    uint32_t loop = 0;
    unsigned long long bok = 0;
    uint32_t blf = 0xffffffffu, e_own = 0;
    for (int64_t x0 = li; x0 < d; x0 += (int64_t)U * G) {
        int32_t jq[U];
        uint32_t wq[U];
        uint64_t nq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t x = x0 + (int64_t)q * G;
            jq[q] = v;
            wq[q] = 0;
            if (x < d) {
                jq[q] = a.col[rs + x];
                wq[q] = cw<W>(a.w, rs + x);
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            nq[q] = 0;
            if (jq[q] != v) nq[q] = a.vw[jq[q]];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (jq[q] == v) {
                loop += wq[q];
            } else if (a.first) {
                const uint32_t hi = (uint32_t)(nq[q] >> 32);
                const unsigned long long ok =
                    ((uint64_t)(uint32_t)tw * wq[q] - (uint64_t)(uint32_t)di * hi_deg(hi)) ^ 0x8000000000000000ull;
                best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32),
                          ((uint32_t)vw_label(nq[q]) << 1) | (hi_single(hi) ? 1u : 0u));
            } else {
                grp_insert(key, es, hs, BITS, vw_label(nq[q]), wq[q], (uint32_t)(nq[q] >> 32));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
        if (a.first) break;
        const int x = li + q * G;
        const int32_t kk = key[x];
        if (kk == kEmpty) continue;
        const uint32_t e = es[x];
        if (kk == ci) {
            e_own += e;
            continue;
        }
        const uint32_t hi = hs[x];
        // TW, delta_i, deg_C, e_{i->C} < 2^31: products of 32-bit operands
        const unsigned long long ok =
            ((uint64_t)(uint32_t)tw * e - (uint64_t)(uint32_t)di * hi_deg(hi)) ^ 0x8000000000000000ull;
        const uint32_t lf = ((uint32_t)kk << 1) | (hi_single(hi) ? 1u : 0u);
        best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32), lf);
    }
    group_best(bok, blf, GW);
#pragma unroll
    for (int off = GW / 2; off > 0; off >>= 1) {
        e_own += __shfl_xor(e_own, off);
        loop += __shfl_xor(loop, off);
    }
    if constexpr (WPG > 1) {
        const int wid = t >> 6;
        if ((t & 63) == 0) {
            r_ok[wid] = bok;
            r_lf[wid] = blf;
            r_eo[wid] = e_own;
            r_lp[wid] = loop;
        }
        __syncthreads();
        if (li == 0) {
            for (int w2 = wid + 1; w2 < wid + WPG; ++w2) {
                if (r_ok[w2] > bok || (r_ok[w2] == bok && r_lf[w2] < blf)) {
                    bok = r_ok[w2];
                    blf = r_lf[w2];
                }
                e_own += r_eo[w2];
                loop += r_lp[w2];
            }
        }
    }
    if (li == 0 && live) {
        a.c_nxt[v] = cpt_decide(a.singlet, tw, ci, own_hi, di, (int64_t)e_own, bok != 0,
                                (int64_t)(bok ^ 0x8000000000000000ull), (int32_t)(blf >> 1), (blf & 1u) != 0);
        a.e_self[v] = e_own + loop;
    }
}

// The LDS cells a lane group writes become visible to the whole group: a
// workgroup barrier when the group spans several wavefronts (G > 64,
// uniform over the workgroup), else a wavefront-scope fence, since a
// wavefront's LDS accesses complete in order and no other wavefront touches
// its groups' cells.  Wavefronts whose groups are their own then never wait
// for the workgroup's slowest one.
__device__ __forceinline__ void group_sync(int G) {
    if (G > 64) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// All packed classes in one launch: workgroups [bo[c], bo[c+1]) take class
// c (S = 16 << c slots per table, G = S/SPL lanes per vertex, 16 SPL >> c
// vertices per workgroup, 256 SPL table slots in all), otherwise as
// k_cpt_group.  SPL (slots per lane, 2, 4 or 8) trades lanes per vertex for
// work per lane: each lane scores SPL slots and takes at most
// ceil(2 SPL / 3) entries of its row.
struct GroupBlocks {
    int64_t bo[kGroupClasses + 1];     // first workgroup of every class
    int64_t cstart[kGroupClasses + 1]; // first row of every class in the class list
};

template <int SPL, int VPG, typename W>
__global__ __launch_bounds__(256) void k_cpt_groups(CArgs a, const int32_t *__restrict__ list,
                                                    const uint64_t *__restrict__ info, GroupBlocks gb) {
    if (single_done(a.gid, a.st)) return;
    static_assert(SPL == 2 || SPL == 4 || SPL == 8, "2, 4 or 8 slots per lane");
    static_assert(VPG == 1 || VPG == 2, "one or two vertices per lane group");
    constexpr int LB = SPL == 2 ? 1 : SPL == 4 ? 2 : 3;   // log2 SPL
    constexpr int U = (2 * SPL + 2) / 3;     // entries per lane at most
    __shared__ int32_t s_key[VPG * 256 * SPL];
    __shared__ uint32_t s_e[VPG * 256 * SPL], s_hi[VPG * 256 * SPL];
    __shared__ unsigned long long r_ok[VPG][4];
    __shared__ uint32_t r_lf[VPG][4];
    // e_{i->c_i} and the loop weight of every vertex of the workgroup: each
    // has one writer (one table slot holds c_i, a row has at most one loop)
    __shared__ uint32_t s_eown[VPG * 128], s_loop[VPG * 128];
    const int t = threadIdx.x;
    int c = 0;
    while (c < kGroupClasses - 1 && (int64_t)blockIdx.x >= gb.bo[c + 1]) ++c;
    const int bits = 4 + c;                  // log2 S
    const int G = (16 >> LB) << c;
    const int NV = (16 * SPL) >> c;          // lane groups per workgroup
    const int kv = t >> (4 - LB + c), li = t & (G - 1);
    const int S = 16 << c;
    // lane group kv sweeps vertices k0 + kv + j * NV, j < VPG, interleaved
    int32_t *key[VPG];
    uint32_t *es[VPG], *hs[VPG];
#pragma unroll
    for (int j = 0; j < VPG; ++j) {
        key[j] = s_key + (j * NV + kv) * S;
        es[j] = s_e + (j * NV + kv) * S;
        hs[j] = s_hi + (j * NV + kv) * S;
        if (!a.first) {   // the first pass from singletons uses no table
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                key[j][li + q * G] = kEmpty;   // lane-consecutive words: no bank conflicts
                es[j][li + q * G] = 0;
            }
        }
        if (li == 0) {
            s_eown[j * NV + kv] = 0;
            s_loop[j * NV + kv] = 0;
        }
    }
    const int64_t k0 = gb.cstart[c] + ((int64_t)blockIdx.x - gb.bo[c]) * NV * VPG;
    bool live[VPG];
    int32_t v[VPG];
    int g[VPG];
    int64_t rs[VPG], d[VPG];
#pragma unroll
    for (int j = 0; j < VPG; ++j) {
        const int64_t k = k0 + kv + (int64_t)j * NV;
        live[j] = false;
        v[j] = 0;
        g[j] = 0;
        rs[j] = 0;
        d[j] = 0;
        if (k < gb.cstart[c + 1]) {
            v[j] = list[k];
            const uint64_t ri = info[k];
            g[j] = graph_of(a.gid, v[j]);
            live[j] = !a.st[g[j]].done;
            if (live[j]) {
                rs[j] = info_start(ri);
                d[j] = info_len(ri);
            }
        }
    }
    // A class-c row has d <= 2S/3 entries, at most U per lane: the loads and
    // gathers of all of a lane's entries are issued before the first insert.
    int32_t jq[VPG][U];
    uint32_t wq[VPG][U];
    uint64_t nq[VPG][U];
#pragma unroll
    for (int j = 0; j < VPG; ++j) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t x = li + (int64_t)q * G;
            jq[j][q] = v[j];
            wq[j][q] = 0;
            if (x < d[j]) {
                jq[j][q] = a.col[rs[j] + x];
                wq[j][q] = cw<W>(a.w, rs[j] + x);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < VPG; ++j)
#pragma unroll
        for (int q = 0; q < U; ++q) {
            nq[j][q] = 0;
            if (jq[j][q] != v[j]) nq[j][q] = a.vw[jq[j][q]];
        }
    // TW, delta_i, deg_C and e_{i->C} are below 2^31 here: scores are
    // products of 32-bit operands
    int32_t ci[VPG];
    uint32_t own_hi[VPG], di[VPG], tw[VPG];
#pragma unroll
    for (int j = 0; j < VPG; ++j) {
        ci[j] = -1;
        own_hi[j] = 0;
        di[j] = 0;
        tw[j] = 0;
        if (live[j]) {
            const uint64_t own = a.vw[v[j]];
            ci[j] = vw_label(own);
            own_hi[j] = (uint32_t)(own >> 32);
            di[j] = (uint32_t)a.delta[v[j]];
            tw[j] = (uint32_t)a.tw[g[j]];
        }
    }
    group_sync(G);
    unsigned long long bok[VPG];
    uint32_t blf[VPG];
#pragma unroll
    for (int j = 0; j < VPG; ++j) {
        bok[j] = 0;
        blf[j] = 0xffffffffu;
    }
    if (a.first) {
        // singletons: every neighbour is its own community (e = the entry's
        // weight, columns are distinct), so entries are scored directly
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int j = 0; j < VPG; ++j) {
                if (jq[j][q] == v[j]) {
                    if (wq[j][q]) s_loop[j * NV + kv] = wq[j][q];
                    continue;
                }
                const uint32_t hi = (uint32_t)(nq[j][q] >> 32);
                const unsigned long long ok =
                    ((uint64_t)tw[j] * wq[j][q] - (uint64_t)di[j] * hi_deg(hi)) ^ 0x8000000000000000ull;
                const uint32_t lf = ((uint32_t)vw_label(nq[j][q]) << 1) | (hi_single(hi) ? 1u : 0u);
                best_take(bok[j], blf[j], (uint32_t)ok, (uint32_t)(ok >> 32), lf);
            }
    } else {
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int j = 0; j < VPG; ++j) {
                if (jq[j][q] == v[j]) {
                    if (wq[j][q]) s_loop[j * NV + kv] = wq[j][q];
                } else
                    grp_insert(key[j], es[j], hs[j], bits, vw_label(nq[j][q]), wq[j][q], (uint32_t)(nq[j][q] >> 32));
            }
    }
#pragma unroll
    for (int j = 0; j < VPG; ++j)
        for (int64_t x = li + (int64_t)U * G; x < d[j]; x += G) {   // not reached for class rows
            const int32_t nb = a.col[rs[j] + x];
            const uint32_t w = cw<W>(a.w, rs[j] + x);
            if (nb == v[j]) {
                s_loop[j * NV + kv] = w;
                continue;
            }
            const uint64_t nw = a.vw[nb];
            if (a.first) {
                const uint32_t hi = (uint32_t)(nw >> 32);
                const unsigned long long ok =
                    ((uint64_t)tw[j] * w - (uint64_t)di[j] * hi_deg(hi)) ^ 0x8000000000000000ull;
                best_take(bok[j], blf[j], (uint32_t)ok, (uint32_t)(ok >> 32),
                          ((uint32_t)vw_label(nw) << 1) | (hi_single(hi) ? 1u : 0u));
            } else {
                grp_insert(key[j], es[j], hs[j], bits, vw_label(nw), w, (uint32_t)(nw >> 32));
            }
        }
    group_sync(G);
#pragma unroll
    for (int j = 0; j < VPG; ++j) {
        if (a.first) break;
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const int x = li + q * G;
            const int32_t kk = key[j][x];
            if (kk == kEmpty) continue;
            const uint32_t e = es[j][x];
            if (kk == ci[j]) {
                s_eown[j * NV + kv] = e;
                continue;
            }
            const uint32_t hi = hs[j][x];
            // TW e - delta_i deg_C as a two's complement word, its sign bit
            // flipped so that unsigned order is signed order
            const unsigned long long ok =
                ((uint64_t)tw[j] * e - (uint64_t)di[j] * hi_deg(hi)) ^ 0x8000000000000000ull;
            const uint32_t lf = ((uint32_t)kk << 1) | (hi_single(hi) ? 1u : 0u);
            best_take(bok[j], blf[j], (uint32_t)ok, (uint32_t)(ok >> 32), lf);
        }
    }
    const int GW = G < 64 ? G : 64;
#pragma unroll
    for (int j = 0; j < VPG; ++j) group_best(bok[j], blf[j], GW);
    if (G > 64) {   // uniform over the workgroup: the class is
        const int wid = t >> 6;
        if ((t & 63) == 0) {
#pragma unroll
            for (int j = 0; j < VPG; ++j) {
                r_ok[j][wid] = bok[j];
                r_lf[j][wid] = blf[j];
            }
        }
        __syncthreads();
        if (li == 0) {
#pragma unroll
            for (int j = 0; j < VPG; ++j)
                for (int w2 = wid + 1; w2 < wid + G / 64; ++w2) {
                    if (r_ok[j][w2] > bok[j] || (r_ok[j][w2] == bok[j] && r_lf[j][w2] < blf[j])) {
                        bok[j] = r_ok[j][w2];
                        blf[j] = r_lf[j][w2];
                    }
                }
        }
    } else {
        group_sync(G);   // the cells written above, visible to lane 0
    }
    if (li == 0) {
#pragma unroll
        for (int j = 0; j < VPG; ++j) {
            if (!live[j]) continue;
            const uint32_t e_own = s_eown[j * NV + kv];
            a.c_nxt[v[j]] = cpt_decide(a.singlet, (int64_t)tw[j], ci[j], own_hi[j], (int64_t)di[j], (int64_t)e_own,
                                       bok[j] != 0, (int64_t)(bok[j] ^ 0x8000000000000000ull),
                                       (int32_t)(blf[j] >> 1), (blf[j] & 1u) != 0);
            a.e_self[v[j]] = e_own + s_loop[j * NV + kv];
        }
    }
}

// The packed classes with software pipelining across tiles: workgroup w of
// class c sweeps tiles [w * TPW, (w + 1) * TPW) of the class (a tile = one
// lane group per vertex, NV vertices, as in k_cpt_groups with one vertex
// per group).  While tile j's neighbours' published words are gathered, the
// columns and weights of tile j + 1 and the class-list words of tile j + 2
// are already in flight, so the three dependent loads of a tile overlap
// with the work of the tiles before it.  Every vertex is decided exactly as
// in k_cpt_groups.
struct PipeBlocks {
    int64_t bo[kGroupClasses + 1];     // first workgroup of every class
    int64_t cstart[kGroupClasses + 1]; // first row of every class in the class list
    int tpw;                           // tiles per workgroup
};

template <int SPL, typename W>
__global__ __launch_bounds__(256) void k_cpt_groups_pipe(CArgs a, const int32_t *__restrict__ list,
                                                         const uint64_t *__restrict__ info, PipeBlocks pb) {
    if (single_done(a.gid, a.st)) return;
    static_assert(SPL == 2 || SPL == 4 || SPL == 8, "2, 4 or 8 slots per lane");
    constexpr int LB = SPL == 2 ? 1 : SPL == 4 ? 2 : 3;   // log2 SPL
    constexpr int U = (2 * SPL + 2) / 3;     // entries per lane at most
    __shared__ int32_t s_key[256 * SPL];
    __shared__ uint32_t s_e[256 * SPL], s_hi[256 * SPL];
    __shared__ unsigned long long r_ok[4];
    __shared__ uint32_t r_lf[4];
    __shared__ uint32_t s_eown[128], s_loop[128];
    const int t = threadIdx.x;
    int c = 0;
    while (c < kGroupClasses - 1 && (int64_t)blockIdx.x >= pb.bo[c + 1]) ++c;
    const int bits = 4 + c;
    const int G = (16 >> LB) << c;
    const int NV = (16 * SPL) >> c;
    const int kv = t >> (4 - LB + c), li = t & (G - 1);
    const int S = 16 << c;
    int32_t *key = s_key + kv * S;
    uint32_t *es = s_e + kv * S, *hs = s_hi + kv * S;
    const int64_t cend = pb.cstart[c + 1];
    const int64_t tile0 = ((int64_t)blockIdx.x - pb.bo[c]) * pb.tpw;
    const int64_t ntile = (cend - pb.cstart[c] + NV - 1) / NV;
    const int64_t tiles = ntile - tile0 < pb.tpw ? ntile - tile0 : pb.tpw;
    // pipeline registers: row k of the class list for tiles j + 1 (entries
    // loaded) and j + 2 (list words loaded)
    auto row_of = [&](int64_t j) { return pb.cstart[c] + j * NV + kv; };
    int32_t v1 = 0, v2 = 0;
    uint64_t ri1 = 0, ri2 = 0;
    {
        const int64_t k = row_of(tile0);
        if (k < cend) {
            v1 = list[k];
            ri1 = info[k];
        } else {
            ri1 = 0;
        }
        const int64_t k2 = row_of(tile0 + 1);
        if (tiles > 1 && k2 < cend) {
            v2 = list[k2];
            ri2 = info[k2];
        }
    }
    int32_t jn[U];
    uint32_t wn[U];
    // entries of the first tile
    {
        const int64_t rs = info_start(ri1), d = info_len(ri1);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t x = li + (int64_t)q * G;
            jn[q] = v1;
            wn[q] = 0;
            if (x < d) {
                jn[q] = a.col[rs + x];
                wn[q] = cw<W>(a.w, rs + x);
            }
        }
    }
    for (int64_t j = 0; j < tiles; ++j) {
        // this tile: vertex v, its row (entries in jq / wq)
        const int64_t k = row_of(tile0 + j);
        const int32_t v = v1;
        const uint64_t ri = ri1;
        int32_t jq[U];
        uint32_t wq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            jq[q] = jn[q];
            wq[q] = wn[q];
        }
        bool live = false;
        int g = 0;
        int64_t d = 0;
        if (k < cend) {
            g = graph_of(a.gid, v);
            live = !a.st[g].done;
            d = live ? info_len(ri) : 0;
        }
        // gathers of this tile
        uint64_t nq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            nq[q] = 0;
            if ((int64_t)(li + q * G) < d && jq[q] != v) nq[q] = a.vw[jq[q]];
        }
        int32_t ci = -1;
        uint32_t own_hi = 0, di = 0, tw = 0;
        if (live) {
            const uint64_t own = a.vw[v];
            ci = vw_label(own);
            own_hi = (uint32_t)(own >> 32);
            di = (uint32_t)a.delta[v];
            tw = (uint32_t)a.tw[g];
        }
        // entries of the next tile, list words of the one after
        v1 = v2;
        ri1 = ri2;
        if (j + 1 < tiles) {
            const int64_t rs = info_start(ri1), dn = info_len(ri1);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int64_t x = li + (int64_t)q * G;
                jn[q] = v1;
                wn[q] = 0;
                if (x < dn) {
                    jn[q] = a.col[rs + x];
                    wn[q] = cw<W>(a.w, rs + x);
                }
            }
            const int64_t k2 = row_of(tile0 + j + 2);
            ri2 = 0;
            if (j + 2 < tiles && k2 < cend) {
                v2 = list[k2];
                ri2 = info[k2];
            }
        }
        // the previous tile's scoring is finished: the tables may be reused
        __syncthreads();
        if (!a.first) {
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                key[li + q * G] = kEmpty;
                es[li + q * G] = 0;
            }
        }
        if (li == 0) {
            s_eown[kv] = 0;
            s_loop[kv] = 0;
        }
        __syncthreads();
        unsigned long long bok = 0;
        uint32_t blf = 0xffffffffu;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if ((int64_t)(li + q * G) >= d) continue;
            if (jq[q] == v) {
                if (wq[q]) s_loop[kv] = wq[q];
                continue;
            }
            const uint32_t hi = (uint32_t)(nq[q] >> 32);
            if (a.first) {
                const unsigned long long ok =
                    ((uint64_t)tw * wq[q] - (uint64_t)di * hi_deg(hi)) ^ 0x8000000000000000ull;
                best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32),
                          ((uint32_t)vw_label(nq[q]) << 1) | (hi_single(hi) ? 1u : 0u));
            } else {
                grp_insert(key, es, hs, bits, vw_label(nq[q]), wq[q], hi);
            }
        }
        __syncthreads();
        if (!a.first) {
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                const int x = li + q * G;
                const int32_t kk = key[x];
                if (kk == kEmpty) continue;
                const uint32_t e = es[x];
                if (kk == ci) {
                    s_eown[kv] = e;
                    continue;
                }
                const uint32_t hi = hs[x];
                const unsigned long long ok =
                    ((uint64_t)tw * e - (uint64_t)di * hi_deg(hi)) ^ 0x8000000000000000ull;
                best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32), ((uint32_t)kk << 1) | (hi_single(hi) ? 1u : 0u));
            }
        }
        const int GW = G < 64 ? G : 64;
        group_best(bok, blf, GW);
        if (G > 64) {   // uniform over the workgroup: the class is
            const int wid = t >> 6;
            if ((t & 63) == 0) {
                r_ok[wid] = bok;
                r_lf[wid] = blf;
            }
            __syncthreads();
            if (li == 0)
                for (int w2 = wid + 1; w2 < wid + G / 64; ++w2)
                    if (r_ok[w2] > bok || (r_ok[w2] == bok && r_lf[w2] < blf)) {
                        bok = r_ok[w2];
                        blf = r_lf[w2];
                    }
        } else {
            // the group's lanes are in one wavefront: its LDS accesses complete
            // in order, so the cells written above are visible to lane 0
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (li == 0 && live) {
            const uint32_t e_own = s_eown[kv];
            a.c_nxt[v] = cpt_decide(a.singlet, (int64_t)tw, ci, own_hi, (int64_t)di, (int64_t)e_own, bok != 0,
                                    (int64_t)(bok ^ 0x8000000000000000ull), (int32_t)(blf >> 1), (blf & 1u) != 0);
            a.e_self[v] = e_own + s_loop[kv];
        }
    }
}

// Table-size class of a row swept from LDS: the smallest packed class c
// with 3d <= 2 * (16 << c), else 2048, 4096 or 16384 slots.
__device__ __forceinline__ int size_class(int64_t d) {
    int c = 0;
    while (c < kGroupClasses && 3 * d > 2 * ((int64_t)16 << c)) ++c;
    if (c < kGroupClasses) return c;
    if (3 * d <= 2 * 2048) return kGroupClasses;
    return 3 * d <= 2 * 4096 ? kGroupClasses + 1 : kGroupClasses + 2;
}

// Rows of up to kCompactBlockMax entries, one 1,024-thread workgroup each
// with a table of S = 16384 slots (key and e_{i->C} only: 128 KB of LDS);
// the degree and size of each candidate community come from its community
// word at scoring time.  Otherwise as k_cpt_group.
constexpr int kBigRowSlots = 16384;
constexpr int kBigRowThreads = 1024;

template <typename W>
__global__ __launch_bounds__(kBigRowThreads) void k_cpt_bigrow(CArgs a, const int32_t *__restrict__ list,
                                                               const uint64_t *__restrict__ info, int64_t count) {
    if (single_done(a.gid, a.st)) return;
    constexpr int S = kBigRowSlots, T = kBigRowThreads, SPL = S / T, NW = T / 64;
    constexpr int BITS = Log2<S>::value;
    __shared__ int32_t key[S];
    __shared__ uint32_t es[S];
    __shared__ unsigned long long r_ok[NW];
    __shared__ uint32_t r_lf[NW];
    __shared__ uint32_t s_eown, s_loop;
    const int t = threadIdx.x;
    if (!a.first) {   // the first pass from singletons uses no table
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            key[t + q * T] = kEmpty;
            es[t + q * T] = 0;
        }
    }
    if (t == 0) {
        s_eown = 0;
        s_loop = 0;
    }
    const int64_t k = blockIdx.x;
    const int32_t v = list[k];
    const uint64_t ri = info[k];
    const int g = graph_of(a.gid, v);
    const bool live = !a.st[g].done;
    const int64_t rs = info_start(ri), d = live ? info_len(ri) : 0;
    const uint64_t own = a.vw[v];
    const int32_t ci = vw_label(own);
    const uint32_t own_hi = (uint32_t)(own >> 32);
    // TW, delta_i, deg_C and e_{i->C} are below 2^31: 32-bit operands
    const uint32_t di = (uint32_t)a.delta[v];
    const uint32_t tw = (uint32_t)a.tw[g];
    __syncthreads();
    unsigned long long bok = 0;
    uint32_t blf = 0xffffffffu;
    constexpr int U = 4;
    for (int64_t x0 = t; x0 < d; x0 += (int64_t)U * T) {
        int32_t jq[U];
        uint32_t wq[U];
        int32_t lq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t x = x0 + (int64_t)q * T;
            jq[q] = -1;
            wq[q] = 0;
            if (x < d) {
                jq[q] = a.col[rs + x];
                wq[q] = cw<W>(a.w, rs + x);
            }
        }
        uint64_t nq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            nq[q] = (jq[q] >= 0 && jq[q] != v) ? a.vw[jq[q]] : 0;
            lq[q] = (jq[q] >= 0 && jq[q] != v) ? vw_label(nq[q]) : -1;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (jq[q] == v) s_loop = wq[q];   // a row has at most one loop
            if (lq[q] < 0) continue;
            if (a.first) {   // singletons: the entry is its own candidate
                const uint32_t hi = (uint32_t)(nq[q] >> 32);
                const unsigned long long ok =
                    ((uint64_t)tw * wq[q] - (uint64_t)di * hi_deg(hi)) ^ 0x8000000000000000ull;
                best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32),
                          ((uint32_t)lq[q] << 1) | (hi_single(hi) ? 1u : 0u));
                continue;
            }
            uint32_t h = ((uint32_t)lq[q] * 0x9E3779B1u) >> (32 - BITS);
            while (true) {
                const int32_t prev = atomicCAS(&key[h], kEmpty, lq[q]);   // claims, or returns the slot's key
                if (prev == kEmpty || prev == lq[q]) break;
                h = (h + 1) & (S - 1);
            }
            atomicAdd(&es[h], wq[q]);
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < SPL; ++q) {
        if (a.first) break;
        const int x = t + q * T;
        const int32_t kk = key[x];
        if (kk == kEmpty) continue;
        const uint32_t e = es[x];
        if (kk == ci) {
            s_eown = e;
            continue;
        }
        const uint64_t dsk = a.ds[kk];
        const unsigned long long ok = ((uint64_t)tw * e - (uint64_t)di * (uint32_t)dsk) ^ 0x8000000000000000ull;
        const uint32_t lf = ((uint32_t)kk << 1) | ((dsk >> 32) == 1 ? 1u : 0u);
        best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32), lf);
    }
    group_best(bok, blf, 64);
    const int wid = t >> 6;
    if ((t & 63) == 0) {
        r_ok[wid] = bok;
        r_lf[wid] = blf;
    }
    __syncthreads();
    if (t == 0 && live) {
        for (int w2 = 1; w2 < NW; ++w2) best_take(bok, blf, (uint32_t)r_ok[w2], (uint32_t)(r_ok[w2] >> 32), r_lf[w2]);
        a.c_nxt[v] = cpt_decide(a.singlet, (int64_t)tw, ci, own_hi, (int64_t)di, (int64_t)s_eown, bok != 0,
                                (int64_t)(bok ^ 0x8000000000000000ull), (int32_t)(blf >> 1), (blf & 1u) != 0);
        a.e_self[v] = s_eown + s_loop;
    }
}

constexpr int kClassTile = 2048;

__global__ __launch_bounds__(256) void k_class_count(const int64_t *__restrict__ rp, const int32_t *__restrict__ list,
                                                     int64_t m, int32_t *counts, int64_t nblocks,
                                                     unsigned long long *cls_nnz) {
    __shared__ int cnt[kLdsClasses];
    __shared__ unsigned long long ecnt[kLdsClasses];
    if (threadIdx.x < kLdsClasses) {
        cnt[threadIdx.x] = 0;
        ecnt[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kClassTile;
    for (int k = 0; k < kClassTile / 256; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i >= m) break;
        const int32_t v = list[i];
        const int64_t d = rp[v + 1] - rp[v];
        const int c = size_class(d);
        atomicAdd(&cnt[c], 1);
        atomicAdd(&ecnt[c], (unsigned long long)d);
    }
    __syncthreads();
    if (threadIdx.x < kLdsClasses) {
        counts[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
        if (ecnt[threadIdx.x]) atomicAdd(&cls_nnz[threadIdx.x], ecnt[threadIdx.x]);
    }
}

// Stable scatter of the packed rows into their classes.
__global__ __launch_bounds__(256) void k_class_scatter(const int64_t *__restrict__ rp, const int32_t *__restrict__ list,
                                                       int64_t m, const int32_t *__restrict__ offs, int64_t nblocks,
                                                       int32_t *out, uint64_t *info) {
    __shared__ int run[kLdsClasses];
    __shared__ int wc[4][kLdsClasses];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t < kLdsClasses) run[t] = offs[t * nblocks + blockIdx.x];
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kClassTile;
    for (int k = 0; k < kClassTile / 256; ++k) {
        const int64_t i = base + k * 256 + t;
        int32_t v = 0;
        int c = -1;
        int64_t rs = 0, d = 0;
        if (i < m) {
            v = list[i];
            rs = rp[v];
            d = rp[v + 1] - rs;
            c = size_class(d);
        }
        int rank = 0;
#pragma unroll
        for (int cc = 0; cc < kLdsClasses; ++cc) {
            const unsigned long long msk = __ballot(c == cc);
            if (c == cc) rank = __popcll(msk & lt);
            if (lane == 0) wc[wid][cc] = __popcll(msk);
        }
        __syncthreads();
        if (c >= 0) {
            int pos = run[c] + rank;
            for (int w2 = 0; w2 < wid; ++w2) pos += wc[w2][c];
            out[pos] = v;
            info[pos] = row_info(rs, d);
        }
        __syncthreads();
        if (t < kLdsClasses) run[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ hubs --

struct CHub {
    const int32_t *v;
    const int64_t *tab_off, *chunk_off, *scan_off, *tab_size;
    const int32_t *chunk_hub, *scan_hub;
    int64_t hubs;
    const int64_t *bkt_off, *reg_off;   // first bucket and first pair slot of each hub (no buckets: table only)
    const int32_t *bkt_hub;             // hub of each bucket
    int shrink;                         // bucket sizes divided by this (1; more only to test the spills)
    unsigned long long *bkey;           // bucket regions: table words (label + 1) << 32 | e
    unsigned int *bcur;                 // words appended to each bucket
    uint64_t *bpart;                    // per bucket: a partial as the scan's
    unsigned int *spill;                // per hub: a bucket went to the table
};

constexpr int kCHubLdsBits = 11;
constexpr unsigned long long kTagMask = 0xffffffff00000000ull;

// Hub tables hold one word per slot: (label + 1) << 32 | e, 0 = empty
// (labels are below 2^31 and e below TW < 2^31, so the add never carries
// into the tag).  Insert or add x for a label into an LDS table of `size`
// slots, probing from slot h.
__device__ __forceinline__ void word_insert(unsigned long long *tab, uint64_t size, uint64_t h, int32_t label,
                                            uint32_t x) {
    const unsigned long long tag = (unsigned long long)(uint32_t)(label + 1) << 32;
    while (true) {
        // the compare-and-swap claims an empty slot, or returns its word
        const unsigned long long prev = atomicCAS(&tab[h], 0ull, tag | x);
        if (prev == 0) return;
        if ((prev & kTagMask) == tag) {
            atomicAdd(&tab[h], (unsigned long long)x);
            return;
        }
        h = (h + 1 == size) ? 0 : h + 1;
    }
}

// The same in an HBM table: a plain read first, so that a slot already
// holding the label takes one add whose result is not waited for.
__device__ __forceinline__ void word_insert_hbm(unsigned long long *tab, uint64_t size, uint64_t h, int32_t label,
                                                uint32_t x) {
    const unsigned long long tag = (unsigned long long)(uint32_t)(label + 1) << 32;
    while (true) {
        const unsigned long long cur = ((volatile unsigned long long *)tab)[h];
        if ((cur & kTagMask) == tag) {
            atomicAdd(&tab[h], (unsigned long long)x);
            return;
        }
        if (cur == 0) {
            const unsigned long long prev = atomicCAS(&tab[h], 0ull, tag | x);
            if (prev == 0) return;
            if ((prev & kTagMask) == tag) {
                atomicAdd(&tab[h], (unsigned long long)x);
                return;
            }
        }
        h = (h + 1 == size) ? 0 : h + 1;
    }
}

// Workgroup per kHubChunk entries of a hub row: LDS pre-aggregation of
// label -> e, then one HBM table insert per distinct label.
template <typename W>
__global__ __launch_bounds__(256) void k_cpt_hub_accum(CArgs a, CHub hm, unsigned long long *gtab,
                                                       unsigned long long *hub_loop, uint64_t *part) {
    if (single_done(a.gid, a.st)) return;
    constexpr int T = 1 << kCHubLdsBits;
    __shared__ unsigned long long s_tab[T];
    __shared__ unsigned int s_cnt[kBktMax], s_base[kBktMax];
    __shared__ unsigned long long r_ok[4];
    __shared__ uint32_t r_lf[4];
    __shared__ int64_t s_h;
    const int t = threadIdx.x;
    if (t == 0) s_h = hm.chunk_hub[blockIdx.x];
    if (!a.first)
        for (int x = t; x < T; x += 256) s_tab[x] = 0;
    __syncthreads();
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int g = graph_of(a.gid, v);
    if (a.st[g].done) return;   // uniform over the workgroup
    const int64_t k = (int64_t)blockIdx.x - hm.chunk_off[h];
    const int64_t row_end = a.row_ptr[v + 1];
    const int64_t rs = a.row_ptr[v] + k * kHubChunk;
    const int64_t re = rs + kHubChunk < row_end ? rs + kHubChunk : row_end;
    // kHubChunk / 256 entries per lane: loads and gathers first, then inserts.
    constexpr int U = kHubChunk / 256;
    static_assert(kHubChunk % 256 == 0, "a chunk is whole rounds of the workgroup");
    int32_t jq[U];
    uint32_t wq[U];
    uint64_t nq[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int64_t e = rs + t + q * 256;
        jq[q] = -1;
        wq[q] = 0;
        if (e < re) {
            jq[q] = a.col[e];
            wq[q] = cw<W>(a.w, e);
        }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) nq[q] = (jq[q] >= 0 && jq[q] != v) ? a.vw[jq[q]] : 0;
    uint32_t loop = 0;
#pragma unroll
    for (int q = 0; q < U; ++q)
        if (jq[q] == v) loop += wq[q];
    if (loop) atomicAdd(&hub_loop[h], (unsigned long long)loop);
    if (a.first) {
        // singletons: every entry is its own candidate; the chunk's best goes
        // to its partial (decided over the hub's chunks), no tables
        const uint32_t di = (uint32_t)a.delta[v], tw = (uint32_t)a.tw[g];
        unsigned long long bok = 0;
        uint32_t blf = 0xffffffffu;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (jq[q] < 0 || jq[q] == v) continue;
            const uint32_t hi = (uint32_t)(nq[q] >> 32);
            const unsigned long long ok = ((uint64_t)tw * wq[q] - (uint64_t)di * hi_deg(hi)) ^ 0x8000000000000000ull;
            best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32),
                      ((uint32_t)vw_label(nq[q]) << 1) | (hi_single(hi) ? 1u : 0u));
        }
        group_best(bok, blf, 64);
        const int wid = t >> 6;
        if ((t & 63) == 0) {
            r_ok[wid] = bok;
            r_lf[wid] = blf;
        }
        __syncthreads();
        if (t == 0) {
            for (int w2 = 1; w2 < 4; ++w2)
                best_take(bok, blf, (uint32_t)r_ok[w2], (uint32_t)(r_ok[w2] >> 32), r_lf[w2]);
            uint64_t *p = part + 4 * (int64_t)blockIdx.x;
            p[0] = bok;
            p[1] = (uint64_t)(blf >> 1) | ((uint64_t)(blf & 1u) << 32);
            p[2] = 0;
            p[3] = 0;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
        if (jq[q] < 0 || jq[q] == v) continue;
        const int32_t l = vw_label(nq[q]);
        word_insert(s_tab, T, ((uint32_t)l * 0x9E3779B1u) >> (32 - kCHubLdsBits), l, wq[q]);
    }
    __syncthreads();
    const int64_t base = hm.tab_off[h], size = hm.tab_size[h];
    const int64_t b0 = hm.bkt_off[h], P = hm.bkt_off[h + 1] - b0;
    if (P == 0) {   // the hub's table
        for (int x = t; x < T; x += 256) {
            const unsigned long long wd = s_tab[x];
            if (wd == 0) continue;
            const int32_t l = (int32_t)(wd >> 32) - 1;
            word_insert_hbm(gtab + base, (uint64_t)size, hash_range(l, (uint64_t)size), l, (uint32_t)wd);
        }
        return;
    }
    // buckets: every distinct label's rank among the workgroup's labels of
    // its bucket, then one cursor add per bucket (as on the general levels)
    for (int b = t; b < P; b += 256) s_cnt[b] = 0;
    __syncthreads();
    constexpr int Q = T / 256;
    int32_t bq[Q];
    uint32_t rq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const unsigned long long wd = s_tab[t + q * 256];
        bq[q] = -1;
        rq[q] = 0;
        if (wd != 0) {
            bq[q] = (int32_t)bkt_of((int32_t)(wd >> 32) - 1, P);
            rq[q] = atomicAdd(&s_cnt[bq[q]], 1u);
        }
    }
    __syncthreads();
    for (int b = t; b < P; b += 256) s_base[b] = s_cnt[b] ? atomicAdd(&hm.bcur[b0 + b], s_cnt[b]) : 0u;
    __syncthreads();
    const int64_t cap = bkt_cap(row_end - a.row_ptr[v], P, hm.shrink);
    bool over = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (bq[q] < 0) continue;
        const unsigned long long wd = s_tab[t + q * 256];
        const int64_t pos = (int64_t)s_base[bq[q]] + rq[q];
        if (pos < cap) {
            hm.bkey[hm.reg_off[h] + (int64_t)bq[q] * cap + pos] = wd;
        } else {   // the bucket's region is full: the bucket goes to the table
            const int32_t l = (int32_t)(wd >> 32) - 1;
            word_insert_hbm(gtab + base, (uint64_t)size, hash_range(l, (uint64_t)size), l, (uint32_t)wd);
            over = true;
        }
    }
    if (over) hm.spill[h] = 1u;
}

// One workgroup per bucket of a hub: sum its words in LDS and score them
// (a partial in the scan's format), or, when its words overflowed its
// region or its table, add all of them to the hub's table instead.  Leaves
// the bucket's cursor at 0.
__global__ __launch_bounds__(256) void k_cpt_hub_bucket(CArgs a, CHub hm, unsigned long long *gtab) {
    if (single_done(a.gid, a.st)) return;
    constexpr int T = 1 << kBktBits;
    __shared__ unsigned long long s_tab[T];
    __shared__ unsigned long long r_ok[4];
    __shared__ uint32_t r_lf[4], r_e[4];
    __shared__ int64_t s_h;
    __shared__ unsigned int s_n;
    __shared__ int s_used, s_over;
    const int t = threadIdx.x;
    const int64_t bk = blockIdx.x;
    if (t == 0) {
        s_h = hm.bkt_hub[bk];
        s_n = hm.bcur[bk];
        s_used = 0;
        s_over = 0;
    }
    for (int x = t; x < T; x += 256) s_tab[x] = 0;
    __syncthreads();
    const int64_t h = s_h;
    const int32_t v = hm.v[h];
    const int g = graph_of(a.gid, v);
    const bool live = !a.st[g].done;   // uniform over the workgroup
    const int64_t b0 = hm.bkt_off[h], P = hm.bkt_off[h + 1] - b0;
    const int64_t cap = bkt_cap(a.row_ptr[v + 1] - a.row_ptr[v], P, hm.shrink);
    const int claim = kBktClaim / hm.shrink > 0 ? kBktClaim / hm.shrink : 1;
    const int64_t reg = hm.reg_off[h] + (bk - b0) * cap;
    const int64_t n = live ? (int64_t)s_n : 0;
    bool spill_all = n > cap;
    if (!spill_all) {
        bool over = false;
        for (int64_t i = t; i < n; i += 256) {
            const unsigned long long wd = hm.bkey[reg + i];
            const unsigned long long tag = wd & kTagMask;
            const uint32_t e = (uint32_t)wd;
            uint32_t x = ((uint32_t)((wd >> 32) - 1) * 0x9E3779B1u) >> (32 - kBktBits);
            while (true) {
                const unsigned long long cur = s_tab[x];
                if ((cur & kTagMask) == tag) {
                    atomicAdd(&s_tab[x], (unsigned long long)e);
                    break;
                }
                if (cur == 0) {
                    if (s_used >= claim) {
                        over = true;
                        break;
                    }
                    const unsigned long long prev = atomicCAS(&s_tab[x], 0ull, wd);
                    if (prev == 0) {
                        atomicAdd(&s_used, 1);
                        break;
                    }
                    if ((prev & kTagMask) == tag) {
                        atomicAdd(&s_tab[x], (unsigned long long)e);
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
    unsigned long long bok = 0;
    uint32_t blf = 0xffffffffu;
    uint32_t e_own = 0;
    if (spill_all) {
        const int64_t m = n < cap ? n : cap;
        const int64_t base = hm.tab_off[h], size = hm.tab_size[h];
        for (int64_t i = t; i < m; i += 256) {
            const unsigned long long wd = hm.bkey[reg + i];
            const int32_t l = (int32_t)(wd >> 32) - 1;
            word_insert_hbm(gtab + base, (uint64_t)size, hash_range(l, (uint64_t)size), l, (uint32_t)wd);
        }
        if (t == 0) hm.spill[h] = 1u;
    } else if (live) {
        const int32_t ci = vw_label(a.vw[v]);
        // TW, delta_i, deg_C and e_{i->C} are below 2^31: 32-bit operands
        const uint32_t di = (uint32_t)a.delta[v];
        const uint32_t tw = (uint32_t)a.tw[g];
        for (int x = t; x < T; x += 256) {
            const unsigned long long wd = s_tab[x];
            if (wd == 0) continue;
            const int32_t k = (int32_t)(wd >> 32) - 1;
            const uint32_t e = (uint32_t)wd;
            if (k == ci) {
                e_own += e;
                continue;
            }
            const uint64_t dsk = a.ds[k];
            const unsigned long long ok = ((uint64_t)tw * e - (uint64_t)di * (uint32_t)dsk) ^ 0x8000000000000000ull;
            const uint32_t lf = ((uint32_t)k << 1) | ((dsk >> 32) == 1 ? 1u : 0u);
            best_take(bok, blf, (uint32_t)ok, (uint32_t)(ok >> 32), lf);
        }
    }
    group_best(bok, blf, 64);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e_own += __shfl_xor(e_own, off);
    const int lane = t & 63, wid = t >> 6;
    if (lane == 0) {
        r_ok[wid] = bok;
        r_lf[wid] = blf;
        r_e[wid] = e_own;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < 4; ++w) {
            best_take(bok, blf, (uint32_t)r_ok[w], (uint32_t)(r_ok[w] >> 32), r_lf[w]);
            e_own += r_e[w];
        }
        uint64_t *p = hm.bpart + 4 * bk;
        p[0] = bok;
        p[1] = (uint64_t)(blf >> 1) | ((uint64_t)(blf & 1u) << 32);
        p[2] = e_own;
        p[3] = 0;
        hm.bcur[bk] = 0u;
    }
}

// Wavefront per hub: combine the partials and decide.  On the first pass
// from singletons the partials are the chunks'; later they are the
// buckets', and a hub whose bucket spilled (or that has no bucket) also
// has pairs in its HBM table, which the wavefront scans and clears here
// (spills are rare, so no launch is spent on the tables of the others).
__global__ __launch_bounds__(256) void k_cpt_hub_decide(CArgs a, CHub hm, const uint64_t *part,
                                                        unsigned long long *hub_loop, unsigned long long *gtab) {
    if (single_done(a.gid, a.st)) return;
    const int lane = threadIdx.x & 63;
    const int64_t h = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (h >= hm.hubs) return;
    const int32_t v = hm.v[h];
    const int g = graph_of(a.gid, v);
    if (a.st[g].done) return;
    unsigned long long bok = 0;
    int32_t bl = 0x7fffffff, bf = 0;
    uint64_t e_own = 0;
    auto take = [&](const uint64_t *p) {
        const unsigned long long ok = p[0];
        const int32_t l = (int32_t)(uint32_t)p[1];
        if (ok > bok || (ok == bok && l < bl)) {
            bok = ok;
            bl = l;
            bf = (int32_t)(p[1] >> 32);
        }
        e_own += p[2];
    };
    if (a.first) {
        for (int64_t b = hm.chunk_off[h] + lane; b < hm.chunk_off[h + 1]; b += 64) take(part + 4 * b);
    } else {
        for (int64_t b = hm.bkt_off[h] + lane; b < hm.bkt_off[h + 1]; b += 64) take(hm.bpart + 4 * b);
        if (hm.bkt_off[h + 1] == hm.bkt_off[h] || hm.spill[h] != 0u) {
            // the table's pairs: (label + 1) << 32 | e per slot, 0 = empty;
            // TW, delta_i, deg_C and e_{i->C} are below 2^31 (32-bit operands)
            const int32_t ci = vw_label(a.vw[v]);
            const uint32_t di = (uint32_t)a.delta[v];
            const uint32_t tw = (uint32_t)a.tw[g];
            const int64_t t0 = hm.tab_off[h], t1 = t0 + hm.tab_size[h];
            for (int64_t x = t0 + lane; x < t1; x += 64) {
                const unsigned long long wd = gtab[x];
                if (wd == 0) continue;
                gtab[x] = 0;
                const int32_t k = (int32_t)(wd >> 32) - 1;
                const uint32_t e = (uint32_t)wd;
                if (k == ci) {
                    e_own += e;
                    continue;
                }
                const uint64_t dsk = a.ds[k];
                const unsigned long long ok = ((uint64_t)tw * e - (uint64_t)di * (uint32_t)dsk) ^ 0x8000000000000000ull;
                if (ok > bok || (ok == bok && k < bl)) {
                    bok = ok;
                    bl = k;
                    bf = (dsk >> 32) == 1 ? 1 : 0;
                }
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long ook = __shfl_xor(bok, off);
        const int32_t ol = __shfl_xor(bl, off);
        const int32_t of = __shfl_xor(bf, off);
        if (ook > bok || (ook == bok && ol < bl)) {
            bok = ook;
            bl = ol;
            bf = of;
        }
        e_own += __shfl_xor(e_own, off);
    }
    if (lane == 0) {
        hm.spill[h] = 0u;
        const uint64_t own = a.vw[v];
        const int32_t ci = vw_label(own);
        const int64_t di = a.delta[v];
        a.c_nxt[v] = cpt_decide(a.singlet, a.tw[g], ci, (uint32_t)(own >> 32), di, (int64_t)e_own, bok != 0,
                                (int64_t)(bok ^ 0x8000000000000000ull), bl, bf != 0);
        a.e_self[v] = (uint32_t)(e_own + hub_loop[h]);
        hub_loop[h] = 0;
    }
}

}  // namespace

// ------------------------------------------------------------------- host --

void compact_classes(const int64_t *rp, const int32_t *list, int64_t m, int32_t *out, uint64_t *info,
                     int64_t *cstart, int64_t *cnnz, hipStream_t s, Timer *t) {
    for (int c = 0; c <= kLdsClasses; ++c) cstart[c] = 0;
    for (int c = 0; c < kLdsClasses; ++c) cnnz[c] = 0;
    if (m <= 0) return;
    const int64_t nblk = (m + kClassTile - 1) / kClassTile;
    const int64_t cm = kLdsClasses * nblk;
    TempBuf counts((size_t)(cm + 1) * sizeof(int32_t), s);
    TempBuf enz(kLdsClasses * sizeof(unsigned long long), s);
    fill<uint64_t>(enz.as<uint64_t>(), 0, kLdsClasses, s);
    {
        TimedLaunch tl(t, TG_LEVEL, "k_class_count", (double)m * 20);
        tl.launch(k_class_count, (unsigned)nblk, 256, 0, s, rp, list, m, counts.as<int32_t>(), nblk,
                  enz.as<unsigned long long>());
        LV_LAUNCHED("k_class_count");
    }
    scan_exclusive<int32_t, int32_t>(counts.as<int32_t>(), counts.as<int32_t>(), cm, counts.as<int32_t>() + cm, s, t);
    {
        TimedLaunch tl(t, TG_LEVEL, "k_class_scatter", (double)m * 32);
        tl.launch(k_class_scatter, (unsigned)nblk, 256, 0, s, rp, list, m, counts.as<int32_t>(), nblk, out, info);
        LV_LAUNCHED("k_class_scatter");
    }
    Readback rb(s);
    const int32_t *hs[kLdsClasses];
    for (int c = 0; c < kLdsClasses; ++c) hs[c] = rb.add(counts.as<int32_t>() + (int64_t)c * nblk);
    const unsigned long long *hn = rb.add(enz.as<unsigned long long>(), kLdsClasses);
    rb.fetch();
    for (int c = 0; c < kLdsClasses; ++c) {
        cstart[c] = *hs[c];
        cnnz[c] = (int64_t)hn[c];
    }
    cstart[kLdsClasses] = m;
}

void compact_init_singletons(int32_t *c0, int32_t *c1, int32_t *c2, const int64_t *delta, uint64_t *ds, uint32_t *es,
                             int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_cpt_init_singletons<<<grid_for(n, 256), 256, 0, s>>>(c0, c1, c2, delta, ds, es, n);
    LV_LAUNCHED("k_cpt_init_singletons");
}

void compact_init_labels(int32_t *c0, int32_t *c1, int32_t *c2, const int32_t *labels, const int64_t *delta,
                         uint64_t *ds, uint32_t *es, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_cpt_init_labels<<<grid_for(n, 256), 256, 0, s>>>(c0, c1, c2, labels, delta, ds, es, n);
    LV_LAUNCHED("k_cpt_init_labels");
}

void compact_final_labels(const int32_t *c0, const int32_t *c1, const int32_t *c2, const int32_t *gid,
                          const PhaseState *st, int64_t n, int32_t *out, hipStream_t s, Timer *t) {
    if (n <= 0) return;
    TimedLaunch tl(t, TG_CONTRACT, "k_cpt_final_labels", (double)n * 12);
    tl.launch(k_cpt_final_labels, grid_for(n, 256), 256, 0, s, c0, c1, c2, gid, st, n, out);
    LV_LAUNCHED("k_cpt_final_labels");
}

void compact_expand(const uint64_t *ds, const uint32_t *es, int64_t n, int64_t *deg, int32_t *size, int64_t *e_self,
                    hipStream_t s) {
    if (n <= 0) return;
    k_cpt_expand<<<grid_for(n, 256), 256, 0, s>>>(ds, es, n, deg, size, e_self);
    LV_LAUNCHED("k_cpt_expand");
}

// The row families are independent within a pass (each reads the
// published words and writes its own rows' labels).  With side streams,
// the one-workgroup rows and the hub kernels run on them beside the rows of
// up to 341 entries on s (each family fills the others' tails; they share
// the device, so each one's own duration grows), and s waits for both.
template <typename W>
static void compact_sweeps(const CArgs &a, const CompactPass &cp, hipStream_t s, SideStreams *side, Timer *t) {
    const char *wn = type_name<W>();
    const std::string sfx = t ? std::string(wn) + ">" : std::string();
    const double eb = 12.0 + sizeof(W);  // column (4), weight, neighbour word (8)
    const double vb = 40.0;
    auto bytes = [&](int b0, int b1) {
        double x = 0;
        for (int b = b0; b < b1; ++b) x += (double)(cp.bstart[b + 1] - cp.bstart[b]) * vb + (double)cp.bnnz[b] * eb;
        return x;
    };
    const bool fork = side && (cp.hubs > 0 || cp.cstart[kLdsClasses] > cp.cstart[kGroupClasses]);
    hipStream_t s1 = s, s2 = s;
    if (fork) {
        side->fork(s);
        s1 = (*side)[0];
        s2 = (*side)[1];
    }
    if (cp.bstart[B_T16] - cp.bstart[B_T8] > 0) {
        TimedLaunch tl(t, TG_SWEEP, "k_cpt_small<", bytes(B_T8, B_T16), sfx.c_str());
        tl.launch(k_cpt_small<W>, grid_for(cp.n, 256), 256, 0, s, a, cp.n, cp.small_max);
        LV_LAUNCHED("k_cpt_small");
    }
    {
        GroupBlocks gb;
        gb.bo[0] = 0;
        double gbytes = 0;
        const int spl = cp.group_slots == 8 ? 8 : cp.group_slots == 2 ? 2 : 4;
        const int vpg = cp.group_vertices == 2 ? 2 : 1;
        for (int c = 0; c < kGroupClasses; ++c) {
            const int64_t cnt = cp.cstart[c + 1] - cp.cstart[c];
            const int nv = ((16 * spl) >> c) * vpg;
            gb.bo[c + 1] = gb.bo[c] + (cnt + nv - 1) / nv;
            gbytes += (double)cnt * vb + (double)cp.cnnz[c] * eb;
        }
        for (int c = 0; c <= kGroupClasses; ++c) gb.cstart[c] = cp.cstart[c];
        if (gb.bo[kGroupClasses] > 0 && cp.group_tiles > 1 && vpg == 1) {
            // several tiles per workgroup, software-pipelined
            PipeBlocks pbk;
            pbk.tpw = cp.group_tiles;
            pbk.bo[0] = 0;
            for (int c = 0; c < kGroupClasses; ++c) {
                const int64_t tiles = gb.bo[c + 1] - gb.bo[c];
                pbk.bo[c + 1] = pbk.bo[c] + (tiles + pbk.tpw - 1) / pbk.tpw;
            }
            for (int c = 0; c <= kGroupClasses; ++c) pbk.cstart[c] = cp.cstart[c];
            const std::string name = "k_cpt_groups_pipe<" + std::to_string(spl) + ",";
            TimedLaunch tl(t, TG_SWEEP, name.c_str(), gbytes, sfx.c_str());
            const unsigned nb = (unsigned)pbk.bo[kGroupClasses];
            if (spl == 8)
                tl.launch(k_cpt_groups_pipe<8, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, pbk);
            else if (spl == 2)
                tl.launch(k_cpt_groups_pipe<2, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, pbk);
            else
                tl.launch(k_cpt_groups_pipe<4, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, pbk);
            LV_LAUNCHED("k_cpt_groups_pipe");
        } else if (gb.bo[kGroupClasses] > 0) {
            const std::string name = "k_cpt_groups<" + std::to_string(spl) + "," + std::to_string(vpg) + ",";
            TimedLaunch tl(t, TG_SWEEP, name.c_str(), gbytes, sfx.c_str());
            const unsigned nb = (unsigned)gb.bo[kGroupClasses];
            if (spl == 8 && vpg == 1)
                tl.launch(k_cpt_groups<8, 1, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, gb);
            else if (spl == 8)
                tl.launch(k_cpt_groups<8, 2, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, gb);
            else if (spl == 2 && vpg == 1)
                tl.launch(k_cpt_groups<2, 1, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, gb);
            else if (spl == 2)
                tl.launch(k_cpt_groups<2, 2, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, gb);
            else if (vpg == 1)
                tl.launch(k_cpt_groups<4, 1, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, gb);
            else
                tl.launch(k_cpt_groups<4, 2, W>, nb, 256, 0, s, a, cp.glist, cp.ginfo, gb);
            LV_LAUNCHED("k_cpt_groups");
        }
    }
    {
        const int c = kGroupClasses;
        const int64_t nw = cp.cstart[c + 1] - cp.cstart[c];
        if (nw > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_cpt_group<2048,256,", (double)nw * vb + (double)cp.cnnz[c] * eb,
                           sfx.c_str());
            tl.launch(k_cpt_group<2048, 256, W>, (unsigned)nw, 256, 0, s1, a, cp.glist + cp.cstart[c],
                      cp.ginfo + cp.cstart[c], nw);
            LV_LAUNCHED("k_cpt_group<2048>");
        }
        const int64_t nx = cp.cstart[c + 2] - cp.cstart[c + 1];
        if (nx > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_cpt_group<4096,256,", (double)nx * vb + (double)cp.cnnz[c + 1] * eb,
                           sfx.c_str());
            tl.launch(k_cpt_group<4096, 256, W>, (unsigned)nx, 256, 0, s1, a, cp.glist + cp.cstart[c + 1],
                      cp.ginfo + cp.cstart[c + 1], nx);
            LV_LAUNCHED("k_cpt_group<4096>");
        }
        const int64_t ny = cp.cstart[c + 3] - cp.cstart[c + 2];
        if (ny > 0) {
            TimedLaunch tl(t, TG_SWEEP, "k_cpt_bigrow<", (double)ny * vb + (double)cp.cnnz[c + 2] * eb, sfx.c_str());
            tl.launch(k_cpt_bigrow<W>, (unsigned)ny, kBigRowThreads, 0, s1, a, cp.glist + cp.cstart[c + 2],
                      cp.ginfo + cp.cstart[c + 2], ny);
            LV_LAUNCHED("k_cpt_bigrow");
        }
    }
    if (cp.hubs > 0) {
        CHub hm{cp.list + cp.bstart[B_HUB], cp.tab_off, cp.chunk_off, cp.scan_off, cp.tab_size,
                cp.chunk_hub, cp.scan_hub, cp.hubs, cp.bkt_off, cp.reg_off, cp.bkt_hub, cp.shrink, cp.bkey,
                cp.bcur, cp.bpart, cp.spill};
        {
            TimedLaunch tl(t, TG_SWEEP, "k_cpt_hub_accum<", (double)cp.bnnz[B_HUB] * eb, sfx.c_str());
            tl.launch(k_cpt_hub_accum<W>, (unsigned)cp.hub_chunks, 256, 0, s2, a, hm, cp.hval, cp.hloop, cp.hpart);
            LV_LAUNCHED("k_cpt_hub_accum");
        }
        if (!a.first && cp.hub_buckets > 0) {
            // per word appended (at most one per hub entry): read
            TimedLaunch tl(t, TG_SWEEP, "k_cpt_hub_bucket", (double)cp.bnnz[B_HUB] * 8.0);
            tl.launch(k_cpt_hub_bucket, (unsigned)cp.hub_buckets, 256, 0, s2, a, hm, cp.hval);
            LV_LAUNCHED("k_cpt_hub_bucket");
        }
        {
            TimedLaunch tl(t, TG_SWEEP, "k_cpt_hub_decide", (double)cp.hubs * vb + (double)cp.hub_buckets * 32.0);
            tl.launch(k_cpt_hub_decide, grid_for(cp.hubs, 4), 256, 0, s2, a, hm, cp.hpart, cp.hloop, cp.hval);
            LV_LAUNCHED("k_cpt_hub_decide");
        }
    }
    if (fork) side->join(s);
}

void compact_pass(const GraphView &g, const CompactPass &cp, const CompactState &cs, int p,
                  const SweepParams &prm, hipStream_t s, Timer *t) {
    const int tile = compact_tile(g.n);
    if (g.n > 0) {
        TimedLaunch tl(t, TG_SWEEP, "k_cpt_publish", (double)g.n * 28);
        const unsigned gb = grid_for(g.n, tile);
        if (tile == 2048)
            tl.launch(k_cpt_publish<2048>, gb, 256, 0, s, cs.ds, cs.c_cur, cs.vw, cs.gid, cs.st, g.n, cs.active + (p & 1),
                      cs.slots);
        else if (tile == 1024)
            tl.launch(k_cpt_publish<1024>, gb, 256, 0, s, cs.ds, cs.c_cur, cs.vw, cs.gid, cs.st, g.n, cs.active + (p & 1),
                      cs.slots);
        else
            tl.launch(k_cpt_publish<512>, gb, 256, 0, s, cs.ds, cs.c_cur, cs.vw, cs.gid, cs.st, g.n, cs.active + (p & 1),
                      cs.slots);
        LV_LAUNCHED("k_cpt_publish");
    }
    CArgs a{g.row_ptr, g.col, g.w, cs.c_cur, cs.c_nxt, g.delta, cs.vw, cs.ds, cs.gid, cs.tw, cs.st, cs.es, prm.singlet,
            cp.first};
    SideStreams *side = cp.overlap ? cs.side : nullptr;
    if (g.wbytes == 4)
        compact_sweeps<int32_t>(a, cp, s, side, t);
    else
        compact_sweeps<int64_t>(a, cp, s, side, t);
    const bool fused = g.n > 0 && cs.ngraphs == 1 && g.n <= kFuseMaxN;
    if (g.n > 0) {
        // a small single graph's acceptance test runs in the last workgroup to finish
        const FinalizeArgs fa{cs.tw, cs.ngraphs, prm.theta_num, prm.theta_den, prm.max_sweeps, p,
                              cs.active + (p & 1), fused ? cs.active + 2 : nullptr, cs.slots};
        TimedLaunch tl(t, TG_SWEEP, "k_cpt_commit", (double)g.n * 12);
        const unsigned gb = grid_for(g.n, tile);
        if (tile == 2048)
            tl.launch(k_cpt_commit<2048>, gb, 256, 0, s, cs.c_cur, cs.c_nxt, g.delta, cs.es, cs.ds, cs.gid, cs.st, g.n, fa);
        else if (tile == 1024)
            tl.launch(k_cpt_commit<1024>, gb, 256, 0, s, cs.c_cur, cs.c_nxt, g.delta, cs.es, cs.ds, cs.gid, cs.st, g.n, fa);
        else
            tl.launch(k_cpt_commit<512>, gb, 256, 0, s, cs.c_cur, cs.c_nxt, g.delta, cs.es, cs.ds, cs.gid, cs.st, g.n, fa);
        LV_LAUNCHED("k_cpt_commit");
    }
    if (!fused) {
        TimedLaunch tl(t, TG_SWEEP, "k_cpt_finalize", 0.0);
        tl.launch(k_cpt_finalize, cs.slots ? 1u : grid_for(cs.ngraphs, 256), 256, 0, s, cs.st, cs.tw, cs.ngraphs,
                  prm.theta_num, prm.theta_den, prm.max_sweeps, p, cs.active + (p & 1), cs.slots);
        LV_LAUNCHED("k_cpt_finalize");
    }
}

}  // namespace lv
