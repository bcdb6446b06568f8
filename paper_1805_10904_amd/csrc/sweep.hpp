// Local-moving phase on the device: degree bucketing, synchronous sweeps,
// commit of community degrees and sizes, exact modularity and the sweep
// acceptance test.
#pragma once

#include <memory>

#include "prims.hpp"

namespace lv {

// A graph as the kernels see it (device pointers).
struct GraphView {
    int64_t n = 0, nnz = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const void *w = nullptr;   // int32 (wbytes 4) or int64 (wbytes 8)
    int wbytes = 4;
    const int64_t *delta = nullptr;
    int64_t tw = 0;
};

// A single graph's per-pass sums (I, movers, sum deg_C^2) are added by
// thousands of workgroups; they go to kAccSlots counters a 128-byte line
// apart (slot = workgroup index mod kAccSlots) instead of one address, where
// device-scope atomics would queue, and the acceptance test sums the slots.
constexpr int kAccSlots = 256;
constexpr int kAccStride = 16;   // 64-bit words per slot

// Device-resident control block of one phase of one graph.
struct PhaseState {
    unsigned long long acc_I;   // sum of e_{i->c_i} (loops included) of the labelling read by the pass
    unsigned long long moved;   // vertices whose label changed in the pass
    unsigned long long s_acc;   // sum of deg_C^2 of the labelling read (compact levels)
    int32_t pass;               // passes finalized in the phase
    int32_t accepted;           // sweeps kept
    int32_t done;               // phase finished
    int32_t limit;              // max_sweeps reached
    int32_t final_slot;         // label ring slot holding the phase result
    int32_t pad;
    uint64_t q_ref[2];          // Q_int of the last kept labelling (lo, hi)
    uint64_t q_last[2];         // Q_int computed by the last finalize
};

// Degree buckets: row length d (entries incl. a loop) -> sweep kernel.
// Row-length buckets.  64-bit scores: <= 8 one thread per vertex, <= 341
// packed workgroups, <= 1024 one workgroup per vertex, <= 10,922 one
// 1,024-thread workgroup on a table of single words (when labels and e fit
// 64 bits together), larger rows the HBM hub path.  128-bit scores: lane
// groups of 4, 16, 64, a workgroup and the same wide kernel.  Compact levels
// sweep every bucket from B_T16 to B_WIDE by their own table-size classes.
enum { B_T8 = 0, B_T16, B_G64, B_MID, B_BLOCK, B_WIDE, B_HUB, NBUCKET };
constexpr int64_t kBucketMax[NBUCKET - 1] = {8, 16, 128, 341, 1024, 10922};

// Packed sweep: one workgroup evaluates up to 64 vertices of row length
// <= kPackMaxDeg (tables of at most 512 slots, see pack_table_bits).
// Vertices are laid out on a line by their cost max(table size,
// kPackMinCost); workgroup b takes the vertices whose line position falls in
// [b * kPackW, (b + 1) * kPackW), so its tables fit kPackW + 512 slots.
constexpr int kPackSlots = 2048;
constexpr int kPackW = 1024;
constexpr int kPackMinCost = kPackW / 256;
constexpr int64_t kPackMaxDeg = 341;
// Compact levels sort the rows they sweep from LDS into table-size classes:
// packed classes c < kGroupClasses with S = 16 << c slots (rows with
// 3d <= 2S, up to 341 entries), then S = 2048 (up to 1,365 entries),
// S = 4096 (up to 2,730) and S = 16384 (up to kCompactBlockMax entries,
// 1,024 threads), one vertex per workgroup.
constexpr int kGroupClasses = 6;
constexpr int kLdsClasses = kGroupClasses + 3;
constexpr int64_t kCompactBlockMax = 10922;

// Launch-shape settings of compact levels (chosen by the autotuner or the
// caller; every setting gives the same results).
struct Tuning {
    int small_max = 4;                  // rows of at most this many entries: one thread per vertex (1..8)
    int64_t block_max = 2730;           // longest row swept from LDS (<= kCompactBlockMax); longer: HBM hub tables
    int pass_batch = 2;                 // sweep passes between host checks
    int group_slots = 4;                // LDS slots per lane of the packed-class sweep (2, 4 or 8)
    int group_vertices = 1;             // vertices per lane group of the packed-class sweep (1 or 2)
    int group_tiles = 1;                // tiles per workgroup of the packed-class sweep (1..8; > 1 pipelined)
    int overlap = 0;                    // 1: row families on side streams, side by side
    int reorder = 0;                    // level-0 vertex order by row length: 0 auto, 1 on, 2 off
};
// log2 of the LDS hash table size of a packed row of d >= 1 entries: the
// smallest b >= 1 with 2^b >= ceil(3d/2) (load at most 2/3).
__device__ __forceinline__ int pack_table_bits(int64_t d) {
    const int64_t need = d + (d + 1) / 2;
    return need <= 2 ? 1 : 64 - __clzll((unsigned long long)(need - 1));
}
constexpr int kHubChunk = 1024;      // row entries per hub accumulation workgroup
constexpr int kHubScan = 1024;       // table slots per hub scan workgroup

// Everything a compact pass needs from the level plan (device pointers).
struct CompactPass {
    int64_t n = 0;
    const int32_t *list = nullptr;
    int64_t bstart[NBUCKET + 1] = {0};
    int64_t bnnz[NBUCKET] = {0};
    const int64_t *pack_pos = nullptr, *pack_first = nullptr;
    int64_t pack_blocks = 0;
    const int32_t *glist = nullptr;            // rows swept from LDS, by class
    const uint64_t *ginfo = nullptr;           // their row start << 12 | length
    int64_t cstart[kLdsClasses + 1] = {0};     // class c: glist[cstart[c], cstart[c+1])
    int64_t cnnz[kLdsClasses] = {0};
    int small_max = 8;                         // rows swept one thread per vertex
    int group_slots = 4;                       // slots per lane of the packed classes
    int group_vertices = 1;                    // vertices per lane group of the packed classes
    int group_tiles = 1;                       // tiles per workgroup of the packed classes
    int first = 0;                             // the labelling read is the singletons (every
                                               // neighbour its own community): no tables
    int overlap = 0;                           // row families side by side on side streams
    int64_t hubs = 0, hub_chunks = 0, hub_scans = 0;
    const int64_t *tab_off = nullptr, *chunk_off = nullptr, *scan_off = nullptr, *tab_size = nullptr;
    const int32_t *chunk_hub = nullptr, *scan_hub = nullptr;
    int32_t *hkey = nullptr;
    unsigned long long *hval = nullptr, *hloop = nullptr;
    uint64_t *hpart = nullptr;
    // hub buckets (see the general levels): offsets, regions, cursors, partials, spill flags
    int64_t hub_buckets = 0;
    const int64_t *bkt_off = nullptr, *reg_off = nullptr;
    const int32_t *bkt_hub = nullptr;
    int shrink = 1;
    unsigned long long *bkey = nullptr;
    unsigned int *bcur = nullptr, *spill = nullptr;
    uint64_t *bpart = nullptr;
};

struct SweepParams {
    int64_t theta_num = 1, theta_den = 1000000;
    int32_t max_sweeps = 1000;
    int singlet = 1;
    int merge = 0;   // the final merge after a phase that kept a sweep (level drivers)
};

// Device state of a compact pass (one graph or a block-diagonal batch).
struct CompactState {
    int32_t *c_cur = nullptr, *c_nxt = nullptr;
    uint64_t *ds = nullptr;        // size_C << 32 | deg_C by label
    uint64_t *vw = nullptr;        // published words by vertex
    uint32_t *es = nullptr;        // e_{i->c_i} incl. loop by vertex
    const int32_t *gid = nullptr;  // graph of every vertex (nullptr: one graph)
    const int64_t *tw = nullptr;   // TW of every graph
    PhaseState *st = nullptr;      // phase state of every graph
    unsigned int *active = nullptr;// two counters of graphs still in their phase (pass parity), then
                                   // the commit's workgroup arrivals (0 between launches)
    int64_t ngraphs = 1;
    SideStreams *side = nullptr;   // optional: streams for the one-workgroup rows and the hubs
    unsigned long long *slots = nullptr;   // one graph: the pass's sums by slot (zero between passes)
};

// Longest row a level of n vertices and total weight tw sweeps from LDS
// (longer rows use the HBM hub tables): the tuned block_max on compact
// levels; on general levels kBucketMax[B_WIDE] when labels and weights fit a
// single 64-bit table word, else kBucketMax[B_BLOCK].
int64_t lds_row_max(int64_t n, int64_t tw, const Tuning &tn);

// Hub buckets (both level kinds): a hub of d entries has one bucket per
// kBktPairs entries (at most kBktMax; longer rows keep their HBM table
// only), each with a region of twice the mean pairs and a
// 2^kBktBits-slot LDS table of which kBktClaim slots may be claimed.
constexpr int kBktPairs = 1024;                 // a hub has one bucket per kBktPairs entries
constexpr int kBktMax = 512;                    // buckets of a hub at most
constexpr int kBktBits = 11;                    // bucket table: 2,048 word-keyed slots (32 KB)
constexpr int kBktClaim = 3 * (1 << kBktBits) / 4;

__device__ __forceinline__ int64_t bkt_count(int64_t d) {
    const int64_t P = (d + kBktPairs - 1) / kBktPairs;
    return P <= kBktMax ? P : 0;
}
// Pair slots of each bucket of a hub of d entries in P buckets: twice the
// mean (divided by the test shrink factor).
__device__ __forceinline__ int64_t bkt_cap(int64_t d, int64_t P, int shrink) {
    const int64_t c = 2 * ((d + P - 1) / P) / shrink;
    return c > 0 ? c : 1;
}
__device__ __forceinline__ int64_t bkt_of(int32_t label, int64_t P) {
    return (int64_t)(((uint64_t)((uint32_t)label * 0x85EBCA6Bu) * (uint64_t)P) >> 32);
}

// Levels whose graphs all have TW < 2^31 run on packed community words
// (sweep_compact.hip).
constexpr int64_t kCompactTwMax = (int64_t)1 << 31;
void compact_init_singletons(int32_t *c0, int32_t *c1, int32_t *c2, const int64_t *delta, uint64_t *ds, uint32_t *es,
                             int64_t n, hipStream_t s);
void compact_init_labels(int32_t *c0, int32_t *c1, int32_t *c2, const int32_t *labels, const int64_t *delta,
                         uint64_t *ds, uint32_t *es, int64_t n, hipStream_t s);
// Stable partition of the m rows in list by table-size class into out,
// with every row's start and length packed in info (start << 12 | length);
// cstart (kLdsClasses + 1) and cnnz (kLdsClasses) receive the class offsets
// and entry counts (synchronises the stream).
void compact_classes(const int64_t *rp, const int32_t *list, int64_t m, int32_t *out, uint64_t *info,
                     int64_t *cstart, int64_t *cnnz, hipStream_t s, Timer *t);
void compact_final_labels(const int32_t *c0, const int32_t *c1, const int32_t *c2, const int32_t *gid,
                          const PhaseState *st, int64_t n, int32_t *out, hipStream_t s, Timer *t);
void compact_expand(const uint64_t *ds, const uint32_t *es, int64_t n, int64_t *deg, int32_t *size, int64_t *e_self,
                    hipStream_t s);
void compact_pass(const GraphView &g, const CompactPass &cp, const CompactState &cs, int p, const SweepParams &prm,
                  hipStream_t s, Timer *t);


class Sweeper {
  public:
    explicit Sweeper(hipStream_t s, Timer *t) : s_(s), t_(t) {}
    // Allocate for levels of at most n vertices and nnz entries.
    void reserve(int64_t n, int64_t nnz);
    // Graphs of the next level: ngraphs graphs laid out as a block-diagonal
    // union, gid (device, per vertex) their ids and tw (device, per graph)
    // their total weights; all TW < 2^31.  Without a call a level is one
    // graph.
    void set_batch(int64_t ngraphs, const int32_t *gid, const int64_t *tw);
    // Degree bucketing of the level's vertices (a3) and hub table set-up.
    void plan(const GraphView &g);
    // Batch, inside a phase: the same plan restricted to graphs whose phase
    // is still running (labels and phase state are kept).
    void replan_active(const GraphView &g);
    // Row-length thresholds of compact levels (before plan).
    void set_tuning(const Tuning &tn) { tuning_ = tn; }
    // Singleton communities (a2): every ring slot = identity, deg = delta, size = 1.
    void init_singletons(const GraphView &g);
    // Singleton communities labelled ids[i] (device int32[n], a permutation
    // of [0, n)): vertex i alone in community ids[i].
    void init_singletons(const GraphView &g, const int32_t *ids);
    // Communities from labels (device int32[n]): ring slots = labels, deg/size recomputed.
    void init_from_labels(const GraphView &g, const int32_t *labels);
    // Enqueue sweep pass p >= 1: reads ring slot (p-1)%3, writes slot p%3,
    // commits the movers to deg_C and sizes, computes Q_int of the labelling
    // it reads and runs the acceptance test.
    void pass(const GraphView &g, int p, const SweepParams &prm, int64_t *e_self_out);
    // Copy the control block of graph 0 to the host (synchronises the stream).
    PhaseState read_state();
    // Number of graphs still in their phase after pass p (synchronises).
    unsigned int active_after(int p);
    // Device address of that count after pass p (for a read-back enqueued
    // right after the pass).
    const unsigned int *active_counter(int p) const { return active_.p + (p & 1); }
    // Control blocks of every graph (device; compact levels).
    PhaseState *states() { return st_.p; }
    // the planned level: compact words, or general levels' score width
    const char *score_kind() const { return compact_ ? "compact" : score64_ ? "64-bit scores" : "128-bit scores"; }
    bool compact() const { return compact_; }
    int64_t ngraphs() const { return ngraphs_; }
    // e_{i->labels_in[i]} incl. loop of the last pass (compact levels, int64 copy)
    void e_self_out(int64_t *dst);
    int32_t *slot(int k) { return c_[k % 3].p; }
    // Batch: every vertex's label from its graph's final ring slot.
    void final_labels(int32_t *out) {
        compact_final_labels(c_[0].p, c_[1].p, c_[2].p, gid_, st_.p, n_, out, s_, t_);
    }
    // deg_C by label of the current labelling (after a pass: of its result)
    int64_t *deg();
    int64_t bucket_count(int b) const { return bstart_[b + 1] - bstart_[b]; }

  private:
    void plan_impl(const GraphView &g, bool active_only);
    Tuning tuning_;
    hipStream_t s_;
    Timer *t_;
    std::unique_ptr<SideStreams> side_;   // leased on the first compact pass
    bool singleton_start_ = false;        // the phase started from singletons
    int64_t cap_n_ = -1, cap_nnz_ = -1;
    DevBuf<int32_t> c_[3];
    DevBuf<int64_t> deg_;           // deg_C by label (updated in place by the commit)
    DevBuf<int32_t> size_;
    bool compact_ = false;          // this level runs on compact words
    DevBuf<uint64_t> ds_;           // compact: size_C << 32 | deg_C by label
    DevBuf<uint64_t> vw_;           // compact: published words by vertex
    DevBuf<uint32_t> es_;           // compact: e_{i->c_i} incl. loop by vertex
    DevBuf<unsigned int> active_;   // compact: graphs still in their phase (two counters)
    DevBuf<int64_t> tw_one_;        // compact single graph: its TW
    int64_t ngraphs_ = 1;
    const int32_t *gid_ = nullptr;
    const int64_t *tw_ = nullptr;
    bool batch_ = false;
    DevBuf<int32_t> list_;          // vertices grouped by bucket, ascending inside a bucket
    DevBuf<int32_t> glist_;         // compact: rows swept from LDS, grouped by table-size class
    DevBuf<uint64_t> ginfo_;        // compact: their row start << 12 | length
    int64_t cstart_[kLdsClasses + 1] = {0};
    int64_t cnnz_[kLdsClasses] = {0};
    bool general_classes_ = false;  // a general level (TW > kTwFastMax) swept by table-size class
    bool score64_ = true;           // the level's scores fit int64 (TW max delta < 2^62)
    DevBuf<unsigned long long> dmax_;   // largest delta of the level
    DevBuf<unsigned long long> acc_;    // general levels: the pass's I and mover count, by slot
    DevBuf<int32_t> bcount_;        // bucketing scratch (per-block counts / offsets)
    DevBuf<PhaseState> st_;
    DevBuf<uint64_t> qpart_;        // per-block partial sums of deg^2 (lo, hi)
    // hubs
    DevBuf<int64_t> hub_meta_;      // 6 arrays of (hubs+1): table offset, chunk offset, scan offset, table size,
                                    // first bucket, first bucket pair slot
    DevBuf<int32_t> hub_key_;
    DevBuf<unsigned long long> hub_val_;
    DevBuf<unsigned long long> hub_loop_;
    DevBuf<uint64_t> hub_part_;     // per scan block: score lo, score hi, label, e_own
    DevBuf<int64_t> pack_pos_;      // line position of every packed vertex (+ total)
    DevBuf<int64_t> pack_first_;    // first packed vertex of every packed workgroup (+ end)
    DevBuf<int32_t> hub_of_chunk_;  // hub of every accumulation workgroup
    DevBuf<int32_t> hub_of_scan_;   // hub of every scan workgroup
    // hubs swept by buckets (levels with 128-bit scores and published words)
    DevBuf<uint64_t> bkt_key_, bkt_val_;   // pair regions: published word, e
    DevBuf<unsigned int> bkt_cur_;         // pairs appended to each bucket
    DevBuf<uint64_t> bkt_part_;            // per bucket: score lo, score hi, label, e_own
    DevBuf<int32_t> hub_of_bkt_;           // hub of every bucket
    DevBuf<unsigned int> hub_spill_;       // per hub: a bucket went to the table
    int64_t hub_buckets_ = 0;
    int64_t pack_count_ = 0, pack_blocks_ = 0;
    int64_t bstart_[NBUCKET + 1] = {0};
    int64_t bucket_nnz_[NBUCKET] = {0};
    int64_t hubs_ = 0, hub_chunks_ = 0, hub_scans_ = 0, hub_slots_ = 0;
    int64_t hub_slot_cap_ = 0;
    int64_t hub_cap_ = 0;           // hubs the hub metadata arrays hold
    int64_t qblocks_ = 0;
    int64_t n_ = 0;
};

}  // namespace lv
