// Renumbering, graph contraction and modularity on the device.
#pragma once

#include <vector>

#include "common.hpp"
#include "sweep.hpp"

namespace lv {

class Contractor {
  public:
    Contractor(hipStream_t s, Timer *t) : s_(s), t_(t) {}
    // Allocate for graphs of at most n vertices and nnz entries.
    void reserve(int64_t n, int64_t nnz);
    // New consecutive IDs of the labels present, in ascending label order:
    // newlab[i] = rank of labels[i] among the distinct labels.  Returns the
    // number of communities (synchronises the stream).
    int64_t renumber(const int32_t *labels, int64_t n, int32_t *newlab);
    // Batched form over a block-diagonal union whose graph s owns vertices
    // [loff[s], loff[s+1]) (device, nslots + 1 entries): only vertices whose
    // graph is kept (keep[gid[i]] != 0) take part, the others get
    // newlab = -1.  Kept graphs' communities get consecutive IDs in ascending
    // label order, so graph s's new IDs are [newoff[s], newoff[s+1])
    // (device, nslots + 1 entries; empty for graphs not kept).
    int64_t renumber_kept(const int32_t *labels, int64_t n, const int32_t *gid, const int32_t *keep,
                          const int64_t *loff, int64_t nslots, int32_t *newlab, int64_t *newoff);
    // final[v] = newlab[final[v]] for v in [0, n0).
    void compose(int32_t *final_labels, int64_t n0, const int32_t *newlab);
    // Contract g so that vertex a of the result is {i : newlab[i] == a};
    // writes row_ptr (n_new + 1), col and weights of wout_bytes = 8 (int64)
    // or 4 (int32: only where every weight of the result is below 2^31, as
    // when 2W < 2^31), capacity g.nnz, and returns the number of entries
    // (synchronises the stream).  delta_out (optional, n_new): the weighted
    // degree of every super-vertex.  Entries of rows with newlab == -1 are
    // dropped.  sorted: columns ascend in every row (the canonical form);
    // otherwise their order within a row is unspecified, which the method
    // does not depend on, except that rows longer than direct_max (the next
    // level's longest row swept from LDS) keep ascending columns, which the
    // hub kernels' pre-aggregation benefits from.
    int64_t contract(const GraphView &g, const int32_t *newlab, int64_t n_new, int64_t *rp_out,
                     int32_t *col_out, void *w_out, int wout_bytes, int64_t *delta_out, bool sorted = false,
                     int64_t direct_max = 2730);

  private:
    // Sort (key_[0], val_[0])[0, m) by the low key_bits of the keys and sum
    // the values of equal keys; *ukeys / *usums receive the unique keys in
    // ascending order and their sums (contractor buffers).  Returns the
    // device address of their number (at most m); does not synchronise.
    const int64_t *sort_sum(int64_t m, int key_bits, const uint64_t **ukeys, const int64_t **usums);

    hipStream_t s_;
    Timer *t_;
    int64_t cap_n_ = -1, cap_nnz_ = -1;
    DevBuf<int32_t> flags_;     // n: label present / renumber map
    DevBuf<uint64_t> key_[2];   // nnz: sort keys of merged pairs
    DevBuf<int64_t> val_[2];    // nnz: their weights
    DevBuf<int32_t> head_;      // nnz: segment heads
    DevBuf<int64_t> uid_;       // nnz: unique index of each sorted entry
    DevBuf<int64_t> seg_off_;   // n + 1: entries per community, then segment offsets
    DevBuf<int64_t> seg_cur_;   // n: per-community placement cursors
    DevBuf<int64_t> seg_start_; // n: place of every vertex's row in its segment
    DevBuf<int64_t> seg_m_;     // n + 1: distinct columns per community
    DevBuf<int32_t> tcol_;      // nnz: grouped entries: new column
    DevBuf<int64_t> tw_;        // nnz: grouped entries: weight
};

// The final merge of a phase (Section 5.1, end of "Generating one level"),
// one synchronous decision from labels (device int32[n] in [0, n)): a
// vertex alone in its community whose neighbours other than itself all
// carry one label C moves to C iff TW*e_{i->C} - delta_i*deg_C beats its own
// score (zero when alone) and, with singlet set, the singlet rule allows it;
// out (device int32[n], not aliasing labels) receives every vertex's label.
void merge_lone(const GraphView &g, const int32_t *labels, int singlet, int32_t *out, hipStream_t s, Timer *t);
// The same over a batch's block-diagonal union u: vertex i belongs to graph
// gid[i] (device), whose total weight is tw_of[gid[i]] (device); only graphs
// with keep[g] != 0 (device) merge, the others keep their labels.
void merge_lone_batch(const GraphView &u, const int32_t *labels, int singlet, const int32_t *gid, const int64_t *tw_of,
                      const int32_t *keep, int32_t *out, hipStream_t s, Timer *t);
// Q_int of every graph of a batch's union under labels: TW_g * I_g - sum of
// deg_C^2 over graph g's communities (tw: host, one per graph; every graph
// of a batch has 2W < 2^31, so the sums fit 64 bits).  Synchronises.
std::vector<i128> modularity_by_graph(const GraphView &u, const int32_t *labels, const int32_t *gid, int64_t ns,
                                      const std::vector<int64_t> &tw, hipStream_t s, Timer *t);

// Q_int = TW*I - sum_C deg_C^2 of labels (device int32[n] in [0, n)).
// Q_int of a labelling (eq. 3).  ws: optional device workspace of
// modularity_ws_bytes(n) bytes (256-byte aligned) used instead of pool
// temporaries.
i128 modularity_int(const GraphView &g, const int32_t *labels, hipStream_t s, Timer *t, void *ws = nullptr);
size_t modularity_ws_bytes(int64_t n);

}  // namespace lv
