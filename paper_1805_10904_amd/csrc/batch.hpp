// Many graphs through the method at once: a block-diagonal union of the
// members' current level graphs is swept, renumbered and contracted with one
// set of launches per pass and per level, while every member keeps its own
// TW, modularity, acceptance test, level count and final labels, so each
// result equals a run on that graph alone.  Members may join between levels
// (a newcomer's level-0 graph is appended to the union beside the contracted
// graphs of members at deeper levels).
#pragma once

#include <vector>

#include "contract.hpp"
#include "sweep.hpp"

namespace lv {

// One phase of one member.
struct LevelRec {
    int64_t n = 0, nnz = 0;
    int32_t executed = 0, accepted = 0, passes = 0;
    i128 q = 0;
};

struct BatchMember {
    GraphView g0;              // the member's level-0 graph (device; TW < 2^31)
    int32_t *fin = nullptr;    // device int32[g0.n]: final labels, composed level by level
    void *tag = nullptr;       // caller data
    // filled by the engine
    int level = 0;             // phases finished
    int64_t n = 0, nnz = 0;    // the member's graph at the current level
    int64_t edges_swept = 0;   // sum over device passes of the level's nnz
    bool done = false;
    int status = 0;            // LOUVAIN_OK or LOUVAIN_ELIMIT
    i128 q = 0;                // Q_int of the final labels
    std::vector<LevelRec> levels;
};

// dst[i][v] = src[src_off[i] + v] for v < n[i] (device pointers; one launch).
void copy_segments(int32_t *const *dst, const int64_t *n, const int64_t *src_off, int64_t count, const int32_t *src,
                   hipStream_t s);

class BatchEngine {
  public:
    BatchEngine(hipStream_t s, Timer *t, const SweepParams &sp, int max_levels, int pass_batch);
    // Queue a member; it joins the union at the start of the next step.
    // Members with n == 0 or TW == 0 finish at once (identity labels, Q 0).
    void admit(BatchMember *m);
    // One level for every member in the union.  Returns the members that
    // finished (their fin, q, status and levels are final once the stream
    // has drained; step() synchronises it before returning).
    std::vector<BatchMember *> step();
    bool idle() const { return slots_.empty() && pending_.empty() && finished_.empty(); }
    void set_tuning(const Tuning &tn) {
        sw_.set_tuning(tn);
        block_max_ = tn.block_max;
    }
    size_t resident() const { return slots_.size(); }
    size_t pending() const { return pending_.size(); }
    // Vertices and entries of the union the next step sweeps.
    int64_t union_vertices() const;
    int64_t union_entries() const;

  private:
    int64_t block_max_ = Tuning().block_max;   // longest row swept from LDS (members are compact)
    struct UBuf {
        DevBuf<int64_t> rp, delta;
        DevBuf<int32_t> col, w32;
    };
    void ensure(UBuf &u, int64_t n, int64_t m, int64_t keep_n, int64_t keep_m);

    hipStream_t s_;
    Timer *t_;
    SweepParams sp_;
    int max_levels_, pass_batch_;
    Sweeper sw_;
    Contractor ct_;
    std::vector<BatchMember *> slots_;     // members whose contracted graphs are in ub_[cur_]
    std::vector<BatchMember *> pending_;   // newcomers
    std::vector<BatchMember *> finished_;  // finished without a step (degenerate)
    UBuf ub_[2];
    int cur_ = 0;
    int64_t un_ = 0, um_ = 0;              // size of the contracted part in ub_[cur_]
    DevBuf<int32_t> gid_, newlab_, labf_, keep_, merged_;
    DevBuf<int64_t> tw_, loff_, newoff_;
};

}  // namespace lv
