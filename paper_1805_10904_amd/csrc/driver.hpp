// The single-graph level driver (Alg. 2), shared by louvain_run and the
// request loop.
#pragma once

#include "common.hpp"
#include "sweep.hpp"

namespace lv {

// Receiver of a run's dendrogram.  With a sink, a run cut by max_levels
// still contracts its last phase, so that the graph handed to last() is the
// one the next phase would run on (its rows in any order).
struct LevelSink {
    virtual ~LevelSink() = default;
    // One level: newlab (device int32[n], valid during the call) sends every
    // vertex of the level's graph to its vertex in the next level's graph,
    // which has k vertices.
    virtual void map(const int32_t *newlab, int64_t n, int64_t k, hipStream_t s) = 0;
    // The graph of the last level (device arrays valid during the call);
    // sorted: its columns already ascend in every row.
    virtual void last(const GraphView &v, bool sorted, hipStream_t s) = 0;
};

// Level-0 vertex order by row length (gather locality): order[p] is the
// given ID of the vertex at position p, pos its inverse, and the CSR is g's
// rebuilt in that order with columns remapped to positions.
struct ReorderedGraph {
    DevBuf<int32_t> order, pos, col, w32;
    DevBuf<int64_t> rp, delta, w64;
    // Build from g (n >= 2) and return the view of the rebuilt graph.
    GraphView build(const GraphView &g, hipStream_t s, Timer *t);
};
// Whether the tuning asks for the level-0 order on g (auto: 2W >= 2^31 and
// at least 2^20 vertices, where the measured sweeps gained from it).
bool reorder_applies(const GraphView &g, const Tuning &tn);

// Phases of sweeps, renumbering and contraction on g0 until a phase keeps no
// sweep or a cap is reached.  fin_p (device int32[g0.n]) receives the final
// labels, *q_out Q_int of them, *stats_out the run record (kernel times when
// timing).  Returns LOUVAIN_OK or LOUVAIN_ELIMIT; throws Error.
// timing: 0 off, 1 every launch, 2 only launches named timer.only.
// tn: launch shapes of compact levels (prm.pass_batch 0 takes tn.pass_batch).
// sink (optional) receives the dendrogram: see LevelSink.
int run_plain(const GraphView &g0, const louvain_params &prm, const Tuning &tn, hipStream_t s, Timer &timer,
              int timing, int32_t *fin_p, i128 *q_out, louvain_run_stats *stats_out,
              struct LevelSink *sink = nullptr);

}  // namespace lv
