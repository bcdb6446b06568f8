// The single-graph level driver (Alg. 2), shared by louvain_run and the
// request loop.
#pragma once

#include "common.hpp"
#include "sweep.hpp"

namespace lv {

// Phases of sweeps, renumbering and contraction on g0 until a phase keeps no
// sweep or a cap is reached.  fin_p (device int32[g0.n]) receives the final
// labels, *q_out Q_int of them, *stats_out the run record (kernel times when
// timing).  Returns LOUVAIN_OK or LOUVAIN_ELIMIT; throws Error.
// timing: 0 off, 1 every launch, 2 only launches named timer.only.
// tn: launch shapes of compact levels (prm.pass_batch 0 takes tn.pass_batch).
int run_plain(const GraphView &g0, const louvain_params &prm, const Tuning &tn, hipStream_t s, Timer &timer,
              int timing, int32_t *fin_p, i128 *q_out, louvain_run_stats *stats_out);

}  // namespace lv
