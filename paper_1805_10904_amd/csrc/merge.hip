// The optional final merge of a phase (Section 5.1, end of "Generating one
// level"): after the last kept sweep, a vertex alone in its community whose
// neighbours (loops aside) all carry one label C joins C when its score
// there beats staying and the singlet rule (Section 3.1) allows it.  Every
// vertex decides from the same labels (one synchronous decision).
#include <climits>

#include "contract.hpp"
#include "prims.hpp"

namespace lv {
namespace {

// deg_C (eq. 2) and |C| of a labelling; deg and size start at zero.
__global__ void k_comm_state(const int32_t *__restrict__ lab, const int64_t *__restrict__ delta, int64_t n,
                             int64_t *deg, int32_t *size) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t c = lab[v];
    atomicAdd((unsigned long long *)&deg[c], (unsigned long long)delta[v]);
    atomicAdd(&size[c], 1);
}

// One wavefront per vertex, grid-stride over vertices.  Vertices that share
// their community are settled by one look at |C(i)| (a wave-uniform branch);
// for a lone vertex the lanes stride over its row and the wave agrees on the
// smallest and largest neighbouring label and on the weight to neighbours.
template <typename W>
__global__ __launch_bounds__(256) void k_merge_lone(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                    const W *__restrict__ w, const int64_t *__restrict__ delta,
                                                    int64_t tw, int64_t n, const int32_t *__restrict__ lab,
                                                    const int64_t *__restrict__ deg,
                                                    const int32_t *__restrict__ size, int singlet, int32_t *out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t ci = lab[i];
        int32_t next = ci;
        if (size[ci] == 1) {
            int32_t lo = INT_MAX, hi = -1;
            int64_t e = 0;
            const int64_t end = rp[i + 1];
            for (int64_t k = rp[i] + lane; k < end; k += 64) {
                const int32_t j = col[k];
                if (j == (int32_t)i) continue;   // loops take no part in moves
                const int32_t cj = lab[j];
                lo = min(lo, cj);
                hi = max(hi, cj);
                e += (int64_t)w[k];
            }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                lo = min(lo, __shfl_xor(lo, m));
                hi = max(hi, __shfl_xor(hi, m));
                e += shfl_xor_any<int64_t>(e, m);
            }
            if (hi >= 0 && lo == hi) {
                const int32_t c = hi;
                const int64_t di = delta[i];
                // alone: e_{i->C(i)\{i}} = 0 and deg_{C(i)} - delta_i = 0
                const i128 s_own = -mul_wide(di, deg[ci] - di);
                const i128 s = mul_wide(tw, e) - mul_wide(di, deg[c]);
                if (s > s_own && !(singlet && size[c] == 1 && c > ci)) next = c;
            }
        }
        if (lane == 0) out[i] = next;
    }
}

}  // namespace

void merge_lone(const GraphView &g, const int32_t *labels, int singlet, int32_t *out, hipStream_t s, Timer *t) {
    if (g.n == 0) return;
    TempBuf deg((size_t)g.n * sizeof(int64_t), s);
    TempBuf size((size_t)g.n * sizeof(int32_t), s);
    fill<int64_t>(deg.as<int64_t>(), 0, g.n, s);
    fill<int32_t>(size.as<int32_t>(), 0, g.n, s);
    {
        TimedLaunch tl(t, TG_CONTRACT, "k_comm_state", (double)g.n * 24);
        tl.launch(k_comm_state, grid_for(g.n, 256), 256, 0, s, labels, g.delta, g.n, deg.as<int64_t>(),
                  size.as<int32_t>());
        LV_LAUNCHED("k_comm_state");
    }
    // one wave per vertex in 4-wave workgroups, at most 16 vertices per wave
    const int64_t waves = (g.n + 15) / 16;
    const unsigned blocks = grid_for(waves, 4);
    TimedLaunch tl(t, TG_CONTRACT, "k_merge_lone", (double)g.n * 24);
    if (g.wbytes == 4)
        tl.launch(k_merge_lone<int32_t>, blocks, 256, 0, s, g.row_ptr, g.col, (const int32_t *)g.w, g.delta, g.tw, g.n,
                  labels, deg.as<int64_t>(), size.as<int32_t>(), singlet, out);
    else
        tl.launch(k_merge_lone<int64_t>, blocks, 256, 0, s, g.row_ptr, g.col, (const int64_t *)g.w, g.delta, g.tw,
                  g.n, labels, deg.as<int64_t>(), size.as<int32_t>(), singlet, out);
    LV_LAUNCHED("k_merge_lone");
}

}  // namespace lv
