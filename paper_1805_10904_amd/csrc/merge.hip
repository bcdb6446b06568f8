// The optional final merge of a phase (Section 5.1, end of "Generating one
// level"): after the last kept sweep, a vertex alone in its community whose
// neighbours (loops aside) all carry one label C joins C when its score
// there beats staying and the singlet rule (Section 3.1) allows it.  Every
// vertex decides from the same labels (one synchronous decision).
#include <climits>
#include <vector>

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
// In a batch (gid set), vertex i belongs to graph gid[i] with total weight
// tw_of[gid[i]], and only graphs with keep[gid[i]] != 0 merge.
template <typename W>
__global__ __launch_bounds__(256) void k_merge_lone(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                    const W *__restrict__ w, const int64_t *__restrict__ delta,
                                                    int64_t tw_one, int64_t n, const int32_t *__restrict__ lab,
                                                    const int64_t *__restrict__ deg,
                                                    const int32_t *__restrict__ size, int singlet,
                                                    const int32_t *__restrict__ gid, const int64_t *__restrict__ tw_of,
                                                    const int32_t *__restrict__ keep, int32_t *out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t ci = lab[i];
        int32_t next = ci;
        int64_t tw = tw_one;
        bool take = true;
        if (gid) {
            const int32_t gi = gid[i];
            tw = tw_of[gi];
            take = keep[gi] != 0;
        }
        if (take && size[ci] == 1) {
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

// Per-graph inner weight I_g = sum of e_{i->C(i)} (loops included): one
// wavefront per vertex, added to acc[gid[i]].
template <typename W>
__global__ __launch_bounds__(256) void k_inner_by_graph(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                        const W *__restrict__ w, int64_t n,
                                                        const int32_t *__restrict__ lab,
                                                        const int32_t *__restrict__ gid, unsigned long long *acc) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t ci = lab[i];
        int64_t e = 0;
        const int64_t end = rp[i + 1];
        for (int64_t k = rp[i] + lane; k < end; k += 64)
            if (lab[col[k]] == ci) e += (int64_t)w[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) e += shfl_xor_any<int64_t>(e, m);
        if (lane == 0 && e) atomicAdd(&acc[gid[i]], (unsigned long long)e);
    }
}

// Per-graph sum of deg_C^2 over the labels present (a label lies in its
// graph's vertex range, so gid[label] is its graph).
__global__ void k_sq_by_graph(const int64_t *__restrict__ deg, int64_t n, const int32_t *__restrict__ gid,
                              unsigned long long *acc) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t d = deg[c];
    if (d) atomicAdd(&acc[gid[c]], (unsigned long long)d * (unsigned long long)d);
}

template <typename W>
void launch_merge(const GraphView &g, const int32_t *labels, const int64_t *deg, const int32_t *size, int singlet,
                  const int32_t *gid, const int64_t *tw_of, const int32_t *keep, int32_t *out, hipStream_t s,
                  Timer *t) {
    // one wave per vertex in 4-wave workgroups, at most 16 vertices per wave
    const int64_t waves = (g.n + 15) / 16;
    TimedLaunch tl(t, TG_CONTRACT, "k_merge_lone", (double)g.n * 24);
    tl.launch(k_merge_lone<W>, grid_for(waves, 4), 256, 0, s, g.row_ptr, g.col, (const W *)g.w, g.delta, g.tw, g.n,
              labels, deg, size, singlet, gid, tw_of, keep, out);
    LV_LAUNCHED("k_merge_lone");
}

void comm_state(const GraphView &g, const int32_t *labels, int64_t *deg, int32_t *size, hipStream_t s, Timer *t) {
    fill<int64_t>(deg, 0, g.n, s);
    fill<int32_t>(size, 0, g.n, s);
    TimedLaunch tl(t, TG_CONTRACT, "k_comm_state", (double)g.n * 24);
    tl.launch(k_comm_state, grid_for(g.n, 256), 256, 0, s, labels, g.delta, g.n, deg, size);
    LV_LAUNCHED("k_comm_state");
}

}  // namespace

void merge_lone_batch(const GraphView &u, const int32_t *labels, int singlet, const int32_t *gid, const int64_t *tw_of,
                      const int32_t *keep, int32_t *out, hipStream_t s, Timer *t) {
    if (u.n == 0) return;
    TempBuf deg((size_t)u.n * sizeof(int64_t), s);
    TempBuf size((size_t)u.n * sizeof(int32_t), s);
    comm_state(u, labels, deg.as<int64_t>(), size.as<int32_t>(), s, t);
    if (u.wbytes == 4)
        launch_merge<int32_t>(u, labels, deg.as<int64_t>(), size.as<int32_t>(), singlet, gid, tw_of, keep, out, s, t);
    else
        launch_merge<int64_t>(u, labels, deg.as<int64_t>(), size.as<int32_t>(), singlet, gid, tw_of, keep, out, s, t);
}

std::vector<i128> modularity_by_graph(const GraphView &u, const int32_t *labels, const int32_t *gid, int64_t ns,
                                      const std::vector<int64_t> &tw, hipStream_t s, Timer *t) {
    std::vector<i128> q((size_t)ns, 0);
    if (u.n == 0 || ns == 0) return q;
    TempBuf deg((size_t)u.n * sizeof(int64_t), s);
    TempBuf size((size_t)u.n * sizeof(int32_t), s);
    TempBuf acc((size_t)(2 * ns) * sizeof(uint64_t), s);
    unsigned long long *inner = (unsigned long long *)acc.p, *sq = inner + ns;
    comm_state(u, labels, deg.as<int64_t>(), size.as<int32_t>(), s, t);
    fill<uint64_t>(acc.as<uint64_t>(), 0, 2 * ns, s);
    {
        const int64_t waves = (u.n + 15) / 16;
        TimedLaunch tl(t, TG_CONTRACT, "k_inner_by_graph", (double)u.nnz * (8 + u.wbytes) + (double)u.n * 16);
        if (u.wbytes == 4)
            tl.launch(k_inner_by_graph<int32_t>, grid_for(waves, 4), 256, 0, s, u.row_ptr, u.col,
                      (const int32_t *)u.w, u.n, labels, gid, inner);
        else
            tl.launch(k_inner_by_graph<int64_t>, grid_for(waves, 4), 256, 0, s, u.row_ptr, u.col,
                      (const int64_t *)u.w, u.n, labels, gid, inner);
        LV_LAUNCHED("k_inner_by_graph");
        tl.launch(k_sq_by_graph, grid_for(u.n, 256), 256, 0, s, (const int64_t *)deg.as<int64_t>(), u.n, gid, sq);
        LV_LAUNCHED("k_sq_by_graph");
    }
    std::vector<uint64_t> h((size_t)(2 * ns));
    LV_HIP(hipMemcpyAsync(h.data(), acc.p, sizeof(uint64_t) * (size_t)(2 * ns), hipMemcpyDeviceToHost, s));
    LV_HIP(hipStreamSynchronize(s));
    for (int64_t g = 0; g < ns; ++g)
        q[(size_t)g] = (i128)tw[(size_t)g] * (i128)h[(size_t)g] - (i128)h[(size_t)(ns + g)];
    return q;
}

void merge_lone(const GraphView &g, const int32_t *labels, int singlet, int32_t *out, hipStream_t s, Timer *t) {
    if (g.n == 0) return;
    TempBuf deg((size_t)g.n * sizeof(int64_t), s);
    TempBuf size((size_t)g.n * sizeof(int32_t), s);
    comm_state(g, labels, deg.as<int64_t>(), size.as<int32_t>(), s, t);
    if (g.wbytes == 4)
        launch_merge<int32_t>(g, labels, deg.as<int64_t>(), size.as<int32_t>(), singlet, nullptr, nullptr, nullptr,
                              out, s, t);
    else
        launch_merge<int64_t>(g, labels, deg.as<int64_t>(), size.as<int32_t>(), singlet, nullptr, nullptr, nullptr,
                              out, s, t);
}

}  // namespace lv
