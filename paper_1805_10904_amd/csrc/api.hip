// The C ABI (include/louvain.h): contexts, graphs, and the method's calls.
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>

#include "contract.hpp"
#include "prims.hpp"
#include "sweep.hpp"

struct louvain_ctx_s {
    std::shared_ptr<lv::Pool> pool = std::make_shared<lv::Pool>();   // destroyed last
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    lv::Timer timer;
};

struct louvain_graph_s {
    std::shared_ptr<lv::Pool> pool;   // keeps the blocks' pool alive; destroyed last
    louvain_ctx ctx = nullptr;
    int device = 0;
    int64_t n = 0, nnz = 0, tw = 0;
    lv::DevBuf<int64_t> row_ptr;
    lv::DevBuf<int32_t> col;
    lv::DevBuf<int32_t> w32;
    lv::DevBuf<int64_t> w64;
    int wbytes = 4;
    lv::DevBuf<int64_t> delta;

    lv::GraphView view() const {
        lv::GraphView v;
        v.n = n;
        v.nnz = nnz;
        v.row_ptr = row_ptr.p;
        v.col = col.p;
        v.w = wbytes == 4 ? (const void *)w32.p : (const void *)w64.p;
        v.wbytes = wbytes;
        v.delta = delta.p;
        v.tw = tw;
        return v;
    }
};

namespace {

using lv::DevBuf;
using lv::Error;
using lv::require;

// Installs a context's pool as the thread's current pool for one call.
struct PoolScope {
    lv::Pool *saved;
    explicit PoolScope(lv::Pool *p) : saved(lv::current_pool()) { lv::current_pool() = p; }
    ~PoolScope() { lv::current_pool() = saved; }
};

template <typename F>
int guarded(louvain_ctx ctx, F &&f) {
    if (!ctx) return LOUVAIN_EINVAL;
    PoolScope scope(ctx->pool.get());
    try {
        LV_HIP(hipSetDevice(ctx->device));
        f();
        ctx->err.clear();
        return LOUVAIN_OK;
    } catch (const Error &e) {
        ctx->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return LOUVAIN_ENOMEM;
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return LOUVAIN_EDEVICE;
    } catch (...) {
        ctx->err = "unknown failure";
        return LOUVAIN_EDEVICE;
    }
}

bool device_ptrs(uint32_t flags) { return (flags & LOUVAIN_DEVICE_PTRS) != 0; }

// Copy count elements from a host or device pointer into device memory.
template <typename T>
void copy_in(T *dst, const T *src, int64_t count, bool dev, hipStream_t s) {
    if (count <= 0) return;
    LV_HIP(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T),
                          dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}

template <typename T>
void copy_out(T *dst, const T *src, int64_t count, bool dev, hipStream_t s) {
    if (count <= 0 || !dst) return;
    LV_HIP(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T),
                          dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
}

__global__ void k_label_range(const int32_t *__restrict__ lab, int64_t n, int *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (lab[i] < 0 || (int64_t)lab[i] >= n)) atomicOr(bad, 1);
}

__global__ void k_widen(const int32_t *__restrict__ in, int64_t *out, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = in[i];
}

// Labels from the caller, copied to the device and range-checked.
DevBuf<int32_t> labels_in(louvain_ctx ctx, const int32_t *labels, int64_t n, uint32_t flags) {
    require(labels != nullptr || n == 0, LOUVAIN_EINVAL, "labels must not be NULL");
    DevBuf<int32_t> d((size_t)n);
    copy_in(d.p, labels, n, device_ptrs(flags), ctx->stream);
    if (n > 0) {
        lv::TempBuf bad(sizeof(int), ctx->stream);
        LV_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), ctx->stream));
        k_label_range<<<lv::grid_for(n, 256), 256, 0, ctx->stream>>>(d.p, n, bad.as<int>());
        LV_LAUNCHED("k_label_range");
        int h = 0;
        LV_HIP(hipMemcpyAsync(&h, bad.p, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
        LV_HIP(hipStreamSynchronize(ctx->stream));
        require(h == 0, LOUVAIN_EINVAL, "label out of range [0, n)");
    }
    return d;
}

louvain_i128 to_abi(lv::i128 v) {
    louvain_i128 r;
    r.lo = (uint64_t)v;
    r.hi = (int64_t)(v >> 64);
    return r;
}

double q_of(lv::i128 q_int, int64_t tw) {
    return tw ? (double)q_int / ((double)tw * (double)tw) : 0.0;
}

// Aggregate the timer's records into per-family statistics.
void collect_kernel_stats(lv::Timer &t, louvain_run_stats *st, size_t first, size_t last, double *ms_sweep,
                          double *ms_contract) {
    for (size_t r = first; r < last; ++r) {
        auto &rec = t.recs[r];
        float ms = 0;
        LV_HIP(hipEventElapsedTime(&ms, rec.a, rec.b));
        const bool sweep_fam = rec.group == lv::TG_SWEEP;
        const bool contract_fam = rec.group == lv::TG_CONTRACT;
        if (ms_sweep && sweep_fam) *ms_sweep += ms;
        if (ms_contract && contract_fam) *ms_contract += ms;
        if (!st) continue;
        int k = 0;
        for (; k < st->n_kernels; ++k)
            if (strncmp(st->kernels[k].name, rec.name.c_str(), sizeof st->kernels[k].name - 1) == 0) break;
        if (k == st->n_kernels) {
            if (k >= LOUVAIN_MAX_KERNEL_STATS) continue;
            memset(&st->kernels[k], 0, sizeof st->kernels[k]);
            strncpy(st->kernels[k].name, rec.name.c_str(), sizeof st->kernels[k].name - 1);
            st->n_kernels++;
        }
        st->kernels[k].launches++;
        st->kernels[k].ms += ms;
        st->kernels[k].alg_bytes += rec.bytes;
    }
}

}  // namespace

extern "C" {

int louvain_ctx_create(int device, void *hip_stream, louvain_ctx *out) {
    if (!out) return LOUVAIN_EINVAL;
    louvain_ctx c = new (std::nothrow) louvain_ctx_s();
    if (!c) return LOUVAIN_ENOMEM;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        delete c;
        return device < 0 ? LOUVAIN_EINVAL : LOUVAIN_EDEVICE;
    }
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->timer.stream = c->stream;
    *out = c;
    return LOUVAIN_OK;
}

int louvain_ctx_destroy(louvain_ctx ctx) {
    if (!ctx) return LOUVAIN_EINVAL;
    (void)hipSetDevice(ctx->device);
    delete ctx;
    return LOUVAIN_OK;
}

const char *louvain_last_error(louvain_ctx ctx) { return ctx ? ctx->err.c_str() : "invalid context"; }

int louvain_graph_create(louvain_ctx ctx, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                         const void *weight, uint32_t flags, louvain_graph *out) {
    return guarded(ctx, [&] {
        require(out != nullptr, LOUVAIN_EINVAL, "out must not be NULL");
        require(n >= 0 && nnz >= 0, LOUVAIN_EINVAL, "n and nnz must be >= 0");
        require(n < ((int64_t)1 << 31), LOUVAIN_EOVERFLOW, "n must be below 2^31");
        require(nnz < ((int64_t)1 << 40), LOUVAIN_EOVERFLOW, "nnz must be below 2^40");
        require(row_ptr != nullptr, LOUVAIN_EINVAL, "row_ptr must not be NULL");
        require(nnz == 0 || (col_idx && weight), LOUVAIN_EINVAL, "col_idx and weight must not be NULL");
        require(n > 0 || nnz == 0, LOUVAIN_EINVAL, "a graph without vertices has no entries");
        const bool dev = device_ptrs(flags);
        std::unique_ptr<louvain_graph_s> g(new louvain_graph_s());
        g->ctx = ctx;
        g->pool = ctx->pool;
        g->device = ctx->device;
        g->n = n;
        g->nnz = nnz;
        g->wbytes = (flags & LOUVAIN_WEIGHTS_I64) ? 8 : 4;
        g->row_ptr.alloc((size_t)n + 1);
        g->col.alloc((size_t)nnz);
        if (g->wbytes == 4) g->w32.alloc((size_t)nnz); else g->w64.alloc((size_t)nnz);
        g->delta.alloc((size_t)n);
        hipStream_t s = ctx->stream;
        copy_in(g->row_ptr.p, row_ptr, n + 1, dev, s);
        copy_in(g->col.p, col_idx, nnz, dev, s);
        lv::Timer *t = ctx->timer.on ? &ctx->timer : nullptr;
        const bool sym = (flags & LOUVAIN_CHECK_SYMMETRY) != 0;
        if (g->wbytes == 4) {
            copy_in(g->w32.p, (const int32_t *)weight, nnz, dev, s);
            lv::ingest_csr<int32_t>(n, nnz, g->row_ptr.p, g->col.p, g->w32.p, g->delta.p, &g->tw, sym, s, t);
        } else {
            copy_in(g->w64.p, (const int64_t *)weight, nnz, dev, s);
            lv::ingest_csr<int64_t>(n, nnz, g->row_ptr.p, g->col.p, g->w64.p, g->delta.p, &g->tw, sym, s, t);
        }
        *out = g.release();
    });
}

int louvain_graph_destroy(louvain_graph g) {
    if (!g) return LOUVAIN_EINVAL;
    (void)hipSetDevice(g->device);
    delete g;
    return LOUVAIN_OK;
}

int louvain_graph_info(louvain_graph g, int64_t *n, int64_t *nnz, int64_t *total_weight) {
    if (!g) return LOUVAIN_EINVAL;
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (total_weight) *total_weight = g->tw;
    return LOUVAIN_OK;
}

int louvain_graph_export(louvain_graph g, int64_t *row_ptr, int32_t *col_idx, int64_t *weight, uint32_t flags) {
    if (!g) return LOUVAIN_EINVAL;
    louvain_ctx ctx = g->ctx;
    return guarded(ctx, [&] {
        require(row_ptr && (g->nnz == 0 || (col_idx && weight)), LOUVAIN_EINVAL, "output must not be NULL");
        const bool dev = device_ptrs(flags);
        hipStream_t s = ctx->stream;
        DevBuf<int64_t> wide;
        const int64_t *w = g->w64.p;
        if (g->wbytes == 4 && g->nnz > 0) {
            wide.alloc((size_t)g->nnz);
            k_widen<<<lv::grid_for(g->nnz, 256), 256, 0, s>>>(g->w32.p, wide.p, g->nnz);
            LV_LAUNCHED("k_widen");
            w = wide.p;
        }
        copy_out(row_ptr, g->row_ptr.p, g->n + 1, dev, s);
        copy_out(col_idx, g->col.p, g->nnz, dev, s);
        copy_out(weight, w, g->nnz, dev, s);
        LV_HIP(hipStreamSynchronize(s));
    });
}

int louvain_local_move(louvain_ctx ctx, louvain_graph g, const int32_t *labels, int32_t *labels_out,
                       int64_t *deg_c_out, int64_t *e_own_out, uint32_t flags) {
    return guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(labels_out != nullptr || g->n == 0, LOUVAIN_EINVAL, "labels_out must not be NULL");
        hipStream_t s = ctx->stream;
        lv::Timer *t = ctx->timer.on ? &ctx->timer : nullptr;
        const lv::GraphView v = g->view();
        DevBuf<int32_t> lin;
        if (labels) lin = labels_in(ctx, labels, g->n, flags);
        lv::Sweeper sw(s, t);
        sw.reserve(v.n, v.nnz);
        sw.plan(v);
        if (labels) sw.init_from_labels(v, lin.p); else sw.init_singletons(v);
        DevBuf<int64_t> eself((size_t)g->n);
        lv::fill<int64_t>(eself.p, 0, g->n, s);
        lv::SweepParams prm;
        prm.singlet = (flags & LOUVAIN_NO_SINGLET) ? 0 : 1;
        sw.pass(v, 1, prm, eself.p);
        LV_HIP(hipStreamSynchronize(s));
        const bool dev = device_ptrs(flags);
        copy_out(labels_out, sw.slot(1), g->n, dev, s);
        copy_out(deg_c_out, sw.deg(), g->n, dev, s);
        copy_out(e_own_out, eself.p, g->n, dev, s);
        LV_HIP(hipStreamSynchronize(s));
    });
}

int louvain_modularity(louvain_ctx ctx, louvain_graph g, const int32_t *labels, louvain_i128 *q_int, double *q,
                       uint32_t flags) {
    return guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(q_int != nullptr, LOUVAIN_EINVAL, "q_int must not be NULL");
        DevBuf<int32_t> lab = labels_in(ctx, labels, g->n, flags);
        lv::Timer *t = ctx->timer.on ? &ctx->timer : nullptr;
        const lv::i128 v = lv::modularity_int(g->view(), lab.p, ctx->stream, t);
        *q_int = to_abi(v);
        if (q) *q = q_of(v, g->tw);
    });
}

int louvain_aggregate(louvain_ctx ctx, louvain_graph g, const int32_t *labels, int32_t *renumber_out,
                      louvain_graph *out, uint32_t flags) {
    return guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(out != nullptr, LOUVAIN_EINVAL, "out must not be NULL");
        hipStream_t s = ctx->stream;
        lv::Timer *t = ctx->timer.on ? &ctx->timer : nullptr;
        DevBuf<int32_t> lab = labels_in(ctx, labels, g->n, flags);
        lv::Contractor ct(s, t);
        ct.reserve(g->n, g->nnz);
        DevBuf<int32_t> newlab((size_t)g->n);
        const int64_t k = ct.renumber(lab.p, g->n, newlab.p);
        std::unique_ptr<louvain_graph_s> g2(new louvain_graph_s());
        g2->ctx = ctx;
        g2->pool = ctx->pool;
        g2->device = ctx->device;
        g2->n = k;
        g2->wbytes = 8;
        g2->row_ptr.alloc((size_t)k + 1);
        g2->col.alloc((size_t)g->nnz);
        g2->w64.alloc((size_t)g->nnz);
        g2->delta.alloc((size_t)k);
        g2->nnz = ct.contract(g->view(), newlab.p, k, g2->row_ptr.p, g2->col.p, g2->w64.p);
        lv::row_sums_i64(k, g2->nnz, g2->row_ptr.p, g2->w64.p, g2->delta.p, s, t);
        g2->tw = g->tw;
        copy_out(renumber_out, newlab.p, g->n, device_ptrs(flags), s);
        LV_HIP(hipStreamSynchronize(s));
        *out = g2.release();
    });
}

int louvain_run(louvain_ctx ctx, louvain_graph g, const louvain_params *params, int32_t *labels_out,
                louvain_i128 *q_int, double *q, louvain_run_stats *stats, uint32_t flags) {
    int status = LOUVAIN_OK;
    const int rc = guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(labels_out != nullptr || g->n == 0, LOUVAIN_EINVAL, "labels_out must not be NULL");
        louvain_params prm{1, 1000000, 1000, 64, 1, 0};
        if (params) prm = *params;
        require(prm.theta_num >= 0 && prm.theta_den > 0, LOUVAIN_EINVAL, "theta must be num >= 0, den > 0");
        require(prm.max_sweeps >= 0 && prm.max_levels >= 1 && prm.max_levels <= 64, LOUVAIN_EINVAL,
                "max_sweeps must be >= 0 and max_levels in [1, 64]");
        const int batch = prm.pass_batch > 0 ? prm.pass_batch : 1;
        hipStream_t s = ctx->stream;
        lv::Timer &timer = ctx->timer;
        const bool timing = stats && stats->timing;
        timer.on = timing;
        timer.reset();
        lv::Timer *t = timing ? &timer : nullptr;
        louvain_run_stats local;
        memset(&local, 0, sizeof local);
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (timing) {
            LV_HIP(hipEventCreate(&ev0));
            LV_HIP(hipEventCreate(&ev1));
            LV_HIP(hipEventRecord(ev0, s));
        }
        struct EvGuard {
            hipEvent_t a, b;
            ~EvGuard() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } evg{ev0, ev1};

        const int64_t n0 = g->n, nnz0 = g->nnz;
        DevBuf<int32_t> fin((size_t)n0);
        lv::iota_i32(fin.p, n0, s);
        lv::i128 q_final = 0;
        lv::GraphView v = g->view();
        if (g->tw > 0) {
            lv::Sweeper sw(s, t);
            lv::Contractor ct(s, t);
            sw.reserve(n0, nnz0);
            ct.reserve(n0, nnz0);
            DevBuf<int32_t> newlab((size_t)n0);
            struct LevelGraph {
                DevBuf<int64_t> rp, delta, w;
                DevBuf<int32_t> col;
            } lg[2];
            int which = 0;
            lv::SweepParams sp;
            sp.theta_num = prm.theta_num;
            sp.theta_den = prm.theta_den;
            sp.max_sweeps = prm.max_sweeps;
            sp.singlet = prm.singlet_rule ? 1 : 0;
            for (int level = 0; level < prm.max_levels; ++level) {
                const size_t rec0 = timer.recs.size();
                sw.plan(v);
                sw.init_singletons(v);
                lv::PhaseState st;
                int p = 0;
                for (;;) {
                    for (int b = 0; b < batch; ++b) sw.pass(v, ++p, sp, nullptr);
                    st = sw.read_state();
                    if (st.done) break;
                    require(p <= prm.max_sweeps + 4 + batch, LOUVAIN_EDEVICE, "sweep loop did not converge");
                }
                auto &ls = local.level[level];
                ls.n = v.n;
                ls.nnz = v.nnz;
                ls.sweeps_accepted = st.accepted;
                ls.sweeps_executed = st.accepted + (st.limit ? 0 : 1);
                ls.gpu_passes = st.pass;
                ls.q_int.lo = st.q_ref[0];
                ls.q_int.hi = (int64_t)st.q_ref[1];
                local.total_edges_swept += (int64_t)st.pass * v.nnz;
                local.levels = level + 1;
                q_final = lv::make_i128(st.q_ref[0], (int64_t)st.q_ref[1]);
                if (st.limit) status = LOUVAIN_ELIMIT;
                if (st.accepted == 0) {
                    if (timing) {
                        LV_HIP(hipStreamSynchronize(s));
                        collect_kernel_stats(timer, nullptr, rec0, timer.recs.size(), &ls.ms_sweep, &ls.ms_contract);
                    }
                    break;
                }
                const int32_t *cfin = sw.slot(st.final_slot);
                const int64_t k = ct.renumber(cfin, v.n, newlab.p);
                ct.compose(fin.p, n0, newlab.p);
                if (level + 1 >= prm.max_levels) {
                    status = LOUVAIN_ELIMIT;
                    if (timing) {
                        LV_HIP(hipStreamSynchronize(s));
                        collect_kernel_stats(timer, nullptr, rec0, timer.recs.size(), &ls.ms_sweep, &ls.ms_contract);
                    }
                    break;
                }
                LevelGraph &nb = lg[which];
                if (!nb.rp.p) {
                    nb.rp.alloc((size_t)n0 + 1);
                    nb.delta.alloc((size_t)n0);
                    nb.w.alloc((size_t)nnz0);
                    nb.col.alloc((size_t)nnz0);
                }
                const int64_t m2 = ct.contract(v, newlab.p, k, nb.rp.p, nb.col.p, nb.w.p);
                lv::row_sums_i64(k, m2, nb.rp.p, nb.w.p, nb.delta.p, s, t);
                lv::GraphView v2;
                v2.n = k;
                v2.nnz = m2;
                v2.row_ptr = nb.rp.p;
                v2.col = nb.col.p;
                v2.w = nb.w.p;
                v2.wbytes = 8;
                v2.delta = nb.delta.p;
                v2.tw = g->tw;
                v = v2;
                which = 1 - which;
                if (timing) {
                    LV_HIP(hipStreamSynchronize(s));
                    collect_kernel_stats(timer, nullptr, rec0, timer.recs.size(), &ls.ms_sweep, &ls.ms_contract);
                }
            }
        }
        local.status = status;
        if (timing) {
            LV_HIP(hipEventRecord(ev1, s));
            LV_HIP(hipStreamSynchronize(s));
            float ms = 0;
            LV_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            local.ms_total = ms;
            collect_kernel_stats(timer, &local, 0, timer.recs.size(), nullptr, nullptr);
        }
        timer.on = false;
        copy_out(labels_out, fin.p, n0, device_ptrs(flags), s);
        LV_HIP(hipStreamSynchronize(s));
        if (q_int) *q_int = to_abi(q_final);
        if (q) *q = q_of(q_final, g->tw);
        if (stats) {
            local.timing = stats->timing;
            *stats = local;
        }
    });
    if (ctx) ctx->timer.on = false;
    return rc != LOUVAIN_OK ? rc : status;
}

}  // extern "C"
