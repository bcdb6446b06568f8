// The C ABI (include/louvain.h): contexts, graphs, and the method's calls.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

#include "batch.hpp"
#include "contract.hpp"
#include "driver.hpp"
#include "prims.hpp"
#include "serve.hpp"
#include "sweep.hpp"

struct louvain_ctx_s {
    std::shared_ptr<lv::Arena> arena;      // the caller's device region (nullptr: hipMalloc)
    std::shared_ptr<lv::Pool> pool;        // destroyed last
    std::string tuning_path;               // launch shapes persisted by louvain_autotune
    std::atomic<long> owner{0};            // thread inside a call on the context (0: none)
    int depth = 0;                         // nesting of the owner's calls
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    lv::Timer timer;
    lv::Tuning tuning;                    // launch shapes of compact levels
    std::mutex serve_mu;                  // guards server creation and serve_budget
    size_t serve_budget = 0;              // 0: a share of the device's free memory
    std::unique_ptr<lv::Server> server;   // request loop, started by the first submit
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

// A run's dendrogram: the renumbering map of every level and the graph of
// the last level (until handed to the caller).
struct louvain_dendro_s {
    std::shared_ptr<lv::Pool> pool;   // keeps the blocks' pool alive; destroyed last
    louvain_ctx ctx = nullptr;
    int device = 0;
    std::vector<lv::DevBuf<int32_t>> maps;    // maps[l]: n[l] entries
    std::vector<int64_t> n;                   // vertices of level l's graph, l = 0..levels
    std::unique_ptr<louvain_graph_s> graph;   // the last level's graph
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

// A small id per host thread (0 is never used).
long thread_id() {
    static std::atomic<long> next{1};
    static thread_local long id = next++;
    return id;
}

// Marks the calling thread as inside a call on ctx; a call from another
// thread meanwhile is refused (LOUVAIN_EBUSY), one nested in it is not.
struct CallScope {
    louvain_ctx ctx;
    bool entered = false;
    explicit CallScope(louvain_ctx c) : ctx(c) {
        const long me = thread_id();
        long cur = 0;
        if (ctx->owner.compare_exchange_strong(cur, me) || cur == me) {
            ctx->depth++;
            entered = true;
        }
    }
    ~CallScope() {
        if (entered && --ctx->depth == 0) ctx->owner.store(0);
    }
};

template <typename F>
int guarded(louvain_ctx ctx, F &&f) {
    if (!ctx) return LOUVAIN_EINVAL;
    CallScope call(ctx);
    if (!call.entered) return LOUVAIN_EBUSY;   // ctx->err belongs to the other thread's call
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

// Launch shapes from the ABI's form, checked.
lv::Tuning tuning_from(const louvain_tuning &t) {
    require(t.small_max >= 1 && t.small_max <= 8, LOUVAIN_EINVAL, "small_max must be in [1, 8]");
    require(t.block_max >= lv::kPackMaxDeg && t.block_max <= lv::kCompactBlockMax, LOUVAIN_EINVAL,
            "block_max must be in [341, 10922]");
    require(t.pass_batch >= 1 && t.pass_batch <= 64, LOUVAIN_EINVAL, "pass_batch must be in [1, 64]");
    require(t.group_slots == 0 || t.group_slots == 2 || t.group_slots == 4 || t.group_slots == 8, LOUVAIN_EINVAL,
            "group_slots must be 0, 2, 4 or 8");
    require(t.group_vertices >= 0 && t.group_vertices <= 2, LOUVAIN_EINVAL, "group_vertices must be 0, 1 or 2");
    require(t.overlap == 0 || t.overlap == 1, LOUVAIN_EINVAL, "overlap must be 0 or 1");
    require(t.reorder >= 0 && t.reorder <= 2, LOUVAIN_EINVAL, "reorder must be 0, 1 or 2");
    require(t.group_tiles >= 0 && t.group_tiles <= 8, LOUVAIN_EINVAL, "group_tiles must be in [0, 8]");
    lv::Tuning tn;
    tn.small_max = t.small_max;
    tn.block_max = t.block_max;
    tn.pass_batch = t.pass_batch;
    tn.group_slots = t.group_slots == 0 ? 4 : t.group_slots;
    tn.group_vertices = t.group_vertices == 0 ? 1 : t.group_vertices;
    tn.overlap = t.overlap;
    tn.reorder = t.reorder;
    tn.group_tiles = t.group_tiles == 0 ? 1 : t.group_tiles;
    return tn;
}

louvain_tuning tuning_to(const lv::Tuning &tn) {
    louvain_tuning t;
    memset(&t, 0, sizeof t);
    t.small_max = tn.small_max;
    t.block_max = (int32_t)tn.block_max;
    t.pass_batch = tn.pass_batch;
    t.group_slots = tn.group_slots;
    t.group_vertices = tn.group_vertices;
    t.overlap = tn.overlap;
    t.reorder = tn.reorder;
    t.group_tiles = tn.group_tiles;
    return t;
}

// Architecture name of a device (the key of a tuning file).
std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    return a.empty() ? "unknown" : a;
}

// Tuning file: text lines "key value" -- "arch <name>" and one line per
// launch-shape field.  Returns false when the file does not exist or was
// written for another architecture (the defaults then stay); throws EINVAL
// for a malformed file or values out of range.
bool load_tuning(const std::string &path, const std::string &arch, lv::Tuning *out) {
    std::ifstream f(path);
    if (!f) return false;
    louvain_tuning t = tuning_to(lv::Tuning());
    std::string line, file_arch;
    int line_no = 0;
    while (std::getline(f, line)) {
        ++line_no;
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string key;
        is >> key;
        if (key == "arch") {
            is >> file_arch;
            continue;
        }
        long long v = 0;
        require((bool)(is >> v), LOUVAIN_EINVAL, path + ":" + std::to_string(line_no) + ": expected 'key value'");
        if (key == "small_max") t.small_max = (int32_t)v;
        else if (key == "block_max") t.block_max = (int32_t)v;
        else if (key == "pass_batch") t.pass_batch = (int32_t)v;
        else if (key == "group_slots") t.group_slots = (int32_t)v;
        else if (key == "group_vertices") t.group_vertices = (int32_t)v;
        else if (key == "overlap") t.overlap = (int32_t)v;
        else if (key == "reorder") t.reorder = (int32_t)v;
        else if (key == "group_tiles") t.group_tiles = (int32_t)v;
        else require(false, LOUVAIN_EINVAL, path + ":" + std::to_string(line_no) + ": unknown key '" + key + "'");
    }
    if (file_arch != arch) return false;
    *out = tuning_from(t);
    return true;
}

void save_tuning(const std::string &path, const std::string &arch, const lv::Tuning &tn, double ms) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        require((bool)f, LOUVAIN_EINVAL, "cannot write the tuning file " + path);
        f << "# launch shapes chosen by louvain_autotune (" << ms << " ms per run)\n";
        f << "arch " << arch << "\n";
        f << "small_max " << tn.small_max << "\n";
        f << "block_max " << tn.block_max << "\n";
        f << "pass_batch " << tn.pass_batch << "\n";
        f << "group_slots " << tn.group_slots << "\n";
        f << "group_vertices " << tn.group_vertices << "\n";
        f << "overlap " << tn.overlap << "\n";
        f << "reorder " << tn.reorder << "\n";
        f << "group_tiles " << tn.group_tiles << "\n";
        require((bool)f, LOUVAIN_EINVAL, "cannot write the tuning file " + path);
    }
    require(std::rename(tmp.c_str(), path.c_str()) == 0, LOUVAIN_EINVAL, "cannot replace the tuning file " + path);
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

__global__ void k_label_range(const int32_t *__restrict__ lab, int64_t n, int64_t bound, int *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (lab[i] < 0 || (int64_t)lab[i] >= bound)) atomicOr(bad, 1);
}

__global__ void k_widen(const int32_t *__restrict__ in, int64_t *out, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = in[i];
}

// Labels from the caller, copied to the device and checked to lie in
// [0, bound) (bound < 0: [0, n)).
DevBuf<int32_t> labels_in(louvain_ctx ctx, const int32_t *labels, int64_t n, uint32_t flags, int64_t bound = -1) {
    if (bound < 0) bound = n;
    require(labels != nullptr || n == 0, LOUVAIN_EINVAL, "labels must not be NULL");
    DevBuf<int32_t> d((size_t)n);
    copy_in(d.p, labels, n, device_ptrs(flags), ctx->stream);
    if (n > 0) {
        lv::TempBuf bad(sizeof(int), ctx->stream);
        LV_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), ctx->stream));
        k_label_range<<<lv::grid_for(n, 256), 256, 0, ctx->stream>>>(d.p, n, bound, bad.as<int>());
        LV_LAUNCHED("k_label_range");
        lv::Readback rb(ctx->stream);
        const int *h = rb.add(bad.as<int>());
        rb.fetch();
        require(*h == 0, LOUVAIN_EINVAL, "label out of range [0, " + std::to_string(bound) + ")");
    }
    return d;
}

// Collects a run's dendrogram (the per-level maps, the last level's graph).
struct DendroSink final : lv::LevelSink {
    louvain_dendro_s *d;
    explicit DendroSink(louvain_dendro_s *dd) : d(dd) {}
    void map(const int32_t *newlab, int64_t n, int64_t k, hipStream_t s) override {
        d->maps.emplace_back((size_t)n);
        copy_in(d->maps.back().p, newlab, n, true, s);
        d->n.push_back(k);
    }
    // The last level's graph in canonical form: copied when its rows are
    // sorted, else contracted by the identity (every vertex its own
    // super-vertex), which sorts every row and keeps the entries, weights
    // and degrees.
    void last(const lv::GraphView &v, bool sorted, hipStream_t s) override {
        std::unique_ptr<louvain_graph_s> g(new louvain_graph_s());
        g->ctx = d->ctx;
        g->pool = d->ctx->pool;
        g->device = d->ctx->device;
        g->n = v.n;
        g->tw = v.tw;
        g->wbytes = v.wbytes;
        g->row_ptr.alloc((size_t)v.n + 1);
        g->col.alloc((size_t)v.nnz);
        if (v.wbytes == 4) g->w32.alloc((size_t)v.nnz); else g->w64.alloc((size_t)v.nnz);
        g->delta.alloc((size_t)v.n);
        if (sorted || v.n == 0 || v.nnz == 0) {
            g->nnz = v.nnz;
            copy_in(g->row_ptr.p, v.row_ptr, v.n + 1, true, s);
            copy_in(g->col.p, v.col, v.nnz, true, s);
            if (v.wbytes == 4)
                copy_in(g->w32.p, (const int32_t *)v.w, v.nnz, true, s);
            else
                copy_in(g->w64.p, (const int64_t *)v.w, v.nnz, true, s);
            copy_in(g->delta.p, v.delta, v.n, true, s);
        } else {
            DevBuf<int32_t> ident((size_t)v.n);
            lv::iota_i32(ident.p, v.n, s);
            lv::Contractor ct(s, nullptr);
            ct.reserve(v.n, v.nnz);
            void *w = v.wbytes == 4 ? (void *)g->w32.p : (void *)g->w64.p;
            g->nnz = ct.contract(v, ident.p, v.n, g->row_ptr.p, g->col.p, w, v.wbytes, g->delta.p, true);
        }
        d->graph = std::move(g);
    }
};

louvain_i128 to_abi(lv::i128 v) {
    louvain_i128 r;
    r.lo = (uint64_t)v;
    r.hi = (int64_t)(v >> 64);
    return r;
}

double q_of(lv::i128 q_int, int64_t tw) {
    return tw ? (double)q_int / ((double)tw * (double)tw) : 0.0;
}

louvain_params checked_params(const louvain_params *params) {
    louvain_params prm{1, 1000000, 1000, 64, 1, 0, 0, 0};
    if (params) prm = *params;
    require(prm.theta_num >= 0 && prm.theta_den > 0, LOUVAIN_EINVAL, "theta must be num >= 0, den > 0");
    require(prm.max_sweeps >= 0 && prm.max_levels >= 1 && prm.max_levels <= 64, LOUVAIN_EINVAL,
            "max_sweeps must be >= 0 and max_levels in [1, 64]");
    require(prm.merge == 0 || prm.merge == 1, LOUVAIN_EINVAL, "merge must be 0 or 1");
    require(prm.reserved == 0, LOUVAIN_EINVAL, "reserved must be 0");
    return prm;
}

lv::SweepParams sweep_params(const louvain_params &prm) {
    lv::SweepParams sp;
    sp.theta_num = prm.theta_num;
    sp.theta_den = prm.theta_den;
    sp.max_sweeps = prm.max_sweeps;
    sp.singlet = prm.singlet_rule ? 1 : 0;
    sp.merge = prm.merge;
    return sp;
}

// A finished batch member's record in the ABI's form.
void member_stats(const lv::BatchMember &m, int32_t timing, louvain_run_stats *st) {
    memset(st, 0, sizeof *st);
    st->timing = timing;
    st->levels = (int32_t)m.levels.size();
    st->status = m.status;
    st->total_edges_swept = m.edges_swept;
    for (size_t l = 0; l < m.levels.size() && l < 64; ++l) {
        const lv::LevelRec &r = m.levels[l];
        louvain_level_stats &ls = st->level[l];
        ls.n = r.n;
        ls.nnz = r.nnz;
        ls.sweeps_executed = r.executed;
        ls.sweeps_accepted = r.accepted;
        ls.gpu_passes = r.passes;
        ls.q_int = to_abi(r.q);
    }
}

// Aggregate the timer's records into per-family statistics.
void collect_kernel_stats(lv::Timer &t, louvain_run_stats *st, size_t first, size_t last, double *ms_sweep,
                          double *ms_contract) {
    for (size_t r = first; r < last; ++r) {
        auto &rec = t.recs[r];
        if (!rec.launched) continue;
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

namespace lv {

// Alg. 2 on one graph: phases of sweeps, renumbering and contraction until a
// phase keeps no sweep.  fin_p (device int32[n]) receives the final labels.
int run_plain(const GraphView &g0, const louvain_params &prm, const Tuning &tn, hipStream_t s, Timer &timer,
              int timing, int32_t *fin_p, i128 *q_out, louvain_run_stats *stats_out, LevelSink *sink) {
    int status = LOUVAIN_OK;
    const int batch = prm.pass_batch > 0 ? prm.pass_batch : tn.pass_batch;
    timer.on = timing != 0;
    if (timing != 2) timer.only.clear();
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

    const int64_t n0 = g0.n, nnz0 = g0.nnz;
    lv::iota_i32(fin_p, n0, s);
    lv::i128 q_final = 0;
    lv::GraphView v = g0;
    if (g0.tw > 0) {
        lv::Sweeper sw(s, t);
        lv::Contractor ct(s, t);
        sw.set_tuning(tn);
        sw.reserve(n0, nnz0);
        ct.reserve(n0, nnz0);
        DevBuf<int32_t> newlab((size_t)n0);
        DevBuf<int32_t> merged;   // labels after the final merge (allocated when used)
        // levels below 2^31 total weight keep int32 weights (every weight
        // of a contracted graph is at most 2W)
        const bool narrow = g0.tw < lv::kCompactTwMax;
        struct LevelGraph {
            DevBuf<int64_t> rp, delta, w64;
            DevBuf<int32_t> col, w32;
        } lg[2];
        int which = 0;
        const lv::SweepParams sp = sweep_params(prm);
        // level 0 in row-length order (results unchanged): v is the rebuilt
        // graph, vertex p starts alone in community order[p], and the final
        // labels start as every vertex's position
        lv::ReorderedGraph rg;
        bool permuted = lv::reorder_applies(g0, tn);
        if (permuted) {
            v = rg.build(g0, s, t);
            LV_HIP(hipMemcpyAsync(fin_p, rg.pos.p, (size_t)n0 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        }
        bool cut_sorted = false;   // the last contraction (a cut run's) sorted its rows
        for (int level = 0; level < prm.max_levels; ++level) {
            const size_t rec0 = timer.recs.size();
            char rname[48];
            snprintf(rname, sizeof rname, "louvain level %d: sweeps", level);
            std::unique_ptr<lv::Range> range(new lv::Range(rname));
            sw.plan(v);
            if (permuted)
                sw.init_singletons(v, rg.order.p);
            else
                sw.init_singletons(v);
            lv::PhaseState st;
            int p = 0;
            std::vector<size_t> pass_rec;   // timer records before each enqueued pass
            auto enqueue = [&](int count) {
                for (int b = 0; b < count; ++b) {
                    pass_rec.push_back(timer.recs.size());
                    sw.pass(v, ++p, sp, nullptr);
                }
            };
            // batch passes per host check of the phase state; one pass is
            // enqueued ahead of each check, so the device does not idle on
            // the round trip (passes after the phase's end return at once)
            enqueue(batch);
            std::unique_ptr<lv::Readback> rb(new lv::Readback(s));
            const lv::PhaseState *hst = rb->add(sw.states());
            rb->issue();
            for (;;) {
                enqueue(1);
                rb->wait();
                st = *hst;
                if (st.done) break;
                require(p <= prm.max_sweeps + 4 + 2 * batch, LOUVAIN_EDEVICE, "sweep loop did not converge");
                enqueue(batch - 1);
                rb.reset(new lv::Readback(s));
                hst = rb->add(sw.states());
                rb->issue();
            }
            // the launches of passes past the phase's end returned at once:
            // they do none of the method's work and stay out of the statistics
            if (timing && st.pass >= 0 && (size_t)st.pass < pass_rec.size())
                for (size_t r = pass_rec[(size_t)st.pass]; r < timer.recs.size(); ++r) timer.recs[r].launched = false;
            range.reset();
            if (lv::log_on())
                fprintf(stderr, "[louvain] level %d: n %lld, nnz %lld, %s, passes %d, sweeps kept %d%s\n", level,
                        (long long)v.n, (long long)v.nnz, sw.score_kind(), st.pass, st.accepted,
                        st.limit ? " (max_sweeps)" : "");
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
                // nothing renumbered: the final labels are the identity, not the level-0 positions
                if (permuted) lv::iota_i32(fin_p, n0, s);
                if (timing == 1) {
                    LV_HIP(hipStreamSynchronize(s));
                    collect_kernel_stats(timer, nullptr, rec0, timer.recs.size(), &ls.ms_sweep, &ls.ms_contract);
                }
                break;
            }
            const int32_t *cfin = sw.slot(st.final_slot);
            if (prm.merge) {
                // the final merge on the phase's labels, then Q once more
                if (!merged.p) merged.alloc((size_t)n0);
                lv::merge_lone(v, cfin, sp.singlet, merged.p, s, t);
                cfin = merged.p;
                q_final = lv::modularity_int(v, cfin, s, t);
                ls.q_int.lo = (uint64_t)q_final;
                ls.q_int.hi = (int64_t)(q_final >> 64);
            }
            snprintf(rname, sizeof rname, "louvain level %d: contraction", level);
            lv::Range crange(rname);
            const int64_t k = ct.renumber(cfin, v.n, newlab.p);
            ct.compose(fin_p, n0, newlab.p);
            // after composing, fin_p holds level 0's map in the given vertex order
            if (sink) sink->map(permuted ? fin_p : newlab.p, v.n, k, s);
            const bool cut = level + 1 >= prm.max_levels;
            if (cut && !sink) {
                status = LOUVAIN_ELIMIT;
                if (timing == 1) {
                    LV_HIP(hipStreamSynchronize(s));
                    collect_kernel_stats(timer, nullptr, rec0, timer.recs.size(), &ls.ms_sweep, &ls.ms_contract);
                }
                break;
            }
            LevelGraph &nb = lg[which];
            if (!nb.rp.p) {
                nb.rp.alloc((size_t)n0 + 1);
                nb.delta.alloc((size_t)n0);
                if (narrow)
                    nb.w32.alloc((size_t)nnz0);
                else
                    nb.w64.alloc((size_t)nnz0);
                nb.col.alloc((size_t)nnz0);
            }
            void *wout = narrow ? (void *)nb.w32.p : (void *)nb.w64.p;
            const int64_t m2 = ct.contract(v, newlab.p, k, nb.rp.p, nb.col.p, wout, narrow ? 4 : 8, nb.delta.p,
                                           sink != nullptr && cut, lv::lds_row_max(k, g0.tw, tn));
            lv::GraphView v2;
            v2.n = k;
            v2.nnz = m2;
            v2.row_ptr = nb.rp.p;
            v2.col = nb.col.p;
            v2.w = wout;
            v2.wbytes = narrow ? 4 : 8;
            v2.delta = nb.delta.p;
            v2.tw = g0.tw;
            v = v2;
            permuted = false;
            which = 1 - which;
            if (timing == 1) {
                LV_HIP(hipStreamSynchronize(s));
                collect_kernel_stats(timer, nullptr, rec0, timer.recs.size(), &ls.ms_sweep, &ls.ms_contract);
            }
            if (cut) {
                status = LOUVAIN_ELIMIT;
                cut_sorted = sink != nullptr;
                break;
            }
        }
        // the caller's graph has ascending columns (checked when it was
        // created); a contraction's are ascending only when it was the cut one
        if (sink) sink->last(permuted ? g0 : v, permuted || v.row_ptr == g0.row_ptr || cut_sorted, s);
    } else if (sink) {
        sink->last(v, true, s);
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
    *q_out = q_final;
    *stats_out = local;
    return status;
}

}  // namespace lv

namespace {

// Timing request of a stats record, installed on the context's timer.
int timing_of(louvain_ctx ctx, const louvain_run_stats *stats) {
    const int timing = stats ? stats->timing : 0;
    require(timing >= 0 && timing <= 2, LOUVAIN_EINVAL, "stats->timing must be 0, 1 or 2");
    if (timing == 2) {
        char only[sizeof stats->timing_only + 1];
        memcpy(only, stats->timing_only, sizeof stats->timing_only);
        only[sizeof stats->timing_only] = 0;
        ctx->timer.only = only;
    }
    return timing;
}

void stats_out(louvain_run_stats *stats, louvain_run_stats &local) {
    if (!stats) return;
    local.timing = stats->timing;
    memcpy(local.timing_only, stats->timing_only, sizeof local.timing_only);
    *stats = local;
}

// louvain_run, keeping the dendrogram when dendro_out is set.
int run_graph(louvain_ctx ctx, louvain_graph g, const louvain_params *params, int32_t *labels_out,
              louvain_i128 *q_int, double *q, louvain_run_stats *stats, louvain_dendro *dendro_out, uint32_t flags) {
    int status = LOUVAIN_OK;
    const int rc = guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(labels_out != nullptr || g->n == 0, LOUVAIN_EINVAL, "labels_out must not be NULL");
        const louvain_params prm = checked_params(params);
        hipStream_t s = ctx->stream;
        const int timing = timing_of(ctx, stats);
        std::unique_ptr<louvain_dendro_s> d;
        std::unique_ptr<DendroSink> sink;
        if (dendro_out) {
            d.reset(new louvain_dendro_s());
            d->pool = ctx->pool;
            d->ctx = ctx;
            d->device = ctx->device;
            d->n.push_back(g->n);
            sink.reset(new DendroSink(d.get()));
        }
        louvain_run_stats local;
        DevBuf<int32_t> fin((size_t)g->n);
        lv::i128 q_final = 0;
        status = lv::run_plain(g->view(), prm, ctx->tuning, s, ctx->timer, timing, fin.p, &q_final, &local,
                               sink.get());
        copy_out(labels_out, fin.p, g->n, device_ptrs(flags), s);
        LV_HIP(hipStreamSynchronize(s));
        if (q_int) *q_int = to_abi(q_final);
        if (q) *q = q_of(q_final, g->tw);
        stats_out(stats, local);
        if (dendro_out) *dendro_out = d.release();
    });
    if (ctx) {
        ctx->timer.on = false;
        ctx->timer.only.clear();
    }
    return rc != LOUVAIN_OK ? rc : status;
}

}  // namespace

// ------------------------------------------------- allocation-free modularity --
//
// louvain_modularity_noalloc uses one file-scope device array as its
// workspace: a label-check flag, a device copy of host labels, and the
// modularity workspace (deg_C by label, per-block partial sums).  Each GPU
// holds its own copy for the life of the process; its address is looked up
// once per device when the first context on that device is created, and
// the kernels get that address (the array's name is only a host-side
// stand-in).  Calls on one GPU take a per-device lock for their whole
// duration (each ends by reading its result back), so they never overlap
// on the array.
namespace {

constexpr int64_t kNoAllocMaxN = LOUVAIN_NOALLOC_MAX_N;
constexpr size_t kScratchFlag = 0;
constexpr size_t kScratchLabels = 256;
constexpr size_t kScratchWs = kScratchLabels + (size_t)kNoAllocMaxN * sizeof(int32_t);
constexpr size_t kScratchBytes =
    kScratchWs + (size_t)kNoAllocMaxN * sizeof(int64_t) + (size_t)(2 * ((kNoAllocMaxN + 2047) / 2048) + 4) * 8;
static_assert(kScratchLabels % 256 == 0 && kScratchWs % 256 == 0, "scratch regions are 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_call_mu[kMaxDevices];

// Address of this device's copy of the scratch array (the device must be current).
int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return LOUVAIN_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return LOUVAIN_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return LOUVAIN_EDEVICE;
    }
    g_scratch_ptr[device] = ptr;
    return LOUVAIN_OK;
}

}  // namespace

extern "C" {

int louvain_ctx_create(int device, void *hip_stream, void *pool, size_t pool_bytes, const char *tuning_path,
                       louvain_ctx *out) {
    if (!out || device < 0) return LOUVAIN_EINVAL;
    if ((pool == nullptr) != (pool_bytes == 0)) return LOUVAIN_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        return LOUVAIN_EDEVICE;
    }
    try {
        std::unique_ptr<louvain_ctx_s> c(new louvain_ctx_s());
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        c->timer.stream = c->stream;
        {
            // the device's copy of the no-allocation scratch array, looked up with the device current
            int prev = 0;
            if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
                (void)hipGetLastError();
                return LOUVAIN_EDEVICE;
            }
            const int rc = scratch_setup(device);
            (void)hipSetDevice(prev);
            if (rc != LOUVAIN_OK) return rc;
        }
        if (pool) {
            // the region must be device memory of this device
            hipPointerAttribute_t attr;
            if (hipPointerGetAttributes(&attr, pool) != hipSuccess || attr.type != hipMemoryTypeDevice ||
                attr.device != device) {
                (void)hipGetLastError();
                return LOUVAIN_EINVAL;
            }
            c->arena = std::make_shared<lv::Arena>(pool, pool_bytes);
        }
        c->pool = std::make_shared<lv::Pool>(c->arena);
        if (const char *f = getenv("LOUVAIN_FAULT_ALLOC_AT")) c->pool->fault_at = atol(f);
        if (tuning_path && *tuning_path) {
            c->tuning_path = tuning_path;
            lv::Tuning tn;
            if (load_tuning(c->tuning_path, device_arch(device), &tn)) c->tuning = tn;
        }
        *out = c.release();
        return LOUVAIN_OK;
    } catch (const Error &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return LOUVAIN_ENOMEM;
    } catch (...) {
        return LOUVAIN_EDEVICE;
    }
}

int louvain_ctx_destroy(louvain_ctx ctx) {
    if (!ctx) return LOUVAIN_EINVAL;
    if (ctx->owner.load() != 0) return LOUVAIN_EBUSY;
    (void)hipSetDevice(ctx->device);
    ctx->server.reset();   // stops the request loop first
    delete ctx;
    return LOUVAIN_OK;
}

int louvain_memory_stats(louvain_ctx ctx, louvain_memory *out) {
    if (!ctx || !out) return LOUVAIN_EINVAL;
    memset(out, 0, sizeof *out);
    {
        std::lock_guard<std::mutex> lk(ctx->pool->mu);
        out->live_bytes = ctx->pool->in_use;
        out->cached_bytes = ctx->pool->cached;
    }
    if (ctx->arena) {
        std::lock_guard<std::mutex> lk(ctx->arena->mu);
        out->pool_bytes = ctx->arena->bytes;
        out->pool_in_use = ctx->arena->in_use;
        out->pool_high_water = ctx->arena->high;
    }
    return LOUVAIN_OK;
}

int louvain_memory_reset_peak(louvain_ctx ctx) {
    if (!ctx) return LOUVAIN_EINVAL;
    if (ctx->arena) {
        std::lock_guard<std::mutex> lk(ctx->arena->mu);
        ctx->arena->high = ctx->arena->in_use;
    }
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
        sw.set_tuning(ctx->tuning);
        sw.reserve(v.n, v.nnz);
        sw.plan(v);
        if (labels) sw.init_from_labels(v, lin.p); else sw.init_singletons(v);
        DevBuf<int64_t> eself((size_t)g->n);
        lv::fill<int64_t>(eself.p, 0, g->n, s);
        lv::SweepParams prm;
        prm.singlet = (flags & LOUVAIN_NO_SINGLET) ? 0 : 1;
        sw.pass(v, 1, prm, eself.p);
        if (sw.compact()) sw.e_self_out(eself.p);
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

int louvain_modularity_noalloc(louvain_ctx ctx, louvain_graph g, const int32_t *labels, louvain_i128 *q_int,
                               double *q, uint32_t flags) {
    return guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(q_int != nullptr, LOUVAIN_EINVAL, "q_int must not be NULL");
        require(g->n <= kNoAllocMaxN, LOUVAIN_EINVAL,
                "n = " + std::to_string(g->n) + " exceeds the limit of louvain_modularity_noalloc (" +
                    std::to_string(kNoAllocMaxN) + " vertices)");
        require(labels != nullptr || g->n == 0, LOUVAIN_EINVAL, "labels must not be NULL");
        require(ctx->device >= 0 && ctx->device < kMaxDevices && g_scratch_ptr[ctx->device], LOUVAIN_EDEVICE,
                "the scratch array of this device was not set up");
        std::lock_guard<std::mutex> lk(g_scratch_call_mu[ctx->device]);
        char *base = (char *)g_scratch_ptr[ctx->device];
        hipStream_t s = ctx->stream;
        const int64_t n = g->n;
        const int32_t *lab = labels;
        if (n > 0) {
            int *flag = (int *)(base + kScratchFlag);
            if (!device_ptrs(flags)) {
                int32_t *copy = (int32_t *)(base + kScratchLabels);
                LV_HIP(hipMemcpyAsync(copy, labels, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
                lab = copy;
            }
            lv::fill<int32_t>(flag, 0, 1, s);
            k_label_range<<<lv::grid_for(n, 256), 256, 0, s>>>(lab, n, n, flag);
            LV_LAUNCHED("k_label_range");
            int bad = 0;
            LV_HIP(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s));
            LV_HIP(hipStreamSynchronize(s));
            require(bad == 0, LOUVAIN_EINVAL, "label out of range [0, " + std::to_string(n) + ")");
        }
        const lv::i128 v = lv::modularity_int(g->view(), lab, s, nullptr, base + kScratchWs);
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
        g2->nnz = ct.contract(g->view(), newlab.p, k, g2->row_ptr.p, g2->col.p, g2->w64.p, 8, g2->delta.p, true);
        g2->tw = g->tw;
        copy_out(renumber_out, newlab.p, g->n, device_ptrs(flags), s);
        LV_HIP(hipStreamSynchronize(s));
        *out = g2.release();
    });
}

int louvain_run(louvain_ctx ctx, louvain_graph g, const louvain_params *params, int32_t *labels_out,
                louvain_i128 *q_int, double *q, louvain_run_stats *stats, uint32_t flags) {
    return run_graph(ctx, g, params, labels_out, q_int, q, stats, nullptr, flags);
}

int louvain_run_dendro(louvain_ctx ctx, louvain_graph g, const louvain_params *params, int32_t *labels_out,
                       louvain_i128 *q_int, double *q, louvain_run_stats *stats, louvain_dendro *dendro_out,
                       uint32_t flags) {
    if (!dendro_out) {
        if (ctx) ctx->err = "dendro_out must not be NULL";
        return LOUVAIN_EINVAL;
    }
    return run_graph(ctx, g, params, labels_out, q_int, q, stats, dendro_out, flags);
}

int louvain_dendro_info(louvain_dendro d, int32_t *levels, int64_t *n) {
    if (!d) return LOUVAIN_EINVAL;
    if (levels) *levels = (int32_t)d->maps.size();
    if (n)
        for (size_t l = 0; l < d->n.size(); ++l) n[l] = d->n[l];
    return LOUVAIN_OK;
}

int louvain_dendro_map(louvain_dendro d, int32_t level, int32_t *map_out, uint32_t flags) {
    if (!d) return LOUVAIN_EINVAL;
    louvain_ctx ctx = d->ctx;
    return guarded(ctx, [&] {
        require(level >= 0 && (size_t)level < d->maps.size(), LOUVAIN_EINVAL, "no such dendrogram level");
        const int64_t n = d->n[(size_t)level];
        require(map_out != nullptr || n == 0, LOUVAIN_EINVAL, "map_out must not be NULL");
        copy_out(map_out, d->maps[(size_t)level].p, n, device_ptrs(flags), ctx->stream);
        LV_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int louvain_dendro_graph(louvain_dendro d, louvain_graph *out) {
    if (!d) return LOUVAIN_EINVAL;
    return guarded(d->ctx, [&] {
        require(out != nullptr, LOUVAIN_EINVAL, "out must not be NULL");
        require(d->graph != nullptr, LOUVAIN_EINVAL, "the dendrogram's graph was already handed out");
        *out = d->graph.release();
    });
}

int louvain_dendro_destroy(louvain_dendro d) {
    if (!d) return LOUVAIN_EINVAL;
    (void)hipSetDevice(d->device);
    delete d;
    return LOUVAIN_OK;
}

int louvain_resume(louvain_ctx ctx, louvain_graph g, const louvain_params *params, int32_t levels_done, int64_t n0,
                   const int32_t *labels_so_far, int32_t *labels_out, louvain_i128 *q_int, double *q,
                   louvain_run_stats *stats, uint32_t flags) {
    int status = LOUVAIN_OK;
    const int rc = guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        require(n0 >= 0 && n0 < ((int64_t)1 << 31), LOUVAIN_EINVAL, "n0 must be in [0, 2^31)");
        require(labels_out != nullptr || n0 == 0, LOUVAIN_EINVAL, "labels_out must not be NULL");
        require(levels_done >= 0, LOUVAIN_EINVAL, "levels_done must be >= 0");
        louvain_params prm = checked_params(params);
        hipStream_t s = ctx->stream;
        const int timing = timing_of(ctx, stats);
        lv::Timer *t = timing ? &ctx->timer : nullptr;
        DevBuf<int32_t> fin = labels_in(ctx, labels_so_far, n0, flags, g->n);
        louvain_run_stats local;
        memset(&local, 0, sizeof local);
        lv::i128 q_final = 0;
        if (levels_done >= prm.max_levels) {
            // no phase left: the partition so far, whose Q_int on g is that of g's singletons
            status = LOUVAIN_ELIMIT;
            local.status = status;
            if (g->tw > 0) {
                DevBuf<int32_t> iota((size_t)g->n);
                lv::iota_i32(iota.p, g->n, s);
                q_final = lv::modularity_int(g->view(), iota.p, s, nullptr);
            }
        } else {
            prm.max_levels -= levels_done;
            DevBuf<int32_t> lvl((size_t)g->n);
            status = lv::run_plain(g->view(), prm, ctx->tuning, s, ctx->timer, timing, lvl.p, &q_final, &local);
            lv::Contractor ct(s, t);
            ct.compose(fin.p, n0, lvl.p);
        }
        copy_out(labels_out, fin.p, n0, device_ptrs(flags), s);
        LV_HIP(hipStreamSynchronize(s));
        if (q_int) *q_int = to_abi(q_final);
        if (q) *q = q_of(q_final, g->tw);
        stats_out(stats, local);
    });
    if (ctx) {
        ctx->timer.on = false;
        ctx->timer.only.clear();
    }
    return rc != LOUVAIN_OK ? rc : status;
}

int louvain_set_tuning(louvain_ctx ctx, const louvain_tuning *tuning) {
    return guarded(ctx, [&] { ctx->tuning = tuning ? tuning_from(*tuning) : lv::Tuning(); });
}

int louvain_get_tuning(louvain_ctx ctx, louvain_tuning *tuning) {
    if (!ctx || !tuning) return LOUVAIN_EINVAL;
    *tuning = tuning_to(ctx->tuning);
    return LOUVAIN_OK;
}

int louvain_autotune(louvain_ctx ctx, louvain_graph g, const louvain_params *params, louvain_tuning *best) {
    return guarded(ctx, [&] {
        require(g != nullptr && g->ctx == ctx, LOUVAIN_EINVAL, "graph missing or from another context");
        louvain_params prm = checked_params(params);
        prm.pass_batch = 0;   // the candidates' pass batching applies
        if (g->tw >= lv::kCompactTwMax || g->n == 0) {
            if (best) {
                *best = tuning_to(ctx->tuning);
                best->ms = -1.0;
            }
            return;
        }
        hipStream_t s = ctx->stream;
        DevBuf<int32_t> fin((size_t)g->n);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        struct EvGuard {
            hipEvent_t *a, *b;
            ~EvGuard() {
                if (*a) (void)hipEventDestroy(*a);
                if (*b) (void)hipEventDestroy(*b);
            }
        } evg{&e0, &e1};
        LV_HIP(hipEventCreate(&e0));
        LV_HIP(hipEventCreate(&e1));
        auto time_run = [&](const lv::Tuning &tn) {
            lv::i128 q;
            louvain_run_stats st;
            LV_HIP(hipEventRecord(e0, s));
            (void)lv::run_plain(g->view(), prm, tn, s, ctx->timer, 0, fin.p, &q, &st);
            LV_HIP(hipEventRecord(e1, s));
            LV_HIP(hipEventSynchronize(e1));
            float ms = 0;
            LV_HIP(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms;
        };
        (void)time_run(ctx->tuning);   // warm-up (allocations, code loading)
        const lv::Tuning cur = ctx->tuning;
        const double cur_ms = std::min(time_run(cur), time_run(cur));
        lv::Tuning pick = cur;
        double pick_ms = cur_ms;
        for (int sm : {4, 8})
            for (int64_t bm : {(int64_t)1365, (int64_t)2730, lv::kCompactBlockMax})
                for (int pb : {1, 2})
                    for (int gv : {1, 2})
                        for (int gt : {1, 4}) {
                            if (gv == 2 && gt > 1) continue;   // pipelining takes one vertex per group
                            lv::Tuning tn;
                            tn.small_max = sm;
                            tn.block_max = bm;
                            tn.pass_batch = pb;
                            tn.group_vertices = gv;
                            tn.group_tiles = gt;
                            tn.overlap = cur.overlap;
                            tn.reorder = cur.reorder;
                            const double ms = std::min(time_run(tn), time_run(tn));
                            if (ms < pick_ms && ms < 0.98 * cur_ms) {
                                pick_ms = ms;
                                pick = tn;
                            }
                        }
        ctx->tuning = pick;
        if (!ctx->tuning_path.empty()) save_tuning(ctx->tuning_path, device_arch(ctx->device), pick, pick_ms);
        if (best) {
            *best = tuning_to(pick);
            best->ms = pick_ms;
        }
    });
}

int louvain_autotune_batch(louvain_ctx ctx, int64_t ngraphs, const louvain_graph *graphs,
                           const louvain_params *params, louvain_tuning *best) {
    return guarded(ctx, [&] {
        require(ngraphs > 0 && graphs != nullptr, LOUVAIN_EINVAL, "ngraphs must be > 0 and graphs not NULL");
        std::vector<lv::GraphView> views;
        int64_t n_total = 0;
        for (int64_t i = 0; i < ngraphs; ++i) {
            require(graphs[i] != nullptr && graphs[i]->ctx == ctx, LOUVAIN_EINVAL,
                    "graph " + std::to_string(i) + " missing or from another context");
            if (graphs[i]->tw < lv::kCompactTwMax) {   // heavier graphs run alone and ignore the shapes
                views.push_back(graphs[i]->view());
                n_total += graphs[i]->n;
            }
        }
        louvain_params prm = checked_params(params);
        prm.pass_batch = 0;   // the candidates' pass batching applies
        if (views.empty() || n_total == 0) {
            if (best) {
                *best = tuning_to(ctx->tuning);
                best->ms = -1.0;
            }
            return;
        }
        hipStream_t s = ctx->stream;
        DevBuf<int32_t> fin((size_t)n_total);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        struct EvGuard {
            hipEvent_t *a, *b;
            ~EvGuard() {
                if (*a) (void)hipEventDestroy(*a);
                if (*b) (void)hipEventDestroy(*b);
            }
        } evg{&e0, &e1};
        LV_HIP(hipEventCreate(&e0));
        LV_HIP(hipEventCreate(&e1));
        // one batched call's device time under a setting (as louvain_run_batch runs it)
        auto time_batch = [&](const lv::Tuning &tn) {
            std::vector<lv::BatchMember> mem(views.size());
            LV_HIP(hipEventRecord(e0, s));
            lv::BatchEngine eng(s, nullptr, sweep_params(prm), prm.max_levels, tn.pass_batch);
            eng.set_tuning(tn);
            int64_t off = 0;
            for (size_t k = 0; k < views.size(); ++k) {
                mem[k].g0 = views[k];
                mem[k].fin = fin.p + off;
                off += views[k].n;
                eng.admit(&mem[k]);
            }
            while (!eng.idle()) eng.step();
            LV_HIP(hipEventRecord(e1, s));
            LV_HIP(hipEventSynchronize(e1));
            float ms = 0;
            LV_HIP(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms;
        };
        auto best_of_two = [&](const lv::Tuning &tn) { return std::min(time_batch(tn), time_batch(tn)); };
        (void)time_batch(ctx->tuning);   // warm-up (allocations, code loading)
        const lv::Tuning cur = ctx->tuning;
        lv::Tuning pick = cur;
        double pick_ms = best_of_two(cur);
        // coordinate descent, one round over the fields: each value of a field
        // with the others at the best setting so far; a change is kept only
        // when it is more than 2% faster than that setting
        auto try_field = [&](auto set, std::initializer_list<int64_t> values) {
            lv::Tuning base = pick;
            const double base_ms = pick_ms;
            for (int64_t v : values) {
                lv::Tuning tn = base;
                set(tn, v);
                const double ms = best_of_two(tn);
                if (ms < pick_ms && ms < 0.98 * base_ms) {
                    pick_ms = ms;
                    pick = tn;
                }
            }
        };
        try_field([](lv::Tuning &t, int64_t v) { t.small_max = (int)v; }, {2, 4, 8});
        try_field([](lv::Tuning &t, int64_t v) { t.group_slots = (int)v; }, {2, 4, 8});
        try_field([](lv::Tuning &t, int64_t v) { t.group_vertices = (int)v; }, {1, 2});
        try_field([](lv::Tuning &t, int64_t v) { t.group_tiles = (int)v; }, {1, 2, 4});
        try_field([](lv::Tuning &t, int64_t v) { t.block_max = v; }, {1365, 2730, lv::kCompactBlockMax});
        try_field([](lv::Tuning &t, int64_t v) { t.pass_batch = (int)v; }, {1, 2, 4});
        ctx->tuning = pick;
        if (!ctx->tuning_path.empty()) save_tuning(ctx->tuning_path, device_arch(ctx->device), pick, pick_ms);
        if (best) {
            *best = tuning_to(pick);
            best->ms = pick_ms;
        }
    });
}

size_t louvain_workspace_bytes(int64_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    return lv::Server::workspace_bytes(n, nnz);
}

int louvain_serve_budget(louvain_ctx ctx, size_t hbm_bytes) {
    if (!ctx) return LOUVAIN_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->serve_mu);
    ctx->serve_budget = hbm_bytes;
    if (ctx->server && hbm_bytes > 0) ctx->server->set_budget(hbm_bytes);
    return LOUVAIN_OK;
}

int louvain_submit(louvain_ctx ctx, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                   const void *weight, const louvain_params *params, int32_t *labels_out, uint32_t flags,
                   uint64_t *ticket) {
    if (!ctx || !ticket) return LOUVAIN_EINVAL;
    if (n < 0 || nnz < 0 || !row_ptr || (nnz > 0 && (!col_idx || !weight)) || (n > 0 && !labels_out) ||
        (n == 0 && nnz > 0))
        return LOUVAIN_EINVAL;
    if (n >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 40)) return LOUVAIN_EOVERFLOW;
    louvain_params prm{1, 1000000, 1000, 64, 1, 0, 0, 0};
    if (params) prm = *params;
    if (prm.theta_num < 0 || prm.theta_den <= 0 || prm.max_sweeps < 0 || prm.max_levels < 1 || prm.max_levels > 64 ||
        (prm.merge != 0 && prm.merge != 1) || prm.reserved != 0)
        return LOUVAIN_EINVAL;
    try {
        std::unique_ptr<lv::ServeRequest> r(new lv::ServeRequest());
        r->n = n;
        r->nnz = nnz;
        r->rp = row_ptr;
        r->col = col_idx;
        r->w = weight;
        r->wbytes = (flags & LOUVAIN_WEIGHTS_I64) ? 8 : 4;
        r->dev = device_ptrs(flags);
        r->check_symmetry = (flags & LOUVAIN_CHECK_SYMMETRY) != 0;
        r->prm = prm;
        r->labels_out = labels_out;
        lv::Server *srv;
        {
            std::lock_guard<std::mutex> lk(ctx->serve_mu);
            if (!ctx->server) {
                size_t budget = ctx->serve_budget;
                if (budget == 0 && ctx->arena) {
                    std::lock_guard<std::mutex> alk(ctx->arena->mu);
                    budget = (ctx->arena->bytes - ctx->arena->in_use) / 10 * 8;
                }
                if (budget == 0) {
                    size_t free_b = 0, total_b = 0;
                    if (hipSetDevice(ctx->device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
                        (void)hipGetLastError();
                        return LOUVAIN_EDEVICE;
                    }
                    budget = free_b / 10 * 8;
                }
                ctx->server.reset(new lv::Server(ctx->device, budget, ctx->tuning, ctx->arena));
            }
            srv = ctx->server.get();
        }
        *ticket = srv->submit(std::move(r));
        return LOUVAIN_OK;
    } catch (const std::bad_alloc &) {
        return LOUVAIN_ENOMEM;
    } catch (...) {
        return LOUVAIN_EDEVICE;
    }
}

int louvain_poll(louvain_ctx ctx, uint64_t ticket, int32_t wait_us, louvain_request_result *result) {
    if (!ctx) return LOUVAIN_EINVAL;
    lv::Server *srv;
    {
        std::lock_guard<std::mutex> lk(ctx->serve_mu);
        srv = ctx->server.get();
    }
    if (!srv) return LOUVAIN_EINVAL;
    std::unique_ptr<lv::ServeRequest> r;
    const int st = srv->poll(ticket, wait_us, &r);
    if (st == LOUVAIN_EAGAIN || !r) return st;
    if (result) {
        memset(result, 0, sizeof *result);
        result->status = r->status;
        result->levels = (int32_t)r->levels.size();
        result->n = r->n;
        result->nnz = r->nnz;
        result->total_edges_swept = r->edges_swept;
        result->q_int = to_abi(r->q);
        result->q = q_of(r->q, r->tw);
        result->t_submit_us = r->t_submit;
        result->t_admit_us = r->t_admit;
        result->t_done_us = r->t_done;
        for (size_t l = 0; l < r->levels.size() && l < 64; ++l) {
            const lv::LevelRec &x = r->levels[l];
            louvain_level_stats &ls = result->level[l];
            ls.n = x.n;
            ls.nnz = x.nnz;
            ls.sweeps_executed = x.executed;
            ls.sweeps_accepted = x.accepted;
            ls.gpu_passes = x.passes;
            ls.q_int = to_abi(x.q);
        }
        strncpy(result->error, r->err.c_str(), sizeof result->error - 1);
    }
    return st;
}

int louvain_run_batch(louvain_ctx ctx, int64_t ngraphs, const louvain_graph *graphs, const louvain_params *params,
                      int32_t *const *labels_out, louvain_i128 *q_int, double *q, int32_t *status_out,
                      louvain_run_stats *stats, uint32_t flags) {
    int status = LOUVAIN_OK;
    const int rc = guarded(ctx, [&] {
        require(ngraphs >= 0, LOUVAIN_EINVAL, "ngraphs must be >= 0");
        if (ngraphs == 0) return;
        require(graphs != nullptr && labels_out != nullptr, LOUVAIN_EINVAL, "graphs and labels_out must not be NULL");
        for (int64_t i = 0; i < ngraphs; ++i) {
            require(graphs[i] != nullptr && graphs[i]->ctx == ctx, LOUVAIN_EINVAL,
                    "graph " + std::to_string(i) + " missing or from another context");
            require(labels_out[i] != nullptr || graphs[i]->n == 0, LOUVAIN_EINVAL,
                    "labels_out[" + std::to_string(i) + "] must not be NULL");
        }
        const louvain_params prm = checked_params(params);
        hipStream_t s = ctx->stream;
        const bool dev = device_ptrs(flags);
        const int32_t timing = stats ? stats[0].timing : 0;
        std::vector<louvain_run_stats> st_local;
        if (stats) st_local.resize((size_t)ngraphs);

        // graphs too heavy for compact words run alone, first
        std::vector<int64_t> eligible;
        std::vector<lv::i128> qv((size_t)ngraphs, 0);
        std::vector<int32_t> sv((size_t)ngraphs, LOUVAIN_OK);
        for (int64_t i = 0; i < ngraphs; ++i) {
            if (graphs[i]->tw < lv::kCompactTwMax) {
                eligible.push_back(i);
                continue;
            }
            louvain_i128 qi;
            louvain_run_stats *si = stats ? &st_local[(size_t)i] : nullptr;
            if (si) si->timing = 0;
            const int r = louvain_run(ctx, graphs[i], &prm, labels_out[i], &qi, nullptr, si, flags);
            if (r != LOUVAIN_OK && r != LOUVAIN_ELIMIT) throw Error(r, ctx->err);
            qv[(size_t)i] = lv::make_i128(qi.lo, qi.hi);
            sv[(size_t)i] = r;
        }

        lv::Timer &timer = ctx->timer;
        require(timing >= 0 && timing <= 2, LOUVAIN_EINVAL, "stats[0].timing must be 0, 1 or 2");
        timer.on = timing != 0;
        timer.only.clear();
        if (timing == 2) {
            char only[sizeof stats[0].timing_only + 1];
            memcpy(only, stats[0].timing_only, sizeof stats[0].timing_only);
            only[sizeof stats[0].timing_only] = 0;
            timer.only = only;
        }
        timer.reset();
        lv::Timer *t = timing ? &timer : nullptr;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        struct EvGuard {
            hipEvent_t *a, *b;
            ~EvGuard() {
                if (*a) (void)hipEventDestroy(*a);
                if (*b) (void)hipEventDestroy(*b);
            }
        } evg{&ev0, &ev1};
        if (timing) {
            LV_HIP(hipEventCreate(&ev0));
            LV_HIP(hipEventCreate(&ev1));
            LV_HIP(hipEventRecord(ev0, s));
        }
        const int64_t ne = (int64_t)eligible.size();
        std::vector<int64_t> off((size_t)ne + 1, 0);
        for (int64_t k = 0; k < ne; ++k) off[(size_t)k + 1] = off[(size_t)k] + graphs[eligible[(size_t)k]]->n;
        DevBuf<int32_t> fin((size_t)off[(size_t)ne]);
        std::vector<lv::BatchMember> mem((size_t)ne);
        lv::BatchEngine eng(s, t, sweep_params(prm), prm.max_levels,
                            prm.pass_batch > 0 ? prm.pass_batch : ctx->tuning.pass_batch);
        eng.set_tuning(ctx->tuning);
        for (int64_t k = 0; k < ne; ++k) {
            lv::BatchMember &m = mem[(size_t)k];
            m.g0 = graphs[eligible[(size_t)k]]->view();
            m.fin = fin.p + off[(size_t)k];
            eng.admit(&m);
        }
        while (!eng.idle()) eng.step();

        // outputs
        if (dev) {
            std::vector<int32_t *> dst((size_t)ne);
            std::vector<int64_t> cnt((size_t)ne);
            for (int64_t k = 0; k < ne; ++k) {
                dst[(size_t)k] = labels_out[eligible[(size_t)k]];
                cnt[(size_t)k] = mem[(size_t)k].g0.n;
            }
            lv::copy_segments(dst.data(), cnt.data(), off.data(), ne, fin.p, s);
        } else if (off[(size_t)ne] > 0) {
            std::vector<int32_t> host((size_t)off[(size_t)ne]);
            LV_HIP(hipMemcpyAsync(host.data(), fin.p, host.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            LV_HIP(hipStreamSynchronize(s));
            for (int64_t k = 0; k < ne; ++k)
                if (mem[(size_t)k].g0.n > 0)
                    memcpy(labels_out[eligible[(size_t)k]], host.data() + off[(size_t)k],
                           (size_t)mem[(size_t)k].g0.n * sizeof(int32_t));
        }
        for (int64_t k = 0; k < ne; ++k) {
            const int64_t i = eligible[(size_t)k];
            qv[(size_t)i] = mem[(size_t)k].q;
            sv[(size_t)i] = mem[(size_t)k].status;
            if (stats) member_stats(mem[(size_t)k], timing, &st_local[(size_t)i]);
        }
        if (timing) {
            LV_HIP(hipEventRecord(ev1, s));
            LV_HIP(hipStreamSynchronize(s));
            float ms = 0;
            LV_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            st_local[0].ms_total = ms;
            st_local[0].n_kernels = 0;
            collect_kernel_stats(timer, &st_local[0], 0, timer.recs.size(), nullptr, nullptr);
        }
        timer.on = false;
        timer.only.clear();
        LV_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < ngraphs; ++i) {
            if (q_int) q_int[i] = to_abi(qv[(size_t)i]);
            if (q) q[i] = q_of(qv[(size_t)i], graphs[i]->tw);
            if (status_out) status_out[i] = sv[(size_t)i];
            if (sv[(size_t)i] == LOUVAIN_ELIMIT) status = LOUVAIN_ELIMIT;
        }
        if (stats) memcpy(stats, st_local.data(), sizeof(louvain_run_stats) * (size_t)ngraphs);
    });
    if (ctx) {
        ctx->timer.on = false;
        ctx->timer.only.clear();
    }
    return rc != LOUVAIN_OK ? rc : status;
}

}  // extern "C"
