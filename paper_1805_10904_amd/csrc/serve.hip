// The request loop (see serve.hpp).
#include <algorithm>
#include <chrono>
#include <cstring>

#include "driver.hpp"
#include "prims.hpp"
#include "serve.hpp"

namespace lv {
namespace {

bool same_params(const louvain_params &a, const louvain_params &b) {
    return a.theta_num == b.theta_num && a.theta_den == b.theta_den && a.max_sweeps == b.max_sweeps &&
           a.max_levels == b.max_levels && (a.singlet_rule != 0) == (b.singlet_rule != 0) &&
           a.pass_batch == b.pass_batch && a.merge == b.merge;
}

SweepParams to_sweep(const louvain_params &p) {
    SweepParams sp;
    sp.theta_num = p.theta_num;
    sp.theta_den = p.theta_den;
    sp.max_sweeps = p.max_sweeps;
    sp.singlet = p.singlet_rule ? 1 : 0;
    sp.merge = p.merge;
    return sp;
}

template <typename T>
void copy_in(T *dst, const T *src, int64_t count, bool dev, hipStream_t s) {
    if (count <= 0) return;
    LV_HIP(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          s));
}

void release_device(ServeRequest *r) {
    r->d_rp.release();
    r->d_delta.release();
    r->d_w64.release();
    r->d_col.release();
    r->d_w32.release();
    r->d_fin.release();
}

// Copy the request's CSR to the device, validate it and compute delta and TW.
void ingest(ServeRequest *r, hipStream_t s) {
    r->d_rp.alloc((size_t)r->n + 1);
    r->d_col.alloc((size_t)r->nnz);
    r->d_delta.alloc((size_t)r->n);
    r->d_fin.alloc((size_t)r->n);
    copy_in(r->d_rp.p, r->rp, r->n + 1, r->dev, s);
    copy_in(r->d_col.p, r->col, r->nnz, r->dev, s);
    if (r->wbytes == 4) {
        r->d_w32.alloc((size_t)r->nnz);
        copy_in(r->d_w32.p, (const int32_t *)r->w, r->nnz, r->dev, s);
        ingest_csr<int32_t>(r->n, r->nnz, r->d_rp.p, r->d_col.p, r->d_w32.p, r->d_delta.p, &r->tw, r->check_symmetry,
                            s, nullptr);
    } else {
        r->d_w64.alloc((size_t)r->nnz);
        copy_in(r->d_w64.p, (const int64_t *)r->w, r->nnz, r->dev, s);
        ingest_csr<int64_t>(r->n, r->nnz, r->d_rp.p, r->d_col.p, r->d_w64.p, r->d_delta.p, &r->tw, r->check_symmetry,
                            s, nullptr);
    }
    GraphView &g = r->member.g0;
    g.n = r->n;
    g.nnz = r->nnz;
    g.row_ptr = r->d_rp.p;
    g.col = r->d_col.p;
    g.w = r->wbytes == 4 ? (const void *)r->d_w32.p : (const void *)r->d_w64.p;
    g.wbytes = r->wbytes;
    g.delta = r->d_delta.p;
    g.tw = r->tw;
    r->member.fin = r->d_fin.p;
    r->member.tag = r;
}

// Labels to the caller's buffer and the result fields from the batch member.
void deliver(ServeRequest *r, hipStream_t s) {
    if (r->n > 0)
        LV_HIP(hipMemcpyAsync(r->labels_out, r->d_fin.p, (size_t)r->n * sizeof(int32_t),
                              r->dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    LV_HIP(hipStreamSynchronize(s));
}

}  // namespace

double Server::now_us() {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t Server::workspace_bytes(int64_t n, int64_t nnz) {
    // resident CSR and labels ~ 20 B/vertex + 12 B/entry; two union buffers
    // with growth slack ~ 40 B/vertex + 30 B/entry; sweep state ~ 80 B/vertex
    // and hub tables up to 24 B/entry, with the hub buckets of levels with
    // 2W >= 2^31 up to 32 B/entry more; contraction sort ~ 45 B/entry
    const double b = 160.0 * (double)n + 160.0 * (double)nnz + (double)(1 << 20);
    return (size_t)b;
}

Server::Server(int device, size_t budget, const Tuning &tn, std::shared_ptr<Arena> arena)
    : device_(device), tuning_(tn), budget_(budget) {
    for (int k = 0; k < kWorkers; ++k) {
        pools_.emplace_back(new Pool(arena));
        workers_.emplace_back(new Worker());
    }
    for (int k = 0; k < kWorkers; ++k)
        workers_[(size_t)k]->th = k == kPlain ? std::thread([this] { loop_plain(); })
                                              : std::thread([this, k] { loop(k); });
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    for (auto &w : workers_)
        if (w->th.joinable()) w->th.join();
    // requests still held release their blocks into the pools, which go last
    all_.clear();
}

uint64_t Server::submit(std::unique_ptr<ServeRequest> r) {
    r->t_submit = now_us();
    r->bytes = workspace_bytes(r->n, r->nnz);
    uint64_t t;
    {
        std::lock_guard<std::mutex> lk(mu_);
        t = next_++;
        r->ticket = t;
        const int k = r->nnz <= kSmallEntries ? kSmall : r->nnz <= kMediumEntries ? kMedium : kLarge;
        workers_[(size_t)k]->incoming.push_back(r.get());
        all_[t] = std::move(r);
    }
    cv_work_.notify_all();
    return t;
}

int Server::poll(uint64_t ticket, int32_t wait_us, std::unique_ptr<ServeRequest> *out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return LOUVAIN_EINVAL;
    ServeRequest *r = it->second.get();
    if (!r->done && wait_us != 0) {
        auto ready = [&] { return r->done; };
        if (wait_us < 0)
            cv_done_.wait(lk, ready);
        else
            cv_done_.wait_for(lk, std::chrono::microseconds(wait_us), ready);
    }
    if (!r->done) return LOUVAIN_EAGAIN;
    const int st = r->status;
    *out = std::move(it->second);
    all_.erase(it);
    return st;
}

void Server::set_budget(size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        budget_ = bytes;
    }
    cv_work_.notify_all();
}

size_t Server::budget() {
    std::lock_guard<std::mutex> lk(mu_);
    return budget_;
}

void Server::finish(ServeRequest *r) {
    release_device(r);
    r->t_done = now_us();
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (r->admitted) in_use_ -= std::min(in_use_, r->bytes);
        r->admitted = false;
        r->done = true;
    }
    cv_done_.notify_all();
    cv_work_.notify_all();   // memory freed: another worker may admit
}

void Server::fail(ServeRequest *r, int code, const std::string &msg) {
    r->status = code;
    r->err = msg;
    finish(r);
}

// Graphs with 2W >= 2^31, ingested by a batched worker: the plain path, one
// at a time, on this worker's stream.
void Server::loop_plain() {
    Worker *w = workers_[kPlain].get();
    current_pool() = pools_[kPlain].get();
    hipStream_t s = nullptr;
    const bool ok =
        hipSetDevice(device_) == hipSuccess && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    Timer timer;
    for (;;) {
        ServeRequest *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_work_.wait(lk, [&] { return stop_ || !w->incoming.empty(); });
            if (stop_) break;
            r = w->incoming.front();
            w->incoming.pop_front();
        }
        if (!ok) {
            fail(r, LOUVAIN_EDEVICE, "the request loop could not set up its device stream");
            continue;
        }
        try {
            louvain_run_stats st;
            r->status = run_plain(r->member.g0, r->prm, tuning_, s, timer, 0, r->d_fin.p, &r->q, &st);
            for (int l = 0; l < st.levels; ++l) {
                LevelRec rec;
                rec.n = st.level[l].n;
                rec.nnz = st.level[l].nnz;
                rec.executed = st.level[l].sweeps_executed;
                rec.accepted = st.level[l].sweeps_accepted;
                rec.passes = st.level[l].gpu_passes;
                rec.q = make_i128(st.level[l].q_int.lo, st.level[l].q_int.hi);
                r->levels.push_back(rec);
            }
            r->edges_swept = st.total_edges_swept;
            deliver(r, s);
            finish(r);
        } catch (const Error &e) {
            (void)hipStreamSynchronize(s);
            fail(r, e.code, e.what());
        } catch (const std::exception &e) {
            (void)hipStreamSynchronize(s);
            fail(r, LOUVAIN_EDEVICE, e.what());
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    for (ServeRequest *r : w->incoming) release_device(r);
    w->incoming.clear();
    if (s) (void)hipStreamDestroy(s);
    current_pool() = nullptr;
}

void Server::loop(int k) {
    Worker *w = workers_[(size_t)k].get();
    current_pool() = pools_[(size_t)k].get();
    hipStream_t s = nullptr;
    bool ok = hipSetDevice(device_) == hipSuccess && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    struct Lane {
        louvain_params prm;
        std::unique_ptr<BatchEngine> eng;
        std::vector<ServeRequest *> members;
    };
    std::vector<std::unique_ptr<Lane>> lanes;
    std::deque<ServeRequest *> queue;
    Timer timer;
    auto busy = [&] {
        for (auto &l : lanes)
            if (!l->eng->idle()) return true;
        return false;
    };
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            // the head of the queue can be admitted (or rejected) now
            auto ready = [&] {
                if (queue.empty()) return false;
                const ServeRequest *r = queue.front();
                return r->bytes > budget_ || in_use_ + r->bytes <= budget_;
            };
            cv_work_.wait(lk, [&] { return stop_ || !w->incoming.empty() || busy() || ready(); });
            if (stop_) break;
            while (!w->incoming.empty()) {
                queue.push_back(w->incoming.front());
                w->incoming.pop_front();
            }
        }
        // admission in arrival order while the footprint fits the budget
        while (!queue.empty()) {
            ServeRequest *r = queue.front();
            bool too_big = false, fits = false;
            {
                std::lock_guard<std::mutex> lk(mu_);
                too_big = r->bytes > budget_;
                fits = !too_big && in_use_ + r->bytes <= budget_;
                if (fits && ok) {
                    in_use_ += r->bytes;
                    r->admitted = true;
                }
            }
            if (!ok) {
                queue.pop_front();
                fail(r, LOUVAIN_EDEVICE, "the request loop could not set up its device stream");
                continue;
            }
            if (too_big) {
                queue.pop_front();
                fail(r, LOUVAIN_ENOMEM, "the graph needs more device memory than the serving budget");
                continue;
            }
            if (!fits) break;
            queue.pop_front();
            r->t_admit = now_us();
            try {
                ingest(r, s);
                if (r->tw >= kCompactTwMax) {
                    // too heavy for the batch's compact words: ingested (its stream
                    // work is complete), handed to the plain worker
                    {
                        std::lock_guard<std::mutex> lk(mu_);
                        workers_[kPlain]->incoming.push_back(r);
                    }
                    cv_work_.notify_all();
                    continue;
                }
                Lane *lane = nullptr;
                for (auto &l : lanes)
                    if (same_params(l->prm, r->prm)) lane = l.get();
                if (!lane) {
                    lanes.emplace_back(new Lane{r->prm, std::unique_ptr<BatchEngine>(new BatchEngine(
                                                    s, nullptr, to_sweep(r->prm), r->prm.max_levels,
                                                    r->prm.pass_batch > 0 ? r->prm.pass_batch : tuning_.pass_batch)),
                                                {}});
                    lane = lanes.back().get();
                    lane->eng->set_tuning(tuning_);
                }
                lane->eng->admit(&r->member);
                lane->members.push_back(r);
            } catch (const Error &e) {
                (void)hipStreamSynchronize(s);
                fail(r, e.code, e.what());
            } catch (const std::exception &e) {
                (void)hipStreamSynchronize(s);
                fail(r, LOUVAIN_EDEVICE, e.what());
            }
        }
        // one level of every lane with work
        for (auto &lp : lanes) {
            Lane &lane = *lp;
            if (lane.eng->idle()) continue;
            std::vector<BatchMember *> fin;
            try {
                fin = lane.eng->step();
                for (BatchMember *m : fin) {
                    ServeRequest *r = (ServeRequest *)m->tag;
                    r->status = m->status;
                    r->q = m->q;
                    r->levels = m->levels;
                    r->edges_swept = m->edges_swept;
                    deliver(r, s);
                }
            } catch (const Error &e) {
                // the lane's device state is lost: fail its members, start afresh
                (void)hipStreamSynchronize(s);
                for (ServeRequest *r : lane.members) fail(r, e.code, e.what());
                lane.members.clear();
                lane.eng.reset(new BatchEngine(s, nullptr, to_sweep(lane.prm), lane.prm.max_levels,
                                               lane.prm.pass_batch > 0 ? lane.prm.pass_batch : tuning_.pass_batch));
                lane.eng->set_tuning(tuning_);
                continue;
            }
            for (BatchMember *m : fin) {
                ServeRequest *r = (ServeRequest *)m->tag;
                lane.members.erase(std::find(lane.members.begin(), lane.members.end(), r));
                finish(r);
            }
        }
    }
    // shutting down: drop the device state of everything still resident
    if (s) (void)hipStreamSynchronize(s);
    for (auto &l : lanes)
        for (ServeRequest *r : l->members) release_device(r);
    lanes.clear();
    if (s) (void)hipStreamDestroy(s);
    current_pool() = nullptr;
}

}  // namespace lv
