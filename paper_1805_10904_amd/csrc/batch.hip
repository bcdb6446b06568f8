// Batched levels over a block-diagonal union of many graphs (see batch.hpp).
//
// Per step: newcomers' level-0 CSRs are appended to the union after the
// contracted graphs of the members that continue; every vertex gets its
// member's slot; the compact sweeps run all members' phases at once (each
// member's acceptance test and stop are its own); the members whose phase
// kept a sweep compose their final labels and, unless their level cap is
// reached, are contracted together into the next union, in slot order, so a
// member's communities stay one contiguous vertex range.
#include <algorithm>
#include <cstring>

#include <memory>

#include "batch.hpp"
#include "prims.hpp"

namespace lv {
namespace {

constexpr int kSegChunk = 4096;
constexpr int64_t kMaxUnionVertices = 0x7fffffffLL;   // int32 labels

// A newcomer's level-0 graph to be appended to the union.
struct UnionSeg {
    const int64_t *rp;
    const int32_t *col;
    const void *w;
    const int64_t *delta;
    int64_t n, nnz, voff, eoff;
    int32_t wbytes, pad;
};

// A per-vertex array of one member (final labels or the union's slot ids).
struct VertSeg {
    int32_t *p;
    int64_t n;
    int64_t slot;
};

enum { SEG_IOTA = 0, SEG_COMPOSE = 1, SEG_SLOT = 2, SEG_COPY = 3 };

// Segment of workgroup b: the largest s with blk0[s] <= b.
__device__ __forceinline__ int seg_of_block(const int64_t *__restrict__ blk0, int nseg, int64_t b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk0[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename WO>
__global__ __launch_bounds__(256) void k_union_copy(const UnionSeg *__restrict__ segs,
                                                    const int64_t *__restrict__ blk0, int nseg, int64_t *rp,
                                                    int32_t *col, WO *w, int64_t *delta) {
    __shared__ int s_seg;
    if (threadIdx.x == 0) s_seg = seg_of_block(blk0, nseg, blockIdx.x);
    __syncthreads();
    const UnionSeg sg = segs[s_seg];
    const int64_t base = ((int64_t)blockIdx.x - blk0[s_seg]) * kSegChunk;
    for (int k = threadIdx.x; k < kSegChunk; k += 256) {
        const int64_t e = base + k;
        if (e < sg.nnz) {
            col[sg.eoff + e] = sg.col[e] + (int32_t)sg.voff;
            w[sg.eoff + e] = sg.wbytes == 4 ? (WO)((const int32_t *)sg.w)[e] : (WO)((const int64_t *)sg.w)[e];
        }
        if (e <= sg.n) {
            // the member's end pointer equals the next member's start (same value)
            rp[sg.voff + e] = sg.rp[e] + sg.eoff;
            if (e < sg.n) delta[sg.voff + e] = sg.delta[e];
        }
    }
}

__global__ __launch_bounds__(256) void k_vert_segments(const VertSeg *__restrict__ segs,
                                                       const int64_t *__restrict__ blk0, int nseg, int mode,
                                                       const int64_t *__restrict__ loff,
                                                       const int64_t *__restrict__ newoff,
                                                       const int32_t *__restrict__ newlab) {
    __shared__ int s_seg;
    if (threadIdx.x == 0) s_seg = seg_of_block(blk0, nseg, blockIdx.x);
    __syncthreads();
    const VertSeg sg = segs[s_seg];
    const int64_t base = ((int64_t)blockIdx.x - blk0[s_seg]) * kSegChunk;
    const int64_t lo = mode == SEG_COMPOSE ? loff[sg.slot] : 0;
    const int64_t no = mode == SEG_COMPOSE ? newoff[sg.slot] : 0;
    for (int k = threadIdx.x; k < kSegChunk; k += 256) {
        const int64_t v = base + k;
        if (v >= sg.n) break;
        if (mode == SEG_IOTA)
            sg.p[v] = (int32_t)v;
        else if (mode == SEG_SLOT)
            sg.p[v] = (int32_t)sg.slot;
        else if (mode == SEG_COPY)
            sg.p[v] = newlab[sg.slot + v];
        else
            sg.p[v] = (int32_t)((int64_t)newlab[lo + sg.p[v]] - no);
    }
}

// out[s] = rp[off[s]] for s in [0, count].
__global__ void k_rp_at(const int64_t *__restrict__ rp, const int64_t *__restrict__ off, int64_t count,
                        int64_t *out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s <= count) out[s] = rp[off[s]];
}

template <typename T>
void grow(DevBuf<T> &b, size_t count, size_t keep, hipStream_t s) {
    if (b.p && b.n >= count) return;
    DevBuf<T> nb(count + count / 4 + 1024);
    if (keep > 0 && b.p) LV_HIP(hipMemcpyAsync(nb.p, b.p, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
    b = std::move(nb);
}

// One host-to-device upload of a descriptor array followed by its block
// prefix (8-byte aligned).
template <typename D>
int64_t *upload(TempBuf &buf, const std::vector<D> &d, const std::vector<int64_t> &blk0, hipStream_t s) {
    static_assert(sizeof(D) % 8 == 0, "descriptor alignment");
    const size_t a = d.size() * sizeof(D), b = blk0.size() * sizeof(int64_t);
    buf = TempBuf(a + b, s);
    std::vector<uint8_t> host(a + b);
    std::memcpy(host.data(), d.data(), a);
    std::memcpy(host.data() + a, blk0.data(), b);
    LV_HIP(hipMemcpyAsync(buf.p, host.data(), a + b, hipMemcpyHostToDevice, s));
    LV_HIP(hipStreamSynchronize(s));   // the staging vector dies here
    return (int64_t *)((uint8_t *)buf.p + a);
}

template <typename T>
void to_device(DevBuf<T> &dst, const std::vector<T> &src, hipStream_t s) {
    dst.reserve(src.size());
    if (!src.empty())
        LV_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

}  // namespace

void copy_segments(int32_t *const *dst, const int64_t *n, const int64_t *src_off, int64_t count, const int32_t *src,
                   hipStream_t s) {
    std::vector<VertSeg> cs;
    std::vector<int64_t> b0;
    int64_t b = 0;
    for (int64_t i = 0; i < count; ++i) {
        if (n[i] <= 0) continue;
        cs.push_back(VertSeg{dst[i], n[i], src_off[i]});
        b0.push_back(b);
        b += (n[i] + kSegChunk - 1) / kSegChunk;
    }
    if (cs.empty()) return;
    TempBuf buf;
    const int64_t *bk = upload(buf, cs, b0, s);
    k_vert_segments<<<(unsigned)b, 256, 0, s>>>(buf.as<VertSeg>(), bk, (int)cs.size(), SEG_COPY, nullptr, nullptr,
                                                src);
    LV_LAUNCHED("k_vert_segments");
    LV_HIP(hipStreamSynchronize(s));
}

BatchEngine::BatchEngine(hipStream_t s, Timer *t, const SweepParams &sp, int max_levels, int pass_batch)
    : s_(s), t_(t), sp_(sp), max_levels_(max_levels), pass_batch_(pass_batch > 0 ? pass_batch : 1), sw_(s, t),
      ct_(s, t) {}

int64_t BatchEngine::union_vertices() const {
    int64_t n = un_;
    for (auto *m : pending_) n += m->g0.n;
    return n;
}

int64_t BatchEngine::union_entries() const {
    int64_t m = um_;
    for (auto *x : pending_) m += x->g0.nnz;
    return m;
}

void BatchEngine::admit(BatchMember *m) {
    m->level = 0;
    m->levels.clear();
    m->edges_swept = 0;
    m->done = false;
    m->status = LOUVAIN_OK;
    m->q = 0;
    m->n = m->g0.n;
    m->nnz = m->g0.nnz;
    require(m->g0.n < kMaxUnionVertices && m->g0.tw < kCompactTwMax, LOUVAIN_EINVAL,
            "batched members need n < 2^31 and TW < 2^31");
    if (m->g0.n == 0 || m->g0.tw == 0) {
        iota_i32(m->fin, m->g0.n, s_);
        m->done = true;
        finished_.push_back(m);
        return;
    }
    pending_.push_back(m);
}

void BatchEngine::ensure(UBuf &u, int64_t n, int64_t m, int64_t keep_n, int64_t keep_m) {
    grow(u.rp, (size_t)n + 1, keep_n > 0 ? (size_t)keep_n + 1 : 0, s_);
    grow(u.delta, (size_t)(n > 0 ? n : 1), (size_t)keep_n, s_);
    grow(u.col, (size_t)(m > 0 ? m : 1), (size_t)keep_m, s_);
    grow(u.w32, (size_t)(m > 0 ? m : 1), (size_t)keep_m, s_);
}

std::vector<BatchMember *> BatchEngine::step() {
    Range range("louvain batched step");
    std::vector<BatchMember *> out;
    out.swap(finished_);
    // newcomers that keep the union's vertex count within int32 labels
    std::vector<BatchMember *> join;
    int64_t n_arr = 0, m_arr = 0;
    {
        size_t k = 0;
        for (; k < pending_.size(); ++k) {
            BatchMember *m = pending_[k];
            if (un_ + n_arr + m->g0.n > kMaxUnionVertices) break;
            join.push_back(m);
            n_arr += m->g0.n;
            m_arr += m->g0.nnz;
        }
        pending_.erase(pending_.begin(), pending_.begin() + (std::ptrdiff_t)k);
    }
    if (slots_.empty() && join.empty()) {
        LV_HIP(hipStreamSynchronize(s_));
        return out;
    }
    // the union keeps int32 weights: every member has 2W < 2^31
    const int64_t N = un_ + n_arr, M = um_ + m_arr;
    UBuf &U = ub_[cur_];
    ensure(U, N, M, slots_.empty() ? 0 : un_, slots_.empty() ? 0 : um_);

    std::vector<BatchMember *> sl = slots_;
    sl.insert(sl.end(), join.begin(), join.end());
    const int64_t ns = (int64_t)sl.size();
    std::vector<int64_t> hloff((size_t)ns + 1), htw((size_t)ns);
    int64_t twmax = 0;
    for (int64_t s = 0, off = 0; s < ns; ++s) {
        hloff[(size_t)s] = off;
        off += sl[(size_t)s]->n;
        htw[(size_t)s] = sl[(size_t)s]->g0.tw;
        twmax = std::max(twmax, sl[(size_t)s]->g0.tw);
        hloff[(size_t)s + 1] = off;
    }
    to_device(loff_, hloff, s_);
    to_device(tw_, htw, s_);
    gid_.reserve((size_t)N);

    TempBuf jb, vb;
    if (!join.empty()) {
        // append the newcomers' CSRs and start their final labels at the identity
        std::vector<UnionSeg> us;
        std::vector<VertSeg> fs;
        std::vector<int64_t> ub0, fb0;
        int64_t vo = un_, eo = um_, b = 0, fb = 0;
        for (auto *m : join) {
            UnionSeg g{m->g0.row_ptr, m->g0.col, m->g0.w, m->g0.delta, m->g0.n, m->g0.nnz, vo, eo, m->g0.wbytes, 0};
            us.push_back(g);
            ub0.push_back(b);
            b += std::max((m->g0.nnz + kSegChunk - 1) / kSegChunk, (m->g0.n + 1 + kSegChunk - 1) / kSegChunk);
            fs.push_back(VertSeg{m->fin, m->g0.n, 0});
            fb0.push_back(fb);
            fb += (m->g0.n + kSegChunk - 1) / kSegChunk;
            vo += m->g0.n;
            eo += m->g0.nnz;
        }
        const int64_t *ubk = upload(jb, us, ub0, s_);
        {
            TimedLaunch tl(t_, TG_LEVEL, "k_union_copy", (double)m_arr * 16 + (double)n_arr * 32);
            tl.launch(k_union_copy<int32_t>, (unsigned)b, 256, 0, s_, jb.as<UnionSeg>(), ubk, (int)us.size(),
                      U.rp.p, U.col.p, U.w32.p, U.delta.p);
            LV_LAUNCHED("k_union_copy");
        }
        const int64_t *fbk = upload(vb, fs, fb0, s_);
        k_vert_segments<<<(unsigned)fb, 256, 0, s_>>>(vb.as<VertSeg>(), fbk, (int)fs.size(), SEG_IOTA, nullptr,
                                                      nullptr, nullptr);
        LV_LAUNCHED("k_vert_segments");
    }
    {
        // slot of every union vertex
        std::vector<VertSeg> gs;
        std::vector<int64_t> gb0;
        int64_t b = 0;
        for (int64_t s = 0; s < ns; ++s) {
            gs.push_back(VertSeg{gid_.p + hloff[(size_t)s], sl[(size_t)s]->n, s});
            gb0.push_back(b);
            b += (sl[(size_t)s]->n + kSegChunk - 1) / kSegChunk;
        }
        TempBuf gbuf;
        const int64_t *gbk = upload(gbuf, gs, gb0, s_);
        TimedLaunch tl(t_, TG_LEVEL, "k_vert_segments", (double)N * 4);
        tl.launch(k_vert_segments, (unsigned)b, 256, 0, s_, gbuf.as<VertSeg>(), gbk, (int)gs.size(), SEG_SLOT, nullptr,
                  nullptr, nullptr);
        LV_LAUNCHED("k_vert_segments");
        LV_HIP(hipStreamSynchronize(s_));
    }

    GraphView v;
    v.n = N;
    v.nnz = M;
    v.row_ptr = U.rp.p;
    v.col = U.col.p;
    v.w = U.w32.p;
    v.wbytes = 4;
    v.delta = U.delta.p;
    v.tw = twmax;

    sw_.reserve(N, M);
    ct_.reserve(N, M);
    sw_.set_batch(ns, gid_.p, tw_.p);
    sw_.plan(v);
    sw_.init_singletons(v);
    int p = 0;
    unsigned int planned = (unsigned int)ns;   // graphs the current bucket lists cover
    // pass_batch passes per host check of the count of graphs still in
    // their phase; one pass is enqueued ahead of each check, so the device
    // does not idle on the round trip (finished graphs' passes return at
    // once; a replan covers the graphs active at the count, a superset of
    // those active when it runs)
    for (int b = 0; b < pass_batch_; ++b) sw_.pass(v, ++p, sp_, nullptr);
    std::unique_ptr<Readback> rb(new Readback(s_));
    const unsigned int *hact = rb->add(sw_.active_counter(p));
    rb->issue();
    for (;;) {
        sw_.pass(v, ++p, sp_, nullptr);
        rb->wait();
        const unsigned int act = *hact;
        if (act == 0) break;
        require(p <= sp_.max_sweeps + 4 + 2 * pass_batch_, LOUVAIN_EDEVICE, "batched sweep loop did not converge");
        if (2 * act <= planned) {
            // most graphs have ended their phase: sweep only the others
            sw_.replan_active(v);
            planned = act;
        }
        for (int b = 1; b < pass_batch_; ++b) sw_.pass(v, ++p, sp_, nullptr);
        rb.reset(new Readback(s_));
        hact = rb->add(sw_.active_counter(p));
        rb->issue();
    }
    std::vector<PhaseState> st((size_t)ns);
    LV_HIP(hipMemcpyAsync(st.data(), sw_.states(), sizeof(PhaseState) * (size_t)ns, hipMemcpyDeviceToHost, s_));
    LV_HIP(hipStreamSynchronize(s_));

    std::vector<int32_t> kc((size_t)ns), kk((size_t)ns);
    bool any_c = false, any_k = false, same = true;
    for (int64_t s = 0; s < ns; ++s) {
        BatchMember *m = sl[(size_t)s];
        const PhaseState &x = st[(size_t)s];
        LevelRec r;
        r.n = m->n;
        r.nnz = m->nnz;
        r.accepted = x.accepted;
        r.executed = x.accepted + (x.limit ? 0 : 1);
        r.passes = x.pass;
        r.q = make_i128(x.q_ref[0], (int64_t)x.q_ref[1]);
        m->levels.push_back(r);
        m->edges_swept += (int64_t)x.pass * m->nnz;
        m->q = r.q;
        if (x.limit) m->status = LOUVAIN_ELIMIT;
        kc[(size_t)s] = x.accepted > 0;
        kk[(size_t)s] = kc[(size_t)s] && m->level + 1 < max_levels_;
        if (kc[(size_t)s] && !kk[(size_t)s]) m->status = LOUVAIN_ELIMIT;
        m->level += 1;
        any_c = any_c || kc[(size_t)s];
        any_k = any_k || kk[(size_t)s];
        same = same && kc[(size_t)s] == kk[(size_t)s];
    }

    TempBuf cb;
    int64_t k = 0;
    if (any_c) {
        labf_.reserve((size_t)N);
        newlab_.reserve((size_t)N);
        newoff_.reserve((size_t)ns + 1);
        sw_.final_labels(labf_.p);
        to_device(keep_, kc, s_);
        const int32_t *lab = labf_.p;
        if (sp_.merge) {
            // the final merge of the graphs that kept a sweep, then their Q once more
            merged_.reserve((size_t)N);
            merge_lone_batch(v, labf_.p, sp_.singlet, gid_.p, tw_.p, keep_.p, merged_.p, s_, t_);
            lab = merged_.p;
            const std::vector<i128> qm = modularity_by_graph(v, lab, gid_.p, ns, htw, s_, t_);
            for (int64_t s = 0; s < ns; ++s) {
                if (!kc[(size_t)s]) continue;
                BatchMember *m = sl[(size_t)s];
                m->levels.back().q = qm[(size_t)s];
                m->q = qm[(size_t)s];
            }
        }
        k = ct_.renumber_kept(lab, N, gid_.p, keep_.p, loff_.p, ns, newlab_.p, newoff_.p);
        std::vector<VertSeg> cs;
        std::vector<int64_t> cb0;
        int64_t b = 0, nv = 0;
        for (int64_t s = 0; s < ns; ++s) {
            if (!kc[(size_t)s]) continue;
            BatchMember *m = sl[(size_t)s];
            cs.push_back(VertSeg{m->fin, m->g0.n, s});
            cb0.push_back(b);
            b += (m->g0.n + kSegChunk - 1) / kSegChunk;
            nv += m->g0.n;
        }
        const int64_t *cbk = upload(cb, cs, cb0, s_);
        {
            TimedLaunch tl(t_, TG_CONTRACT, "k_compose_batch", (double)nv * 12);
            tl.launch(k_vert_segments, (unsigned)b, 256, 0, s_, cb.as<VertSeg>(), cbk, (int)cs.size(), SEG_COMPOSE,
                      loff_.p, newoff_.p, newlab_.p);
            LV_LAUNCHED("k_compose_batch");
        }
        if (any_k && !same) {
            to_device(keep_, kk, s_);
            k = ct_.renumber_kept(lab, N, gid_.p, keep_.p, loff_.p, ns, newlab_.p, newoff_.p);
        }
    }
    std::vector<BatchMember *> next;
    if (any_k) {
        UBuf &D = ub_[1 - cur_];
        ensure(D, k, M, 0, 0);
        // every member has 2W < 2^31, so every contracted weight fits int32
        const int64_t m2 = ct_.contract(v, newlab_.p, k, D.rp.p, D.col.p, D.w32.p, 4, D.delta.p, false, block_max_);
        std::vector<int64_t> hno((size_t)ns + 1), hrp((size_t)ns + 1);
        TempBuf rpb((size_t)(ns + 1) * sizeof(int64_t), s_);
        k_rp_at<<<grid_for(ns + 1, 256), 256, 0, s_>>>(D.rp.p, newoff_.p, ns, rpb.as<int64_t>());
        LV_LAUNCHED("k_rp_at");
        LV_HIP(hipMemcpyAsync(hno.data(), newoff_.p, sizeof(int64_t) * (size_t)(ns + 1), hipMemcpyDeviceToHost, s_));
        LV_HIP(hipMemcpyAsync(hrp.data(), rpb.p, sizeof(int64_t) * (size_t)(ns + 1), hipMemcpyDeviceToHost, s_));
        LV_HIP(hipStreamSynchronize(s_));
        for (int64_t s = 0; s < ns; ++s) {
            if (!kk[(size_t)s]) continue;
            BatchMember *m = sl[(size_t)s];
            m->n = hno[(size_t)s + 1] - hno[(size_t)s];
            m->nnz = hrp[(size_t)s + 1] - hrp[(size_t)s];
            next.push_back(m);
        }
        un_ = k;
        um_ = m2;
        cur_ = 1 - cur_;
    } else {
        un_ = um_ = 0;
    }
    slots_.swap(next);
    for (int64_t s = 0; s < ns; ++s)
        if (!kk[(size_t)s]) {
            sl[(size_t)s]->done = true;
            out.push_back(sl[(size_t)s]);
        }
    LV_HIP(hipStreamSynchronize(s_));
    return out;
}

}  // namespace lv
