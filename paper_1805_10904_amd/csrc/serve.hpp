// Request loop of the served form: graphs are submitted from any thread and
// routed by size to one of three batched workers (each a thread with its own
// stream, device pool and batch engines, so a graph is not held back by the
// level steps of much larger ones: a batch's members advance one level per
// step together, and a step lasts as long as its largest member's level; the
// streams overlap on the device).  A
// worker admits its requests in arrival order while their estimated device
// footprints fit the shared memory budget, and every admitted graph joins
// the worker's running batch at the next level boundary (continuous
// batching: newcomers at level 0 are swept in the same launches as members
// at deeper levels).  A graph whose total weight 2W reaches 2^31 cannot use
// the batch's compact words; after its ingest it is handed to a third
// worker that runs it on the plain path on its own stream, so the worker
// that admitted it keeps stepping its batch meanwhile.  Results are
// identical to louvain_run on each graph alone.
#pragma once

#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>

#include "batch.hpp"

namespace lv {

struct ServeRequest {
    uint64_t ticket = 0;
    // input: caller memory, read when the request is admitted
    int64_t n = 0, nnz = 0;
    const int64_t *rp = nullptr;
    const int32_t *col = nullptr;
    const void *w = nullptr;
    int wbytes = 4;
    bool dev = false;            // input and output pointers are device pointers
    bool check_symmetry = false;
    louvain_params prm{};
    int32_t *labels_out = nullptr;
    // result
    size_t bytes = 0;            // footprint estimate
    bool admitted = false;       // bytes are counted against the budget
    bool done = false;
    int status = LOUVAIN_OK;
    std::string err;
    int64_t tw = 0;
    i128 q = 0;
    std::vector<LevelRec> levels;
    int64_t edges_swept = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;   // microseconds, steady clock
    // device state while resident
    DevBuf<int64_t> d_rp, d_delta, d_w64;
    DevBuf<int32_t> d_col, d_w32, d_fin;
    BatchMember member;
};

class Server {
  public:
    // arena: the context's backing store of device memory (nullptr: hipMalloc)
    Server(int device, size_t budget, const Tuning &tn, std::shared_ptr<Arena> arena);
    ~Server();
    // Queue a request (thread-safe); returns its ticket.
    uint64_t submit(std::unique_ptr<ServeRequest> r);
    // LOUVAIN_EAGAIN while the request is pending after waiting up to wait_us
    // microseconds (< 0: without limit); otherwise hands the finished request
    // over (*out) and returns its status.  Unknown tickets: LOUVAIN_EINVAL.
    int poll(uint64_t ticket, int32_t wait_us, std::unique_ptr<ServeRequest> *out);
    void set_budget(size_t bytes);
    size_t budget();
    // Estimated peak device bytes of one graph of n vertices and nnz entries
    // in the batch (its resident CSR plus its share of every level buffer).
    static size_t workspace_bytes(int64_t n, int64_t nnz);
    static double now_us();

    // Requests with at most kSmallEntries entries go to the small-graph
    // worker, up to kMediumEntries to the medium one, larger to the large one.
    static constexpr int64_t kSmallEntries = (int64_t)1 << 20;
    static constexpr int64_t kMediumEntries = (int64_t)1 << 23;

  private:
    struct Worker {
        std::thread th;
        std::deque<ServeRequest *> incoming;
    };
    void loop(int k);
    void loop_plain();
    void finish(ServeRequest *r);
    void fail(ServeRequest *r, int code, const std::string &msg);

    // worker k: 0 small, 1 medium, 2 large graphs (batched), 3 graphs with
    // 2W >= 2^31 (plain path, after their ingest by a batched worker)
    enum { kSmall = 0, kMedium = 1, kLarge = 2, kPlain = 3, kWorkers = 4 };

    int device_;
    Tuning tuning_;
    // device pools of the workers; they outlive the threads and the requests
    // (a request ingested by one worker may be released by the plain worker)
    std::vector<std::unique_ptr<Pool>> pools_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::unordered_map<uint64_t, std::unique_ptr<ServeRequest>> all_;
    uint64_t next_ = 1;
    bool stop_ = false;
    size_t budget_;
    size_t in_use_ = 0;   // footprints of admitted, unfinished requests
    std::vector<std::unique_ptr<Worker>> workers_;
};

}  // namespace lv
