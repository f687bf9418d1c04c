// pmp_server.cpp -- continuous-batching request server over libpmp.
//
// A server owns `max_slots` worker threads on one device, each with its own
// HIP stream (default priority) and a pinned host staging buffer.  All device
// memory is one arena of hbm_budget_bytes, allocated when the server is
// created: each admitted request's series and workspace are carved from it
// (first fit, 256-byte aligned, freed blocks coalesce), so no request
// allocates or frees device memory, and a request whose memory cannot be
// carved yet stays queued.
//
// Admission: whenever a slot is free, the queued request of least estimated
// work (cells times mean window length) whose memory can be carved is
// admitted, so short requests do not wait behind long ones.  A request that
// has waited kAgingSeconds or more goes first (oldest first), and while it
// cannot be carved nothing else is admitted, so memory drains for it and no
// request starves.  Admitted requests run concurrently on their streams and
// their kernels overlap on the GPU.  Each request's result depends only on
// its own input (the pipeline shares no state between requests), so it is the
// same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pmp.h"

namespace {

constexpr double kAgingSeconds = 10.0;         // waiting time that overrides least-work order
constexpr size_t kStageBytes = (size_t)16 << 20;   // pinned staging per slot
constexpr size_t kAlign = 256;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator of offsets in [0, cap), blocks coalesce when freed.
class ArenaAlloc {
public:
    explicit ArenaAlloc(size_t cap = 0) { if (cap) free_[0] = cap; }
    // offset of a block of `bytes` (a multiple of kAlign), or SIZE_MAX
    size_t take(size_t bytes) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return off;
        }
        return SIZE_MAX;
    }
    void give(size_t off, size_t bytes) {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    std::map<size_t, size_t> free_;    // offset -> size
};

struct Request {
    uint64_t id = 0;
    std::vector<double> series;
    int32_t m_min = 0, m_max = 0, k = 0, excl = 0, budget = 0;
    pmp_options opt{};
    bool has_opt = false;
    size_t ws = 0;          // workspace bound (pmp_workspace_bytes)
    size_t bytes = 0;       // arena bytes: series + workspace, aligned
    size_t off = 0;         // arena offset once admitted
    uint64_t cells = 0;
    double work = 0.0;      // cells x mean window length: the admission order
    // results
    bool done = false;
    int status = PMP_OK;
    std::string error;
    std::vector<pmp_motif> out;
    pmp_timing timing{};
};

}  // namespace

struct pmp_server {
    int device = 0;
    size_t budget = 0;
    int slots = 1;
    char *arena = nullptr;
    ArenaAlloc alloc;
    std::vector<hipStream_t> streams;
    std::vector<double *> stage;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::list<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    bool stop = false;
    uint64_t next_id = 1;
    std::vector<std::thread> workers;

    Request *admit();
    void work(int slot);
};

// Caller holds mu.  The request to run next, with its memory carved, or
// nullptr if none can run now.
Request *pmp_server::admit() {
    if (queue.empty()) return nullptr;
    const double now = now_s();
    Request *oldest = queue.front();
    if (now - oldest->timing.submit_s >= kAgingSeconds) {
        const size_t off = alloc.take(oldest->bytes);
        if (off == SIZE_MAX) return nullptr;     // let memory drain for it
        oldest->off = off;
        queue.pop_front();
        return oldest;
    }
    std::vector<std::list<Request *>::iterator> order;
    for (auto it = queue.begin(); it != queue.end(); ++it) order.push_back(it);
    std::stable_sort(order.begin(), order.end(),
                     [](const auto &a, const auto &b) { return (*a)->work < (*b)->work; });
    for (auto it : order) {
        const size_t off = alloc.take((*it)->bytes);
        if (off == SIZE_MAX) continue;
        Request *r = *it;
        r->off = off;
        queue.erase(it);
        return r;
    }
    return nullptr;
}

void pmp_server::work(int slot) {
    if (hipSetDevice(device) != hipSuccess) return;
    const hipStream_t s = streams[slot];
    double *stg = stage[slot];
    const size_t stage_n = kStageBytes / sizeof(double);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop && queue.empty()) break;
                r = admit();
                if (r) break;
                // wake on a submission or a completion, and at least every
                // second so that a request reaching its aging time is seen
                cv_work.wait_for(lk, std::chrono::seconds(1));
            }
            if (!r) break;
        }
        r->timing.start_s = now_s();
        const int64_t n = (int64_t)r->series.size();
        double *d_t = (double *)(arena + r->off);
        void *d_ws = arena + r->off + align_up((size_t)n * sizeof(double));
        int rc = PMP_OK;
        // series to the device through the pinned staging buffer
        for (int64_t x = 0; x < n && !rc; x += (int64_t)stage_n) {
            const int64_t c = std::min<int64_t>((int64_t)stage_n, n - x);
            std::memcpy(stg, r->series.data() + x, (size_t)c * sizeof(double));
            if (hipMemcpyAsync(d_t + x, stg, (size_t)c * sizeof(double), hipMemcpyHostToDevice,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = PMP_EDEVICE;
                r->error = "copy of the series failed";
            }
        }
        std::vector<pmp_motif> out((size_t)r->k);
        int32_t n_out = 0;
        if (!rc) {
            rc = pmp_run_device(d_t, n, r->m_min, r->m_max, r->k, r->excl, r->budget,
                                r->has_opt ? &r->opt : nullptr, d_ws, r->ws, (void *)s, out.data(),
                                &n_out, nullptr);
            if (rc) r->error = pmp_last_error();
        }
        (void)hipStreamSynchronize(s);   // the arena block is reused after this
        out.resize(rc ? 0 : (size_t)n_out);
        {
            std::lock_guard<std::mutex> lk(mu);
            r->out = std::move(out);
            r->status = rc;
            r->timing.end_s = now_s();
            r->timing.cells = r->cells;
            r->timing.workspace_bytes = r->bytes;
            r->done = true;
            alloc.give(r->off, r->bytes);
            std::vector<double>().swap(r->series);
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

static void release(pmp_server *srv) {
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    for (double *p : srv->stage) (void)hipHostFree(p);
    if (srv->arena) (void)hipFree(srv->arena);
    delete srv;
}

extern "C" {

pmp_server *pmp_server_create(int device, size_t hbm_budget_bytes, int32_t max_slots) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return nullptr;
    if (max_slots < 1 || hbm_budget_bytes < kAlign) return nullptr;
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    pmp_server *srv = new pmp_server();
    srv->device = device;
    srv->budget = hbm_budget_bytes & ~(kAlign - 1);
    srv->slots = max_slots;
    if (hipMalloc((void **)&srv->arena, srv->budget) != hipSuccess) {
        srv->arena = nullptr;
        release(srv);
        return nullptr;
    }
    srv->alloc = ArenaAlloc(srv->budget);
    for (int i = 0; i < max_slots; ++i) {
        hipStream_t s;
        double *p = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            release(srv);
            return nullptr;
        }
        srv->streams.push_back(s);
        if (hipHostMalloc((void **)&p, kStageBytes, hipHostMallocDefault) != hipSuccess) {
            release(srv);
            return nullptr;
        }
        srv->stage.push_back(p);
    }
    for (int i = 0; i < max_slots; ++i) srv->workers.emplace_back([srv, i] { srv->work(i); });
    return srv;
}

int pmp_submit(pmp_server *srv, const double *series, int64_t n, int32_t m_min, int32_t m_max,
               int32_t k, int32_t exclusion, int32_t budget, const pmp_options *opt,
               uint64_t *req_id) {
    if (!srv || !series || !req_id) return PMP_EINVAL;
    if (k < 1 || exclusion < 1 || budget < 1) return PMP_EINVAL;
    const size_t ws = pmp_workspace_bytes(n, m_min, m_max, k, opt);
    if (ws == 0) return PMP_EINVAL;
    const size_t bytes = align_up((size_t)n * sizeof(double)) + align_up(ws);
    if (bytes > srv->budget) return PMP_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        if (!(series[i] - series[i] == 0.0)) return PMP_EINVAL;   // NaN or inf
    Request *r = new Request();
    r->series.assign(series, series + n);
    r->m_min = m_min;
    r->m_max = m_max;
    r->k = k;
    r->excl = exclusion;
    r->budget = budget;
    if (opt) {
        r->opt = *opt;
        r->has_opt = true;
    }
    r->ws = ws;
    r->bytes = bytes;
    const int step = opt ? opt->m_step : 1;
    for (int64_t m = m_min; m <= m_max; m += step) {
        r->cells += (uint64_t)(n - m + 1);
        r->work += (double)(n - m + 1) * (double)m;
    }
    r->timing.submit_s = now_s();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        r->id = srv->next_id++;
        srv->reqs[r->id] = r;
        srv->queue.push_back(r);
    }
    srv->cv_work.notify_all();
    *req_id = r->id;
    return PMP_OK;
}

static int finish(pmp_server *srv, Request *r, pmp_motif *out, int32_t *n_out, pmp_timing *tm) {
    // caller holds srv->mu and r->done
    const int rc = r->status;
    if (out) memcpy(out, r->out.data(), r->out.size() * sizeof(pmp_motif));
    if (n_out) *n_out = (int32_t)r->out.size();
    if (tm) *tm = r->timing;
    srv->reqs.erase(r->id);
    delete r;
    return rc;
}

int pmp_poll(pmp_server *srv, uint64_t req_id, pmp_motif *out, int32_t *n_out, pmp_timing *tm) {
    if (!srv) return PMP_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return PMP_ENOTFOUND;
    if (!it->second->done) return PMP_EBUSY;
    return finish(srv, it->second, out, n_out, tm);
}

int pmp_wait(pmp_server *srv, uint64_t req_id, pmp_motif *out, int32_t *n_out, pmp_timing *tm) {
    if (!srv) return PMP_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return PMP_ENOTFOUND;
    Request *r = it->second;
    srv->cv_done.wait(lk, [&] { return r->done; });
    return finish(srv, r, out, n_out, tm);
}

void pmp_server_destroy(pmp_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &w : srv->workers) w.join();
    for (auto &kv : srv->reqs) delete kv.second;
    release(srv);
}

}  // extern "C"
