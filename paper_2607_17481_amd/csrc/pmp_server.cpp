// pmp_server.cpp -- continuous-batching request server over libpmp.
//
// A server owns `max_slots` worker threads on one device, each with its own
// HIP stream (default priority).  Requests queue in arrival order; whenever a
// slot is free, the first queued request whose workspace fits in the HBM
// budget still unreserved is admitted (first fit, so small requests can pass a
// large one that does not fit yet).  Admitted requests run concurrently on
// their streams, so their kernels overlap on the GPU.  Each request's result
// depends only on its own input (the pipeline shares no state between
// requests), so it is the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pmp.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    std::vector<double> series;
    int32_t m_min = 0, m_max = 0, k = 0, excl = 0, budget = 0;
    pmp_options opt{};
    bool has_opt = false;
    size_t ws = 0;
    uint64_t cells = 0;
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
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    size_t reserved = 0;
    int running = 0;
    bool stop = false;
    uint64_t next_id = 1;
    std::vector<std::thread> workers;

    void work();
};

void pmp_server::work() {
    if (hipSetDevice(device) != hipSuccess) return;
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop && queue.empty()) break;
                for (auto it = queue.begin(); it != queue.end(); ++it)
                    if (reserved + (*it)->ws <= budget) {
                        r = *it;
                        queue.erase(it);
                        break;
                    }
                if (r) break;
                cv_work.wait(lk);
            }
            if (!r) break;
            reserved += r->ws;
            ++running;
        }
        r->timing.start_s = now_s();
        double *d_t = nullptr;
        void *d_ws = nullptr;
        int rc = PMP_OK;
        const int64_t n = (int64_t)r->series.size();
        if (hipMalloc(&d_t, (size_t)n * sizeof(double)) != hipSuccess ||
            hipMalloc(&d_ws, r->ws) != hipSuccess) {
            rc = PMP_ENOMEM;
            r->error = "device allocation failed";
        }
        if (!rc && hipMemcpyAsync(d_t, r->series.data(), (size_t)n * sizeof(double),
                                  hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = PMP_EDEVICE;
            r->error = "copy of the series failed";
        }
        std::vector<pmp_motif> out((size_t)r->k);
        int32_t n_out = 0;
        if (!rc) {
            rc = pmp_run_device(d_t, n, r->m_min, r->m_max, r->k, r->excl, r->budget,
                                r->has_opt ? &r->opt : nullptr, d_ws, r->ws, (void *)s, out.data(),
                                &n_out, nullptr);
            if (rc) r->error = pmp_last_error();
        }
        (void)hipStreamSynchronize(s);
        if (d_ws) (void)hipFree(d_ws);
        if (d_t) (void)hipFree(d_t);
        out.resize(rc ? 0 : (size_t)n_out);
        {
            std::lock_guard<std::mutex> lk(mu);
            r->out = std::move(out);
            r->status = rc;
            r->timing.end_s = now_s();
            r->timing.cells = r->cells;
            r->timing.workspace_bytes = r->ws;
            r->done = true;
            reserved -= r->ws;
            --running;
            std::vector<double>().swap(r->series);
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    (void)hipStreamDestroy(s);
}

extern "C" {

pmp_server *pmp_server_create(int device, size_t hbm_budget_bytes, int32_t max_slots) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return nullptr;
    if (max_slots < 1 || hbm_budget_bytes == 0) return nullptr;
    pmp_server *srv = new pmp_server();
    srv->device = device;
    srv->budget = hbm_budget_bytes;
    srv->slots = max_slots;
    for (int i = 0; i < max_slots; ++i) srv->workers.emplace_back([srv] { srv->work(); });
    return srv;
}

int pmp_submit(pmp_server *srv, const double *series, int64_t n, int32_t m_min, int32_t m_max,
               int32_t k, int32_t exclusion, int32_t budget, const pmp_options *opt,
               uint64_t *req_id) {
    if (!srv || !series || !req_id) return PMP_EINVAL;
    if (k < 1 || exclusion < 1 || budget < 1) return PMP_EINVAL;
    const size_t ws = pmp_workspace_bytes(n, m_min, m_max, k, opt);
    if (ws == 0) return PMP_EINVAL;
    if (ws > srv->budget) return PMP_ENOMEM;
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
    const int step = opt ? opt->m_step : 1;
    for (int64_t m = m_min; m <= m_max; m += step) r->cells += (uint64_t)(n - m + 1);
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
    delete srv;
}

}  // extern "C"
