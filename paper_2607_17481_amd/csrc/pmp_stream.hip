// pmp_stream.hip -- stream sessions: samples ingested in order, in batches of
// beta <= excl, with the state resident on the GPU (Sec. 3.1, 3.5,
// Algorithm 1; kernels in k_stream.hip).
//
// The host keeps what decides each batch's shape without reading the device
// back: the change-point counts of the samples (a window is constant when
// none lies inside it, Sec. 2), every anchor's indexed count, depth and run
// bounds.  A batch is then one upload of its descriptor and five to seven
// launches on the session's stream.
#include "pmp_dev.h"
#include "pmp_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace pmp;

struct pmp_stream {
    int device = 0;
    hipStream_t hs = nullptr;
    Opt o;
    int K = kMaxK;
    int m_min = 0, m_max = 0, k = 0, excl = 0, alpha = 0, beta = 0, R = 0;
    int64_t cap = 0;                      // samples the session holds
    std::vector<int> ms;                  // every length of the interval
    std::vector<SAnchor> anc;             // anchor lengths (host copy)
    std::vector<std::vector<uint32_t>> runs;   // run bounds per anchor
    int64_t cells = 0;                    // anchor cells at capacity
    int max_am = 0;                       // longest anchor
    // host state of the series
    int64_t n_in = 0;                     // samples appended
    int64_t n_done = 0;                   // samples whose batch ran
    double last = 0.0;                    // the sample before n_in
    std::vector<uint32_t> E;              // E[x] = change points among samples 1..x-1
    // device state
    double *t = nullptr, *F = nullptr, *mu = nullptr, *isig = nullptr, *basis = nullptr;
    uint64_t *P = nullptr;
    int32_t *I = nullptr, *Icand = nullptr;
    uint32_t *perm = nullptr, *skey = nullptr, *ptmp = nullptr, *ktmp = nullptr, *cellid = nullptr;
    float *gproj = nullptr;
    unsigned long long *counters = nullptr;
    // per batch
    SAnchor *d_anc = nullptr;
    int32_t *d_list = nullptr;            // la[listcap], lq[listcap]
    uint32_t *bkey = nullptr;
    float *bmarg = nullptr;
    SUpdate *upd = nullptr;
    uint32_t *nupd = nullptr;
    SMerge *d_merge = nullptr;
    int listcap = 0;
    uint32_t updcap = 0;
    // pinned staging for the per-batch uploads (a ring, each slot reused
    // only after its copy finished)
    static constexpr int kSlots = 4;
    char *stage[kSlots] = {};
    hipEvent_t stage_ev[kSlots] = {};
    size_t stage_bytes = 0;
    int slot = 0;
    // selection (one-pass top-k)
    char *selblk = nullptr;
    unsigned int *hist = nullptr;
    uint32_t *sel_cnt = nullptr, *scan_tmp = nullptr;
    int64_t need = 0;
    // exact queries: workspace grown on demand
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // statistics
    uint64_t batches = 0, windows = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double ms_ingest = 0.0;
    std::vector<void *> allocs;
    uint64_t dev_bytes = 0;               // device memory held (without the exact query's)
};

namespace {

template <typename T>
int dalloc(pmp_stream *s, T **p, int64_t count) {
    void *v = nullptr;
    const size_t bytes = std::max<size_t>(256, (size_t)count * sizeof(T));
    if (hipMalloc(&v, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PMP_ENOMEM, "stream: hipMalloc of %zu bytes failed", bytes);
    }
    s->allocs.push_back(v);
    s->dev_bytes += bytes;
    *p = (T *)v;
    return PMP_OK;
}

void release(pmp_stream *s) {
    if (!s) return;
    if (s->hs) (void)hipStreamSynchronize(s->hs);
    for (void *p : s->allocs) (void)hipFree(p);
    for (int i = 0; i < pmp_stream::kSlots; ++i) {
        if (s->stage[i]) (void)hipHostFree(s->stage[i]);
        if (s->stage_ev[i]) (void)hipEventDestroy(s->stage_ev[i]);
    }
    if (s->ws) (void)hipFree(s->ws);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->hs) (void)hipStreamDestroy(s->hs);
    delete s;
}

StreamDev dev_args(pmp_stream *s, int nlist) {
    StreamDev S{};
    S.t = s->t;
    S.F = s->F;
    S.mu = s->mu;
    S.isig = s->isig;
    S.P = s->P;
    S.I = s->I;
    S.Icand = s->Icand;
    S.perm = s->perm;
    S.skey = s->skey;
    S.ptmp = s->ptmp;
    S.ktmp = s->ktmp;
    S.basis = s->basis;
    S.gproj = s->gproj;
    S.anc = s->d_anc;
    S.la = s->d_list;
    S.lq = s->d_list + s->listcap;
    S.nlist = nlist;
    S.B = s->o.B;
    S.R = s->R;
    S.excl = s->excl;
    S.bkey = s->bkey;
    S.bmarg = s->bmarg;
    S.upd = s->upd;
    S.nupd = s->nupd;
    S.updcap = s->updcap;
    S.counters = s->counters;
    return S;
}

// Directory depth of an anchor holding n windows (Prop. 4: the smallest d
// with n <= alpha 2^d, up to the signature's bits) and its Hamming-1 probes
// (1 + max(0, d - d0), capped by d and the probe cap), as in the request
// path.
void depth_of(const pmp_stream *s, int64_t n, int &d, int &h) {
    d = 0;
    while (d < s->o.B && n > ((int64_t)s->alpha << d)) ++d;
    h = d > 0 ? 1 + std::max(0, d - s->o.d0) : 0;
    h = std::min(h, std::min(d, s->o.probe_cap));
}

// One batch: the samples [n_done, end) (already resident and counted in E).
int run_batch(pmp_stream *s, int64_t end) {
    const int na = (int)s->anc.size();
    const int64_t t0 = s->n_done, t1 = end;             // sample range of the batch
    std::vector<int32_t> la, lq;
    la.reserve((size_t)na * (t1 - t0));
    lq.reserve((size_t)na * (t1 - t0));
    std::vector<SMerge> merges;
    for (int a = 0; a < na; ++a) {
        SAnchor &A = s->anc[a];
        const int m = A.m;
        A.j0 = (int32_t)la.size();
        int nn = 0;
        // windows completed by samples t0..t1-1: starts tau - m + 1 >= 0
        for (int64_t tau = std::max<int64_t>(t0, m - 1); tau < t1; ++tau) {
            const int64_t q = tau - m + 1;
            if (s->E[q + m] == s->E[q + 1]) continue;   // constant window
            la.push_back(a);
            lq.push_back((int32_t)q);
            ++nn;
        }
        A.nnew = nn;
        int d, h;
        depth_of(s, (int64_t)A.nidx + nn, d, h);
        A.depth = d;
        A.probes = h;
        const std::vector<uint32_t> &rb = s->runs[a];
        A.nruns = (int32_t)rb.size() - 1;
        std::copy(rb.begin(), rb.end(), A.runs);
    }
    const int nlist = (int)la.size();
    if (nlist > s->listcap) return fail(PMP_EINTERNAL, "stream batch list overflow");
    // the runs after this batch: the new run, then the binary-counter merge
    // of the newest runs (a run absorbs the newer ones once they are as
    // large), at most one merge per anchor
    int64_t nthreads = 0;
    for (int a = 0; a < na; ++a) {
        SAnchor &A = s->anc[a];
        if (A.nnew == 0) continue;
        std::vector<uint32_t> &rb = s->runs[a];
        rb.push_back((uint32_t)(A.nidx + A.nnew));
        const int last = (int)rb.size() - 2;             // the new run
        int first = last;
        while (first > 0 && rb[first] - rb[first - 1] <= rb.back() - rb[first]) --first;
        // (the counter keeps about log2 N runs; this bound is not reached in practice)
        while (first > 0 && (int)rb.size() - 1 - (last - first) > kStreamMaxRuns) --first;
        if (first < last) {
            SMerge M{};
            M.cbase = A.cbase;
            M.first = nthreads;
            M.nruns = last - first + 1;
            for (int r = 0; r <= M.nruns; ++r) M.runs[r] = rb[first + r];
            nthreads += M.runs[M.nruns] - M.runs[0];
            merges.push_back(M);
            rb.erase(rb.begin() + first + 1, rb.end() - 1);
        }
        if ((int)rb.size() - 1 > kStreamMaxRuns) return fail(PMP_EINTERNAL, "stream run table overflow");
    }
    // one upload: anchors, list, merges
    const size_t b_anc = (size_t)na * sizeof(SAnchor);
    const size_t b_list = (size_t)2 * s->listcap * sizeof(int32_t);
    const size_t b_mg = merges.size() * sizeof(SMerge);
    char *st = s->stage[s->slot];
    HIPCHK(hipEventSynchronize(s->stage_ev[s->slot]));
    std::memcpy(st, s->anc.data(), b_anc);
    int32_t *sl = (int32_t *)(st + b_anc);
    std::memcpy(sl, la.data(), (size_t)nlist * sizeof(int32_t));
    std::memcpy(sl + s->listcap, lq.data(), (size_t)nlist * sizeof(int32_t));
    std::memcpy(st + b_anc + b_list, merges.data(), b_mg);
    // the device descriptor block is laid out the same way
    HIPCHK(hipMemcpyAsync(s->d_anc, st, b_anc + b_list + b_mg, hipMemcpyHostToDevice, s->hs));
    HIPCHK(hipEventRecord(s->stage_ev[s->slot], s->hs));
    s->slot = (s->slot + 1) % pmp_stream::kSlots;

    const StreamDev S = dev_args(s, nlist);
    launch_stream_windows(S, s->max_am, s->hs);
    launch_stream_probe(S, s->hs);
    if (nlist > 0) launch_stream_apply(S, s->hs);
    launch_stream_newruns(S, na, s->hs);
    launch_stream_merge(S, s->d_merge, (int)merges.size(), nthreads, s->hs);
    HIPCHK(hipGetLastError());
    for (int a = 0; a < na; ++a) s->anc[a].nidx += s->anc[a].nnew;
    s->windows += (uint64_t)nlist;
    s->batches += 1;
    s->n_done = end;
    return PMP_OK;
}

int ingest(pmp_stream *s, bool partial) {
    HIPCHK(hipEventRecord(s->ev0, s->hs));
    while (s->n_in - s->n_done >= s->beta || (partial && s->n_in > s->n_done)) {
        const int64_t end = std::min(s->n_done + s->beta, s->n_in);
        const int rc = run_batch(s, end);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(s->ev1, s->hs));
    HIPCHK(hipEventSynchronize(s->ev1));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, s->ev0, s->ev1) == hipSuccess) s->ms_ingest += ms;
    return PMP_OK;
}

}  // namespace

extern "C" {

int pmp_stream_create(int device, int64_t capacity, int32_t m_min, int32_t m_max, int32_t k,
                      int32_t exclusion, int32_t budget, int32_t batch, const pmp_options *opt,
                      pmp_stream **out) {
    clear_error();
    if (!out) return fail(PMP_EINVAL, "out is NULL");
    *out = nullptr;
    Opt o;
    int rc = read_options(opt, o);
    if (rc) return rc;
    if (o.precision != PMP_PREC_FP64)
        return fail(PMP_EINVAL, "stream sessions compute in the FP64 form only");
    if (m_min < 3 || m_max < m_min || m_max > kMaxM || capacity < m_max || k < 1 ||
        exclusion < 1 || budget < 1)
        return fail(PMP_EINVAL, "bad stream arguments");
    if (batch == 0) batch = exclusion;
    if (batch < 1 || batch > exclusion) return fail(PMP_EINVAL, "batch must be in [1, exclusion]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(PMP_EDEVICE, "no HIP device %d", device);
    if (hipSetDevice(device) != hipSuccess) return fail(PMP_EDEVICE, "hipSetDevice failed");

    pmp_stream *s = new pmp_stream();
    s->device = device;
    s->o = o;
    s->K = o.K ? o.K : kMaxK;
    s->m_min = m_min;
    s->m_max = m_max;
    s->k = k;
    s->excl = exclusion;
    s->alpha = budget;
    s->beta = batch;
    s->R = o.gamma * budget;
    s->cap = capacity;
    for (int64_t m = m_min; m <= m_max; m += o.m_step) s->ms.push_back((int)m);
    // anchor lengths (Sec. 3.3): every stride-th length of the list and the
    // last one
    const int L = (int)s->ms.size();
    int64_t cb = 0, bb = 0;
    for (int l = 0; l < L; ++l) {
        if (!(l % o.stride == 0 || l == L - 1)) continue;
        SAnchor A{};
        A.m = s->ms[l];
        A.kprime = kprime_of(s->K, A.m);
        A.cbase = cb;
        A.bbase = bb;
        cb += capacity - A.m + 1;
        bb += (int64_t)2 * A.kprime * A.m;
        s->max_am = std::max(s->max_am, A.m);
        s->anc.push_back(A);
        s->runs.push_back({0u});
    }
    s->cells = cb;
    const int na = (int)s->anc.size();
    if (cb > INT32_MAX) {
        release(s);
        return fail(PMP_EINVAL, "stream capacity times anchor lengths exceeds 2^31 cells");
    }
    s->E.assign((size_t)capacity + 1, 0u);
    s->listcap = std::max(1, na * batch);
    s->updcap = (uint32_t)std::min<int64_t>((int64_t)s->listcap * s->R, UINT32_MAX);
    s->need = need_select(k, s->max_am);

#define SCHK(x)            \
    do {                   \
        rc = (x);          \
        if (rc) {          \
            release(s);    \
            return rc;     \
        }                  \
    } while (0)
    SCHK(dalloc(s, &s->t, capacity));
    SCHK(dalloc(s, &s->F, cb * kRec));
    SCHK(dalloc(s, &s->mu, cb));
    SCHK(dalloc(s, &s->isig, cb));
    SCHK(dalloc(s, &s->P, cb));
    SCHK(dalloc(s, &s->I, cb));
    SCHK(dalloc(s, &s->Icand, cb));
    SCHK(dalloc(s, &s->perm, cb));
    SCHK(dalloc(s, &s->skey, cb));
    SCHK(dalloc(s, &s->ptmp, cb));
    SCHK(dalloc(s, &s->ktmp, cb));
    SCHK(dalloc(s, &s->cellid, cb));
    SCHK(dalloc(s, &s->basis, bb));
    SCHK(dalloc(s, &s->gproj, (int64_t)na * kMaxBits * kFD));
    SCHK(dalloc(s, &s->counters, kStreamCounters));
    {
        // anchors, batch list and merge descriptors in one block
        char *blk = nullptr;
        const size_t bytes = (size_t)na * sizeof(SAnchor) + (size_t)2 * s->listcap * sizeof(int32_t) +
                             (size_t)na * sizeof(SMerge);
        SCHK(dalloc(s, &blk, (int64_t)bytes));
        s->d_anc = (SAnchor *)blk;
        s->d_list = (int32_t *)(blk + (size_t)na * sizeof(SAnchor));
        s->d_merge = (SMerge *)(blk + (size_t)na * sizeof(SAnchor) +
                                (size_t)2 * s->listcap * sizeof(int32_t));
        s->stage_bytes = bytes;
    }
    SCHK(dalloc(s, &s->bkey, s->listcap));
    SCHK(dalloc(s, &s->bmarg, (int64_t)s->listcap * kMaxBits));
    SCHK(dalloc(s, &s->upd, s->updcap));
    SCHK(dalloc(s, &s->nupd, 1));
    SCHK(dalloc(s, &s->selblk, (int64_t)select_block_bytes(s->need)));
    SCHK(dalloc(s, &s->hist, kSelBins));
    SCHK(dalloc(s, &s->sel_cnt, select_blocks(cb) + 1));
    SCHK(dalloc(s, &s->scan_tmp, (int64_t)scan_temp_bytes(select_blocks(cb) + 1) / 4 + 1));
#undef SCHK
    auto hchk = [&](hipError_t e, const char *what) {
        if (e == hipSuccess) return PMP_OK;
        release(s);
        return fail(PMP_EDEVICE, "stream: %s failed: %s", what, hipGetErrorString(e));
    };
    if ((rc = hchk(hipStreamCreateWithFlags(&s->hs, hipStreamNonBlocking), "hipStreamCreate")))
        return rc;
    for (int i = 0; i < pmp_stream::kSlots; ++i) {
        if ((rc = hchk(hipHostMalloc((void **)&s->stage[i], s->stage_bytes), "hipHostMalloc")))
            return rc;
        if ((rc = hchk(hipEventCreateWithFlags(&s->stage_ev[i], hipEventDisableTiming),
                       "hipEventCreate")))
            return rc;
        if ((rc = hchk(hipEventRecord(s->stage_ev[i], s->hs), "hipEventRecord"))) return rc;
    }
    if ((rc = hchk(hipEventCreate(&s->ev0), "hipEventCreate"))) return rc;
    if ((rc = hchk(hipEventCreate(&s->ev1), "hipEventCreate"))) return rc;

    // projections, basis tables, an empty profile
    std::vector<float> gp((size_t)na * kMaxBits * kFD);
    for (int a = 0; a < na; ++a) projections(o.seed, s->anc[a].m, gp.data() + (size_t)a * kMaxBits * kFD);
    if ((rc = hchk(hipMemcpyAsync(s->gproj, gp.data(), gp.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s->hs), "hipMemcpyAsync")))
        return rc;
    if ((rc = hchk(hipMemcpyAsync(s->d_anc, s->anc.data(), (size_t)na * sizeof(SAnchor),
                                  hipMemcpyHostToDevice, s->hs), "hipMemcpyAsync")))
        return rc;
    int64_t max_elems = 0;
    for (const SAnchor &A : s->anc) max_elems = std::max<int64_t>(max_elems, 2 * A.kprime * A.m);
    launch_stream_basis(s->d_anc, na, max_elems, s->basis, s->hs);
    launch_fill_u64(s->P, cb, kInfBits, s->hs);
    launch_fill_u32((uint32_t *)s->I, cb, 0xFFFFFFFFu, s->hs);
    launch_fill_u32(s->nupd, 1, 0u, s->hs);
    launch_fill_u64((uint64_t *)s->counters, kStreamCounters, 0ull, s->hs);
    launch_iota_u32(s->cellid, cb, s->hs);
    if ((rc = hchk(hipGetLastError(), "launch"))) return rc;
    if ((rc = hchk(hipStreamSynchronize(s->hs), "hipStreamSynchronize"))) return rc;
    *out = s;
    return PMP_OK;
}

int pmp_stream_append(pmp_stream *s, const double *samples, int64_t count) {
    clear_error();
    if (!s || (count > 0 && !samples) || count < 0) return fail(PMP_EINVAL, "bad arguments");
    if (count > s->cap - s->n_in)
        return fail(PMP_EINVAL, "append of %lld samples exceeds the capacity (%lld held of %lld)",
                    (long long)count, (long long)s->n_in, (long long)s->cap);
    for (int64_t x = 0; x < count; ++x)
        if (!std::isfinite(samples[x])) return fail(PMP_EINVAL, "non-finite sample at %lld", (long long)x);
    if (count == 0) return PMP_OK;
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipMemcpyAsync(s->t + s->n_in, samples, (size_t)count * sizeof(double),
                          hipMemcpyHostToDevice, s->hs));
    for (int64_t x = 0; x < count; ++x) {
        const int64_t r = s->n_in + x;
        const bool chg = r > 0 && samples[x] != (x > 0 ? samples[x - 1] : s->last);
        s->E[r + 1] = s->E[r] + (chg ? 1u : 0u);
    }
    s->last = samples[count - 1];
    s->n_in += count;
    return ingest(s, false);
}

int pmp_stream_flush(pmp_stream *s) {
    clear_error();
    if (!s) return fail(PMP_EINVAL, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    return ingest(s, true);
}

int pmp_stream_topk(pmp_stream *s, pmp_motif *out, int32_t *n_out) {
    clear_error();
    if (!s || !out || !n_out) return fail(PMP_EINVAL, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    *n_out = 0;
    const int64_t need = s->need;
    SelState *sel = (SelState *)s->selblk;
    uint64_t *less_val = (uint64_t *)(s->selblk + kSelHead);
    uint32_t *less_k = (uint32_t *)(less_val + need);
    uint32_t *less_cell = less_k + need;
    uint32_t *eq_k = less_cell + need;
    uint32_t *eq_cell = eq_k + need;
    launch_select(s->P, s->cells, need, sel, s->hist, s->sel_cnt, s->scan_tmp, less_k, less_val,
                  eq_k, less_cell, eq_cell, s->cellid, s->hs);
    HIPCHK(hipGetLastError());
    std::vector<char> host(select_block_bytes(need));
    HIPCHK(hipMemcpyAsync(host.data(), s->selblk, host.size(), hipMemcpyDeviceToHost, s->hs));
    HIPCHK(hipStreamSynchronize(s->hs));
    SelState st;
    std::memcpy(&st, host.data(), sizeof(st));
    if (!st.done || st.nless > (uint32_t)need) return fail(PMP_EINTERNAL, "stream selection failed");
    const uint64_t *lv = (const uint64_t *)(host.data() + kSelHead);
    const uint32_t *lc = (const uint32_t *)(lv + need) + need;
    const uint32_t *ec = lc + 2 * need;
    struct C {
        double d;
        int a;
        int64_t q;
    };
    auto anchor_of = [&](uint32_t cell) {
        int a = 0;
        while (a + 1 < (int)s->anc.size() && s->anc[a + 1].cbase <= (int64_t)cell) ++a;
        return a;
    };
    std::vector<C> c;
    for (uint32_t x = 0; x < st.nless; ++x) {
        double d;
        std::memcpy(&d, &lv[x], 8);
        const int a = anchor_of(lc[x]);
        c.push_back({d, a, (int64_t)lc[x] - s->anc[a].cbase});
    }
    // key (P, m, i): anchors are in ascending m and cells ascending within
    std::sort(c.begin(), c.end(), [](const C &x, const C &y) {
        if (x.d != y.d) return x.d < y.d;
        if (x.a != y.a) return x.a < y.a;
        return x.q < y.q;
    });
    if (st.pivot != kInfBits) {
        double pv;
        std::memcpy(&pv, &st.pivot, 8);
        for (int64_t x = 0; x < st.need_eq; ++x) {
            const int a = anchor_of(ec[x]);
            c.push_back({pv, a, (int64_t)ec[x] - s->anc[a].cbase});
        }
    }
    // greedy (Sec. 2): skip a cell within m/2 of an accepted cell of its length
    std::vector<C> acc;
    for (const C &x : c) {
        if (!std::isfinite(x.d)) break;
        bool skip = false;
        for (const C &y : acc)
            if (y.a == x.a && 2 * std::llabs(y.q - x.q) <= s->anc[x.a].m) {
                skip = true;
                break;
            }
        if (skip) continue;
        acc.push_back(x);
        if ((int)acc.size() == s->k) break;
    }
    for (size_t x = 0; x < acc.size(); ++x) {
        int32_t nb = -1;
        HIPCHK(hipMemcpy(&nb, s->I + s->anc[acc[x].a].cbase + acc[x].q, sizeof(int32_t),
                         hipMemcpyDeviceToHost));
        out[x].i = acc[x].q;
        out[x].j = nb;
        out[x].m = s->anc[acc[x].a].m;
        out[x].flags = 0;
        out[x].dist = acc[x].d;
    }
    *n_out = (int32_t)acc.size();
    return PMP_OK;
}

int pmp_stream_exact(pmp_stream *s, pmp_motif *out, int32_t *n_out, pmp_stats *stats) {
    clear_error();
    if (!s || !out || !n_out) return fail(PMP_EINVAL, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    *n_out = 0;
    if (s->n_in < s->m_max) return fail(PMP_EINVAL, "the stream holds fewer samples than m_max");
    pmp_options po;
    memset(&po, 0, sizeof(po));
    po.size = sizeof(po);
    po.m_step = s->o.m_step;
    po.precision = s->o.precision;
    po.spectral_width = s->o.K;
    po.seed = s->o.seed;
    po.certify = 1;
    po.signature_bits = s->o.B;
    po.gamma = s->o.gamma;
    po.probe_ref_depth = s->o.d0;
    po.probe_cap = s->o.probe_cap;
    po.anchor_stride = s->o.stride;
    po.sieve_width = s->o.sieve_w;
    po.complete_rounds = s->o.compl_rounds;
    po.complete_dm = s->o.compl_dm;
    po.complete_dp = s->o.compl_dp;
    const size_t need = pmp_workspace_bytes(s->n_in, s->m_min, s->m_max, s->k, &po);
    if (need == 0) return fail(PMP_EINVAL, "bad arguments for the exact query");
    if (need > s->ws_bytes) {
        if (s->ws) HIPCHK(hipFree(s->ws));
        s->ws = nullptr;
        s->ws_bytes = 0;
        if (hipMalloc(&s->ws, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(PMP_ENOMEM, "stream: exact query workspace of %zu bytes", need);
        }
        s->ws_bytes = need;
    }
    return pmp_run_device(s->t, s->n_in, s->m_min, s->m_max, s->k, s->excl, s->alpha, &po, s->ws,
                          s->ws_bytes, (void *)s->hs, out, n_out, stats);
}

int pmp_stream_profile(pmp_stream *s, int32_t anchor, double *P, int64_t *I, int64_t *W) {
    clear_error();
    if (!s || anchor < 0 || anchor >= (int32_t)s->anc.size() || !W)
        return fail(PMP_EINVAL, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    const SAnchor &A = s->anc[anchor];
    const int64_t w = s->n_done >= A.m ? s->n_done - A.m + 1 : 0;
    *W = w;
    HIPCHK(hipStreamSynchronize(s->hs));
    if (w == 0) return PMP_OK;
    if (P) {
        HIPCHK(hipMemcpy(P, s->P + A.cbase, (size_t)w * sizeof(double), hipMemcpyDeviceToHost));
    }
    if (I) {
        std::vector<int32_t> tmp((size_t)w);
        HIPCHK(hipMemcpy(tmp.data(), s->I + A.cbase, (size_t)w * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
        for (int64_t x = 0; x < w; ++x) I[x] = tmp[(size_t)x];
    }
    return PMP_OK;
}

int pmp_stream_info(pmp_stream *s, pmp_stream_stats *st, int32_t *lengths, int32_t capacity) {
    clear_error();
    if (!s || !st) return fail(PMP_EINVAL, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    unsigned long long c[kStreamCounters] = {};
    HIPCHK(hipMemcpyAsync(c, s->counters, sizeof(c), hipMemcpyDeviceToHost, s->hs));
    HIPCHK(hipStreamSynchronize(s->hs));
    std::memset(st, 0, sizeof(*st));
    st->appended = (uint64_t)s->n_in;
    st->processed = (uint64_t)s->n_done;
    st->batches = s->batches;
    st->windows = s->windows;
    st->candidates = c[CS_CAND];
    st->verified = c[CS_VER];
    st->updates = c[CS_UPD];
    st->dropped = c[CS_DROP];
    st->anchors = (int32_t)s->anc.size();
    st->K = s->K;
    st->batch = s->beta;
    st->ms_ingest = s->ms_ingest;
    st->device_bytes = s->dev_bytes + s->ws_bytes;
    if (lengths)
        for (int a = 0; a < (int)s->anc.size() && a < capacity; ++a) lengths[a] = s->anc[a].m;
    return PMP_OK;
}

void pmp_stream_destroy(pmp_stream *s) { release(s); }

}  // extern "C"
