// k_probe.hip -- streaming candidate generation, Parseval prune and exact
// verification (paper Sec. 3.4, Algorithm 1 phase B).
//
// Every indexed window q is a query.  Its candidates are the windows stored
// in its own bucket (the d-bit signature prefix) and then in the Hamming-1
// buckets of its `probes` lowest-margin prefix bits, in increasing margin
// order.  As in the stream, a query only sees earlier windows, and only valid
// ones (i <= q - excl); each bucket is sorted by start, so those form a prefix
// of the bucket.  Inspections are capped at R = gamma * alpha per query; when
// a bucket holds more valid entries than the remaining budget, half of it goes
// to the most recent entries and half to entries at even intervals over the
// rest of the bucket.
//
// A candidate c is evaluated exactly only if its certified Parseval bound is
// below max(P[q], P[c]) -- the two cells the pair can lower (Sec. 3.4, the
// definition of S_stream).  Each exact distance lowers both cells through a
// 64-bit atomic min on the FP64 bit pattern (non-negative doubles order like
// their bit patterns), which is order independent.  Which candidates pass the
// prune depends on how far the cells have been lowered when they are
// inspected, so the upper profile may differ slightly between runs; the exact
// top-k built on it by the certificate does not (the role of the fixed merge
// order of Prop. 5).
//
// GPU mapping: one lane per query searches its candidates (lane-parallel
// bound tests) until every lane still working holds a proposal; a lane that
// holds one already (and whose own cell is finite) keeps searching for a
// second meanwhile, so the wait for the slowest lane's search is used.  The
// exact distances of the proposals are then computed for the whole
// wavefront (verify_proposals), first slot, then second.
//
// One departure from the paper: a query stops once its own cell reaches 0
// (the smallest possible value); the remaining candidates could only lower
// their own cells, which their own queries, or the certificate, cover.
#include "pmp_dev.h"

namespace pmp {

// The query windows of a wavefront, staged in LDS when they share one length
// and lie within a short span of the series (dynamic size: kQwinExtra + the
// longest window, in doubles).  The staged samples are the series' own, so a
// distance read through them has the same bits.
extern __shared__ double probe_qwin[];
constexpr int kQwinExtra = 256;
struct QwinA {
    int64_t base;
    __device__ __forceinline__ double operator()(int64_t x) const { return probe_qwin[x - base]; }
};

// Queries are taken in (length, start) order (indexed position k), so that
// neighbouring windows, which tend to cost alike, share a wavefront; only the
// anchor lengths are probed (Sec. 3.3), each from its first probe block, so a
// wavefront never spans two lengths.  A block is one wavefront: wavefront
// times vary over two orders of magnitude, and a single-wave block lets a
// compute unit start new work as soon as any one wavefront ends, not when a
// slot for four is free.  Whenever a verification lowers a cell, the partner's
// start is recorded as the cell's hint (any partner that lowered it will do:
// the hints only propose pairs at the lengths between anchors).
// Four wavefronts per SIMD (128 registers, a few spilled) hide more of the
// candidate chain's latency than three without spills.
template <typename FT>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4)))
void k_probe(Req q, const uint32_t *__restrict__ bstart, int qcap, int64_t blk0) {
    // the anchor length of this block (blocks [blk0, blk0 + gridDim.x) of
    // the probe): the last length whose first probe block is at or below it
    // (uniform)
    const int64_t gb = blk0 + (int64_t)blockIdx.x;
    int lb = 0;
    {
        int hi = q.L - 1;
        while (lb < hi) {
            const int mid = (lb + hi + 1) >> 1;
            if (q.len[mid].pblk_base <= gb) lb = mid; else hi = mid - 1;
        }
    }
    const int64_t k_first = q.len[lb].kbase + (gb - q.len[lb].pblk_base) * kWave;
    const int64_t k = k_first + threadIdx.x;
    uint32_t n_cand = 0, n_ver = 0;

    // ---- per-lane query state
    bool done = k >= q.len[lb].kbase + q.len[lb].n_index;
    int l = -1, m = 0, d = 0, probes = 0;
    int64_t cell_base = 0;
    uint32_t cq = 0, prefix = 0, lim = 0;
    int64_t iq = 0;
    uint64_t kw = 0;
    double Pq = 0.0, muq = 0.0, isq = 0.0;
    float sqrt2m = 0.0f;
    const uint32_t *bb = bstart;
    const FT *fq = (const FT *)q.F;
    if (!done) {
        l = lb;
        const LenInfo L = q.len[l];
        m = L.m;
        d = L.depth;
        probes = L.probes;
        cell_base = L.cell_base;
        bb = bstart + L.bucket_base;
        sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
        cq = q.cell[k];
        iq = (int64_t)cq - cell_base;
        kw = q.keyw[k];
        prefix = d ? (uint32_t)(kw & 0xFFFFFFu) >> (q.B - d) : 0u;
        Pq = bitsd(q.P[k]);
        muq = q.mu[k];
        isq = q.isig[k];
        fq += k * kRec;
        done = Pq == 0.0 || iq - q.excl < 0;
        lim = (uint32_t)(cell_base + iq - q.excl);
    }
    // ---- stage the query windows (uniform decision): one length, and the
    // span from the first start to the last window's end fits
    bool staged = false;
    int64_t qlo = 0;
    {
        const uint64_t valid = __ballot(l >= 0);
        const int last = 63 - __clzll((long long)valid);
        const int l0 = __shfl(l, 0, kWave);
        qlo = __shfl(iq, 0, kWave);
        const int64_t qhi = __shfl(iq, last, kWave) + __shfl(m, last, kWave);
        staged = __ballot(l >= 0 && l != l0) == 0 && qhi - qlo <= (int64_t)qcap;
        if (staged) {
            for (int64_t x = lane_id(); x < qhi - qlo; x += kWave) probe_qwin[x] = q.t[qlo + x];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    // candidate iterator
    int pr = -1, budget = q.budget_R;
    int64_t bs = 0, cut = 0, span = 0;
    int take = 0, rec = 0, str = 1, j = 0;
    // current proposals (two slots), kept in LDS from the search that finds
    // them to the verification that reads them, so that they hold no
    // registers through the search loop
    __shared__ double s_Pc[2][kWave], s_mu[2][kWave], s_is[2][kWave], s_lim[2][kWave];
    __shared__ int64_t s_ic[2][kWave];
    __shared__ uint32_t s_c[2][kWave];
    const int ln = threadIdx.x;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        s_Pc[sl][ln] = 0.0;
        s_mu[sl][ln] = 0.0;
        s_is[sl][ln] = 0.0;
        s_lim[sl][ln] = INFINITY;
        s_ic[sl][ln] = 0;
        s_c[sl][ln] = 0;
    }
    bool has = false, has1 = false;

    for (;;) {
        // ---- the wavefront searches until every lane still working holds a
        // proposal; a lane that holds one already looks for a second meanwhile
        while (__ballot(!done && !has) != 0) {
            // a second proposal only once the query's own cell is finite
            // (before that, its first distance often ends it: a repeat at 0)
            if (done || has1 || (has && Pq == INFINITY)) continue;
            if (j >= take) {
                // open the next bucket
                ++pr;
                if (pr > probes || budget <= 0) { done = true; continue; }
                uint32_t b = prefix;
                if (pr > 0) {
                    const int bit = (int)((kw >> (24 + 5 * (pr - 1))) & 31u);
                    b = prefix ^ (1u << (d - 1 - bit));
                }
                bs = bb[b];
                // the valid entries (cell <= lim) form a prefix of the bucket
                // (in the own bucket the query and everything after it lie
                // past the prefix)
                int64_t lo = bs, hi = (int64_t)bb[b + 1];
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (q.pcell[mid] <= lim) lo = mid + 1; else hi = mid;
                }
                cut = lo;
                const int64_t cnt = cut - bs;
                j = 0;
                if (cnt <= 0) { take = 0; continue; }
                if (cnt <= budget) {
                    take = (int)cnt; rec = take; span = 0;
                } else {
                    take = budget; rec = budget - budget / 2; span = cnt - rec;
                }
                str = take - rec > 0 ? take - rec : 1;
                budget -= take;
                continue;
            }
            const int64_t cs = j < rec ? cut - 1 - j : bs + ((int64_t)(j - rec) * span) / str;
            ++j;
            ++n_cand;
            const uint32_t kc = q.perm[cs];
            const double Pc = bitsd(q.P[kc]);
            const double thr = fmax(Pq, Pc);
            if (thr == 0.0) continue;
            // no bound can prune below +inf: skip the record reads
            if (thr != INFINITY) {
                const float lb = lb_mem<FT>(fq, (const FT *)q.F + (int64_t)kc * kRec, sqrt2m);
                if ((double)lb >= thr) continue;
            }
            {
                const int sl = has ? 1 : 0;
                s_lim[sl][ln] = exit_bound(thr);
                s_c[sl][ln] = kc;
                s_ic[sl][ln] = (int64_t)q.pcell[cs] - cell_base;
                s_Pc[sl][ln] = Pc;
                s_mu[sl][ln] = q.mu[kc];
                s_is[sl][ln] = q.isig[kc];
                if (has) has1 = true; else has = true;
            }
        }
        // ---- the wavefront verifies the first proposals
        const uint64_t mask = __ballot(has);
        if (mask == 0) break;
        const double pPc = s_Pc[0][ln], pmu = s_mu[0][ln], pis = s_is[0][ln], plim = s_lim[0][ln];
        const int64_t pic = s_ic[0][ln];
        const uint32_t pc = s_c[0][ln];
        auto on_result = [&](double dd) {
            ++n_ver;
            const unsigned long long db = (unsigned long long)dbits(dd);
            if (dd < Pq) {
                atomicMin((unsigned long long *)&q.P[k], db);
                Pq = dd;
                q.hint[k] = (uint32_t)pic;
            }
            if (dd < pPc) {
                atomicMin((unsigned long long *)&q.P[pc], db);
                q.hint[pc] = (uint32_t)iq;
            }
            has = false;
            if (Pq == 0.0) done = true;
        };
        if (staged)
            verify_proposals(mask, QwinA{qlo}, q.t, iq, muq, isq, pic, pmu, pis, m, on_result, plim);
        else
            verify_proposals(mask, SeriesA{q.t}, q.t, iq, muq, isq, pic, pmu, pis, m, on_result,
                             plim);
        // the second slot (a lane whose own cell reached 0 drops it)
        const uint64_t mask1 = __ballot(has1 && !done);
        auto on_result1 = [&](double dd) {
            const double pPc1 = s_Pc[1][ln];
            const uint32_t pc1 = s_c[1][ln];
            ++n_ver;
            const unsigned long long db = (unsigned long long)dbits(dd);
            if (dd < Pq) {
                atomicMin((unsigned long long *)&q.P[k], db);
                Pq = dd;
                q.hint[k] = (uint32_t)s_ic[1][ln];
            }
            if (dd < pPc1) {
                atomicMin((unsigned long long *)&q.P[pc1], db);
                q.hint[pc1] = (uint32_t)iq;
            }
            if (Pq == 0.0) done = true;
        };
        if (mask1) {
            const double pmu1 = s_mu[1][ln], pis1 = s_is[1][ln], plim1 = s_lim[1][ln];
            const int64_t pic1 = s_ic[1][ln];
            if (staged)
                verify_proposals(mask1, QwinA{qlo}, q.t, iq, muq, isq, pic1, pmu1, pis1, m, on_result1,
                                 plim1);
            else
                verify_proposals(mask1, SeriesA{q.t}, q.t, iq, muq, isq, pic1, pmu1, pis1, m,
                                 on_result1, plim1);
        }
        has1 = false;
    }
    // stats: one atomic per wave
    unsigned long long a = n_cand, v = n_ver;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, kWave);
        v += __shfl_xor(v, off, kWave);
    }
    if (lane_id() == 0) {
        if (a) atomicAdd(&q.counters[C_PASS_CAND], a);
        if (v) atomicAdd(&q.counters[C_PASS_VER], v);
    }
}

// Buckets holding more than R entries (hot classes, Sec. 3.6) -- statistics.
__global__ __launch_bounds__(kBlock) void k_hot_buckets(const uint32_t *__restrict__ bstart,
                                                        int64_t nb, int R,
                                                        unsigned long long *__restrict__ cnt) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long h = 0;
    if (b < nb) h = (bstart[b + 1] - bstart[b]) > (uint32_t)R;
    for (int off = kWave / 2; off > 0; off >>= 1) h += __shfl_xor(h, off, kWave);
    if (lane_id() == 0 && h) atomicAdd(cnt, h);
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_probe(int precision, const Req &q, const uint32_t *bstart, int64_t blk0,
                  int64_t nblocks, int max_m, hipStream_t s) {
    if (nblocks <= 0) return;
    const dim3 grid((unsigned)nblocks);
    const int qcap = kQwinExtra + max_m;
    const size_t lds = (size_t)qcap * sizeof(double);
    if (precision == 0)
        hipLaunchKernelGGL(k_probe<double>, grid, dim3(kWave), lds, s, q, bstart, qcap, blk0);
    else
        hipLaunchKernelGGL(k_probe<float>, grid, dim3(kWave), lds, s, q, bstart, qcap, blk0);
}

void launch_hot_buckets(const uint32_t *bstart, int64_t nb, int R, unsigned long long *cnt,
                        hipStream_t s) {
    if (nb > 0)
        hipLaunchKernelGGL(k_hot_buckets, dim3(nblk(nb)), dim3(kBlock), 0, s, bstart, nb, R, cnt);
}

}  // namespace pmp
