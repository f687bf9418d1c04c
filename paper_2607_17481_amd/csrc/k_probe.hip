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
// their bit patterns), which is order independent, so the profile does not
// depend on the schedule (the role of the fixed merge order of Prop. 5).
//
// One departure from the paper: a query stops once its own cell reaches 0
// (the smallest possible value); the remaining candidates could only lower
// their own cells, which their own queries, or the certificate, cover.
#include "pmp_dev.h"

namespace pmp {

template <typename FT>
__global__ __launch_bounds__(kBlock) void k_probe(Req q, const uint32_t *__restrict__ bstart,
                                                  int64_t N) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t n_cand = 0, n_ver = 0;
    if (s < N) {
        const int l = find_len_slot(q.len, q.L, s);
        const LenInfo L = q.len[l];
        const int m = L.m;
        const int d = L.depth;
        const int kp = L.kprime;
        const float sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
        const uint32_t cq = q.perm[s];
        const int64_t iq = (int64_t)cq - L.cell_base;
        const uint64_t kw = q.keyw[s];
        const uint32_t sig = (uint32_t)(kw & 0xFFFFFFu);
        const uint32_t prefix = d ? sig >> (q.B - d) : 0u;
        const FT *fq = (const FT *)q.F + s * kRec;
        double Pq = bitsd(q.P[cq]);
        const double muq = q.mu[cq], isq = q.isig[cq];
        const int64_t last_valid = iq - q.excl;          // candidates i <= iq - excl
        int budget = q.budget_R;
        const uint32_t *bb = bstart + L.bucket_base;
        for (int pr = 0; pr <= L.probes && budget > 0 && Pq > 0.0; ++pr) {
            uint32_t b = prefix;
            if (pr > 0) {
                const int bit = (int)((kw >> (24 + 5 * (pr - 1))) & 31u);
                b = prefix ^ (1u << (d - 1 - bit));
            }
            const int64_t bs = bb[b], be = bb[b + 1];
            if (be <= bs || last_valid < 0) continue;
            // first entry with start > last_valid
            int64_t lo = bs, hi = be;
            const uint32_t lim = (uint32_t)(L.cell_base + last_valid);
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (q.perm[mid] <= lim) lo = mid + 1; else hi = mid;
            }
            const int64_t cut = lo;
            const int64_t cnt = cut - bs;
            if (cnt <= 0) continue;
            int take, rec;
            int64_t strided_span;
            if (cnt <= budget) {
                take = (int)cnt; rec = take; strided_span = 0;
            } else {
                take = budget; rec = budget - budget / 2; strided_span = cnt - rec;
            }
            const int str = take - rec;
            budget -= take;
            for (int j = 0; j < take && Pq > 0.0; ++j) {
                int64_t cs;
                if (j < rec) cs = cut - 1 - j;                         // most recent first
                else cs = bs + ((int64_t)(j - rec) * strided_span) / str;   // even intervals
                ++n_cand;
                const uint32_t cc = q.perm[cs];
                const double Pc = bitsd(q.P[cc]);
                const double thr = fmax(Pq, Pc);
                if (thr == 0.0) continue;
                const FT *fc = (const FT *)q.F + cs * kRec;
                const float lb = lb_safe<FT>(fq, fc, kp, sqrt2m);
                if ((double)lb >= thr) continue;
                ++n_ver;
                const double dd = snap(zdist(q.t, iq, muq, isq, (int64_t)cc - L.cell_base,
                                             q.mu[cc], q.isig[cc], m));
                const uint64_t db = dbits(dd);
                if (dd < Pq) {
                    atomicMin((unsigned long long *)&q.P[cq], (unsigned long long)db);
                    Pq = dd;
                }
                if (dd < Pc) atomicMin((unsigned long long *)&q.P[cc], (unsigned long long)db);
            }
        }
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

void launch_probe(int precision, const Req &q, const uint32_t *bstart, int64_t N, hipStream_t s) {
    if (N <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_probe<double>, dim3(nblk(N)), dim3(kBlock), 0, s, q, bstart, N);
    else
        hipLaunchKernelGGL(k_probe<float>, dim3(nblk(N)), dim3(kBlock), 0, s, q, bstart, N);
}

void launch_hot_buckets(const uint32_t *bstart, int64_t nb, int R, unsigned long long *cnt,
                        hipStream_t s) {
    if (nb > 0)
        hipLaunchKernelGGL(k_hot_buckets, dim3(nblk(nb)), dim3(kBlock), 0, s, bstart, nb, R, cnt);
}

}  // namespace pmp
