// k_complete.hip -- the emit stage of the one pass (paper Sec. 3.3 anchor
// lengths, Sec. 3.6 emit-time completion, Algorithm 2): the hot-class sieve,
// the hints at the lengths between anchors, and local completion.
//
// Every step here only lowers cells of the upper profile through exact
// distances (the canonical FP64 distance of pmp_dev.h), so soundness (Prop. 1)
// holds as for the probe; the certificate that follows makes the reported
// top-k exact whatever these steps find.  They matter for speed: the lower
// the upper profile before the certificate, the smaller its threshold and the
// fewer windows it treats as queries.
//
//  * Sieve (S_hot): a bucket of an anchor length holding more than R entries
//    was never scanned in full.  Its members are sorted by their projection
//    on one seeded Gaussian direction of that length, and every member is
//    verified against the w members after it in that order (Lemma 3 bounds
//    how far apart the closest pair of the class lands).
//  * Hints: a length between anchors has no index of its own.  Each of its
//    windows is re-cut with the partners that the nearest anchor lengths below
//    and above recorded for the window at the same start (their hints), the
//    "index or hint" rule of the paper's emit refinement applied once to every
//    cell.  (A departure: the paper re-cuts only around its seeds; here a cell
//    left without a value would become a query of the certificate.)  Both
//    anchors are used, not chains through the neighbouring lengths: a window
//    constant at one length (no change point inside, so no hint) may not be at
//    the next, and a chain would break there for every member of its class.
//  * Local completion (S_local): around each seed (m0, i0) with partner j0,
//    every (m, i, j) with |m - m0| <= dm, |i - i0| <= dp, |j - j0| <= dp,
//    |i - j| >= excl is evaluated exactly; improved cells take the partner as
//    their hint.  The seeds are the current top-k cells, re-selected every
//    round, for at most P_max rounds or until no cell improves.
#include "pmp_dev.h"

namespace pmp {

namespace {

// Lowers both cells of a verified pair; the hint of a lowered cell becomes
// its partner's start.  Returns true if either cell went down.
__device__ __forceinline__ bool lower_pair(const Req &q, uint32_t ka, int64_t ia, uint32_t kb,
                                           int64_t ib, double d) {
    const unsigned long long db = (unsigned long long)dbits(d);
    bool lowered = false;
    if (atomicMin((unsigned long long *)&q.P[ka], db) > db) {
        q.hint[ka] = (uint32_t)ib;
        lowered = true;
    }
    if (atomicMin((unsigned long long *)&q.P[kb], db) > db) {
        q.hint[kb] = (uint32_t)ia;
        lowered = true;
    }
    return lowered;
}

// one candidate pair of a lane, tested (Parseval prune against the two cells
// it could lower) and, if it survives, proposed for verification
template <typename FT>
struct Proposal {
    bool on = false;
    uint32_t kb = 0;
    int64_t ib = 0;
    double mub = 0.0, isb = 0.0, lim = INFINITY;
};

template <typename FT>
__device__ __forceinline__ Proposal<FT> propose(const Req &q, uint32_t ka, uint32_t kb, int64_t ib,
                                                float sqrt2m) {
    Proposal<FT> pr;
    const double thr = fmax(bitsd(q.P[ka]), bitsd(q.P[kb]));
    if (thr == 0.0) return pr;
    if (thr != INFINITY) {
        const FT *F = (const FT *)q.F;
        const float lb = lb_mem<FT>(F + (int64_t)ka * kRec, F + (int64_t)kb * kRec, sqrt2m);
        if ((double)lb >= thr) return pr;
    }
    pr.on = true;
    pr.kb = kb;
    pr.ib = ib;
    pr.mub = q.mu[kb];
    pr.isb = q.isig[kb];
    pr.lim = exit_bound(thr);
    return pr;
}

}  // namespace

// ------------------------------------------------------------------ hints

// One wavefront per 64 indexed windows of a length between anchors: the
// length of a block is the last whose first hint block is at or below it
// (the bases are non-decreasing; anchors own no hint blocks).
template <typename FT>
__global__ __launch_bounds__(kWave) void k_hints(Req q) {
    const int64_t blk = blockIdx.x;
    int l = 0;
    {
        int hi = q.L - 1;
        while (l < hi) {
            const int mid = (l + hi + 1) >> 1;
            if (q.len[mid].hblk_base <= blk) l = mid; else hi = mid - 1;
        }
    }
    const LenInfo L = q.len[l];
    const int64_t k = L.kbase + (blk - L.hblk_base) * kWave + threadIdx.x;
    const bool live = !L.anchor && k < L.kbase + L.n_index;
    const int m = L.m;
    const float sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
    int64_t i = 0;
    double mua = 0.0, isa = 0.0;
    if (live) {
        i = (int64_t)q.cell[k] - L.cell_base;
        mua = q.mu[k];
        isa = q.isig[k];
    }
    uint32_t jprev = kNone;
    unsigned long long n_ver = 0;
    for (int side = 0; side < 2; ++side) {
        const int a = side ? L.a_hi : L.a_lo;
        uint32_t j = kNone, kj = kNone;
        // both sides even when the first brought the cell to 0: the second
        // partner's own cell, at this length, may still come down
        if (live && a >= 0) {
            const LenInfo A = q.len[a];
            if (i < A.W) {
                const uint32_t ka = q.kmap[A.cell_base + i];
                if (ka != kNone) j = q.hint[ka];
            }
            if (j != kNone && j != jprev && (int64_t)j < L.W) {
                const int64_t gap = (int64_t)j > i ? (int64_t)j - i : i - (int64_t)j;
                if (gap >= q.excl) kj = q.kmap[L.cell_base + j];
            }
            jprev = j;
        }
        Proposal<FT> pr;
        if (kj != kNone) pr = propose<FT>(q, (uint32_t)k, kj, (int64_t)j, sqrt2m);
        const uint64_t mask = __ballot(pr.on);
        if (mask == 0) continue;
        verify_proposals(mask, SeriesA{q.t}, q.t, i, mua, isa, pr.ib, pr.mub, pr.isb, m,
                         [&](double dd) {
                             ++n_ver;
                             lower_pair(q, (uint32_t)k, i, pr.kb, pr.ib, dd);
                         },
                         pr.lim);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) n_ver += __shfl_xor(n_ver, off, kWave);
    if (lane_id() == 0 && n_ver) atomicAdd(&q.counters[C_HINT_VER], n_ver);
}

// ------------------------------------------------------------------ sieve

// Members of the hot buckets (more than R entries) of the anchor lengths:
// cnt[b] = the bucket's size if it is hot, else 0.
__global__ __launch_bounds__(kBlock) void k_sieve_count(Req q, const uint32_t *__restrict__ bstart,
                                                        int64_t nbuckets, int R,
                                                        uint32_t *__restrict__ cnt) {
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nbuckets) return;
    int lo = 0, hi = q.L - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (q.len[mid].bucket_base <= b) lo = mid; else hi = mid - 1;
    }
    const uint32_t size = bstart[b + 1] - bstart[b];
    cnt[b] = (q.len[lo].anchor && size > (uint32_t)R) ? size : 0u;
}

// bucket of member x: the last bucket whose offset is at or below x
__device__ __forceinline__ int64_t member_bucket(const uint32_t *__restrict__ off, int64_t nbuckets,
                                                 uint32_t x) {
    int64_t lo = 0, hi = nbuckets - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sort keys of the members: the projection <g, F> (one seeded direction per
// length, FP32) as an order-preserving 32-bit pattern, the member index, and
// the member's bucket.
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_sieve_keys(Req q, const uint32_t *__restrict__ bstart,
                                                       const uint32_t *__restrict__ off,
                                                       int64_t nbuckets, uint32_t total,
                                                       const float *__restrict__ dir,
                                                       uint32_t *__restrict__ key,
                                                       uint32_t *__restrict__ val,
                                                       uint32_t *__restrict__ seg) {
    const uint32_t x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= total) return;
    const int64_t b = member_bucket(off, nbuckets, x);
    const uint32_t slot = bstart[b] + (x - off[b]);
    const uint32_t kk = q.perm[slot];
    const int l = find_len_k(q.len, q.L, kk);
    const FT *F = (const FT *)q.F + (int64_t)kk * kRec;
    const float *g = dir + l * (2 * (kMaxK - 1));
    float p = 0.0f;
#pragma unroll
    for (int c = 0; c < 2 * (kMaxK - 1); ++c) p = fmaf(g[c], (float)F[c], p);
    const uint32_t u = __float_as_uint(p);
    key[x] = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    val[x] = x;
    seg[x] = (uint32_t)b;
}

// After the sort by projection: the bucket of each sorted position, for the
// stable sort by bucket that follows.
__global__ __launch_bounds__(kBlock) void k_sieve_regroup(const uint32_t *__restrict__ val,
                                                          const uint32_t *__restrict__ seg,
                                                          uint32_t total,
                                                          uint32_t *__restrict__ key2) {
    const uint32_t y = blockIdx.x * kBlock + threadIdx.x;
    if (y < total) key2[y] = seg[val[y]];
}

// One lane per member in (bucket, projection) order: the w members after it
// in its bucket are its candidates (valid pairs only, Parseval prune first).
template <typename FT>
__global__ __launch_bounds__(kWave) void k_sieve_verify(Req q, const uint32_t *__restrict__ bstart,
                                                        const uint32_t *__restrict__ off,
                                                        const uint32_t *__restrict__ order,
                                                        const uint32_t *__restrict__ seg,
                                                        uint32_t total, int w) {
    const uint32_t y = blockIdx.x * kWave + threadIdx.x;
    const bool live = y < total;
    uint32_t ka = 0, end = 0, b = 0;
    int64_t ia = 0;
    double mua = 0.0, isa = 0.0;
    int m = 0;
    float sqrt2m = 0.0f;
    if (live) {
        const uint32_t x = order[y];
        b = seg[x];
        end = off[b] + (bstart[b + 1] - bstart[b]);
        ka = q.perm[bstart[b] + (x - off[b])];
        const int l = find_len_k(q.len, q.L, ka);
        m = q.len[l].m;
        sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
        ia = (int64_t)q.cell[ka] - q.len[l].cell_base;
        mua = q.mu[ka];
        isa = q.isig[ka];
    }
    unsigned long long n_ver = 0;
    for (int s = 1; s <= w; ++s) {
        Proposal<FT> pr;
        if (live && y + (uint32_t)s < end) {
            const uint32_t x2 = order[y + s];
            const uint32_t kb = q.perm[bstart[b] + (x2 - off[b])];
            const int64_t ib = (int64_t)q.cell[kb] - (q.cell[ka] - ia);
            const int64_t gap = ib > ia ? ib - ia : ia - ib;
            if (gap >= q.excl) pr = propose<FT>(q, ka, kb, ib, sqrt2m);
        }
        const uint64_t mask = __ballot(pr.on);
        if (mask == 0) continue;
        verify_proposals(mask, SeriesA{q.t}, q.t, ia, mua, isa, pr.ib, pr.mub, pr.isb, m,
                         [&](double dd) {
                             ++n_ver;
                             lower_pair(q, ka, ia, pr.kb, pr.ib, dd);
                         },
                         pr.lim);
    }
    for (int off2 = kWave / 2; off2 > 0; off2 >>= 1) n_ver += __shfl_xor(n_ver, off2, kWave);
    if (lane_id() == 0 && n_ver) atomicAdd(&q.counters[C_SIEVE_VER], n_ver);
}

// ------------------------------------------------------- local completion

// One block per seed; seeds[s] = indexed position of the seed cell.
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_complete(Req q, const uint32_t *__restrict__ seeds,
                                                     int dm, int dp) {
    const uint32_t ks = seeds[blockIdx.x];
    const int l0 = find_len_k(q.len, q.L, ks);
    const int m0 = q.len[l0].m;
    const int64_t i0 = (int64_t)q.cell[ks] - q.len[l0].cell_base;
    const uint32_t j0u = q.hint[ks];
    if (j0u == kNone) return;
    const int64_t j0 = (int64_t)j0u;
    // the lengths of the box: a contiguous range of length indices
    int la = l0, lb = l0;
    while (la > 0 && m0 - q.len[la - 1].m <= dm) --la;
    while (lb + 1 < q.L && q.len[lb + 1].m - m0 <= dm) ++lb;
    const int side = 2 * dp + 1;
    const int per_len = side * side;
    const int total = (lb - la + 1) * per_len;
    unsigned long long n_ver = 0, n_low = 0;
    for (int p = threadIdx.x; p < total; p += kBlock) {
        const int l = la + p / per_len;
        const int r = p % per_len;
        const LenInfo L = q.len[l];
        const int64_t i = i0 - dp + r / side, j = j0 - dp + r % side;
        if (i < 0 || j < 0 || i >= L.W || j >= L.W) continue;
        const int64_t gap = i > j ? i - j : j - i;
        if (gap < q.excl) continue;
        const uint32_t ki = q.kmap[L.cell_base + i], kj = q.kmap[L.cell_base + j];
        if (ki == kNone || kj == kNone) continue;
        const float sqrt2m = (float)sqrt(2.0 / (double)L.m) * (1.0f + 1e-7f);
        const Proposal<FT> pr = propose<FT>(q, ki, kj, j, sqrt2m);
        if (!pr.on) continue;
        const double d = snap(lane_zdist(q.t, i, q.mu[ki], q.isig[ki], j, pr.mub, pr.isb, L.m,
                                         pr.lim));
        ++n_ver;
        if (d != INFINITY && lower_pair(q, ki, i, kj, j, d)) ++n_low;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        n_ver += __shfl_xor(n_ver, off, kWave);
        n_low += __shfl_xor(n_low, off, kWave);
    }
    if (lane_id() == 0) {
        if (n_ver) atomicAdd(&q.counters[C_COMPL_VER], n_ver);
        if (n_low) atomicAdd(&q.counters[C_COMPL_IMPROVED], n_low);
    }
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_hints(int precision, const Req &q, int64_t nblocks, hipStream_t s) {
    if (nblocks <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_hints<double>, dim3((unsigned)nblocks), dim3(kWave), 0, s, q);
    else
        hipLaunchKernelGGL(k_hints<float>, dim3((unsigned)nblocks), dim3(kWave), 0, s, q);
}

void launch_sieve_count(const Req &q, const uint32_t *bstart, int64_t nbuckets, int R,
                        uint32_t *cnt, hipStream_t s) {
    if (nbuckets > 0)
        hipLaunchKernelGGL(k_sieve_count, dim3(nblk(nbuckets)), dim3(kBlock), 0, s, q, bstart,
                           nbuckets, R, cnt);
}

void launch_sieve_keys(int precision, const Req &q, const uint32_t *bstart, const uint32_t *off,
                       int64_t nbuckets, uint32_t total, const float *dir, uint32_t *key,
                       uint32_t *val, uint32_t *seg, hipStream_t s) {
    if (total == 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_sieve_keys<double>, dim3(nblk(total)), dim3(kBlock), 0, s, q, bstart,
                           off, nbuckets, total, dir, key, val, seg);
    else
        hipLaunchKernelGGL(k_sieve_keys<float>, dim3(nblk(total)), dim3(kBlock), 0, s, q, bstart,
                           off, nbuckets, total, dir, key, val, seg);
}

void launch_sieve_regroup(const uint32_t *val, const uint32_t *seg, uint32_t total, uint32_t *key2,
                          hipStream_t s) {
    if (total > 0)
        hipLaunchKernelGGL(k_sieve_regroup, dim3(nblk(total)), dim3(kBlock), 0, s, val, seg, total,
                           key2);
}

void launch_sieve_verify(int precision, const Req &q, const uint32_t *bstart, const uint32_t *off,
                         const uint32_t *order, const uint32_t *seg, uint32_t total, int w,
                         hipStream_t s) {
    if (total == 0 || w <= 0) return;
    const unsigned g = (unsigned)((total + kWave - 1) / kWave);
    if (precision == 0)
        hipLaunchKernelGGL(k_sieve_verify<double>, dim3(g), dim3(kWave), 0, s, q, bstart, off,
                           order, seg, total, w);
    else
        hipLaunchKernelGGL(k_sieve_verify<float>, dim3(g), dim3(kWave), 0, s, q, bstart, off,
                           order, seg, total, w);
}

void launch_complete(int precision, const Req &q, const uint32_t *seeds, int nseeds, int dm,
                     int dp, hipStream_t s) {
    if (nseeds <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_complete<double>, dim3((unsigned)nseeds), dim3(kBlock), 0, s, q,
                           seeds, dm, dp);
    else
        hipLaunchKernelGGL(k_complete<float>, dim3((unsigned)nseeds), dim3(kBlock), 0, s, q,
                           seeds, dm, dp);
}

}  // namespace pmp
