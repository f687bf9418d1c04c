// pmp_dev.h -- internal declarations shared by the HIP translation units of
// libpmp (not a public header).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pmp {

// ------------------------------------------------------------ constants
constexpr int    kBlock      = 256;       // threads per block (4 waves of 64)
constexpr int    kWave       = 64;
constexpr int    kMaxK       = 16;        // largest spectral width K
constexpr int    kRec        = 32;        // feature record: 30 features + e_i + |F|
constexpr int    kSlotErr    = 30;        // record slot of the error bound e_i
constexpr int    kSlotNorm   = 31;        // record slot of ||F||
constexpr int    kMaxBits    = 24;        // SimHash bits B (Sec. 4: B = 24)
constexpr int    kProbeSlots = 8;         // Hamming-1 probes kept per key word
constexpr int    kMaxM       = 2048;      // longest window supported
constexpr int    kTileW      = 1024;      // windows per sketch tile
constexpr int    kSegW       = 64;        // windows per sliding-DFT segment
constexpr int    kSegs       = kTileW / kSegW;   // 16 segments, one per 16 lanes
constexpr double kEps0       = 1e-6;      // zero snap (Sec. 3.6)
constexpr uint64_t kInfBits  = 0x7FF0000000000000ull;   // +inf as FP64 bits

// Per-length metadata, device resident.  Every per-window array is indexed
// by the compacted position k of the non-constant ("indexed") windows in
// (length, start) order; the windows of length l are k in [kbase, kbase + n_index).
struct LenInfo {
    int32_t m;            // window length
    int32_t kprime;       // K' = min(K-1, ceil(m/2)-1)
    int32_t depth;        // directory depth d (Prop. 4 final state)
    int32_t probes;       // Hamming-1 probes h = min(cap, d, 1 + max(0, d - d0))
    int64_t W;            // windows n - m + 1
    int64_t cell_base;    // first cell of this length in (length, start) order
    int64_t kbase;        // first indexed position of this length
    int64_t bucket_base;  // first bucket of this length
    int64_t n_index;      // non-constant windows (entries of the directory)
    int64_t tile_base;    // first sketch tile of this length
    int64_t blk_base;     // first block of this length in k_keys (anchors own blocks)
    // anchor lengths (Sec. 3.3): the one pass probes only these.  pblk_base
    // is non-decreasing over the lengths: an anchor owns probe blocks
    // [pblk_base, pblk_base + ceil(n_index / 64)), a non-anchor none.
    // Likewise hblk_base for the hint blocks of the non-anchor lengths.
    int32_t anchor;       // 1: an anchor length
    int32_t a_lo, a_hi;   // a non-anchor's nearest anchors below and above
                          // (indices; -1: none)
    int32_t pad_;
    int64_t pblk_base;    // first probe block of this length
    int64_t hblk_base;    // first hint block of this length
    // Keys and buckets exist at the anchor lengths only (nothing else reads
    // them): a non-anchor has depth 0 and no k_keys blocks, and an anchor's
    // sort entries sit at [abase, abase + n_index) of the anchor windows
    int64_t abase;        // first slot of this length among the anchor windows
};

// Everything a kernel needs to know about one request.
struct Req {
    const double *t;       // series
    int64_t n;
    int32_t L;             // number of lengths
    int32_t K;             // spectral width
    int32_t B;             // signature bits
    int32_t excl;          // exclusion zone
    int32_t budget_R;      // inspections per query (R = gamma * alpha)
    int32_t key_shift;     // bucket key: len_idx << key_shift | prefix << (key_shift - d)
    int32_t jkey_shift;    // join key: len_idx << jkey_shift | quantized p1
    int32_t precision;
    const LenInfo *len;    // [L]
    // per indexed window k, in (length, start) order
    uint32_t *cell;        // [N] cell id (cell_base of its length + start)
    double  *mu;           // [N] window mean
    double  *isig;         // [N] 1 / sigma (population standard deviation)
    uint64_t *P;           // [N] profile, FP64 bits (atomicMin)
    void    *F;            // [N][kRec] features (float or double)
    uint64_t *keyw;        // [N] key word: signature | probe order << 24
    uint4   *jop;          // [N][8] join operands: 32 bf16 hi, then 32 bf16 lo (G = hi + lo)
    float4  *jmeta;        // [N] |G|^2, e' >= |G - F|, bound on |G|, 0
    float4  *gp;           // [N] principal coordinates of the FP32 feature copy, and
                           //     0.5 |G|^2 (rounded down) with the sign bit = (P != 0)
    const double *udir;    // [L][kJoinDirs][32] principal directions (null: none)
    // bucket order (slots)
    uint32_t *skey;        // [N] sort keys
    uint32_t *sval;        // [N] sort values (k)
    uint32_t *perm;        // [N] slot -> k
    uint32_t *pcell;       // [N] slot -> cell
    const float *gproj;    // [L][B][30] SimHash projections
    uint32_t *kmap;        // [cells] cell -> indexed position k (kNone: constant);
                           // written by the sketch when not null
    uint32_t *hint;        // [N] start of a partner that lowered the cell
                           // (kNone: none), written when a cell is lowered
    float   *emax;         // [L] largest e_i of each length
    unsigned long long *counters;   // stats counters
    int     *bad;          // raised on inputs the library cannot represent
};

enum Counter {
    C_PASS_CAND = 0, C_PASS_VER, C_JOIN_CAND, C_JOIN_VER, C_HOT, C_JOIN_PAIRS,
    C_SIEVE_VER, C_HINT_VER, C_COMPL_VER, C_COMPL_IMPROVED, C_NCOUNTERS
};

constexpr uint32_t kNone = 0xFFFFFFFFu;      // no entry (kmap, hint)

// ------------------------------------------------------------- helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Snapped distance (Sec. 3.6: values below eps0 are reported as 0).
__device__ __forceinline__ double snap(double d) { return d < kEps0 ? 0.0 : d; }

__device__ __forceinline__ uint64_t dbits(double d) {
    return (uint64_t)__double_as_longlong(d);
}
__device__ __forceinline__ double bitsd(uint64_t b) {
    return __longlong_as_double((long long)b);
}

// Length index of a cell (binary search over cell_base, L is small).
__device__ __forceinline__ int find_len(const LenInfo *len, int L, int64_t cell) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (len[mid].cell_base <= cell) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Length index of an indexed position k (slots share the per-length ranges).
__device__ __forceinline__ int find_len_k(const LenInfo *len, int L, int64_t k) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (len[mid].kbase <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int kJoinTile = 32;             // windows per threshold-join tile
constexpr int kJoinBlock = 4;             // join tiles per block (they share candidate tiles)
constexpr int kJoinDirs = 3;              // principal directions per length in the join
constexpr int kJoinNb = 1;                // join grid cells are 1/kJoinNb of the radius wide; a
                                          // pair within it lies at most kJoinNb cells apart

// Per length, one round of the threshold join (k_join.hip).
struct GridLen {
    int64_t blk_base;     // first join block (kJoinBlock tiles) of this length
    double qlo;           // grid origin of both coordinates
    double hinv;          // 1 / cell width of the first coordinate (0: one cell)
    double hinv2;         // 1 / cell width of the second and third coordinates
    double R2;            // squared radius on the join vectors G (+inf: every pair)
    double eps_c;         // MFMA dot-product error per unit |G_q| (times the largest |G_c|)
    double nmax2;         // square of the largest |G|
    float sqrt2m;         // sqrt(2/m) (1 + 1e-7)
    float rp;             // bound on any coordinate difference of a pair within R_f
};

// State of the device-side radix select (k_certify.hip).
constexpr int kSelBins = 2048;            // bins of one select pass (11 bits)
struct SelState {
    uint64_t high;        // bits of the selected prefix so far
    uint64_t pivot;       // FP64 bits of the boundary value (kInfBits: take all)
    int64_t remaining;    // values still wanted at or below the prefix
    int64_t need_eq;      // values equal to the pivot to take, in cell order
    uint32_t nless;       // values below the pivot found by the emit pass
    int32_t done;         // the pivot is known
};

struct RowReq {
    int32_t l;          // length index
    int32_t pad;
    int64_t k;          // indexed position of the cell
    uint64_t target;    // pass 2: FP64 bits of the value whose smallest j is wanted
};

// The canonical exact distance, computed by a group of kGroup consecutive
// lanes (kPerRound groups per wavefront, each with its own pair): lane g of
// the group sums the terms r = g, g + kGroup, ... in ascending order, then a
// butterfly over the group adds the partial sums.  Every kernel that writes,
// compares or reports a distance calls this function, so they all agree bit
// for bit; every step is symmetric in (a, b), so d(a, b) == d(b, a).  Loads
// of a group are contiguous.  All 64 lanes of the wavefront must call it.
constexpr int kGroup = 8;                 // lanes per exact distance
constexpr int kPerRound = kWave / kGroup; // distances per wavefront round
constexpr int kZBatch = 8;                // terms per lane loaded together
constexpr int kLaneMode = 32;             // proposals from which each lane takes its own,
constexpr int kLaneModeMaxM = 100;        // for windows up to this length: longer ones
                                          // read better in groups (contiguous loads);
                                          // measured crossover between 100 and 124

// The first window's samples are read through an accessor: the series
// itself, or a copy of the same samples staged in LDS; the second window's
// come from the series.
struct SeriesA {
    const double *t;
    __device__ __forceinline__ double operator()(int64_t x) const { return t[x]; }
};

template <int kB = kZBatch, class A>
__device__ __forceinline__ double group_zdist_a(A qa, const double *__restrict__ t, int64_t a,
                                                double mua, double ia, int64_t b, double mub,
                                                double ib, int m, double lim2 = INFINITY) {
#pragma clang fp contract(off)
    double acc = 0.0;
    // kB terms per lane are loaded before they are summed (in order), so that
    // a window of up to kB * kGroup samples costs one memory latency (kB = 1:
    // the fewest registers; the sum and its order are the same for any kB)
    for (int r0 = lane_id() & (kGroup - 1); r0 < m; r0 += kB * kGroup) {
        double xa[kB], xb[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int r = r0 + u * kGroup;
            xa[u] = r < m ? qa(a + r) : 0.0;
            xb[u] = r < m ? t[b + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (r0 + u * kGroup < m) {
                const double za = (xa[u] - mua) * ia;
                const double zb = (xb[u] - mub) * ib;
                const double e = za - zb;
                acc = fma(e, e, acc);
            }
        }
        // early exit: the partial sums only grow (every term is >= 0 and
        // rounding is monotone), so once their total reaches lim2 the
        // finished sum would too; the group decides together (all its lanes
        // compute the same total)
        if (lim2 != INFINITY && (r0 | (kGroup - 1)) + 1 + (kB - 1) * kGroup < m) {
            double sp = acc;
#pragma unroll
            for (int off = 1; off < kGroup; off <<= 1) sp += __shfl_xor(sp, off, kGroup);
            if (sp >= lim2) return INFINITY;
        }
    }
#pragma unroll
    for (int off = 1; off < kGroup; off <<= 1) acc += __shfl_xor(acc, off, kGroup);
    return sqrt(acc);
}
__device__ __forceinline__ double group_zdist(const double *__restrict__ t, int64_t a, double mua,
                                              double ia, int64_t b, double mub, double ib, int m,
                                              double lim2 = INFINITY) {
    return group_zdist_a(SeriesA{t}, t, a, mua, ia, b, mub, ib, m, lim2);
}

// The same canonical distance evaluated by one lane alone, bit for bit: the
// kGroup partial sums of group_zdist become kGroup accumulators of the lane
// (accumulator g takes the terms r = g, g + kGroup, ... in ascending order),
// combined in the order of group_zdist's butterfly.  Used when most lanes of a
// wavefront have a pair of their own, where it avoids the group's shuffles.
static_assert(kGroup == 8, "lane_zdist combines eight partial sums");
__device__ __forceinline__ double butterfly8(const double *p) {
    return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}
template <class A>
__device__ __forceinline__ double lane_zdist_a(A qa, const double *__restrict__ t, int64_t a,
                                               double mua, double ia, int64_t b, double mub,
                                               double ib, int m, double lim2 = INFINITY) {
#pragma clang fp contract(off)
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
    for (int r0 = 0; r0 < m; r0 += kGroup) {
        double xa[kGroup], xb[kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            xa[g] = r0 + g < m ? qa(a + r0 + g) : 0.0;
            xb[g] = r0 + g < m ? t[b + r0 + g] : 0.0;
        }
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            if (r0 + g < m) {
                const double za = (xa[g] - mua) * ia;
                const double zb = (xb[g] - mub) * ib;
                const double e = za - zb;
                acc[g] = fma(e, e, acc[g]);
            }
        }
        // early exit as in group_zdist (any partial total is a lower bound
        // of the finished sum), tested every kZBatch terms per accumulator
        if (lim2 != INFINITY && ((r0 / kGroup) % kZBatch) == kZBatch - 1 && r0 + kGroup < m &&
            butterfly8(acc) >= lim2)
            return INFINITY;
    }
    return sqrt(butterfly8(acc));
}
__device__ __forceinline__ double lane_zdist(const double *__restrict__ t, int64_t a, double mua,
                                             double ia, int64_t b, double mub, double ib, int m,
                                             double lim2 = INFINITY) {
    return lane_zdist_a(SeriesA{t}, t, a, mua, ia, b, mub, ib, m, lim2);
}

// Squared bound for group_zdist's early exit: a sum that reaches it has a
// computed root >= thr (the factor covers the roundings of thr^2 and sqrt).
__device__ __forceinline__ double exit_bound(double thr) {
    return thr == INFINITY ? INFINITY : thr * thr * (1.0 + 8.0 * 1.1102230246251565e-16);
}

// Length index of the indexed positions handled by a wavefront: a scalar
// binary search for the wavefront's first position (uniform, so it runs on
// the scalar unit), then a short per-lane step forward.
__device__ __forceinline__ int find_len_k_wave(const LenInfo *len, int L, int64_t k_first,
                                               int64_t k) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (len[mid].kbase <= k_first) lo = mid; else hi = mid - 1;
    }
    while (lo + 1 < L && len[lo + 1].kbase <= k) ++lo;
    return lo;
}

// Canonical moments of one window x[0..m) (Sec. 3.2: population, two
// passes): returns sigma and sets mu.  Four partial sums in a fixed order
// keep the loads independent; every caller gets the same bits for the same
// samples, which the distances below depend on.
__device__ __forceinline__ double window_moments(const double *x, int m, double &mu) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int r = 0;
    for (; r + 4 <= m; r += 4) {
        a0 += x[r];
        a1 += x[r + 1];
        a2 += x[r + 2];
        a3 += x[r + 3];
    }
    for (; r < m; ++r) a0 += x[r];
    mu = ((a0 + a1) + (a2 + a3)) / (double)m;
    a0 = a1 = a2 = a3 = 0.0;
    for (r = 0; r + 4 <= m; r += 4) {
        const double c0 = x[r] - mu, c1 = x[r + 1] - mu;
        const double c2 = x[r + 2] - mu, c3 = x[r + 3] - mu;
        a0 = fma(c0, c0, a0);
        a1 = fma(c1, c1, a1);
        a2 = fma(c2, c2, a2);
        a3 = fma(c3, c3, a3);
    }
    for (; r < m; ++r) {
        const double c0 = x[r] - mu;
        a0 = fma(c0, c0, a0);
    }
    return sqrt(((a0 + a1) + (a2 + a3)) / (double)m);
}

// Certified lower bound on d_m(q, c) from two stored feature records: the
// Parseval bound (Lemma 2) of the true features is at least
//   sqrt(2/m) (||F~q - F~c|| - e_q - e_c),
// and every rounding of this evaluation is absorbed by the relative slacks
// (applied to the norm before the subtraction, so the result never exceeds
// the true bound even when the two terms nearly cancel).  All 30 slots are
// used: slots beyond 2K' are zero on both sides and add nothing.
template <typename FT>
__device__ __forceinline__ float lb_mem(const FT *__restrict__ fq, const FT *__restrict__ fc,
                                        float sqrt2m) {
    FT acc = 0;
    if (sizeof(FT) == 8) {
        const double2 *a = (const double2 *)fq;
        const double2 *b = (const double2 *)fc;
#pragma unroll
        for (int x = 0; x < kMaxK - 1; ++x) {
            const double2 u = a[x], v = b[x];
            const double e0 = u.x - v.x, e1 = u.y - v.y;
            acc = fma(e0, e0, acc);
            acc = fma(e1, e1, acc);
        }
    } else {
        const float4 *a = (const float4 *)fq;
        const float4 *b = (const float4 *)fc;
#pragma unroll
        for (int x = 0; x < 7; ++x) {
            const float4 u = a[x], v = b[x];
            const float e0 = u.x - v.x, e1 = u.y - v.y, e2 = u.z - v.z, e3 = u.w - v.w;
            acc = fmaf(e0, e0, acc);
            acc = fmaf(e1, e1, acc);
            acc = fmaf(e2, e2, acc);
            acc = fmaf(e3, e3, acc);
        }
        const float2 u = ((const float2 *)fq)[14], v = ((const float2 *)fc)[14];
        const float e0 = u.x - v.x, e1 = u.y - v.y;
        acc = fmaf(e0, e0, acc);
        acc = fmaf(e1, e1, acc);
    }
    const FT nd = sqrt(acc);
    const FT es = fq[kSlotErr] + fc[kSlotErr];
    if (sizeof(FT) == 4) {
        float v = (float)nd * (1.0f - 1e-5f) - (float)es * (1.0f + 1e-5f);
        return v > 0.0f ? v * sqrt2m * (1.0f - 1e-6f) : 0.0f;
    } else {
        double v = (double)nd * (1.0 - 1e-12) - (double)es * (1.0 + 1e-12);
        return v > 0.0 ? __double2float_rd(v * (double)sqrt2m * (1.0 - 1e-6)) : 0.0f;
    }
}

// Verification of the proposals of a wavefront.  Every lane whose bit is set
// in `mask` has a proposal (a, b: window starts; mua, ia, mub, ib: moments;
// m; lim2: the squared distance at or above which the result is of no use,
// see exit_bound).  With at least kLaneMode proposals of windows up to
// kLaneModeMaxM samples (the length of the first proposal decides for the
// wavefront) every proposing lane evaluates its own (lane_zdist); otherwise
// they are taken kPerRound at a time,
// one per group of kGroup lanes (group_zdist).  Both give the same bits.
// `on_result(d)` runs on the proposing lane with its snapped distance (+inf
// when the sum stopped early).
template <bool kLaneForm = true, int kB = kZBatch, class A, typename F>
__device__ __forceinline__ void verify_proposals(uint64_t mask, A qa, const double *__restrict__ t,
                                                 int64_t a, double mua, double ia, int64_t b,
                                                 double mub, double ib, int m, F &&on_result,
                                                 double lim2 = INFINITY) {
    const int lane = lane_id();
    if (kLaneForm && __popcll(mask) >= kLaneMode &&
        __shfl(m, __ffsll((unsigned long long)mask) - 1, kWave) <= kLaneModeMaxM) {
        // most lanes propose short windows: each evaluates its own pair
        if ((mask >> lane) & 1ull)
            on_result(snap(lane_zdist_a(qa, t, a, mua, ia, b, mub, ib, m, lim2)));
        return;
    }
    const int grp = lane / kGroup;
    while (mask) {
        // the next kPerRound proposing lanes, in lane order
        int src[kPerRound];
        int cnt = 0;
#pragma unroll
        for (int g = 0; g < kPerRound; ++g) {
            src[g] = -1;
            if (mask) {
                src[g] = __ffsll((unsigned long long)mask) - 1;
                mask &= mask - 1;
                ++cnt;
            }
        }
        int mys = src[0];
#pragma unroll
        for (int g = 1; g < kPerRound; ++g)
            if (grp == g && src[g] >= 0) mys = src[g];
        const bool live = grp == 0 || (grp < cnt);
        const int my = mys;
        const int64_t ga = __shfl(a, my, kWave);
        const int64_t gb = __shfl(b, my, kWave);
        const double gmua = __shfl(mua, my, kWave), gia = __shfl(ia, my, kWave);
        const double gmub = __shfl(mub, my, kWave), gib = __shfl(ib, my, kWave);
        const double glim = __shfl(lim2, my, kWave);
        int gm = __shfl(m, my, kWave);
        if (!live) gm = 0;
        const double d = snap(group_zdist_a<kB>(qa, t, ga, gmua, gia, gb, gmub, gib, gm, glim));
        // hand each result back to its proposing lane
#pragma unroll
        for (int g = 0; g < kPerRound; ++g) {
            const double dg = __shfl(d, g * kGroup, kWave);
            if (g < cnt && lane == src[g]) on_result(dg);
        }
    }
}

// ------------------------------------------------------------- stream

// One anchor length of a stream session, as the kernels of one batch see it
// (Sec. 3.1, 3.5, Algorithm 1).  Cells of the anchor are its window starts
// q at cbase + q.  The directory is the anchor's indexed windows in
// arrival order, cut into sorted runs: run r holds the indexed positions
// [runs[r], runs[r + 1]), sorted by (SimHash key, start).
constexpr int kStreamMaxRuns = 48;
struct SAnchor {
    int32_t m, kprime;
    int64_t cbase;        // first cell
    int64_t bbase;        // offset of the basis table (2 K' rows of m doubles)
    int32_t nidx;         // indexed windows before this batch
    int32_t nnew;         // indexed windows this batch completes
    int32_t j0;           // first entry of the batch list that is this anchor's
    int32_t depth;        // directory depth d (Prop. 4)
    int32_t probes;       // Hamming-1 probes h
    int32_t nruns;
    uint32_t runs[kStreamMaxRuns + 1];
};

// A candidate endpoint's improvement, merged after the batch's searches.
struct SUpdate {
    uint32_t cell;
    int32_t j;            // the query start that reached it
    uint64_t d;           // FP64 bits of the distance
};

// One merge of the newest runs of one anchor into a single run.
struct SMerge {
    int64_t cbase;
    int64_t first;        // first thread of this merge in the launch
    int32_t nruns;        // runs merged
    int32_t pad_;
    uint32_t runs[kStreamMaxRuns + 1];
};

// Kernel arguments of a stream batch.
struct StreamDev {
    const double *t;      // resident series
    double *F;            // [cells][kRec] records
    double *mu, *isig;    // [cells]
    uint64_t *P;          // [cells] upper profile (FP64 bits; +inf: none)
    int32_t *I;           // [cells] its neighbour (-1: none)
    int32_t *Icand;       // [cells] merge scratch
    uint32_t *perm, *skey;   // [cells] directory runs (start, key) by position
    uint32_t *ptmp, *ktmp;   // [cells] merge scratch
    const double *basis;
    const float *gproj;   // [anchor][kMaxBits][30] SimHash projections
    const SAnchor *anc;
    const int32_t *la, *lq;  // batch list: anchor, start
    int32_t nlist;
    int32_t B;            // signature bits
    int32_t R;            // budget per query (gamma alpha)
    int32_t excl;
    uint32_t *bkey;       // [list] SimHash key
    float *bmarg;         // [list][kMaxBits] projection margins
    SUpdate *upd;
    uint32_t *nupd;
    uint32_t updcap;
    unsigned long long *counters;   // kStreamCounters
};
enum { CS_CAND = 0, CS_VER, CS_UPD, CS_DROP, kStreamCounters };

// --------------------------------------------------- host-side launchers
// (k_scan.hip)
size_t scan_temp_bytes(int64_t n);
// out[i] = sum_{j<i} in[j]; total (optional, device) = sum of all.
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                        void *temp, hipStream_t s);
size_t sort_temp_bytes(int64_t n);
// Stable LSD radix sort of (key, val) pairs on key bits [lo, hi).  Result in
// (k0, v0), or, after an odd number of passes with copy_back false, in
// (k1, v1): the return value is 1 then, 0 otherwise.  (k1, v1) are scratch
// of the same size.
int radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                     int lo, int hi, void *temp, hipStream_t s, bool copy_back = true);

// (k_sketch.hip)
void launch_changepoints(const double *t, int64_t n, uint32_t *flag, int *bad, hipStream_t s);
void launch_tile_counts(const LenInfo *len, int L, const uint32_t *E, int64_t ntiles,
                        uint32_t *tile_cnt, hipStream_t s);
// Which tiles of [0, ntiles) the sketch gives records: every length
// (kSketchAll), the anchor lengths only, the moments and positions of every
// tile still written (kSketchAnchors), or the lengths between anchors, whose
// moments and positions a kSketchAnchors pass already wrote (kSketchBetween;
// it re-writes them with the same values and resets their cells to +inf, so
// it runs before anything lowers a cell of those lengths)
enum { kSketchAll = 0, kSketchAnchors = 1, kSketchBetween = 2 };
void launch_sketch(int precision, const Req &q, const uint32_t *E, const uint32_t *tile_off,
                   int64_t ntiles, int max_m, int mode, hipStream_t s);
void launch_keys(int precision, const Req &q, int64_t nblocks, hipStream_t s);
void launch_join_ops(int precision, const Req &q, int64_t k0, int64_t k1, hipStream_t s);
int64_t basis_elems(const LenInfo *len_host, int L, std::vector<int64_t> &base);
void launch_basis(const LenInfo *len, int L, const int64_t *base, uint16_t *bh, uint16_t *bm,
                  uint16_t *bl, int max_m, hipStream_t s);
void launch_sketch_mfma(int precision, const Req &q, const uint32_t *E, const uint32_t *tile_off,
                        int64_t ntiles, int max_m, const int64_t *bbase, const uint16_t *bh,
                        const uint16_t *bm, const uint16_t *bl, int mode, hipStream_t s);
void launch_bucket_bounds(const Req &q, int64_t N, int64_t nbuckets, uint32_t *bstart,
                          hipStream_t s);
// (k_probe.hip)
// one wavefront per 64 indexed windows of each anchor length (LenInfo.pblk_base):
// the probe blocks [blk0, blk0 + nblocks)
void launch_probe(int precision, const Req &q, const uint32_t *bstart, int64_t blk0,
                  int64_t nblocks, int max_m, hipStream_t s);
void launch_hot_buckets(const uint32_t *bstart, int64_t nb, int R, unsigned long long *cnt,
                        hipStream_t s);
// (k_complete.hip): the emit stage
// the hints: one wavefront per 64 indexed windows of each length between
// anchors (LenInfo.hblk_base)
void launch_hints(int precision, const Req &q, int64_t nblocks, hipStream_t s);
void launch_sieve_count(const Req &q, const uint32_t *bstart, int64_t nbuckets, int R,
                        uint32_t *cnt, hipStream_t s);
void launch_sieve_keys(int precision, const Req &q, const uint32_t *bstart, const uint32_t *off,
                       int64_t nbuckets, uint32_t total, const float *dir, uint32_t *key,
                       uint32_t *val, uint32_t *seg, hipStream_t s);
void launch_sieve_regroup(const uint32_t *val, const uint32_t *seg, uint32_t total, uint32_t *key2,
                          hipStream_t s);
void launch_sieve_verify(int precision, const Req &q, const uint32_t *bstart, const uint32_t *off,
                         const uint32_t *order, const uint32_t *seg, uint32_t total, int w,
                         hipStream_t s);
void launch_complete(int precision, const Req &q, const uint32_t *seeds, int nseeds, int dm,
                     int dp, hipStream_t s);
// (k_certify.hip)
int64_t select_blocks(int64_t n);
// The first `need` values of P in (value, position) order: positions below the
// pivot go to less (unordered, with their values in less_val), positions
// equal to it to eq (position order); less_cell / eq_cell hold cell[position].
// Everything runs on the stream; st holds the counts when the stream reaches
// the end.
void launch_select(const uint64_t *P, int64_t n, int64_t need, SelState *st,
                   unsigned int *hist, uint32_t *cnt, uint32_t *scan_tmp, uint32_t *less,
                   uint64_t *less_val, uint32_t *eq, uint32_t *less_cell, uint32_t *eq_cell,
                   const uint32_t *cell, hipStream_t s);
// (k_join.hip)
size_t join_cov_doubles(int L);
// principal directions: covariance of a sample, then power iteration (GPU)
// principal directions of the lengths [0, nlen) (the lengths whose records
// exist)
void launch_join_dirs(int precision, const Req &q, int nlen, double *cov, double *udir,
                      hipStream_t s);
// grid keys over cb1 (and cb2, cb3 when nonzero) bits of the principal
// coordinates, of the first N indexed windows; queries are the cells not at 0
// with (length, start) <= (l_lim, i_lim)
void launch_grid_keys(const Req &q, const GridLen *gl, int64_t N, int cb1, int cb2, int cb3,
                      int l_lim, int64_t i_lim, uint32_t *gkey, uint32_t *gval, uint8_t *qf,
                      float4 *gp, hipStream_t s);
// the join operands and coordinates of the first n sorted positions, in
// sorted order
void launch_join_gather(const uint32_t *gval, const uint4 *jop, const float4 *gp, int64_t n,
                        uint4 *jop_s, float4 *gp_s, hipStream_t s);
// one block of kJoinBlock query tiles per GridLen block: the blocks
// [blk0, blk0 + nblocks) of the round; kept pairs go to `pairs` (capacity
// cap, fill count *pcount), or are verified in place once it is full
void launch_join_tiles(int precision, const Req &q, const GridLen *gl, const uint32_t *gkey,
                       const uint32_t *gval, const uint8_t *qf, const uint4 *jop_s,
                       const float4 *jmeta, const float4 *gp_s, int64_t blk0, int64_t nblocks,
                       int cb1, int cb2, int cb3, double T, uint2 *pairs,
                       unsigned long long *pcount, int64_t cap, hipStream_t s);
// the exact stage of the first min(*pcount, cap) pairs of the buffer
void launch_join_verify(int precision, const Req &q, const GridLen *gl, const uint2 *pairs,
                        const unsigned long long *pcount, int64_t cap, double T, hipStream_t s);
void launch_rows(const Req &q, const RowReq *rr, int nrows, int64_t maxN,
                 unsigned long long *out_min, unsigned long long *out_arg, hipStream_t s);
void launch_stream_basis(const SAnchor *anc, int na, int64_t elems, double *basis,
                         hipStream_t s);
void launch_stream_windows(const StreamDev &S, int max_m, hipStream_t s);
void launch_stream_probe(const StreamDev &S, hipStream_t s);
void launch_stream_apply(const StreamDev &S, hipStream_t s);
void launch_stream_newruns(const StreamDev &S, int na, hipStream_t s);
void launch_stream_merge(const StreamDev &S, const SMerge *mg, int nmerge, int64_t nthreads,
                         hipStream_t s);
void launch_iota_u32(uint32_t *p, int64_t n, hipStream_t s);
void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
// *out += the number of zeros among P[0 .. n)
void launch_count_zero(const uint64_t *P, int64_t n, unsigned long long *out, hipStream_t s);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void launch_gather_u32(const uint32_t *src, const uint32_t *idx, int64_t n, uint32_t *out,
                       hipStream_t s);

}  // namespace pmp
