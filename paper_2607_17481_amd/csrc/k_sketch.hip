// k_sketch.hip -- moments, normalized spectral features and SimHash keys.
//
// Paper Sec. 3.2: the retained feature of window (i, m) is
//   F_{i,m} = (X_1 .. X_{K'}) / sigma,  X_k = sum_r t_{i+r} e^{-2 pi i k r / m},
// K' = min(K-1, ceil(m/2)-1), zero-padded to K-1 bins; by Lemma 1 it equals the
// leading non-DC bins of the DFT of the z-normalized window.  The paper keeps
// one sliding state per length and updates it in O(K) per slide
//   X_{i+1,k} = e^{2 pi i k / m} (X_{i,k} - t_i + t_{i+m}),
// recomputing from the raw samples every 4096 slides.  On the GPU each block
// takes a tile of 1024 consecutive windows of one length, staged in LDS; the
// tile is split into 16 segments of 64 windows, and thread (segment, bin)
// computes its bin directly at the segment start and slides it 63 times, in
// FP64.  Samples are shifted by a per-segment constant c first, which leaves
// every bin k >= 1 unchanged (Lemma 1) and keeps the magnitudes small.
//
// Each window also gets a rigorous bound e_i >= ||F~_i - F_i|| on the error of
// its stored features (computation in FP64 + rounding to the storage type),
// so that the Parseval bound can be shrunk into a true lower bound at every
// magnitude (replacing the paper's relative (1 - lambda) shrink, Lemma 4,
// which it proves only above a threshold).
//
// One pass writes, for every non-constant window k (compacted, in (length,
// start) order): its cell, moments, feature record, key word (signature +
// Hamming-1 probe order), join record and bucket sort key.  Records are
// staged in LDS and leave in whole, coalesced rows.
#include "pmp_dev.h"

namespace pmp {

// ------------------------------------------------------- change points

// flag[r] = [t_r != t_{r-1}] for 1 <= r < n; flag[0] = flag[n] = 0.  Also
// raises *bad if any sample is not finite.
__global__ __launch_bounds__(kBlock) void k_changepoints(const double *__restrict__ t, int64_t n,
                                                         uint32_t *__restrict__ flag,
                                                         int *__restrict__ bad) {
    int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r > n) return;
    uint32_t f = 0;
    if (r < n) {
        double x = t[r];
        if (!isfinite(x)) atomicOr(bad, 1);
        if (r > 0 && x != t[r - 1]) f = 1;
    }
    flag[r] = f;
}

namespace {

__device__ __forceinline__ int find_tile_len(const LenInfo *len, int L, int64_t tile) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (len[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace

// Non-constant windows per tile: window [i, i+m) is constant iff no change
// point lies in (i, i+m), i.e. E[i+m] == E[i+1] for the exclusive prefix E.
__global__ __launch_bounds__(kBlock) void k_tile_counts(const LenInfo *__restrict__ len, int L,
                                                        const uint32_t *__restrict__ E,
                                                        uint32_t *__restrict__ tile_cnt) {
    __shared__ uint32_t ws[kBlock / kWave];
    const int64_t tile = blockIdx.x;
    const int l = find_tile_len(len, L, tile);
    const int m = len[l].m;
    const int64_t i0 = (tile - len[l].tile_base) * kTileW;
    const int nw = (int)min<int64_t>(kTileW, len[l].W - i0);
    uint32_t c = 0;
    for (int w = threadIdx.x; w < nw; w += kBlock) c += E[i0 + w + m] != E[i0 + w + 1];
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (lane_id() == 0) ws[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) tile_cnt[tile] = ws[0] + ws[1] + ws[2] + ws[3];
}

// ---------------------------------------------------------------- sketch

namespace {

constexpr int kFD = 2 * (kMaxK - 1);          // 30 feature reals
constexpr int kRowsC = 128;                   // staged windows per chunk
constexpr int kSlidesC = kRowsC / kSegs;      // slides per segment per chunk (8)
constexpr int kStageLd = 31;                  // doubles per staged row (odd: the
                                              // row threads' 8-byte reads spread
                                              // over all banks)

struct SketchSmem {
    int32_t kpos[kTileW];                     // indexed position, -1: constant window
    float ymax[kSegs];                        // largest |t - c| of each segment
    uint32_t wsum[kBlock / kWave];
    int emax;
};

// Post-processing of one indexed window (one thread): two-pass moments, the
// normalized features F = X / sigma written to the record, SimHash bits and
// the Hamming-1 probe order (Sec. 3.4), the join projections, and the
// error bound e_i of the stored features.
template <typename FT>
__device__ __forceinline__ void sketch_row(const Req &q, const LenInfo &L, int l, int64_t cell,
                                           const double *__restrict__ x, int rot,
                                           const double *__restrict__ X, float Ymax, int kk,
                                           const float *__restrict__ gl,
                                           const double *__restrict__ uj, float &emax) {
    const int m = L.m;
    // ---- moments, two passes (Sec. 3.2); each sum starts at sample `rot`
    // and wraps around, so that the row groups of a wavefront, whose windows
    // lie 64 apart, read different LDS banks
    double a0 = 0.0, a1 = 0.0;
    {
        int r = rot;
        for (int j = 0; j < m; ++j) {
            if (j & 1) a1 += x[r]; else a0 += x[r];
            r = r + 1 == m ? 0 : r + 1;
        }
    }
    const double mu = (a0 + a1) / (double)m;
    a0 = 0.0;
    a1 = 0.0;
    {
        int r = rot;
        for (int j = 0; j < m; ++j) {
            const double c = x[r] - mu;
            if (j & 1) a1 = fma(c, c, a1); else a0 = fma(c, c, a0);
            r = r + 1 == m ? 0 : r + 1;
        }
    }
    const double sg = sqrt((a0 + a1) / (double)m);
    double is = 1.0 / sg;
    if (!(sg > 0.0) || !isfinite(sg) || !(is > 0.0) || !isfinite(is)) {
        // samples differ but sigma underflows or overflows: outside the
        // range the library represents; the window stays indexed so every
        // count stays consistent, and the call fails
        atomicOr(q.bad, 2);
        is = 1.0;
    }
    q.cell[kk] = (uint32_t)cell;
    q.mu[kk] = mu;
    q.isig[kk] = is;
    q.P[kk] = kInfBits;

    // ---- features: scale, store, keep an FP32 copy
    FT *rec = (FT *)q.F + (int64_t)kk * kRec;
    float f[kFD];
    double n2 = 0.0;
#pragma unroll
    for (int p = 0; p < kFD / 2; ++p) {
        const double vr = X[2 * p] * is, vi = X[2 * p + 1] * is;
        f[2 * p] = (float)vr;
        f[2 * p + 1] = (float)vi;
        if (sizeof(FT) == 8) {
            double2 v;
            v.x = vr;
            v.y = vi;
            *(double2 *)(rec + 2 * p) = v;
        }
    }
    if (sizeof(FT) == 4) {
#pragma unroll
        for (int p = 0; p < 7; ++p)
            *(float4 *)(rec + 4 * p) = make_float4(f[4 * p], f[4 * p + 1], f[4 * p + 2], f[4 * p + 3]);
    }
#pragma unroll
    for (int x2 = 0; x2 < kFD; ++x2) n2 = fma((double)f[x2], (double)f[x2], n2);

    // ---- SimHash bits: bit b = [<g_b, F> >= 0], most significant first
    uint32_t sig = 0;
    uint32_t key[kMaxBits];
#pragma unroll
    for (int bt = 0; bt < kMaxBits; ++bt) {
        key[bt] = 0xFFFFFFFFu;
        if (bt < q.B) {
            float dot = 0.0f;
#pragma unroll
            for (int c = 0; c < kFD; ++c) dot = fmaf(gl[bt * kFD + c], f[c], dot);
            if (dot >= 0.0f) sig |= 1u << (q.B - 1 - bt);
            // probe key: the margin |dot| (its order is the order of the
            // bit patterns) with the bit index in the low five bits
            if (bt < L.depth) key[bt] = (__float_as_uint(fabsf(dot)) & ~31u) | (uint32_t)bt;
        }
    }
    // ---- Hamming-1 probe order: the `probes` smallest margins among the
    // d prefix bits, ascending (Sec. 3.4 multi-probe)
    uint64_t order = 0;
    for (int h = 0; h < L.probes; ++h) {
        uint32_t mn = key[0];
#pragma unroll
        for (int bt = 1; bt < kMaxBits; ++bt) mn = min(mn, key[bt]);
        order |= (uint64_t)(mn & 31u) << (5 * h);
#pragma unroll
        for (int bt = 0; bt < kMaxBits; ++bt) key[bt] = key[bt] == mn ? 0xFFFFFFFFu : key[bt];
    }
    q.keyw[kk] = (uint64_t)sig | (order << 24);
    const uint32_t prefix = L.depth ? sig >> (q.B - L.depth) : 0u;
    q.skey[kk] = ((uint32_t)l << q.key_shift) | (prefix << (q.key_shift - L.depth));
    q.sval[kk] = (uint32_t)kk;

    // ---- join record: orthonormal projections of the FP32 copy, FP64 dots
    float jp[kJoinDims];
#pragma unroll
    for (int dm = 0; dm < kJoinDims; ++dm) {
        double p = 0.0;
#pragma unroll
        for (int c = 0; c < kFD; ++c) p = fma(uj[dm * kFD + c], (double)f[c], p);
        jp[dm] = (float)p;
    }
    float4 *jr = (float4 *)(q.jrec + (int64_t)kk * 8);
    jr[0] = make_float4(jp[0], jp[1], jp[2], jp[3]);
    jr[1] = make_float4(jp[4], jp[5], __uint_as_float((uint32_t)kk), 0.0f);

    // ---- error bound of the stored features: the direct start (four
    // quarters) and up to 63 slides in FP64, the scaling by 1/sigma, and the
    // rounding to FT; the FP32 copy is within u32 |F| of the FP64 value, which
    // also bounds the norm used here
    const double nrm = sqrt(n2) * (1.0 + 1e-6) + 1e-30;
    const double u64 = 1.1102230246251565e-16;
    const double ust = sizeof(FT) == 4 ? 5.9604644775390625e-08 : u64;
    const double Ebin = (6.0 * m * (double)m + 8.0 * kSegW * (m + 2.0) + 2.0 * m) * u64 * (double)Ymax;
    const double ecomp = sqrt(2.0 * L.kprime) * Ebin * is * 1.001;
    const double estore = (ust + 4.0 * u64) * (nrm + 6e-8 * nrm) * 1.001;
    const float e = (float)((ecomp + estore) * (1.0 + 1e-6)) * (1.0f + 2.4e-7f) + 1e-30f;
    if (sizeof(FT) == 8) {
        double2 v;
        v.x = (double)e;
        v.y = nrm;
        *(double2 *)(rec + kSlotErr) = v;
    } else {
        *(float4 *)(rec + 28) = make_float4(f[28], f[29], e, (float)nrm);
    }
    emax = fmaxf(emax, e);
}

}  // namespace

// One block per tile of 1024 consecutive windows of one length.
//  1. samples into LDS; compacted position of every non-constant window;
//  2. thread (segment g = tid / 16, bin b = tid % 16) owns bin k = b + 1 of
//     the 64 windows of segment g: it computes the bin directly at the
//     segment start (four independent phasor chains, so the sum is not one
//     long dependent chain) and slides it 63 times, in FP64;
//  3. every 8 slides the 128 new windows' raw bins are staged in LDS and one
//     thread per window finishes it (sketch_row).
template <typename FT>
__global__ __launch_bounds__(kBlock, 3) void k_sketch(Req q, const uint32_t *__restrict__ E,
                                                      const uint32_t *__restrict__ tile_off,
                                                      int st_len,
                                                      const float *__restrict__ gproj,
                                                      const double *__restrict__ ujoin) {
    extern __shared__ double dyn[];
    __shared__ SketchSmem sm;
    const int64_t tile = blockIdx.x;
    const int l = find_tile_len(q.len, q.L, tile);
    const LenInfo L = q.len[l];
    const int m = L.m;
    const int kp = L.kprime;
    const int64_t i0 = (tile - L.tile_base) * kTileW;
    const int nw = (int)min<int64_t>(kTileW, L.W - i0);
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / kWave;
    double *st = dyn;                                            // samples, 1024 + m - 1
    double(*stage)[kStageLd] = (double(*)[kStageLd])(dyn + st_len);   // kRowsC rows

    if (tid == 0) sm.emax = 0;
    for (int r = tid; r < nw + m - 1; r += kBlock) st[r] = q.t[i0 + r];

    // ---- compacted positions: thread tid takes windows 4 tid .. 4 tid + 3
    {
        bool ix[4];
        int c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int w = 4 * tid + j;
            ix[j] = w < nw && E[i0 + w + m] != E[i0 + w + 1];
            c += ix[j];
        }
        int x = c;                                               // inclusive wave scan
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int y = __shfl_up(x, off, kWave);
            if (lane >= off) x += y;
        }
        if (lane == kWave - 1) sm.wsum[wv] = (uint32_t)x;
        __syncthreads();
        uint32_t pos = tile_off[tile] + (uint32_t)(x - c);
        for (int v = 0; v < wv; ++v) pos += sm.wsum[v];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int w = 4 * tid + j;
            if (w < nw) sm.kpos[w] = ix[j] ? (int32_t)pos++ : -1;
        }
    }
    __syncthreads();

    // ---- sliding DFT in FP64: thread (segment g, bin b)
    const int b = tid & 15;
    const int g = tid >> 4;
    const int s0 = g * kSegW;
    const int segn = max(0, min(kSegW, nw - s0));
    const double c = segn > 0 ? st[s0] : 0.0;
    int any = 0;
    {
        // does the segment hold an indexed window; the largest |t - c| over
        // its samples, for the error bound
        double Y = 0.0;
        for (int r = b; r < segn; r += 16) any |= sm.kpos[s0 + r] >= 0;
        for (int r = b; r < segn + m - 1; r += 16) Y = fmax(Y, fabs(st[s0 + r] - c));
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            any |= __shfl_xor(any, off, 16);
            Y = fmax(Y, __shfl_xor(Y, off, 16));
        }
        if (b == 0) sm.ymax[g] = (float)(Y * (1.0 + 1e-6)) * (1.0f + 1e-6f);
    }
    double xr = 0.0, xi = 0.0, wcos = 1.0, wsin = 0.0;
    // a segment of constant windows only has no feature to compute
    const bool own = any && b < kp;
    if (own) {
        const int k = b + 1;
        sincospi(2.0 * (double)k / (double)m, &wsin, &wcos);   // omega = e^{+2 pi i k/m}
        // X = sum_r y_r e^{-2 pi i k r/m} over four quarters, each with its
        // own exactly started phasor
        const int ql = (m + 3) / 4;
        double ar[4], ai[4], pr[4], pi[4];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const int j = (int)(((int64_t)k * (int64_t)(ch * ql)) % m);
            double sn, cs;
            sincospi(2.0 * (double)j / (double)m, &sn, &cs);
            pr[ch] = cs;
            pi[ch] = -sn;
            ar[ch] = 0.0;
            ai[ch] = 0.0;
        }
        for (int u = 0; u < ql; ++u) {
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const int r = ch * ql + u;
                if (r < m) {
                    const double y = st[s0 + r] - c;
                    ar[ch] = fma(y, pr[ch], ar[ch]);
                    ai[ch] = fma(y, pi[ch], ai[ch]);
                    // phasor *= conj(omega)
                    const double npr = fma(pr[ch], wcos, pi[ch] * wsin);
                    const double npi = fma(pi[ch], wcos, -(pr[ch] * wsin));
                    pr[ch] = npr;
                    pi[ch] = npi;
                }
            }
        }
        xr = (ar[0] + ar[1]) + (ar[2] + ar[3]);
        xi = (ai[0] + ai[1]) + (ai[2] + ai[3]);
    }

    float emax = 0.0f;
    for (int chunk = 0; chunk < kSegW / kSlidesC; ++chunk) {
        // ---- 8 slides of every (segment, bin), raw bins into the staging rows
        for (int u = 0; u < kSlidesC; ++u) {
            const int sl = chunk * kSlidesC + u;
            const int s = s0 + sl;
            double *rw = stage[g * kSlidesC + u];
            if (sl < segn) {
                if (own) {
                    if (sl > 0) {
                        const double ya = st[s - 1] - c;
                        const double yb = st[s - 1 + m] - c;
                        const double a_r = xr - ya + yb;
                        const double a_i = xi;
                        xr = fma(a_r, wcos, -(a_i * wsin));
                        xi = fma(a_r, wsin, a_i * wcos);
                    }
                    rw[2 * b] = xr;
                    rw[2 * b + 1] = xi;
                } else if (any && b < kMaxK - 1) {
                    rw[2 * b] = 0.0;
                    rw[2 * b + 1] = 0.0;
                }
            }
        }
        __syncthreads();

        // ---- one thread per staged window
        if (tid < kRowsC) {
            const int row = tid;
            const int sg = row / kSlidesC;
            const int s = sg * kSegW + chunk * kSlidesC + (row % kSlidesC);
            const int32_t kk = s < nw ? sm.kpos[s] : -1;
            if (kk >= 0)
                sketch_row<FT>(q, L, l, L.cell_base + i0 + s, st + s, (8 * sg) % m, stage[row],
                               sm.ymax[sg], kk, gproj + (int64_t)l * q.B * kFD, ujoin, emax);
        }
        __syncthreads();
    }
    // largest e_i of the tile: one LDS atomic per wavefront
    int eb = __float_as_int(emax);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) eb = max(eb, __shfl_xor(eb, off, kWave));
    if (lane == 0 && eb) atomicMax(&sm.emax, eb);
    __syncthreads();
    if (tid == 0 && sm.emax) atomicMax((int *)&q.emax[l], sm.emax);
}

// First slot of every bucket from the sorted keys: between two consecutive
// sorted entries, every bucket index in (previous, current] starts at the
// current slot (empty buckets included); the entry past the end closes the
// last buckets.
__global__ __launch_bounds__(kBlock) void k_bucket_bounds(Req q, int64_t N, int64_t nbuckets,
                                                          uint32_t *__restrict__ bstart) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s > N) return;
    const uint32_t mask = (1u << q.key_shift) - 1u;
    auto gidx = [&](uint32_t key) -> int64_t {
        const int l = (int)(key >> q.key_shift);
        const int d = q.len[l].depth;
        return q.len[l].bucket_base + (int64_t)((key & mask) >> (q.key_shift - d));
    };
    const int64_t cur = s < N ? gidx(q.skey[s]) : nbuckets;
    const int64_t prev = s > 0 ? gidx(q.skey[s - 1]) : -1;
    for (int64_t b = prev + 1; b <= cur; ++b) bstart[b] = (uint32_t)s;
}

// Slot maps after the sort: k -> slot and slot -> cell.
__global__ __launch_bounds__(kBlock) void k_slot_maps(Req q, int64_t N) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    const uint32_t k = q.perm[s];
    q.inv[k] = (uint32_t)s;
    q.pcell[s] = q.cell[k];
}

__global__ __launch_bounds__(kBlock) void k_invert(const uint32_t *__restrict__ perm, int64_t N,
                                                   uint32_t *__restrict__ inv) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < N) inv[perm[s]] = (uint32_t)s;
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_changepoints(const double *t, int64_t n, uint32_t *flag, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_changepoints, dim3(nblk(n + 1)), dim3(kBlock), 0, s, t, n, flag, bad);
}

void launch_tile_counts(const LenInfo *len, int L, const uint32_t *E, int64_t ntiles,
                        uint32_t *tile_cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_counts, dim3((unsigned)ntiles), dim3(kBlock), 0, s, len, L, E,
                       tile_cnt);
}

void launch_sketch(int precision, const Req &q, const uint32_t *E, const uint32_t *tile_off,
                   int64_t ntiles, int max_m, hipStream_t s) {
    // samples (1024 + m - 1 doubles, rounded up to an even count so the
    // staging rows that follow are 16-byte aligned), then the staging rows,
    // sized for the longest window of the request
    const int st_len = (kTileW + max_m + 1) & ~1;
    const size_t dyn = (size_t)(st_len + kRowsC * kStageLd) * sizeof(double);
    if (precision == 0)
        hipLaunchKernelGGL((k_sketch<double>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_off, st_len, q.gproj, q.ujoin);
    else
        hipLaunchKernelGGL((k_sketch<float>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_off, st_len, q.gproj, q.ujoin);
}

void launch_bucket_bounds(const Req &q, int64_t N, int64_t nbuckets, uint32_t *bstart,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_bounds, dim3(nblk(N + 1)), dim3(kBlock), 0, s, q, N, nbuckets,
                       bstart);
}

void launch_slot_maps(const Req &q, int64_t N, hipStream_t s) {
    if (N > 0) hipLaunchKernelGGL(k_slot_maps, dim3(nblk(N)), dim3(kBlock), 0, s, q, N);
}

void launch_invert(const uint32_t *perm, int64_t N, uint32_t *inv, hipStream_t s) {
    if (N > 0) hipLaunchKernelGGL(k_invert, dim3(nblk(N)), dim3(kBlock), 0, s, perm, N, inv);
}

}  // namespace pmp
