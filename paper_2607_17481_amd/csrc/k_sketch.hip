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

constexpr int kFD = 2 * (kMaxK - 1);      // 30 feature reals
constexpr int kRows = kSegs * kChunk;     // windows per post-processing step (64)

struct SketchSmem {
    double isig[kTileW];
    int32_t kpos[kTileW];                 // indexed position, -1 for constant windows
    float ymax[kSegs];
    float mg[kRows][kMaxBits + 1];        // |<g_l, F>| of each row
    uint32_t sigp[kRows][4];              // signature bits, one part per quad thread
    int32_t seg_any[kSegs];               // segment holds an indexed window
    float g[kMaxBits][kFD];
    uint32_t wsum[kBlock / kWave];
    int emax;
};

}  // namespace

// One block per tile of 1024 consecutive windows of one length.  Thread
// (segment g = tid / 16, bin b = tid % 16) owns bin k = b + 1 of the 64
// windows of segment g: it computes the bin directly at the segment start
// (four independent phasor chains, so the sum is not one long dependent
// chain) and slides it 63 times.  Every 4 slides the 64 new windows are
// post-processed by four threads each.
template <typename FT>
__global__ __launch_bounds__(kBlock, 3) void k_sketch(Req q, const uint32_t *__restrict__ E,
                                                      const uint32_t *__restrict__ tile_off) {
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
    double *st = dyn;                                        // samples, 1024 + m - 1
    FT(*stage)[kRec + 1] = (FT(*)[kRec + 1])(dyn + kTileW + m);   // then kRows records

    if (tid == 0) sm.emax = 0;
    for (int r = tid; r < nw + m - 1; r += kBlock) st[r] = q.t[i0 + r];
    for (int c = tid; c < q.B * kFD; c += kBlock)
        sm.g[c / kFD][c % kFD] = q.gproj[(int64_t)l * q.B * kFD + c];
    __syncthreads();

    // ---- moments (two-pass, population; Sec. 3.2) and compacted positions
    {
        uint32_t run = tile_off[tile];
        for (int w0 = 0; w0 < kTileW; w0 += kBlock) {
            const int w = w0 + tid;
            const bool in = w < nw;
            const bool ix = in && E[i0 + w + m] != E[i0 + w + 1];
            const uint64_t bal = __ballot(ix);
            if (lane == 0) sm.wsum[wv] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t pos = run + (uint32_t)__popcll(bal & lanemask_lt()), tot = 0;
            for (int x = 0; x < kBlock / kWave; ++x) {
                if (x < wv) pos += sm.wsum[x];
                tot += sm.wsum[x];
            }
            double is = 0.0;
            if (ix) {
                // four partial sums per pass keep the LDS loads independent
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int r = 0;
                for (; r + 4 <= m; r += 4) {
                    a0 += st[w + r];
                    a1 += st[w + r + 1];
                    a2 += st[w + r + 2];
                    a3 += st[w + r + 3];
                }
                for (; r < m; ++r) a0 += st[w + r];
                const double mu = ((a0 + a1) + (a2 + a3)) / (double)m;
                a0 = a1 = a2 = a3 = 0.0;
                for (r = 0; r + 4 <= m; r += 4) {
                    const double c0 = st[w + r] - mu, c1 = st[w + r + 1] - mu;
                    const double c2 = st[w + r + 2] - mu, c3 = st[w + r + 3] - mu;
                    a0 = fma(c0, c0, a0);
                    a1 = fma(c1, c1, a1);
                    a2 = fma(c2, c2, a2);
                    a3 = fma(c3, c3, a3);
                }
                for (; r < m; ++r) {
                    const double c0 = st[w + r] - mu;
                    a0 = fma(c0, c0, a0);
                }
                const double sg = sqrt(((a0 + a1) + (a2 + a3)) / (double)m);
                is = 1.0 / sg;
                if (!(sg > 0.0) || !isfinite(sg) || !(is > 0.0) || !isfinite(is)) {
                    // samples differ but sigma underflows or overflows:
                    // outside the range the library represents; keep the
                    // window indexed so every count stays consistent
                    atomicOr(q.bad, 2);
                    is = 1.0;
                }
                q.cell[pos] = (uint32_t)(L.cell_base + i0 + w);
                q.mu[pos] = mu;
                q.isig[pos] = is;
                q.P[pos] = kInfBits;
            }
            if (in) {
                sm.isig[w] = is;
                sm.kpos[w] = ix ? (int32_t)pos : -1;
            }
            run += tot;
            __syncthreads();
        }
        if (tid < kSegs) {
            int any = 0;
            for (int w = tid * kSegW; w < min(nw, (tid + 1) * kSegW); ++w) any |= sm.kpos[w] >= 0;
            sm.seg_any[tid] = any;
        }
        __syncthreads();
    }

    // ---- sliding DFT in FP64: thread (segment g, bin b)
    const int b = tid & 15;
    const int g = tid >> 4;
    const int s0 = g * kSegW;
    const int segn = max(0, min(kSegW, nw - s0));
    const double c = segn > 0 ? st[s0] : 0.0;
    {
        // largest |t - c| over the segment's samples, for the error bound
        double Y = 0.0;
        for (int r = b; r < segn + m - 1; r += 16) Y = fmax(Y, fabs(st[s0 + r] - c));
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) Y = fmax(Y, __shfl_xor(Y, off, 16));
        if (b == 0) sm.ymax[g] = (float)(Y * (1.0 + 1e-6)) * (1.0f + 1e-6f);
    }
    double xr = 0.0, xi = 0.0, wcos = 1.0, wsin = 0.0;
    // a segment of constant windows only has no feature to compute
    const bool own = segn > 0 && b < kp && sm.seg_any[g];
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

    const int row = tid >> 2;         // post-processing: four threads per row
    const int quad = tid & 3;
    const int pg = row / kChunk, pu = row % kChunk;
    for (int chunk = 0; chunk < kSegW / kChunk; ++chunk) {
        // ---- 4 slides of every (segment, bin), into the staging rows
        for (int u = 0; u < kChunk; ++u) {
            const int sl = chunk * kChunk + u;
            const int s = s0 + sl;
            FT *rw = stage[g * kChunk + u];
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
                    const double is = sm.isig[s];
                    rw[2 * b] = (FT)(xr * is);
                    rw[2 * b + 1] = (FT)(xi * is);
                } else if (b < kMaxK - 1) {
                    rw[2 * b] = (FT)0;
                    rw[2 * b + 1] = (FT)0;
                }
            }
        }
        __syncthreads();

        // ---- post-processing of the 64 rows
        const int s = pg * kSegW + chunk * kChunk + pu;
        const bool valid = s < nw;
        const int32_t kk = valid ? sm.kpos[s] : -1;
        const bool indexed = kk >= 0;
        // constant windows (no cell) skip the arithmetic below
        float f[kFD];
        double n2 = 0.0;
        if (indexed) {
#pragma unroll
            for (int x = 0; x < kFD; ++x) f[x] = (float)stage[row][x];
            // SimHash bits (Sec. 3.4): bit l = [<g_l, F> >= 0], six per
            // thread; margins and bits go to LDS, so no register array is
            // indexed at run time and no cross-lane exchange is needed
            uint32_t sig = 0;
#pragma unroll
            for (int h = 0; h < 6; ++h) {
                const int bt = quad * 6 + h;
                if (bt < q.B) {
                    float dot = 0.0f;
#pragma unroll
                    for (int x = 0; x < kFD; ++x) dot = fmaf(sm.g[bt][x], f[x], dot);
                    sm.mg[row][bt] = fabsf(dot);
                    if (dot >= 0.0f) sig |= 1u << (q.B - 1 - bt);
                }
            }
            sm.sigp[row][quad] = sig;
            // join record: orthonormal projections of the FP32 copy, FP64 dots
            float *jr = q.jrec + (int64_t)kk * 8;
#pragma unroll
            for (int dd = 0; dd < 2; ++dd) {
                const int dim = quad + 4 * dd;
                if (dim < kJoinDims) {
                    double p = 0.0;
#pragma unroll
                    for (int x = 0; x < kFD; ++x) p = fma(q.ujoin[dim * kFD + x], (double)f[x], p);
                    jr[dim] = (float)p;
                }
            }
            // norm of the FP32 copy (static register indices only)
            if (quad == 0) {
#pragma unroll
                for (int x = 0; x < kFD; ++x) n2 = fma((double)f[x], (double)f[x], n2);
            }
        }
        __syncthreads();                      // margins and bits visible to the quad leader
        if (indexed && quad == 0) {
            // Hamming-1 probe order: the `probes` smallest margins among the
            // d prefix bits, ascending (Sec. 3.4 multi-probe)
            uint64_t order = 0;
            uint32_t used = 0;
            for (int h = 0; h < L.probes; ++h) {
                int best = -1;
                float bm = 0.0f;
                for (int bt = 0; bt < L.depth; ++bt) {
                    if (used & (1u << bt)) continue;
                    const float v = sm.mg[row][bt];
                    if (best < 0 || v < bm) { best = bt; bm = v; }
                }
                used |= 1u << best;
                order |= (uint64_t)best << (5 * h);
            }
            const uint32_t sig = sm.sigp[row][0] | sm.sigp[row][1] | sm.sigp[row][2] | sm.sigp[row][3];
            q.keyw[kk] = (uint64_t)sig | (order << 24);
            const uint32_t prefix = L.depth ? sig >> (q.B - L.depth) : 0u;
            q.skey[kk] = ((uint32_t)l << q.key_shift) | (prefix << (q.key_shift - L.depth));
            q.sval[kk] = (uint32_t)kk;
            float *jr = q.jrec + (int64_t)kk * 8;
            jr[6] = __uint_as_float((uint32_t)kk);
            jr[7] = 0.0f;
            // error bound of the stored features (see file comment): direct
            // start (4 quarters) + 63 slides in FP64, the multiplication by
            // 1/sigma, and the rounding to FT; the FP32 copy differs from the
            // FP64 value by <= u32 |F|, which also bounds the norm used here
            const double nrm = sqrt(n2) * (1.0 + 1e-6) + 1e-30;
            const double u64 = 1.1102230246251565e-16;
            const double ust = sizeof(FT) == 4 ? 5.9604644775390625e-08 : u64;
            const double Y = (double)sm.ymax[pg];
            const double Ebin = (6.0 * m * (double)m + 8.0 * kSegW * (m + 2.0) + 2.0 * m) * u64 * Y;
            const double ecomp = sqrt(2.0 * kp) * Ebin * sm.isig[s] * 1.001;
            const double estore = (ust + 4.0 * u64) * (nrm + 6e-8 * nrm) * 1.001;
            const float e = (float)((ecomp + estore) * (1.0 + 1e-6)) * (1.0f + 2.4e-7f) + 1e-30f;
            stage[row][kSlotErr] = (FT)e;
            stage[row][kSlotNorm] = (FT)nrm;
            atomicMax(&sm.emax, __float_as_int(e));
        }
        __syncthreads();
        // ---- whole records out, 16 bytes per thread and store
        constexpr int kPer = 16 / (int)sizeof(FT);           // FT values per 16 bytes
        constexpr int kParts = kRec / kPer;                  // 16-byte parts per record
        for (int flat = tid; flat < kRows * kParts; flat += kBlock) {
            const int r = flat / kParts, part = flat % kParts;
            const int sr = (r / kChunk) * kSegW + chunk * kChunk + (r % kChunk);
            if (sr < nw) {
                const int32_t kr = sm.kpos[sr];
                if (kr >= 0) {
                    const FT *src = &stage[r][part * kPer];
                    FT *dst = (FT *)q.F + (int64_t)kr * kRec + part * kPer;
                    if (sizeof(FT) == 8) {
                        double2 v;
                        v.x = (double)src[0];
                        v.y = (double)src[1];
                        *(double2 *)dst = v;
                    } else {
                        float4 v;
                        v.x = (float)src[0];
                        v.y = (float)src[1];
                        v.z = (float)src[kPer > 2 ? 2 : 0];
                        v.w = (float)src[kPer > 3 ? 3 : 0];
                        *(float4 *)dst = v;
                    }
                }
            }
        }
        __syncthreads();
    }
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
    // samples (1024 + m - 1 doubles) then the staging rows, sized for the
    // longest window of the request
    if (precision == 0) {
        const size_t dyn = (size_t)(kTileW + max_m) * sizeof(double) +
                           (size_t)kSegs * kChunk * (kRec + 1) * sizeof(double);
        hipLaunchKernelGGL((k_sketch<double>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_off);
    } else {
        const size_t dyn = (size_t)(kTileW + max_m) * sizeof(double) +
                           (size_t)kSegs * kChunk * (kRec + 1) * sizeof(float);
        hipLaunchKernelGGL((k_sketch<float>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_off);
    }
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
