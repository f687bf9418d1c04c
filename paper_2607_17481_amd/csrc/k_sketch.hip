// k_sketch.hip -- moments, normalized spectral features and SimHash keys.
//
// Paper Sec. 3.2: the retained feature of window (i, m) is
//   F_{i,m} = (X_1 .. X_{K'}) / sigma,  X_k = sum_r t_{i+r} e^{-2 pi i k r / m},
// K' = min(K-1, ceil(m/2)-1), zero-padded to K-1 bins; by Lemma 1 it equals the
// leading non-DC bins of the DFT of the z-normalized window.  The paper keeps
// one sliding state per length and updates it in O(K) per slide
//   X_{i+1,k} = e^{2 pi i k / m} (X_{i,k} - t_i + t_{i+m}),
// recomputing from the raw samples every 4096 slides.  On the GPU each block
// takes a tile of 256 consecutive windows of one length, staged in LDS; the
// tile is split into 16 segments of 16 windows, and thread (segment, bin)
// computes its bin directly at the segment start and slides it 15 times, in
// FP64.  Samples are shifted by a per-segment constant c first, which leaves
// every bin k >= 1 unchanged (Lemma 1) and keeps the magnitudes small.
//
// Each window also gets a rigorous bound e_i >= ||F~_i - F_i|| on the error of
// its stored features (computation in FP64 + rounding to the storage type),
// so that the Parseval bound can be shrunk into a true lower bound at every
// magnitude (replacing the paper's relative (1 - lambda) shrink, Lemma 4,
// which it proves only above a threshold).
//
// Pass A writes the window moments and the key word (signature bits plus the
// Hamming-1 probe order); pass B, after the bucket sort, recomputes the same
// features and writes them in bucket (slot) order together with the join
// record.
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

// Non-constant windows per length: window [i, i+m) is constant iff no change
// point lies in (i, i+m), i.e. E[i+m] == E[i+1] for the exclusive prefix E.
__global__ __launch_bounds__(kBlock) void k_count_index(const LenInfo *__restrict__ len,
                                                        const uint32_t *__restrict__ E,
                                                        unsigned long long *__restrict__ cnt) {
    const int l = blockIdx.y;
    const int m = len[l].m;
    const int64_t W = len[l].W;
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < W;
         i += (int64_t)gridDim.x * kBlock)
        c += E[i + m] != E[i + 1];
    // wave reduction then one atomic per wave
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (lane_id() == 0 && c) atomicAdd(&cnt[l], c);
}

// ---------------------------------------------------------------- sketch

namespace {

__device__ __forceinline__ int find_tile_len(const LenInfo *len, int L, int64_t tile) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (len[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct SketchSmem {
    double mu[kTileW];
    double isig[kTileW];
    float ymax[kTileW / kSegW];
    float f[kTileW][kRec + 1];   // +1 pads the row to avoid bank conflicts
    float g[kMaxBits][2 * (kMaxK - 1)];
    uint32_t wcount[kBlock / kWave];
};

}  // namespace

template <int PASS, typename FT>
__global__ __launch_bounds__(kBlock) void k_sketch(Req q, const uint32_t *__restrict__ E,
                                                   uint32_t *__restrict__ tile_cnt) {
    extern __shared__ double st[];                 // tile samples, 256 + m - 1
    __shared__ SketchSmem sm;
    const int64_t tile = blockIdx.x;
    const int l = find_tile_len(q.len, q.L, tile);
    const LenInfo L = q.len[l];
    const int m = L.m;
    const int kp = L.kprime;
    const int64_t i0 = (tile - L.tile_base) * kTileW;
    const int nw = (int)min<int64_t>(kTileW, L.W - i0);
    const int tid = threadIdx.x;

    for (int r = tid; r < nw + m - 1; r += kBlock) st[r] = q.t[i0 + r];
    if (PASS == 0) {
        for (int c = tid; c < q.B * 2 * (kMaxK - 1); c += kBlock)
            sm.g[c / (2 * (kMaxK - 1))][c % (2 * (kMaxK - 1))] =
                q.gproj[((int64_t)l * q.B) * 2 * (kMaxK - 1) + c];
    }
    __syncthreads();

    // ---- moments: two-pass population mean / standard deviation (Sec. 3.2)
    if (tid < nw) {
        const int64_t cell = L.cell_base + i0 + tid;
        double mu = 0.0, is = 0.0;
        if (PASS == 0) {
            const bool cst = E[i0 + tid + m] == E[i0 + tid + 1];
            if (!cst) {
#pragma clang fp contract(off)
                double s = 0.0;
                for (int r = 0; r < m; ++r) s += st[tid + r];
                mu = s / (double)m;
                double qq = 0.0;
                for (int r = 0; r < m; ++r) {
                    double c = st[tid + r] - mu;
                    qq += c * c;
                }
                double sg = sqrt(qq / (double)m);
                is = 1.0 / sg;
                if (!(sg > 0.0) || !isfinite(sg) || !(is > 0.0) || !isfinite(is)) {
                    // samples differ but sigma underflows: outside the range
                    // the library represents; keep the window indexed so
                    // every count stays consistent and report the input
                    atomicOr(q.bad, 2);
                    is = 1.0;
                }
            } else {
                mu = st[tid];
            }
            q.mu[cell] = mu;
            q.isig[cell] = is;
        } else {
            mu = q.mu[cell];
            is = q.isig[cell];
        }
        sm.mu[tid] = mu;
        sm.isig[tid] = is;
    }
    __syncthreads();

    // ---- sliding DFT in FP64: thread (segment g, bin b)
    {
        const int b = tid & 15;          // bin k = b + 1
        const int g = tid >> 4;          // segment
        const int s0 = g * kSegW;
        double Y = 0.0;
        if (s0 < nw) {
            const double c = sm.mu[s0];
            if (b < kp) {
                const int k = b + 1;
                double wsin, wcos;
                sincospi(2.0 * (double)k / (double)m, &wsin, &wcos);   // omega = e^{+2 pi i k/m}
                // direct DFT of the segment's first window by a rotating phasor
                double xr = 0.0, xi = 0.0, pr = 1.0, pi = 0.0;
                for (int r = 0; r < m; ++r) {
                    double y = st[s0 + r] - c;
                    Y = fmax(Y, fabs(y));
                    xr = fma(y, pr, xr);
                    xi = fma(y, pi, xi);
                    // phasor *= conj(omega)
                    double npr = fma(pr, wcos, pi * wsin);
                    double npi = fma(pi, wcos, -(pr * wsin));
                    pr = npr;
                    pi = npi;
                }
                for (int s = s0; s < s0 + kSegW && s < nw; ++s) {
                    if (s > s0) {
                        double ya = st[s - 1] - c;
                        double yb = st[s - 1 + m] - c;
                        Y = fmax(Y, fabs(yb));
                        double ar = xr - ya + yb;
                        double ai = xi;
                        xr = fma(ar, wcos, -(ai * wsin));
                        xi = fma(ar, wsin, ai * wcos);
                    }
                    const double is = sm.isig[s];
                    const double fr = xr * is, fi = xi * is;
                    sm.f[s][2 * b] = (float)fr;
                    sm.f[s][2 * b + 1] = (float)fi;
                    if (PASS == 1 && is != 0.0) {
                        const uint32_t slot = q.inv[L.cell_base + i0 + s];
                        FT *rec = (FT *)q.F + (int64_t)slot * kRec;
                        rec[2 * b] = (FT)fr;
                        rec[2 * b + 1] = (FT)fi;
                    }
                }
                if (b == 0) sm.ymax[g] = (float)(Y * (1.0 + 1e-6));
            } else if (b < kMaxK - 1) {
                for (int s = s0; s < s0 + kSegW && s < nw; ++s) {
                    sm.f[s][2 * b] = 0.0f;
                    sm.f[s][2 * b + 1] = 0.0f;
                    if (PASS == 1 && sm.isig[s] != 0.0) {
                        const uint32_t slot = q.inv[L.cell_base + i0 + s];
                        FT *rec = (FT *)q.F + (int64_t)slot * kRec;
                        rec[2 * b] = (FT)0;
                        rec[2 * b + 1] = (FT)0;
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- per-window post-processing
    const int w = tid;
    bool indexed = false;
    if (w < nw) {
        const int64_t cell = L.cell_base + i0 + w;
        const double is = sm.isig[w];
        indexed = is != 0.0;     // 0 exactly for constant windows, > 0 otherwise
        if (PASS == 0) {
            uint64_t kw = ~0ull;
            if (indexed) {
                float f[2 * (kMaxK - 1)];
#pragma unroll
                for (int c = 0; c < 2 * (kMaxK - 1); ++c) f[c] = sm.f[w][c];
                float mg[kMaxBits];
                uint32_t sig = 0;
                for (int b = 0; b < q.B; ++b) {
                    float dot = 0.0f;
#pragma unroll
                    for (int c = 0; c < 2 * (kMaxK - 1); ++c) dot = fmaf(sm.g[b][c], f[c], dot);
                    mg[b] = fabsf(dot);
                    if (dot >= 0.0f) sig |= 1u << (q.B - 1 - b);
                }
                // Hamming-1 probe order: the `probes` smallest margins among
                // the d prefix bits, ascending (Sec. 3.4 multi-probe)
                uint64_t order = 0;
                uint32_t used = 0;
                for (int h = 0; h < L.probes; ++h) {
                    int best = -1;
                    float bm = 0.0f;
                    for (int b = 0; b < L.depth; ++b) {
                        if (used & (1u << b)) continue;
                        if (best < 0 || mg[b] < bm) { best = b; bm = mg[b]; }
                    }
                    used |= 1u << best;
                    order |= (uint64_t)best << (5 * h);
                }
                kw = (uint64_t)sig | (order << 24);
            }
            q.keyw_nat[cell] = kw;
        } else if (indexed) {
            const uint32_t slot = q.inv[cell];
            double n2 = 0.0;
            float f[2 * (kMaxK - 1)];
#pragma unroll
            for (int c = 0; c < 2 * (kMaxK - 1); ++c) {
                f[c] = sm.f[w][c];
                n2 += (double)f[c] * (double)f[c];
            }
            const double nrm = sqrt(n2) * (1.0 + 1e-6) + 1e-30;
            // error bound of the stored features (see file comment)
            const double u64 = 1.1102230246251565e-16;
            const double ust = sizeof(FT) == 4 ? 5.9604644775390625e-08 : u64;
            const double Y = (double)sm.ymax[w / kSegW];
            const double Ebin = (6.0 * m * (double)m + 8.0 * kSegW * (m + 2.0) + 2.0 * m) * u64 * Y;
            const double ecomp = sqrt(2.0 * kp) * Ebin * is * 1.001;
            // the FP32 copy in LDS differs from the FP64 value by <= u32 |F|;
            // that covers FP32 storage, and bounds the norm used here
            const double estore = (ust + 4.0 * u64) * (nrm + 6e-8 * nrm) * 1.001;
            const float e = (float)((ecomp + estore) * (1.0 + 1e-6)) * (1.0f + 2.4e-7f) + 1e-30f;
            FT *rec = (FT *)q.F + (int64_t)slot * kRec;
            rec[kSlotErr] = (FT)e;
            rec[kSlotNorm] = (FT)nrm;
            atomicMax((int *)&q.emax[l], __float_as_int(e));
            q.keyw[slot] = q.keyw_nat[cell];
            // join record: orthonormal projections of the FP32 copy, FP64 dots
            float *jr = q.jrec + (int64_t)slot * 8;
#pragma unroll
            for (int d = 0; d < kJoinDims; ++d) {
                double p = 0.0;
#pragma unroll
                for (int c = 0; c < 2 * (kMaxK - 1); ++c)
                    p = fma(q.ujoin[d * 2 * (kMaxK - 1) + c], (double)f[c], p);
                jr[d] = (float)p;
            }
            jr[6] = __uint_as_float(slot);
            jr[7] = 0.0f;
        }
    }
    if (PASS == 0) {
        uint64_t bal = __ballot(indexed);
        if (lane_id() == 0) sm.wcount[tid / kWave] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (tid == 0) {
            uint32_t s = 0;
            for (int k = 0; k < kBlock / kWave; ++k) s += sm.wcount[k];
            tile_cnt[tile] = s;
        }
    }
}

// Sort input in (length, start) order: key = len << key_shift | prefix <<
// (key_shift - d), value = cell.  Also counts bucket populations.
__global__ __launch_bounds__(kBlock) void k_emit_sortin(Req q, const uint32_t *__restrict__ tile_off) {
    __shared__ uint32_t wc[kBlock / kWave];
    const int64_t tile = blockIdx.x;
    const int l = find_tile_len(q.len, q.L, tile);
    const LenInfo L = q.len[l];
    const int64_t i0 = (tile - L.tile_base) * kTileW;
    const int nw = (int)min<int64_t>(kTileW, L.W - i0);
    const int tid = threadIdx.x;
    uint64_t kw = ~0ull;
    const int64_t cell = L.cell_base + i0 + tid;
    if (tid < nw) kw = q.keyw_nat[cell];
    const bool ix = kw != ~0ull;
    const uint64_t bal = __ballot(ix);
    if (lane_id() == 0) wc[tid / kWave] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (ix) {
        uint32_t pos = tile_off[tile] + (uint32_t)__popcll(bal & lanemask_lt());
        for (int k = 0; k < tid / kWave; ++k) pos += wc[k];
        const uint32_t sig = (uint32_t)(kw & 0xFFFFFFu);
        const uint32_t prefix = L.depth ? sig >> (q.B - L.depth) : 0u;
        q.skey[pos] = ((uint32_t)l << q.key_shift) | (prefix << (q.key_shift - L.depth));
        q.sval[pos] = (uint32_t)cell;
        atomicAdd(&q.bucket_cnt[L.bucket_base + prefix], 1u);
    }
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

void launch_count_index(const LenInfo *len, int L, const uint32_t *E, unsigned long long *cnt,
                        int64_t maxW, hipStream_t s) {
    int64_t bx = (maxW + kBlock * 8 - 1) / (kBlock * 8);
    if (bx < 1) bx = 1;
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(k_count_index, dim3((unsigned)bx, (unsigned)L), dim3(kBlock), 0, s, len, E,
                       cnt);
}

void launch_sketch(int pass, int precision, const Req &q, const uint32_t *E, uint32_t *tile_cnt,
                   int64_t ntiles, int max_m, hipStream_t s) {
    const size_t dyn = (size_t)(kTileW + max_m) * sizeof(double);
    if (pass == 0)
        hipLaunchKernelGGL((k_sketch<0, float>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_cnt);
    else if (precision == 0)
        hipLaunchKernelGGL((k_sketch<1, double>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_cnt);
    else
        hipLaunchKernelGGL((k_sketch<1, float>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                           tile_cnt);
}

void launch_emit_sortin(const Req &q, const uint32_t *tile_off, int64_t ntiles, hipStream_t s) {
    hipLaunchKernelGGL(k_emit_sortin, dim3((unsigned)ntiles), dim3(kBlock), 0, s, q, tile_off);
}

void launch_invert(const uint32_t *perm, int64_t N, uint32_t *inv, hipStream_t s) {
    if (N > 0) hipLaunchKernelGGL(k_invert, dim3(nblk(N)), dim3(kBlock), 0, s, perm, N, inv);
}

}  // namespace pmp
