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

#include <algorithm>
#include <vector>

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

// bf16 with round to nearest even (finite input), as its 16 bits.
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
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
constexpr int kGLd = 32;                      // floats per SimHash projection in LDS
constexpr int kStageLd = 31;                  // doubles per staged row (odd: the
                                              // row threads' 8-byte reads spread
                                              // over all banks)

struct SketchSmem {
    int32_t kpos[kTileW];                     // indexed position, -1: constant window
    uint16_t widx[kTileW];                    // the tile's non-constant windows, in order
    float ymax[kSegs];                        // largest |t - c| of each segment
    uint32_t wsum[kBlock / kWave];
    int emax;
};

// Finishing of one non-constant window (one thread): the normalized
// features F = X / sigma written to its record, with the norm of their FP32
// copy and the error bound e_i of the stored features.
template <typename FT>
__device__ __forceinline__ void sketch_record(const Req &q, int m, int kprime,
                                              const double *__restrict__ X, double is,
                                              float Ymax, int kk, float &emax) {
    FT *rec = (FT *)q.F + (int64_t)kk * kRec;
    float f[kFD];
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
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < kFD; ++c) n2 = fma((double)f[c], (double)f[c], n2);
    // error bound: the direct start (four quarters) and up to 63 slides in
    // FP64, the scaling by 1/sigma, and the rounding to FT; the FP32 copy is
    // within u32 |F| of the FP64 value, which also bounds the norm used here
    const double nrm = sqrt(n2) * (1.0 + 1e-6) + 1e-30;
    const double u64 = 1.1102230246251565e-16;
    const double ust = sizeof(FT) == 4 ? 5.9604644775390625e-08 : u64;
    const double Ebin = (6.0 * m * (double)m + 8.0 * kSegW * (m + 2.0) + 2.0 * m) * u64 * (double)Ymax;
    const double ecomp = sqrt(2.0 * kprime) * Ebin * is * 1.001;
    // the FP64 two-pass sigma is within (m + 8) u64 of its exact value
    // (relative), which scales F by as much
    const double estore = (ust + (4.0 + m + 8.0) * u64) * (nrm + 6e-8 * nrm) * 1.001;
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

// A tile's samples into LDS: st[r] = t[i0 + r] for r < nvalid, 0 up to
// ntotal.  Every load of a thread is issued before the first LDS write, so a
// tile waits for memory once, not once per 256 samples.
__device__ __forceinline__ void load_tile_samples(const double *__restrict__ t, int64_t i0,
                                                  int nvalid, int ntotal, double *st) {
    constexpr int kLd = (kTileW + kMaxM + 64) / kBlock + 1;   // covers every tile and halo
    const int tid = threadIdx.x;
    double v[kLd];
#pragma unroll
    for (int x = 0; x < kLd; ++x) {
        const int r = tid + x * kBlock;
        v[x] = r < nvalid ? t[i0 + r] : 0.0;
    }
#pragma unroll
    for (int x = 0; x < kLd; ++x) {
        const int r = tid + x * kBlock;
        if (r < ntotal) st[r] = v[x];
    }
}

// Shared first steps of a sketch tile (samples already in LDS): the
// compacted position k of every non-constant window (thread tid takes
// windows 4 tid .. 4 tid + 3; a block scan) and the list of those windows,
// then their two-pass moments (Sec. 3.2), dealt evenly over the threads from
// the list, with their cell and the initial profile value.  Ends with the
// block synchronized and kpos final (and, when given, smu / sis: the mean
// and 1 / sigma of each non-constant window by its place in the tile).
__device__ __forceinline__ void tile_positions_and_moments(
    const Req &q, const LenInfo &L, int64_t i0, int nw, int64_t tile, const double *st,
    const uint32_t *__restrict__ E, const uint32_t *__restrict__ tile_off, int32_t *kpos,
    uint16_t *widx, uint32_t *wsum, double *smu = nullptr, double *sis = nullptr) {
    const int m = L.m;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / kWave;
    {
        // the eight change-point counts are loaded together (indices
        // clamped to the tile's last window, which stays within E[0..n])
        uint32_t ea[4], eb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t w = i0 + min(4 * tid + j, nw - 1);
            ea[j] = E[w + m];
            eb[j] = E[w + 1];
        }
        bool ix[4];
        int c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ix[j] = 4 * tid + j < nw && ea[j] != eb[j];
            c += ix[j];
        }
        int x = c;                                               // inclusive wave scan
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int y = __shfl_up(x, off, kWave);
            if (lane >= off) x += y;
        }
        if (lane == kWave - 1) wsum[wv] = (uint32_t)x;
        __syncthreads();
        uint32_t loc = (uint32_t)(x - c);
        for (int v = 0; v < wv; ++v) loc += wsum[v];
        const uint32_t base = tile_off[tile];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int w = 4 * tid + j;
            if (w < nw) {
                kpos[w] = ix[j] ? (int32_t)(base + loc) : -1;
                if (ix[j]) widx[loc++] = (uint16_t)w;
            }
        }
    }
    __syncthreads();
    // the cell -> indexed position map (anchors and hints need it)
    if (q.kmap)
        for (int w = tid; w < nw; w += kBlock)
            q.kmap[L.cell_base + i0 + w] = kpos[w] < 0 ? kNone : (uint32_t)kpos[w];
    int nix = 0;                                        // non-constant windows of the tile
    for (int v = 0; v < kBlock / kWave; ++v) nix += (int)wsum[v];

    // ---- moments (two-pass, population; Sec. 3.2), one thread per
    // non-constant window
    for (int xi = tid; xi < nix; xi += kBlock) {
        const int w = widx[xi];
        const int32_t kk = kpos[w];
        double mu;
        const double sg = window_moments(st + w, m, mu);
        double is = 1.0 / sg;
        if (!(sg > 0.0) || !isfinite(sg) || !(is > 0.0) || !isfinite(is)) {
            // samples differ but sigma underflows or overflows: outside the
            // range the library represents; the window stays indexed so
            // every count stays consistent, and the call fails
            atomicOr(q.bad, 2);
            is = 1.0;
        }
        q.cell[kk] = (uint32_t)(L.cell_base + i0 + w);
        q.mu[kk] = mu;
        q.isig[kk] = is;
        q.P[kk] = kInfBits;
        if (smu) {
            smu[w] = mu;
            sis[w] = is;
        }
    }
    __syncthreads();
}

}  // namespace

// One block per tile of 1024 consecutive windows of one length.
//  1. samples into LDS; compacted position of every non-constant window;
//     two-pass moments of those windows (one thread per window);
//  2. thread (segment g = tid / 16, bin b = tid % 16) owns bin k = b + 1 of
//     the 64 windows of segment g: it computes the bin directly at the
//     segment start (four independent phasor chains, so the sum is not one
//     long dependent chain) and slides it 63 times, in FP64;
//  3. every 8 slides the new windows' raw bins are staged in LDS, and each
//     wavefront gives the non-constant ones of its four segments their
//     records, one per lane (sketch_record), with no barrier of the block:
//     the wavefronts of a tile run their segments independently.
// Keys and join records follow in k_keys, one thread per non-constant
// window with every lane busy.
template <typename FT>
__global__ __launch_bounds__(kBlock, 3) void k_sketch(Req q, const uint32_t *__restrict__ E,
                                                      const uint32_t *__restrict__ tile_off,
                                                      int st_len, int mode) {
    extern __shared__ double dyn[];
    __shared__ SketchSmem sm;
    const int64_t tile = blockIdx.x;
    const int l = find_tile_len(q.len, q.L, tile);
    const LenInfo L = q.len[l];
    if (mode == kSketchBetween && L.anchor) return;       // done by the first pass
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
    load_tile_samples(q.t, i0, nw + m - 1, nw + m - 1, st);
    // feature slots beyond K' stay zero in every staging row
    for (int x = tid; x < kRowsC * (kFD - 2 * kp); x += kBlock)
        stage[x / (kFD - 2 * kp)][2 * kp + x % (kFD - 2 * kp)] = 0.0;

    tile_positions_and_moments(q, L, i0, nw, tile, st, E, tile_off, sm.kpos, sm.widx, sm.wsum);
    if (mode == kSketchAnchors && !L.anchor) return;      // records later, if needed
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

    // Each wavefront owns segments 4 wv .. 4 wv + 3, i.e. staging rows
    // 32 wv .. 32 wv + 31, and finishes their windows itself: from here on it
    // synchronizes with no other wavefront.
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // the record lane's 1/sigma for a chunk, loaded one chunk ahead so that
    // the slides hide its latency
    auto isig_of = [&](int chunk) -> double {
        const int row = 4 * kSlidesC * wv + lane;
        const int s = (row / kSlidesC) * kSegW + chunk * kSlidesC + (row % kSlidesC);
        const int32_t kk = lane < 4 * kSlidesC && s < nw ? sm.kpos[s] : -1;
        return kk >= 0 ? q.isig[kk] : 0.0;
    };
    double is_next = isig_of(0);
    float emax = 0.0f;
    for (int chunk = 0; chunk < kSegW / kSlidesC; ++chunk) {
        const double is_cur = is_next;
        if (chunk + 1 < kSegW / kSlidesC) is_next = isig_of(chunk + 1);
        // ---- 8 slides of every (segment, bin), raw bins into the staging rows
        if (own) {
            const int u_end = min(kSlidesC, segn - chunk * kSlidesC);
            for (int u = 0; u < u_end; ++u) {
                const int s = s0 + chunk * kSlidesC + u;
                if (s > s0) {
                    const double ya = st[s - 1] - c;
                    const double yb = st[s - 1 + m] - c;
                    const double a_r = xr - ya + yb;
                    const double a_i = xi;
                    xr = fma(a_r, wcos, -(a_i * wsin));
                    xi = fma(a_r, wsin, a_i * wcos);
                }
                double *rw = stage[g * kSlidesC + u];
                rw[2 * b] = xr;
                rw[2 * b + 1] = xi;
            }
        }
        wave_sync();
        // ---- the chunk's non-constant windows of this wavefront's segments,
        // one per lane
        if (lane < 4 * kSlidesC) {
            const int row = 4 * kSlidesC * wv + lane;
            const int sg = row / kSlidesC;
            const int s = sg * kSegW + chunk * kSlidesC + (row % kSlidesC);
            const int32_t kk = s < nw ? sm.kpos[s] : -1;
            if (kk >= 0) sketch_record<FT>(q, m, kp, stage[row], is_cur, sm.ymax[sg], kk, emax);
        }
        wave_sync();
    }
    // largest e_i of the tile: one LDS atomic per wavefront
    int eb = __float_as_int(emax);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) eb = max(eb, __shfl_xor(eb, off, kWave));
    if (lane == 0 && eb) atomicMax(&sm.emax, eb);
    __syncthreads();
    if (tid == 0 && sm.emax) atomicMax((int *)&q.emax[l], sm.emax);
}

// ------------------------------------------------------- MFMA sketch

// Precision forms 1 and 2: the projection of a block of 32 consecutive
// windows onto the truncated DFT basis is a dense product
//   X[w][f] = sum_r y_w[r] B[r][f],   y_w = t[w + .] - mu_w (by Lemma 1 the
//   shift leaves every bin k >= 1 unchanged),
//   B[r][2k-2] = cos(2 pi k r / m),  B[r][2k-1] = -sin(2 pi k r / m),
// done on the matrix cores with FP32 accumulation.  Form 1 splits the
// float values of y and B exactly into three bf16 parts each (hi + mid +
// lo) and keeps the six products of weight 2^-16 and above (hi.hi in an
// accumulator of its own, the other five in a second); only mid.lo, lo.mid
// and lo.lo (below 2^-23 of each product) are dropped, so the results are
// FP32-grade.  Form 2 uses one bf16 product.  Each window's record carries
// the derived bound e_i on its error, so the Parseval prune stays a true
// lower bound; moments stay FP64 (shared with the FP64 form).

// Basis as float values split into three bf16 parts, per length: [f (32)][r
// (m rounded up to 16)], one table per part.  Computed in FP64 from the
// exact phase (k r mod m) / m.
__global__ __launch_bounds__(kBlock) void k_basis(const LenInfo *__restrict__ len, int L,
                                                  const int64_t *__restrict__ base,
                                                  uint16_t *__restrict__ bh,
                                                  uint16_t *__restrict__ bm,
                                                  uint16_t *__restrict__ bl) {
    const int l = blockIdx.y;
    if (l >= L) return;
    const int m = len[l].m, kp = len[l].kprime;
    const int mp = (m + 15) & ~15;
    const int64_t o = base[l];
    for (int x = blockIdx.x * kBlock + threadIdx.x; x < 32 * mp; x += gridDim.x * kBlock) {
        const int f = x / mp, r = x % mp;
        const int k = f / 2 + 1;
        double v = 0.0;
        if (f < 2 * kp && r < m) {
            double sn, cs;
            sincospi(2.0 * (double)(((int64_t)k * r) % m) / (double)m, &sn, &cs);
            v = (f & 1) ? -sn : cs;
        }
        const float vf = (float)v;
        const uint32_t h = bf16_bits(vf);
        const float r1 = vf - __uint_as_float(h << 16);   // exact
        const uint32_t md = bf16_bits(r1);
        bh[o + x] = (uint16_t)h;
        bm[o + x] = (uint16_t)md;
        bl[o + x] = (uint16_t)bf16_bits(r1 - __uint_as_float(md << 16));   // exact
    }
}

namespace {
constexpr int kMBlk = 32;                     // windows per MFMA block
typedef __attribute__((ext_vector_type(8))) __bf16 mbf16x8;
typedef __attribute__((ext_vector_type(16))) float mf32x16;

__device__ __forceinline__ mbf16x8 u4_as_bf16x8(uint4 v) {
    union {
        uint4 u;
        mbf16x8 b;
    } c;
    c.u = v;
    return c.b;
}
}  // namespace

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_sketch_mfma(Req q, const uint32_t *__restrict__ E,
                                                        const uint32_t *__restrict__ tile_off,
                                                        const int64_t *__restrict__ bbase,
                                                        const uint16_t *__restrict__ bh,
                                                        const uint16_t *__restrict__ bm,
                                                        const uint16_t *__restrict__ bl, int mode) {
    extern __shared__ double dyn[];
    __shared__ int32_t kpos[kTileW];
    __shared__ uint16_t widx[kTileW];
    __shared__ uint32_t wsum[kBlock / kWave];
    __shared__ double smu[kTileW], sis[kTileW];
    __shared__ int emax_s;
    const int64_t tile = blockIdx.x;
    const int l = find_tile_len(q.len, q.L, tile);
    const LenInfo L = q.len[l];
    if (mode == kSketchBetween && L.anchor) return;       // done by the first pass
    const int m = L.m;
    const int mp = (m + 15) & ~15;
    const int64_t i0 = (tile - L.tile_base) * kTileW;
    const int nw = (int)min<int64_t>(kTileW, L.W - i0);
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / kWave;
    double *st = dyn;                              // samples, 1024 + m - 1 (+ zero pad)

    if (tid == 0) emax_s = 0;
    load_tile_samples(q.t, i0, nw + m - 1, nw + mp + kMBlk, st);
    tile_positions_and_moments(q, L, i0, nw, tile, st, E, tile_off, kpos, widx, wsum, smu, sis);
    if (mode == kSketchAnchors && !L.anchor) return;      // records later, if needed

    const uint4 *Bh = (const uint4 *)(bh + bbase[l]);
    const uint4 *Bm = (const uint4 *)(bm + bbase[l]);
    const uint4 *Bl = (const uint4 *)(bl + bbase[l]);
    const int i = lane % kMBlk, hh = lane / kMBlk;
    const double u64 = 1.1102230246251565e-16;
    // Error bound.  Each window is centred on its own mean, y = t - mu, so
    // |y|^2 = m sigma^2.  Every rounding of a component (basis row B, the
    // cos or sin of one bin) is below per * sum_r |y_r| |B_r|, and over the
    // 2K' rows sum (sum_r |y_r||B_r|)^2 <= |y|^2 sum_rows |B_row|^2 = m
    // sigma^2 K' m, since cos^2 + sin^2 = 1 at every sample (Cauchy-Schwarz).
    // The feature vector X / sigma is therefore within sqrt(K') m per.
    // per: y and B rounded to float (2 x 2^-24) and the FP64 centring and
    // chunk sums ((m / 8 + 4) u64); then, with u = 2^-8 the bf16 unit
    // roundoff and every FP32 addition rounding by up to 2^-23:
    // mid.lo + lo.mid + lo.lo <= (2 (1 + u) u^3 + u^4) < 2^-23 (|mid| <=
    // (1 + u) u |y|, |lo| <= u^2 |y|); hi.hi summed from zero per chunk of 16
    // samples (16 additions over products within (1 + u)^2 of |y_r B_r|);
    // the other five products, together below 1.03 x 2^-7 of |y_r B_r|,
    // summed from zero over groups of 4 chunks (320 additions).
    // The float and bf16 values of normal-range samples are exact splits;
    // flushed subnormals (the parts, products and partial sums of one
    // sample, at most 16 of them) add at most 2^-122 per sample in absolute
    // terms, counted separately below.
    const double per = 2.0 * 0x1.0p-24 + ((double)m / 8.0 + 4.0) * u64 + 0x1.0p-23 * 1.01 +
                       16.0 * 0x1.0p-23 * 1.01 + 320.0 * 0x1.0p-23 * 1.03 * 0x1.0p-7 * 1.01;
    const double ecomp = sqrt((double)L.kprime) * per * (double)m * (1.0 + 1e-6);
    const double eabs = sqrt(2.0 * L.kprime) * (double)m * 0x1.0p-122;
    float emax = 0.0f;
    // blocks of 32 non-constant windows, from the tile's compacted list
    // (lanes past its end project window 0 and store nothing)
    int nix = 0;
    for (int v = 0; v < kBlock / kWave; ++v) nix += (int)wsum[v];
    for (int blk = wv; blk * kMBlk < nix; blk += kBlock / kWave) {
        const int x0 = blk * kMBlk;
        const bool has = x0 + i < nix;
        const int wi = has ? (int)widx[x0 + i] : 0;
        const double mu = has ? smu[wi] : 0.0;
        const double *x = st + wi + 8 * hh;          // window i, this lane's half of each chunk

        double sum[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) sum[v] = 0.0;
        mf32x16 acc2 = {};
        // B operands of feature i, samples r0 + 8 hh .. + 7: loaded one chunk
        // ahead
        int bo = (i * mp + 8 * hh) / 8;
        uint4 nbh = Bh[bo], nbm = Bm[bo], nbl = Bl[bo];
        for (int r0 = 0; r0 < mp; r0 += 16) {
            const mbf16x8 bhv = u4_as_bf16x8(nbh);
            const mbf16x8 bmv = u4_as_bf16x8(nbm), blv = u4_as_bf16x8(nbl);
            if (r0 + 16 < mp) {
                bo += 2;
                nbh = Bh[bo];
                nbm = Bm[bo];
                nbl = Bl[bo];
            }
            // A: window i, the same samples (centred, split by the
            // hardware's round-to-nearest-even conversion of the float
            // value; the empty asm keeps the compiler from rounding the
            // FP64 difference to bf16 directly, which gives the same bits
            // through a longer sequence)
            float yf[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                yf[e] = (float)(x[r0 + e] - mu);
                asm("" : "+v"(yf[e]));
            }
            mbf16x8 ah, am, al;
#pragma unroll
            for (int e = 0; e < 8; ++e) ah[e] = (__bf16)yf[e];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                yf[e] -= (float)ah[e];                                    // exact
                am[e] = (__bf16)yf[e];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) al[e] = (__bf16)(yf[e] - (float)am[e]);   // exact
            mf32x16 acc = {};
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bhv, acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bmv, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bhv, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, blv, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bhv, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bmv, acc2, 0, 0, 0);
            // the smaller products go to FP64 every 4 chunks
            if ((r0 & 63) == 48 || r0 + 16 >= mp) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    sum[v] += (double)acc2[v];
                    acc2[v] = 0.0f;
                }
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) sum[v] += (double)acc[v];
        }
        // records: lane i holds feature i of 16 windows (rows 8 (v/4) + 4 hh
        // + v % 4); the 16 norms are summed over the 32 feature lanes together
        float fv[16], n2[16];
        int wr[16];                                   // the window of each row, or -1
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int xr = x0 + 8 * (v / 4) + 4 * hh + (v % 4);
            wr[v] = xr < nix ? (int)widx[xr] : -1;
            const double is = wr[v] >= 0 ? sis[wr[v]] : 0.0;
            fv[v] = (float)(sum[v] * is);
            n2[v] = fv[v] * fv[v];
        }
#pragma unroll
        for (int off = kMBlk / 2; off > 0; off >>= 1)
#pragma unroll
            for (int v = 0; v < 16; ++v) n2[v] += __shfl_xor(n2[v], off, kMBlk);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int w = wr[v];
            if (w >= 0) {
                const int32_t kk = kpos[w];
                const double is = sis[w];
                float *rec = (float *)q.F + (int64_t)kk * kRec;
                // the FP32 sum of 30 squares is within 32 u32 of exact
                const double nrm = sqrt((double)n2[v]) * (1.0 + 64.0 * 5.9604644775390625e-08) + 1e-30;
                // ecomp is per unit of sigma / sigma; the stored value adds
                // its float rounding and the FP64 sigma's (m + 8) u64
                const double estore = (5.9604644775390625e-08 + (m + 12.0) * u64) * nrm;
                const float e = (float)(((ecomp + eabs * is) * (1.0 + 1e-9) + estore) * (1.0 + 1e-5)) *
                                    (1.0f + 2.4e-7f) + 1e-30f;
                float val = i < kFD ? fv[v] : 0.0f;
                if (i == kSlotErr) val = e;
                if (i == kSlotNorm) val = (float)nrm * (1.0f + 2.4e-7f);
                rec[i] = val;
                emax = fmaxf(emax, e);
            }
        }
    }
    int eb = __float_as_int(emax);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) eb = max(eb, __shfl_xor(eb, off, kWave));
    if (lane == 0 && eb) atomicMax(&emax_s, eb);
    __syncthreads();
    if (tid == 0 && emax_s) atomicMax((int *)&q.emax[l], emax_s);
}

// SimHash keys, probe order and bucket sort key of every non-constant
// window of an anchor length (Sec. 3.3: only they are indexed), from its
// stored record.  Blocks are laid out per anchor length (blk_base), so the
// length's projections sit in LDS for all threads.
namespace {

// The FP32 copy f of a window's stored features (zeros when !valid), with
// the record's error bound and norm.
template <typename FT>
__device__ __forceinline__ void load_fcopy(const Req &q, int64_t kk, bool valid, float f[kFD],
                                           float &erec, float &nrec) {
    const FT *rec = (const FT *)q.F + kk * kRec;
    erec = nrec = 0.0f;
#pragma unroll
    for (int c = 0; c < kFD; ++c) f[c] = 0.0f;
    if (valid && sizeof(FT) == 8) {
#pragma unroll
        for (int p = 0; p < kFD / 2; ++p) {
            const double2 v = *(const double2 *)(rec + 2 * p);
            f[2 * p] = (float)v.x;
            f[2 * p + 1] = (float)v.y;
        }
        const double2 v = *(const double2 *)(rec + kSlotErr);
        erec = (float)v.x;
        nrec = (float)(v.y * (1.0 + 1e-7));
    } else if (valid) {
#pragma unroll
        for (int p = 0; p < 7; ++p) {
            const float4 v = *(const float4 *)(rec + 4 * p);
            f[4 * p] = v.x;
            f[4 * p + 1] = v.y;
            f[4 * p + 2] = v.z;
            f[4 * p + 3] = v.w;
        }
        const float4 v = *(const float4 *)(rec + 28);
        f[28] = v.x;
        f[29] = v.y;
        erec = v.z;
        nrec = v.w;
    }
}

// The FP32 copy as bf16 pairs: G = hi + lo, hi = bf16(f), lo = bf16(f - hi);
// each component of G is within 2^-17 of f (relative).  n2 = |G|^2 (FP64).
__device__ __forceinline__ void bf16_pairs(const float f[kFD], uint32_t hw[16], uint32_t lw[16],
                                           double &n2) {
    n2 = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        uint32_t hp = 0, lp = 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = 2 * w + e;
            const float x = c < kFD ? f[c] : 0.0f;
            const uint32_t hb = bf16_bits(x);
            const float xh = __uint_as_float(hb << 16);
            const uint32_t lb = bf16_bits(x - xh);
            const double gx = (double)xh + (double)__uint_as_float(lb << 16);
            n2 = fma(gx, gx, n2);
            hp |= hb << (16 * e);
            lp |= lb << (16 * e);
        }
        hw[w] = hp;
        lw[w] = lp;
    }
}

}  // namespace

// The threshold join's operands of the indexed windows [k0, k1), one thread
// each, written only when a join runs and only for the windows it queries
// (lengths up to the key bound): the bf16 pairs G, their metadata and the
// principal coordinates of the FP32 copy (FP64 dots) that place the grid.
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_join_ops(Req q, int64_t k0, int64_t k1) {
    const int64_t kk = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (kk >= k1) return;
    const int64_t k_first = k0 + (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1));
    const int l = find_len_k_wave(q.len, q.L, k_first, kk);
    float f[kFD];
    float erec, nrec;
    load_fcopy<FT>(q, kk, true, f, erec, nrec);
    uint32_t hw[16], lw[16];
    double n2;
    bf16_pairs(f, hw, lw, n2);
    const double *u = q.udir + (int64_t)l * kJoinDirs * 32;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
#pragma unroll
    for (int c = 0; c < kFD; ++c) {
        p0 = fma(u[c], (double)f[c], p0);
        p1 = fma(u[32 + c], (double)f[c], p1);
        p2 = fma(u[64 + c], (double)f[c], p2);
    }
    // f is within u32 |F~| of the stored record F~, itself within e of F;
    // so e' = e + (u32 + 2^-17) |F~| bounds |G - F|
    uint4 *jo = q.jop + kk * 8;
#pragma unroll
    for (int part = 0; part < 4; ++part) {
        jo[part] = make_uint4(hw[4 * part], hw[4 * part + 1], hw[4 * part + 2], hw[4 * part + 3]);
        jo[4 + part] = make_uint4(lw[4 * part], lw[4 * part + 1], lw[4 * part + 2], lw[4 * part + 3]);
    }
    // w: the join's candidate Gram term 0.5 |G|^2, rounded down (its sign
    // bit is set per certify round by the grid keys)
    q.gp[kk] = make_float4((float)p0, (float)p1, (float)p2,
                           (float)(0.5 * (double)(float)n2 * (1.0 - 0x1.0p-23)));
    const double ep =
        ((double)erec + (5.9604644775390625e-08 + 0x1.0p-17) * (double)nrec) * (1.0 + 1e-6);
    q.jmeta[kk] = make_float4((float)n2, (float)ep * (1.0f + 2.4e-7f),
                              (float)((double)nrec * (1.0 + 0x1.0p-16)) * (1.0f + 2.4e-7f), 0.0f);
}

namespace {
struct KeysSmem {
    // SimHash projections (bit x feature), bf16 hi, lo; rows of 40 (80 bytes,
    // an odd multiple of 16) so that the lanes' 16-byte reads of different
    // rows fall in different banks
    uint16_t gh[32][40], gl[32][40];
    float dots[kBlock / kWave][2][32][33];    // each wavefront's 64 x 32 projections
};

}  // namespace

template <typename FT, bool kBf16Keys>
__global__ __launch_bounds__(kBlock) void k_keys(Req q, const float *__restrict__ gproj) {
    __shared__ KeysSmem sm;
    int l;
    {
        int lo = 0, hi = q.L - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (q.len[mid].blk_base <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
        }
        l = lo;
    }
    const LenInfo L = q.len[l];
    const int tid = threadIdx.x;
    for (int x = tid; x < 32 * 32; x += kBlock) {
        const int bt = x / 32, c = x % 32;
        const float gv = bt < q.B && c < kFD ? gproj[((int64_t)l * q.B + bt) * kFD + c] : 0.0f;
        const uint32_t h = bf16_bits(gv);
        sm.gh[bt][c] = (uint16_t)h;
        sm.gl[bt][c] = (uint16_t)bf16_bits(gv - __uint_as_float(h << 16));
    }
    __syncthreads();
    const int64_t j = ((int64_t)blockIdx.x - L.blk_base) * kBlock + tid;
    // every lane takes part in the wavefront's matrix products; lanes past
    // the length's last window carry zeros and write nothing
    const bool valid = j < L.n_index;
    const int64_t kk = L.kbase + (valid ? j : 0);

    float f[kFD];
    float erec = 0.0f, nrec = 0.0f;
    load_fcopy<FT>(q, kk, valid, f, erec, nrec);
    uint32_t hw[16], lw[16];
    double n2;
    bf16_pairs(f, hw, lw, n2);

    // ---- SimHash projections <g_b, G> of the wavefront's 64 windows on the
    // matrix cores: two blocks of 32 windows x 32 bits (B used) over 32
    // features (30 used), split bf16 (hi.hi + hi.lo + lo.hi, FP32 sums;
    // within about 2^-16 |g| |f| of the FP32 dot), or with the BF16 keys of
    // precision form 2, hi.hi alone (within about 2^-7); bits near zero may
    // flip either way -- keys steer candidates only, never validity.  Operand A of a
    // block: lane L holds window (L mod 32) of the block and features
    // 8 (L / 32) .. +8 of each 16-feature slice; a lane's other half comes
    // from its partner L ^ 32.
    const int lane = lane_id();
    const int wv = tid / kWave;
    const bool upper = lane >= 32;
    const int col = lane & 31, koff = 8 * (lane >> 5);
#pragma unroll 1
    for (int bk = 0; bk < 2; ++bk) {
        // block bk holds windows 32 bk .. 32 bk + 31: the lanes of that half
        // own them, the other half holds their partners' features
        const bool own = upper == (bk == 1);
        mf32x16 c = {};
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            uint32_t ah[4], al[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t h0 = hw[8 * sl + i], h1 = hw[8 * sl + 4 + i];
                const uint32_t l0 = lw[8 * sl + i], l1 = lw[8 * sl + 4 + i];
                const uint32_t sh = (uint32_t)__shfl_xor((int)(upper ? h0 : h1), 32, kWave);
                const uint32_t sl_ = (uint32_t)__shfl_xor((int)(upper ? l0 : l1), 32, kWave);
                ah[i] = own ? (upper ? h1 : h0) : sh;
                al[i] = own ? (upper ? l1 : l0) : sl_;
            }
            const mbf16x8 Ah = u4_as_bf16x8(make_uint4(ah[0], ah[1], ah[2], ah[3]));
            const mbf16x8 Al = u4_as_bf16x8(make_uint4(al[0], al[1], al[2], al[3]));
            const mbf16x8 bh = u4_as_bf16x8(*(const uint4 *)&sm.gh[col][16 * sl + koff]);
            const mbf16x8 bl = u4_as_bf16x8(*(const uint4 *)&sm.gl[col][16 * sl + koff]);
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, bh, c, 0, 0, 0);
            if (!kBf16Keys) {
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, bl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, bh, c, 0, 0, 0);
            }
        }
        // to LDS: register r of lane L is row 8 (r / 4) + 4 (L / 32) + r % 4,
        // column L mod 32
#pragma unroll
        for (int r = 0; r < 16; ++r)
            sm.dots[wv][bk][8 * (r / 4) + 4 * (lane >> 5) + (r % 4)][col] = c[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (!valid) return;

    // ---- SimHash bits: bit b = [<g_b, F> >= 0], most significant first;
    // the margins |<g_b, F>| of the d prefix bits feed a sorted list of the
    // kProbeSlots smallest (Hamming-1 probe order, Sec. 3.4 multi-probe).
    // A list entry is the margin's bit pattern (ordered like the margin)
    // with the bit index in its low five bits.
    const float *mydots = sm.dots[wv][lane >> 5][lane & 31];
    uint32_t sig = 0;
    uint32_t top[kProbeSlots];
#pragma unroll
    for (int h = 0; h < kProbeSlots; ++h) top[h] = 0xFFFFFFFFu;
#pragma unroll 1
    for (int bt = 0; bt < q.B; ++bt) {
        const float dot = mydots[bt];
        if (dot >= 0.0f) sig |= 1u << (q.B - 1 - bt);
        if (bt < L.depth) {
            uint32_t v = (__float_as_uint(fabsf(dot)) & ~31u) | (uint32_t)bt;
#pragma unroll
            for (int h = 0; h < kProbeSlots; ++h) {
                const uint32_t lo = min(top[h], v);
                v = max(top[h], v);
                top[h] = lo;
            }
        }
    }
    uint64_t order = 0;
#pragma unroll
    for (int h = 0; h < kProbeSlots; ++h)
        if (h < L.probes) order |= (uint64_t)(top[h] & 31u) << (5 * h);
    q.keyw[kk] = (uint64_t)sig | (order << 24);
    const uint32_t prefix = L.depth ? sig >> (q.B - L.depth) : 0u;
    // the sort entries of the anchor windows only, compacted
    q.skey[L.abase + j] = ((uint32_t)l << q.key_shift) | (prefix << (q.key_shift - L.depth));
    q.sval[L.abase + j] = (uint32_t)kk;
}

// First slot of every bucket from the sorted keys: between two consecutive
// sorted entries, every bucket index in (previous, current] starts at the
// current slot (empty buckets included); the entry past the end closes the
// last buckets.  Also the slot map: slot -> cell.
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
    if (s < N) q.pcell[s] = q.cell[q.perm[s]];
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
                   int64_t ntiles, int max_m, int mode, hipStream_t s) {
    if (ntiles <= 0) return;
    // samples (1024 + m - 1 doubles, rounded up to an even count so the
    // staging rows that follow are 16-byte aligned), then the staging rows,
    // sized for the longest window of the request
    const int st_len = (kTileW + max_m + 1) & ~1;
    const size_t dyn = (size_t)(st_len + kRowsC * kStageLd) * sizeof(double);
    // the FP64 form only: the precision forms sketch on the matrix cores
    // (k_sketch_mfma)
    (void)precision;
    hipLaunchKernelGGL((k_sketch<double>), dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                       tile_off, st_len, mode);
}

int64_t basis_elems(const LenInfo *len_host, int L, std::vector<int64_t> &base) {
    base.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) base[l + 1] = base[l] + 32 * (int64_t)((len_host[l].m + 15) & ~15);
    return base[L];
}

void launch_basis(const LenInfo *len, int L, const int64_t *base, uint16_t *bh, uint16_t *bm,
                  uint16_t *bl, int max_m, hipStream_t s) {
    const int mp = (max_m + 15) & ~15;
    const unsigned gx = (unsigned)std::min<int64_t>((32 * (int64_t)mp + kBlock - 1) / kBlock, 64);
    hipLaunchKernelGGL(k_basis, dim3(gx, (unsigned)L), dim3(kBlock), 0, s, len, L, base, bh, bm,
                       bl);
}

void launch_sketch_mfma(int precision, const Req &q, const uint32_t *E, const uint32_t *tile_off,
                        int64_t ntiles, int max_m, const int64_t *bbase, const uint16_t *bh,
                        const uint16_t *bm, const uint16_t *bl, int mode, hipStream_t s) {
    if (ntiles <= 0) return;
    // samples of the tile, padded with zeros for the last block's reads
    const size_t dyn = (size_t)(kTileW + ((max_m + 15) & ~15) + kMBlk) * sizeof(double);
    // both precision forms take FP32-grade features (form 2 differs in its
    // keys only)
    (void)precision;
    hipLaunchKernelGGL(k_sketch_mfma, dim3((unsigned)ntiles), dim3(kBlock), dyn, s, q, E,
                       tile_off, bbase, bh, bm, bl, mode);
}

void launch_join_ops(int precision, const Req &q, int64_t k0, int64_t k1, hipStream_t s) {
    if (k1 <= k0) return;
    const unsigned g = (unsigned)((k1 - k0 + kBlock - 1) / kBlock);
    if (precision == 0)
        hipLaunchKernelGGL(k_join_ops<double>, dim3(g), dim3(kBlock), 0, s, q, k0, k1);
    else
        hipLaunchKernelGGL(k_join_ops<float>, dim3(g), dim3(kBlock), 0, s, q, k0, k1);
}

void launch_keys(int precision, const Req &q, int64_t nblocks, hipStream_t s) {
    if (nblocks <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL((k_keys<double, false>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, q,
                           q.gproj);
    else if (precision == 1)
        hipLaunchKernelGGL((k_keys<float, false>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, q,
                           q.gproj);
    else
        hipLaunchKernelGGL((k_keys<float, true>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, q,
                           q.gproj);
}

void launch_bucket_bounds(const Req &q, int64_t N, int64_t nbuckets, uint32_t *bstart,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_bounds, dim3(nblk(N + 1)), dim3(kBlock), 0, s, q, N, nbuckets,
                       bstart);
}

}  // namespace pmp
