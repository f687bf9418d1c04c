// k_join.hip -- the certificate's exact threshold join, as MFMA tiles.
//
// After the one pass the profile is a sound upper bound (Prop. 1); let T be
// the k-th value the greedy accepts on it.  A pair at distance d <= T has, by
// Lemma 2, true features within T sqrt(m/2) of each other, hence working
// vectors G (the stored features as a sum of two bf16 numbers) within
//   R = T sqrt(m/2) + e'_i + e'_j,     e' >= ||G - F|| (stored record bound
// plus the FP32 and bf16 roundings).  The join finds every such pair:
//
//  * grid: each length's windows get coordinates, the projections of their
//    FP32 feature copies f on the leading principal directions of that
//    length's features (orthonormal, so a coordinate moves by at most
//    ||df|| <= R_f = T sqrt(m/2) + e_i + e_j + u32 (|F~_i| + |F~_j|)); two of
//    them, in cells of width h >= R_f, place a pair within R_f in adjacent
//    cells (or one, in finer cells, when R_f is below the two-coordinate
//    grid's resolution), and all three must differ by at most R_f;
//  * tiles: windows sorted by (length, cell) are cut into tiles of 32; a
//    tile's candidates are the windows of the cells next to its queries' cells
//    (each a contiguous run of the order), taken 32 at a time;
//  * filter: for a 32 x 32 tile, <G_q, G_c> comes from six MFMA products in
//    bf16 with FP32 accumulation (hi.hi + hi.lo + lo.hi), and
//      ||dG||^2 = |G_q|^2 + |G_c|^2 - 2 <G_q, G_c>
//    is bounded below with a rigorous rounding margin; a pair is kept unless
//    that bound exceeds R^2;
//  * exact: kept pairs pass the exclusion test, the certified Parseval bound
//    from the stored records (<= T and below one of the two cells) and are
//    verified with the canonical FP64 distance, lowering both cells.  The
//    tiles hand their kept pairs to a buffer, and the exact stage runs as a
//    kernel of its own (k_join_verify) after each chunk of tiles: the tiles
//    walk in step as a block, so an exact stage inside them would hold the
//    block's other wavefronts at the next barrier.
//
// Every unordered pair is examined once: a pair whose other end is itself a
// query and comes earlier in the order is left to that end's tile (both ends
// see each other, since cell adjacency is symmetric and the filter is
// conservative on both sides).
#include "pmp_dev.h"

namespace pmp {

namespace {

constexpr int kJT = kJoinTile;                // queries / candidates per tile
constexpr int kQueueHigh = 128;               // kept pairs buffered before they are handed on
constexpr int kQueueCap = kQueueHigh + kJT * kJT;   // room for one more whole tile
constexpr int kCovSample = 1024;              // windows per length for the principal directions

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
    union {
        uint4 u;
        bf16x8 b;
    } c;
    c.u = v;
    return c.b;
}

// Lower bound (first index with key >= target) in the sorted keys[lo, hi),
// by a 64-ary search of the whole wavefront (uniform result).
__device__ __forceinline__ int64_t wave_lower_bound(const uint32_t *__restrict__ keys, int64_t lo,
                                                    int64_t hi, uint32_t target) {
    const int lane = lane_id();
    while (hi - lo > kWave) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t idx = lo + (int64_t)lane * step;
        const bool below = idx < hi && keys[idx] < target;
        const int cnt = __popcll(__ballot(below));
        if (cnt == 0) return lo;
        const int64_t nlo = lo + (int64_t)(cnt - 1) * step + 1;
        const int64_t nhi = min(hi, lo + (int64_t)cnt * step);
        lo = nlo;
        hi = nhi;
    }
    const int64_t idx = lo + lane;
    const bool below = idx < hi && keys[idx] < target;
    return lo + __popcll(__ballot(below));
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// G of one window, in FP64 (hi + lo is exact).
__device__ __forceinline__ void load_g(const uint4 *__restrict__ op, double g[2 * kMaxK]) {
#pragma unroll
    for (int part = 0; part < 4; ++part) {
        const uint4 h = op[part], w = op[4 + part];
        const uint32_t hs[4] = {h.x, h.y, h.z, h.w}, ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            g[8 * part + 2 * e] = (double)__uint_as_float(hs[e] << 16) +
                                  (double)__uint_as_float(ws[e] << 16);
            g[8 * part + 2 * e + 1] = (double)__uint_as_float(hs[e] & 0xFFFF0000u) +
                                      (double)__uint_as_float(ws[e] & 0xFFFF0000u);
        }
    }
}

}  // namespace

// ------------------------------------------------- principal directions

// Mean and second moments of the FP32 feature copies over an even sample of
// each length's windows: out[l] = {count, sum[32], sum of products [32 x 32]
// (upper)}.
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_join_cov(Req q, double *__restrict__ out) {
    __shared__ float rows[64][2 * kMaxK + 1];
    const int l = blockIdx.x;
    const LenInfo L = q.len[l];
    const int64_t n = L.n_index;
    const int S = (int)min<int64_t>(n, kCovSample);
    double *o = out + (int64_t)l * (1 + 32 + 32 * 32);
    // thread -> pairs (a <= b < 32) of the upper triangle, or a sum entry
    double acc[5] = {0, 0, 0, 0, 0};
    int pa[5], pb[5];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
        int p = threadIdx.x + x * kBlock;           // 0 .. 1279: 528 pairs, then 32 sums
        pa[x] = -1;
        pb[x] = -1;
        if (p < 528) {
            int a = 0;
            while (p >= 32 - a) { p -= 32 - a; ++a; }
            pa[x] = a;
            pb[x] = a + p;
        } else if (p < 528 + 32) {
            pa[x] = p - 528;
            pb[x] = 32;                              // the sum entry
        }
    }
    for (int s0 = 0; s0 < S; s0 += 64) {
        __syncthreads();
        for (int x = threadIdx.x; x < 64 * 32; x += kBlock) {
            const int r = x / 32, c = x % 32;
            float v = 0.0f;
            if (s0 + r < S && c < 2 * (kMaxK - 1)) {
                const int64_t k = L.kbase + (int64_t)(((double)(s0 + r) + 0.5) * (double)n / (double)S);
                v = (float)((const FT *)q.F)[k * kRec + c];
            }
            rows[r][c] = v;
        }
        if (threadIdx.x < 64) rows[threadIdx.x][32] = 1.0f;
        __syncthreads();
        const int rn = min(64, S - s0);
        for (int r = 0; r < rn; ++r) {
#pragma unroll
            for (int x = 0; x < 5; ++x)
                if (pa[x] >= 0) acc[x] = fma((double)rows[r][pa[x]], (double)rows[r][pb[x]], acc[x]);
        }
    }
    if (threadIdx.x == 0) o[0] = (double)S;
#pragma unroll
    for (int x = 0; x < 5; ++x) {
        if (pa[x] < 0) continue;
        if (pb[x] == 32) o[1 + pa[x]] = acc[x];
        else o[33 + pa[x] * 32 + pb[x]] = acc[x];
    }
}

namespace {
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
}  // namespace

// The kJoinDirs leading principal directions of each length's sample (power
// iteration on the covariance, each deflated against the ones before), made
// orthonormal in FP64; one wavefront per length, lane i holds component i.
// Any orthonormal set keeps the threshold join exact; the leading directions
// make its cells selective.  udir[l][v][0..31] (components 30, 31 are 0).
__global__ __launch_bounds__(kWave) void k_pca(const double *__restrict__ cov, int L,
                                               double *__restrict__ udir) {
    constexpr int D = 2 * (kMaxK - 1);
    __shared__ double C[D][D + 1];
    __shared__ double xs[32];
    const int l = blockIdx.x;
    if (l >= L) return;
    const int i = threadIdx.x;
    const double *c = cov + (int64_t)l * (1 + 32 + 32 * 32);
    const double S = c[0];
    if (i < D)
        for (int b = 0; b < D; ++b) {
            const int lo = min(i, b), hi = max(i, b);
            C[i][b] = S >= 2.0 ? c[33 + lo * 32 + hi] / S - (c[1 + i] / S) * (c[1 + b] / S) : 0.0;
        }
    __syncthreads();
    double u[kJoinDirs];
    for (int v = 0; v < kJoinDirs; ++v) {
        double x = i < D ? 1.0 + 0.37 * ((i * (v + 3)) % 7) - 0.5 * (i % (v + 2)) : 0.0;
        // deflate against the directions before, then normalize
        for (int w = 0; w < v; ++w) x -= wave_sum_d(x * u[w]) * u[w];
        double nn = sqrt(wave_sum_d(x * x));
        if (nn > 1e-300) {
            x /= nn;
            for (int it = 0; it < 64; ++it) {
                __syncthreads();
                if (i < 32) xs[i] = x;
                __syncthreads();
                double y = 0.0;
                if (i < D)
                    for (int j = 0; j < D; ++j) y = fma(C[i][j], xs[j], y);
                for (int w = 0; w < v; ++w) y -= wave_sum_d(y * u[w]) * u[w];
                const double ny = sqrt(wave_sum_d(y * y));
                if (!(ny > 1e-300)) break;
                x = y / ny;
            }
        }
        // exact orthonormality against the ones before (twice, for
        // rounding); a degenerate vector falls back to a unit vector
        for (int e = 0;; ++e) {
            for (int r = 0; r < 2; ++r)
                for (int w = 0; w < v; ++w) x -= wave_sum_d(x * u[w]) * u[w];
            const double nx = sqrt(wave_sum_d(x * x));
            if (nx > 1e-300) { x /= nx; break; }
            x = i == e ? 1.0 : 0.0;
        }
        for (int r = 0; r < 2; ++r) {
            for (int w = 0; w < v; ++w) x -= wave_sum_d(x * u[w]) * u[w];
            x /= sqrt(wave_sum_d(x * x));
        }
        u[v] = i < D ? x : 0.0;
        if (i < 32) udir[((int64_t)l * kJoinDirs + v) * 32 + i] = u[v];
    }
}

// ------------------------------------------------------------ grid keys

// Sort key (length, cell1, cell2) and value k of every indexed window (from
// its principal coordinates, computed by k_keys), and its query flag (cell
// not yet at 0) for this round.  With cb2 = 0 the grid
// has one coordinate only, in finer cells (a band), for radii below the
// resolution of the two-coordinate grid.
__global__ __launch_bounds__(kBlock) void k_grid_keys(Req q, const GridLen *__restrict__ gl,
                                                      int64_t N, int cb1, int cb2, int cb3,
                                                      int l_lim, int64_t i_lim,
                                                      uint32_t *__restrict__ gkey,
                                                      uint32_t *__restrict__ gval,
                                                      uint8_t *__restrict__ qf,
                                                      float4 *__restrict__ gp) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= N) return;
    const int64_t k_first = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1));
    const int l = find_len_k_wave(q.len, q.L, k_first, k);
    const GridLen &G = gl[l];
    const float4 c = gp[k];
    const double p1 = c.x, p2 = c.y, p3 = c.z;
    auto cell = [&](double p, int bits, double hinv) -> uint32_t {
        const uint32_t top = (1u << bits) - 1u;
        const double x = (p - G.qlo) * hinv;
        if (!(x > 0.0)) return 0u;
        if (x >= (double)top) return top;
        return (uint32_t)x;
    };
    gkey[k] = ((uint32_t)l << (cb1 + cb2 + cb3)) | (cell(p1, cb1, G.hinv) << (cb2 + cb3)) |
              (cb2 ? cell(p2, cb2, G.hinv2) << cb3 : 0u) | (cb3 ? cell(p3, cb3, G.hinv2) : 0u);
    gval[k] = (uint32_t)k;
    // a query: a cell not yet at 0 whose (length, start) lies at or before
    // the bound (the bound is the last length when it does not apply)
    const int64_t i = (int64_t)q.cell[k] - q.len[l].cell_base;
    const bool f = q.P[k] != 0ull && (l < l_lim || (l == l_lim && i <= i_lim));
    qf[k] = f;
    // the same flag in the sign of the candidate's Gram term, so that a
    // candidate tile reads one 16-byte word per window besides its operands
    gp[k].w = f ? -fabsf(c.w) : fabsf(c.w);
}

// The join operands and coordinates in sorted (grid) order, so that a tile
// of the order reads one contiguous block, with no index load before it.
__global__ __launch_bounds__(kBlock) void k_join_gather(const uint32_t *__restrict__ gval,
                                                        const uint4 *__restrict__ jop,
                                                        const float4 *__restrict__ gp, int64_t n,
                                                        uint4 *__restrict__ jop_s,
                                                        float4 *__restrict__ gp_s) {
    // eight threads per window: one 16-byte part of its operands each
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t pos = x >> 3;
    const int part = (int)(x & 7);
    if (pos >= n) return;
    const uint32_t k = gval[pos];
    jop_s[pos * 8 + part] = jop[(int64_t)k * 8 + part];
    if (part == 0) gp_s[pos] = gp[k];
}

// ------------------------------------------------------------ the tiles

// The exact stage of kept pairs, one pair (ki, kc) of indexed windows of one
// length per lane (whole wavefront; `valid` false on lanes without one).  A
// pair outside the exclusion zone gets the certified Parseval bound from the
// stored records, and if the bound leaves it able to lower one of its cells
// below T, the canonical FP64 distance, which lowers both cells.  The
// window's loads are issued together (one memory latency before the tests).
// Returns the distances this lane's pair needed (0 or 1).  kLean: the form
// with the fewest registers (no record bound, one term per lane per load):
// a pair the bound would have skipped then has its distance computed and
// discarded at the exit bound, which leaves every cell as the full form does.
template <typename FT, bool kLaneForm, bool kLean = false>
__device__ __forceinline__ uint32_t join_exact(const Req &q, bool valid, uint32_t ki, uint32_t kc,
                                               int m, int64_t cell_base, float sqrt2m, double T) {
    bool has = false;
    int64_t si = 0, sc = 0;
    double Pi = 0.0, Pc = 0.0, mui = 0.0, isi = 0.0, muc = 0.0, isc = 0.0, lim = INFINITY;
    if (valid) {
        si = (int64_t)q.cell[ki] - cell_base;
        sc = (int64_t)q.cell[kc] - cell_base;
        Pi = bitsd(q.P[ki]);
        Pc = bitsd(q.P[kc]);
        mui = q.mu[ki];
        isi = q.isig[ki];
        muc = q.mu[kc];
        isc = q.isig[kc];
        const int64_t gap = si > sc ? si - sc : sc - si;
        const double thr = fmin(T, fmax(Pi, Pc));
        if (gap >= q.excl && thr > 0.0) {
            const float lb = kLean ? 0.0f
                                   : lb_mem<FT>((const FT *)q.F + (int64_t)ki * kRec,
                                                (const FT *)q.F + (int64_t)kc * kRec, sqrt2m);
            if ((double)lb <= T && ((double)lb < Pi || (double)lb < Pc)) {
                has = true;
                lim = exit_bound(thr);
            }
        }
    }
    uint32_t n_ver = 0;
    const uint64_t mask = __ballot(has);
    if (mask) {
        uint64_t *P = q.P;
        verify_proposals<kLaneForm, kLean ? 1 : kZBatch>(mask, SeriesA{q.t}, q.t, si, mui, isi, sc,
                                                         muc, isc, m,
                                    [&](double dd) {
            ++n_ver;
            const unsigned long long db = (unsigned long long)dbits(dd);
            if (dd < Pi) atomicMin((unsigned long long *)&P[ki], db);
            if (dd < Pc) atomicMin((unsigned long long *)&P[kc], db);
        }, lim);
    }
    return n_ver;
}

// A block of kJB wavefronts takes kJB consecutive query tiles of 32 sorted
// windows of one length.  It walks the candidate runs of the union of their
// queries' neighbourhoods together, and each candidate tile is loaded once
// by the whole block into LDS (double-buffered: the next tile's loads are in
// flight while the current one goes through the matrix cores and the
// filter) and read from there by every wavefront, so the kJB query tiles,
// whose neighbourhoods nearly coincide, share its global traffic.  Every
// wavefront keeps its own queries, filter terms and queue of kept pairs (as
// window indices (k_q, k_c)).  A full queue is copied to the pair buffer,
// whose pairs k_join_verify takes after the launch; a wavefront that finds
// the buffer full runs the exact stage of the rest in place.  The launch
// covers the blocks [blk0, blk0 + gridDim.x) of the round.
constexpr int kJB = kJoinBlock;               // query tiles (wavefronts) per block
constexpr int kJRow = 9;                      // uint4 per LDS operand row (8 + 1: no bank conflicts)

template <typename FT>
__global__ __launch_bounds__(kJB * kWave) __attribute__((amdgpu_waves_per_eu(3)))
void k_join_tiles(Req q, const GridLen *__restrict__ gl, const uint32_t *__restrict__ gkey,
                  const uint32_t *__restrict__ gval, const uint8_t *__restrict__ qf,
                  const uint4 *__restrict__ jop_s, const float4 *__restrict__ jmeta,
                  const float4 *__restrict__ gp_s, int cb1, int cb2, int cb3, double T,
                  int64_t blk0, uint2 *__restrict__ pairs, unsigned long long *__restrict__ pcount,
                  int64_t cap) {
    __shared__ uint2 queue[kJB][kQueueCap];
    __shared__ uint32_t rowk[kJB][kJT];               // the queries' window indices
    __shared__ uint32_t ck[2][kJT];                   // the candidates' window indices
    __shared__ float roww[kJB][kJT];                  // the queries' Gram filter terms
    __shared__ float4 rowc[kJB][kJT];                 // the queries' principal coordinates
    __shared__ uint4 cop[2][kJT][kJRow];              // candidate operands, two tiles
    __shared__ float4 cgp[2][kJT];                    // candidate coordinates and Gram terms
    __shared__ int red[2][kJB];                       // block reductions
    const int tid = threadIdx.x;
    const int wv = tid / kWave;
    const int lane = lane_id();
    const int64_t gb = blk0 + (int64_t)blockIdx.x;
    int l;
    {
        int lo = 0, hi = q.L - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (gl[mid].blk_base <= gb) lo = mid; else hi = mid - 1;
        }
        l = lo;
    }
    const GridLen &G = gl[l];
    const LenInfo L = q.len[l];
    const int m = L.m;
    const int64_t pbeg = L.kbase, pend = L.kbase + L.n_index;
    const int64_t p0 = pbeg + ((gb - G.blk_base) * kJB + wv) * kJT;
    const int i = lane % kJT, hh = lane / kJT;
    const int64_t pq = p0 + i;
    const bool validq = pq < pend;
    const uint32_t kq = validq ? gval[pq] : 0u;
    const bool isq = validq && qf[kq];

    // block-wide min and max of one wave-uniform value per wavefront
    auto block_minmax = [&](int vmin, int vmax, int &omin, int &omax) {
        if (lane == 0) {
            red[0][wv] = vmin;
            red[1][wv] = vmax;
        }
        __syncthreads();
        omin = red[0][0];
        omax = red[1][0];
#pragma unroll
        for (int w = 1; w < kJB; ++w) {
            omin = min(omin, red[0][w]);
            omax = max(omax, red[1][w]);
        }
        __syncthreads();
    };
    {
        int none, anyq;
        block_minmax(0, __ballot(isq) ? 1 : 0, none, anyq);
        if (!anyq) return;                        // uniform over the block
    }

    // ---- query operands (A) and filter terms
    bf16x8 aH0, aH1, aL0, aL1;
    {
        const uint4 *o = jop_s + pq * 8;
        const uint4 z = make_uint4(0, 0, 0, 0);
        aH0 = as_bf16x8(isq ? o[hh] : z);
        aH1 = as_bf16x8(isq ? o[2 + hh] : z);
        aL0 = as_bf16x8(isq ? o[4 + hh] : z);
        aL1 = as_bf16x8(isq ? o[6 + hh] : z);
    }
    float a = INFINITY;                                   // filter term of query i
    if (isq) {
        const float4 mt = jmeta[kq];                      // |G|^2, e', |G| bound, 0
        const double nG2 = (double)mt.x * (1.0 - 0x1.0p-23);
        double v = 0.5 * (nG2 - G.R2) - G.eps_c * (double)mt.z - 1e-30;
        v -= 0x1.0p-22 * (fabs(v) + G.nmax2);
        a = (float)v;
    }
    if (hh == 0) {
        roww[wv][i] = a;
        rowk[wv][i] = kq;
        rowc[wv][i] = isq ? gp_s[pq] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }

    // ---- the rows of adjacent cells, over the block's queries
    const uint32_t mask1 = (1u << cb1) - 1u, mask2 = (1u << cb2) - 1u, mask3 = (1u << cb3) - 1u;
    const uint32_t key_q = validq ? gkey[pq] : 0u;
    const int c1q = (int)((key_q >> (cb2 + cb3)) & mask1), c2q = (int)((key_q >> cb3) & mask2);
    const int c3q = (int)(key_q & mask3);
    int c1min, c1max;
    block_minmax(wave_min_i(isq ? c1q : INT_MAX), wave_max_i(isq ? c1q : -1), c1min, c1max);
    const uint32_t lbits = (uint32_t)l << (cb1 + cb2 + cb3);
    unsigned long long n_pairs = 0, n_kept = 0, n_ver = 0;
    int qn = 0;                                           // queued pairs (wave-uniform)

    // hand the queued pairs of this wavefront to the pair buffer: one
    // reservation for the whole queue; the part past the buffer's end gets
    // the exact stage here
    auto spill = [&]() {
        // the queue is written and read by lanes of this wavefront only
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(pcount, (unsigned long long)qn);
            n_kept += (unsigned long long)qn;
        }
        base = __shfl(base, 0, kWave);
        const int fit = base >= (unsigned long long)cap
                            ? 0 : (int)min((unsigned long long)qn, (unsigned long long)cap - base);
        for (int e = lane; e < fit; e += kWave) pairs[base + e] = queue[wv][e];
        for (int b = fit; b < qn; b += kWave) {
            const int e = b + lane;
            const uint2 pr = e < qn ? queue[wv][e] : make_uint2(0u, 0u);
            n_ver += join_exact<FT, false, true>(q, e < qn, pr.x, pr.y, m, L.cell_base, G.sqrt2m, T);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        qn = 0;
    };

    // the block's candidate runs (one per grid row next to a query's cell);
    // every decision below is uniform over the block, so that every
    // wavefront passes the same barriers
    int c1p = max(c1min - kJoinNb, 0) - 1;
    const int c1end = min(c1max + kJoinNb, (int)mask1);
    int64_t c0 = 0, cend = 0;
    int c2p = 0, c2end = -1;                              // three coordinates: the row's c2 range
    // move [c0, cend) to the next non-empty run once the current one is used
    // up; false when there is none
    auto next_run = [&]() -> bool {
        if (cb3 > 0) {
            // three coordinates: one run per pair of adjacent (c1, c2) cells,
            // over the c3 cells next to the queries of that pair
            while (c0 >= cend && (c2p < c2end || c1p < c1end)) {
                if (c2p >= c2end) {
                    ++c1p;
                    const bool near1 = isq && abs(c1q - c1p) <= kJoinNb;
                    int lo2, hi2;
                    block_minmax(wave_min_i(near1 ? max(c2q - kJoinNb, 0) : INT_MAX),
                                 wave_max_i(near1 ? min(c2q + kJoinNb, (int)mask2) : -1), lo2, hi2);
                    if (lo2 > hi2) continue;
                    c2p = lo2 - 1;
                    c2end = hi2;
                    continue;
                }
                ++c2p;
                const bool near = isq && abs(c1q - c1p) <= kJoinNb && abs(c2q - c2p) <= kJoinNb;
                int c3lo, c3hi;
                block_minmax(wave_min_i(near ? max(c3q - kJoinNb, 0) : INT_MAX),
                             wave_max_i(near ? min(c3q + kJoinNb, (int)mask3) : -1), c3lo, c3hi);
                if (c3lo > c3hi) continue;
                const uint32_t rk = lbits | ((uint32_t)c1p << (cb2 + cb3)) | ((uint32_t)c2p << cb3);
                c0 = wave_lower_bound(gkey, pbeg, pend, rk | (uint32_t)c3lo);
                cend = wave_lower_bound(gkey, c0, pend, (rk | (uint32_t)c3hi) + 1u);
            }
        } else if (cb2 == 0) {
            // one coordinate: the cells next to the queries' cells form a
            // single run of the order
            if (c0 >= cend && c1p < c1end) {
                const uint32_t klo = lbits | (uint32_t)(c1p + 1);
                c1p = c1end;
                c0 = wave_lower_bound(gkey, pbeg, pend, klo);
                cend = wave_lower_bound(gkey, c0, pend, (lbits | (uint32_t)c1end) + 1u);
            }
        } else {
            while (c0 >= cend && c1p < c1end) {
                ++c1p;
                const bool near = isq && abs(c1q - c1p) <= kJoinNb;
                int c2lo, c2hi;
                block_minmax(wave_min_i(near ? max(c2q - kJoinNb, 0) : INT_MAX),
                             wave_max_i(near ? min(c2q + kJoinNb, (int)mask2) : -1), c2lo, c2hi);
                if (c2lo > c2hi) continue;
                const uint32_t rk = lbits | ((uint32_t)c1p << cb2);
                c0 = wave_lower_bound(gkey, pbeg, pend, rk | (uint32_t)c2lo);
                cend = wave_lower_bound(gkey, c0, pend, (rk | (uint32_t)c2hi) + 1u);
            }
        }
        return c0 < cend;
    };
    // a candidate tile is the positions [tc0, min(tc0 + 32, tend)); the block
    // loads it with one 16-byte part of one candidate per thread (and the
    // coordinates of one candidate on each of the first 32 threads)
    const int ld_c = tid / 8, ld_part = tid % 8;
    auto load_part = [&](bool have_t, int64_t tc0, int64_t tend, uint4 &op, float4 &cg,
                         uint32_t &kc) {
        const int64_t pc = tc0 + ld_c;
        op = have_t && pc < tend ? jop_s[pc * 8 + ld_part] : make_uint4(0, 0, 0, 0);
        if (tid < kJT) {
            const int64_t pg = tc0 + tid;
            const bool in = have_t && pg < tend;
            cg = in ? gp_s[pg] : make_float4(0.0f, 0.0f, 0.0f, INFINITY);
            kc = in ? gval[pg] : 0u;
        }
    };
    auto store_part = [&](int buf, const uint4 &op, const float4 &cg, uint32_t kc) {
        cop[buf][ld_c][ld_part] = op;
        if (tid < kJT) {
            cgp[buf][tid] = cg;
            ck[buf][tid] = kc;
        }
    };

    bool have = next_run();
    int64_t tc0 = c0;
    {
        uint4 op;
        float4 cg;
        uint32_t kc = 0;
        load_part(have, tc0, cend, op, cg, kc);
        store_part(0, op, cg, kc);
    }
    __syncthreads();
    // the Gram filter terms of the 16 rows this lane holds, in registers for
    // the whole walk (rows 8 (r / 4) + 4 hh + r % 4 of the result)
    float rw[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rw[r] = roww[wv][8 * (r / 4) + 4 * hh + (r % 4)];
    int cur = 0;
    c0 += kJT;
    bool have1 = have && next_run();
    while (have) {
        // the next tile's loads, in flight through this tile's work
        const int64_t nc0 = c0, nend = cend;
        uint4 op;
        float4 cg;
        uint32_t kcn = 0;
        load_part(have1, nc0, nend, op, cg, kcn);
        // this tile: operands from LDS (lane (i, hh) holds candidate tc0 + i)
        const bf16x8 bH0 = as_bf16x8(cop[cur][i][hh]), bH1 = as_bf16x8(cop[cur][i][2 + hh]);
        const bf16x8 bL0 = as_bf16x8(cop[cur][i][4 + hh]), bL1 = as_bf16x8(cop[cur][i][6 + hh]);
        const float4 gc = cgp[cur][i];
        const float bj = fabsf(gc.w);
        f32x16 acc = {};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH0, bH0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH1, bH1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH0, bL0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH1, bL1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aL0, bH0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aL1, bH1, acc, 0, 0, 0);
        n_pairs += 16;
        // the Gram test of the 16 rows this lane holds, as a bit mask (bit r:
        // row 8 (r / 4) + 4 hh + r % 4); most tiles keep nothing
        uint32_t km = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) km |= (acc[r] >= rw[r] + bj ? 1u : 0u) << r;
        if (__ballot(km != 0u)) {
            // keep (row, candidate) unless a coordinate rules it out, the
            // candidate is a query earlier in the order (its tile takes the
            // pair) or it is the row itself (positions relative to the query
            // tile p0); each lane walks only its own passing rows
            const int pcr = (int)(tc0 + i - p0);
            const bool qc = gc.w != INFINITY && signbit(gc.w);
            uint32_t kk = 0;
            for (uint32_t b = km; b != 0u; b &= b - 1u) {
                const int r = __builtin_ctz(b);
                const int row = 8 * (r >> 2) + 4 * hh + (r & 3);
                const float4 rc = rowc[wv][row];
                if (fabsf(rc.x - gc.x) <= G.rp && fabsf(rc.y - gc.y) <= G.rp &&
                    fabsf(rc.z - gc.z) <= G.rp && pcr != row && !(qc && pcr < row))
                    kk |= 1u << r;
            }
            // queue positions: an exclusive prefix sum of the counts
            const int cnt = __popc(kk);
            int pre = cnt;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int v = __shfl_up(pre, off, kWave);
                if (lane >= off) pre += v;
            }
            const int total = __shfl(pre, kWave - 1, kWave);
            int pos = qn + pre - cnt;
            const uint32_t kcand = ck[cur][i];
            for (uint32_t b = kk; b != 0u; b &= b - 1u) {
                const int r = __builtin_ctz(b);
                queue[wv][pos++] = make_uint2(rowk[wv][8 * (r >> 2) + 4 * hh + (r & 3)], kcand);
            }
            qn += total;
            if (qn > kQueueHigh) spill();
        }
        // stage the next tile; after the barrier it is the current one
        store_part(cur ^ 1, op, cg, kcn);
        __syncthreads();
        cur ^= 1;
        have = have1;
        tc0 = nc0;
        if (have) {
            c0 += kJT;
            have1 = next_run();
        }
    }
    if (qn > 0) spill();
    // statistics: one atomic per wavefront
    for (int off = kWave / 2; off > 0; off >>= 1) {
        n_pairs += __shfl_xor(n_pairs, off, kWave);
        n_kept += __shfl_xor(n_kept, off, kWave);
        n_ver += __shfl_xor(n_ver, off, kWave);
    }
    if (lane == 0) {
        atomicAdd(&q.counters[C_JOIN_PAIRS], n_pairs);
        if (n_kept) atomicAdd(&q.counters[C_JOIN_CAND], n_kept);
        if (n_ver) atomicAdd(&q.counters[C_JOIN_VER], n_ver);
    }
}

// The exact stage of the pairs in the buffer (the first min(*pcount, cap)
// entries), one pair per lane, the wavefronts striding over the buffer.
// Pairs of one length sit together in the buffer (a queue holds one
// length), so a wavefront's pairs mostly share their window length.
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_join_verify(Req q, const GridLen *__restrict__ gl,
                                                        const uint2 *__restrict__ pairs,
                                                        const unsigned long long *__restrict__ pcount,
                                                        int64_t cap, double T) {
    const int64_t n = min((int64_t)*pcount, cap);
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    uint32_t n_ver = 0;
    for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1)); base < n;
         base += stride) {
        const int64_t e = base + lane;
        const bool valid = e < n;
        const uint2 pr = valid ? pairs[e] : make_uint2(0u, 0u);
        const int l = valid ? find_len_k(q.len, q.L, (int64_t)pr.x) : 0;
        const LenInfo &L = q.len[l];
        n_ver += join_exact<FT, true>(q, valid, pr.x, pr.y, L.m, L.cell_base, gl[l].sqrt2m, T);
    }
    unsigned long long v = n_ver;
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane == 0 && v) atomicAdd(&q.counters[C_JOIN_VER], v);
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

size_t join_cov_doubles(int L) { return (size_t)L * (1 + 32 + 32 * 32); }

void launch_join_dirs(int precision, const Req &q, int nlen, double *cov, double *udir,
                      hipStream_t s) {
    if (nlen <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_join_cov<double>, dim3((unsigned)nlen), dim3(kBlock), 0, s, q, cov);
    else
        hipLaunchKernelGGL(k_join_cov<float>, dim3((unsigned)nlen), dim3(kBlock), 0, s, q, cov);
    hipLaunchKernelGGL(k_pca, dim3((unsigned)nlen), dim3(kWave), 0, s, cov, nlen, udir);
}

void launch_grid_keys(const Req &q, const GridLen *gl, int64_t N, int cb1, int cb2, int cb3,
                      int l_lim, int64_t i_lim, uint32_t *gkey, uint32_t *gval, uint8_t *qf,
                      float4 *gp, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_grid_keys, dim3(nblk(N)), dim3(kBlock), 0, s, q, gl, N, cb1, cb2, cb3,
                       l_lim, i_lim, gkey, gval, qf, gp);
}

void launch_join_gather(const uint32_t *gval, const uint4 *jop, const float4 *gp, int64_t n,
                        uint4 *jop_s, float4 *gp_s, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_join_gather, dim3((unsigned)((n * 8 + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, gval, jop, gp, n, jop_s, gp_s);
}

void launch_join_tiles(int precision, const Req &q, const GridLen *gl, const uint32_t *gkey,
                       const uint32_t *gval, const uint8_t *qf, const uint4 *jop_s,
                       const float4 *jmeta, const float4 *gp_s, int64_t blk0, int64_t nblocks,
                       int cb1, int cb2, int cb3, double T, uint2 *pairs,
                       unsigned long long *pcount, int64_t cap, hipStream_t s) {
    if (nblocks <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_join_tiles<double>, dim3((unsigned)nblocks), dim3(kJB * kWave), 0, s,
                           q, gl, gkey, gval, qf, jop_s, jmeta, gp_s, cb1, cb2, cb3, T, blk0,
                           pairs, pcount, cap);
    else
        hipLaunchKernelGGL(k_join_tiles<float>, dim3((unsigned)nblocks), dim3(kJB * kWave), 0, s,
                           q, gl, gkey, gval, qf, jop_s, jmeta, gp_s, cb1, cb2, cb3, T, blk0,
                           pairs, pcount, cap);
}

void launch_join_verify(int precision, const Req &q, const GridLen *gl, const uint2 *pairs,
                        const unsigned long long *pcount, int64_t cap, double T, hipStream_t s) {
    // enough wavefronts to keep every SIMD busy with eight, each striding
    const int64_t want = (cap + kBlock - 1) / kBlock;
    const unsigned nb = (unsigned)(want < 2048 ? want : 2048);
    if (precision == 0)
        hipLaunchKernelGGL(k_join_verify<double>, dim3(nb), dim3(kBlock), 0, s, q, gl, pairs,
                           pcount, cap, T);
    else
        hipLaunchKernelGGL(k_join_verify<float>, dim3(nb), dim3(kBlock), 0, s, q, gl, pairs,
                           pcount, cap, T);
}

}  // namespace pmp
