// k_certify.hip -- top-k selection, exact threshold join and exact rows.
//
// Selection (paper Sec. 2 top-k rule; Sec. 3.6 final report): the greedy
// reads cells in (distance, m, i) order and accepts a cell unless an accepted
// cell of the same length lies within m/2.  Each accepted cell excludes at
// most m others, so the first k(m_max + 1) cells of that order decide the
// first k acceptances; they are found by a radix select on the FP64 bit
// pattern of the profile followed by an ordered compaction.
//
// Certificate (not in the paper): after the one pass the profile is a sound
// upper bound (Prop. 1).  Let T be the k-th value the greedy accepts on it.
// Every cell whose exact value is <= T has a partner at distance <= T, and by
// Lemma 2 that partner's true features lie within T sqrt(m/2) of its own; with
// the per-window error bounds e_i, within T sqrt(m/2) + e_q + e_c of the
// stored ones.  The join sorts each length's windows by a projection onto
// orthonormal directions and verifies, for every cell not yet at 0, all
// partners inside that radius whose certified bound is <= T.  Afterwards every
// cell with exact value <= T holds its exact value; if the greedy's k-th
// acceptance is still <= T the top-k is exact, otherwise T grows and the join
// repeats.
//
// Rows: the nearest neighbour j of each reported cell is the smallest j at
// the minimum, found by a brute-force scan of the whole row (two passes: the
// minimum, then the smallest j attaining it).
#include "pmp_dev.h"

namespace pmp {

// ---------------------------------------------------------------- select

// Histogram of bits [shift, shift + nbits) of P over cells whose bits above
// shift + nbits equal `high`.
__global__ __launch_bounds__(kBlock) void k_select_hist(const uint64_t *__restrict__ P,
                                                        int64_t n, int shift, int nbits,
                                                        uint64_t high,
                                                        unsigned int *__restrict__ hist) {
    __shared__ unsigned int h[2048];
    for (int i = threadIdx.x; i < (1 << nbits); i += kBlock) h[i] = 0;
    __syncthreads();
    const int top = shift + nbits;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const uint64_t v = P[i];
        if (v >= kInfBits) continue;                       // no value
        if (top < 64 && (v >> top) != high) continue;
        atomicAdd(&h[(v >> shift) & ((1ull << nbits) - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (1 << nbits); i += kBlock)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Per-block counts of cells equal to the pivot (for the ordered compaction).
constexpr int kSelTile = kBlock * 16;

__global__ __launch_bounds__(kBlock) void k_select_count(const uint64_t *__restrict__ P, int64_t n,
                                                         uint64_t pivot,
                                                         uint32_t *__restrict__ cnt) {
    __shared__ uint32_t wc[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kSelTile;
    uint32_t c = 0;
    for (int r = 0; r < 16; ++r) {
        int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        if (i < n && P[i] == pivot) ++c;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (lane_id() == 0) wc[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int k = 0; k < kBlock / kWave; ++k) s += wc[k];
        cnt[blockIdx.x] = s;
    }
}

// Cells below the pivot are appended (any order); cells equal to the pivot are
// written in natural order up to `need` of them.
__global__ __launch_bounds__(kBlock) void k_select_emit(const uint64_t *__restrict__ P, int64_t n,
                                                        uint64_t pivot, uint32_t need,
                                                        const uint32_t *__restrict__ off,
                                                        uint32_t *__restrict__ less,
                                                        uint64_t *__restrict__ less_val,
                                                        uint32_t *__restrict__ nless, uint32_t cap,
                                                        uint32_t *__restrict__ eq) {
    __shared__ uint32_t wc[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kSelTile;
    uint32_t run = off[blockIdx.x];
    if (run >= need) {
        // still emit the cells below the pivot
        for (int r = 0; r < 16; ++r) {
            int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
            if (i < n && P[i] < pivot) {
                uint32_t p = atomicAdd(nless, 1u);
                if (p < cap) {
                    less[p] = (uint32_t)i;
                    less_val[p] = P[i];
                }
            }
        }
        return;
    }
    for (int r = 0; r < 16; ++r) {
        int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        const bool ok = i < n;
        const uint64_t v = ok ? P[i] : kInfBits;
        if (ok && v < pivot) {
            uint32_t p = atomicAdd(nless, 1u);
            if (p < cap) {
                less[p] = (uint32_t)i;
                less_val[p] = v;
            }
        }
        const bool e = ok && v == pivot;
        const uint64_t bal = __ballot(e);
        if (lane_id() == 0) wc[threadIdx.x / kWave] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t pos = run + (uint32_t)__popcll(bal & lanemask_lt());
        uint32_t tot = 0;
        for (int k = 0; k < kBlock / kWave; ++k) {
            if (k < (int)(threadIdx.x / kWave)) pos += wc[k];
            tot += wc[k];
        }
        if (e && pos < need) eq[pos] = (uint32_t)i;
        run += tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ join

// Join sort key: length index in the high bits, quantized first projection
// below.  Quantization is monotone, so a band [p - r, p + r] maps to a key
// range.
__device__ __forceinline__ uint32_t jquant(float p, float R, int jshift) {
    const double scale = (double)(1u << jshift) / (2.0 * (double)R);
    double x = ((double)p + (double)R) * scale;
    if (!(x > 0.0)) return 0u;
    const double top = (double)((1u << jshift) - 1u);
    if (x >= top) return (1u << jshift) - 1u;
    return (uint32_t)x;
}

__global__ __launch_bounds__(kBlock) void k_join_keys(Req q, const float *__restrict__ prange,
                                                      int64_t N, uint32_t *__restrict__ jk,
                                                      uint32_t *__restrict__ jv) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= N) return;
    const int l = find_len_k(q.len, q.L, k);
    const float p = q.jrec[k * 8];
    jk[k] = ((uint32_t)l << q.jkey_shift) | jquant(p, prange[l], q.jkey_shift);
    jv[k] = (uint32_t)k;
}

__global__ __launch_bounds__(kBlock) void k_join_gather(const float *__restrict__ jrec,
                                                        const uint32_t *__restrict__ jperm,
                                                        int64_t N, float *__restrict__ jsorted) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    const float4 *src = (const float4 *)(jrec + (int64_t)jperm[p] * 8);
    float4 *dst = (float4 *)(jsorted + p * 8);
    dst[0] = src[0];
    dst[1] = src[1];
}

// One lane per sorted position searches its band (lane-parallel filters and
// bounds); the wavefront verifies the proposals one per lane per round with
// the canonical distance.  The exact distance lowers both cells.
// Join queries: the indexed windows not yet at 0, in (length, start) order,
// as positions of the join order (wave-aggregated append).
__global__ __launch_bounds__(kBlock) void k_join_queries(Req q, const uint32_t *__restrict__ jinv,
                                                         int64_t N, uint32_t *__restrict__ jq,
                                                         uint32_t *__restrict__ count) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool want = k < N && q.P[k] != 0ull;
    const uint64_t bal = __ballot(want);
    uint32_t base = 0;
    if (lane_id() == 0 && bal) base = atomicAdd(count, (uint32_t)__popcll(bal));
    base = __shfl(base, 0, kWave);
    if (want) jq[base + __popcll(bal & lanemask_lt())] = jinv[k];
}

template <typename FT>
__global__ __launch_bounds__(kBlock) void k_join(Req q, const float *__restrict__ js,
                                                 const uint32_t *__restrict__ jkey,
                                                 const JoinLen *__restrict__ jl,
                                                 const uint32_t *__restrict__ jq, int64_t nq,
                                                 int64_t N, double T) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t n_cand = 0, n_ver = 0;
    bool done = k >= nq;
    const int64_t p = done ? 0 : (int64_t)jq[k];
    uint32_t kq = 0, klo = 0, khi = 0;
    double Pq = 0.0, muq = 0.0, isq = 0.0;
    int m = 0;
    int64_t iq = 0, cell_base = 0;
    float sqrt2m = 0.0f, rf2 = 0.0f;
    bool inf_r = false;
    float pq[kJoinDims];
    const FT *fq = (const FT *)q.F;
    if (!done) {
        const float *rq = js + p * 8;
        kq = __float_as_uint(rq[6]);
        Pq = bitsd(q.P[kq]);
        done = Pq == 0.0;
        if (!done) {
            const int l = find_len_k(q.len, q.L, kq);
            const LenInfo L = q.len[l];
            const JoinLen J = jl[l];
            m = L.m;
            cell_base = L.cell_base;
            sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
            iq = (int64_t)q.cell[kq] - cell_base;
            muq = q.mu[kq];
            isq = q.isig[kq];
            fq += (int64_t)kq * kRec;
#pragma unroll
            for (int x = 0; x < kJoinDims; ++x) pq[x] = rq[x];
            const uint32_t lbase = (uint32_t)l << q.jkey_shift;
            inf_r = !isfinite(J.r_key);
            klo = inf_r ? lbase : lbase | jquant(pq[0] - J.r_key, J.prange, q.jkey_shift);
            khi = inf_r ? (lbase | ((1u << q.jkey_shift) - 1u))
                        : lbase | jquant(pq[0] + J.r_key, J.prange, q.jkey_shift);
            rf2 = J.r_filter * J.r_filter;
        }
    }
    int dir = 0;
    int64_t c = p - 1;
    bool has = false;
    uint32_t pc = 0;
    int64_t pic = 0;
    double pmu = 0.0, pis = 0.0;
    for (;;) {
        while (!done && !has) {
            if (dir == 0) {
                if (c < 0 || jkey[c] < klo) { dir = 1; c = p + 1; continue; }
            } else if (c >= N || jkey[c] > khi) {
                done = true;
                break;
            }
            const int64_t cur = c;
            c += dir == 0 ? -1 : 1;
            const float *rc = js + cur * 8;
            if (!inf_r) {
                float s2 = 0.0f;
#pragma unroll
                for (int x = 0; x < kJoinDims; ++x) {
                    const float e = rc[x] - pq[x];
                    s2 = fmaf(e, e, s2);
                }
                if (!(s2 <= rf2)) continue;
            }
            const uint32_t kc = __float_as_uint(rc[6]);
            const int64_t ic = (int64_t)q.cell[kc] - cell_base;
            const int64_t gap = ic > iq ? ic - iq : iq - ic;
            if (gap < q.excl) continue;
            ++n_cand;
            const float lb = lb_mem<FT>(fq, (const FT *)q.F + (int64_t)kc * kRec, sqrt2m);
            if ((double)lb > T || (double)lb >= Pq) continue;
            has = true;
            pc = kc;
            pic = ic;
            pmu = q.mu[kc];
            pis = q.isig[kc];
        }
        const uint64_t mask = __ballot(has);
        if (mask == 0) break;
        verify_proposals(mask, q.t, iq, muq, isq, pic, pmu, pis, m,
                         [&](double dd) {
                             ++n_ver;
                             const unsigned long long db = (unsigned long long)dbits(dd);
                             if (dd < Pq) {
                                 atomicMin((unsigned long long *)&q.P[kq], db);
                                 Pq = dd;
                             }
                             atomicMin((unsigned long long *)&q.P[pc], db);
                             has = false;
                             if (Pq == 0.0) done = true;
                         });
    }
    unsigned long long a = n_cand, v = n_ver;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, kWave);
        v += __shfl_xor(v, off, kWave);
    }
    if (lane_id() == 0) {
        if (a) atomicAdd(&q.counters[C_JOIN_CAND], a);
        if (v) atomicAdd(&q.counters[C_JOIN_VER], v);
    }
}

// ------------------------------------------------------------------ rows

// Pass 1 (find_min = 1): out_min[c] = min over valid j of the snapped
// distance.  Pass 2: out_arg[c] = smallest valid j whose snapped distance
// equals req[c].target.  Constant windows are not indexed and never scanned.
// Each 16-lane group takes every (groups)-th window of the length.
__global__ __launch_bounds__(kBlock) void k_rows(Req q, const RowReq *__restrict__ rr, int find_min,
                                                 unsigned long long *__restrict__ out_min,
                                                 unsigned long long *__restrict__ out_arg) {
    const RowReq R = rr[blockIdx.y];
    const LenInfo L = q.len[R.l];
    const int m = L.m;
    const int64_t i = (int64_t)q.cell[R.k] - L.cell_base;
    const double mui = q.mu[R.k], isi = q.isig[R.k];
    constexpr int kGroupsPerBlock = kBlock / kGroup;
    const int64_t g0 = (int64_t)blockIdx.x * kGroupsPerBlock + threadIdx.x / kGroup;
    const int64_t ng = (int64_t)gridDim.x * kGroupsPerBlock;
    // every group runs the same number of iterations (uniform control flow)
    const int64_t iters = (L.n_index + ng - 1) / ng;
    unsigned long long best = find_min ? (unsigned long long)kInfBits : ~0ull;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t x = g0 + it * ng;
        bool ok = x < L.n_index;
        const int64_t kc = L.kbase + (ok ? x : 0);
        const int64_t j = (int64_t)q.cell[kc] - L.cell_base;
        const int64_t gap = j > i ? j - i : i - j;
        ok = ok && gap >= q.excl;
        const double dd = snap(group_zdist(q.t, i, mui, isi, ok ? j : i, ok ? q.mu[kc] : 0.0,
                                           ok ? q.isig[kc] : 0.0, ok ? m : 0));
        if (ok) {
            const unsigned long long b = (unsigned long long)dbits(dd);
            if (find_min) best = b < best ? b : best;
            else if (b == R.target && (unsigned long long)j < best) best = (unsigned long long)j;
        }
    }
    // all lanes of a group hold the same value; reduce across the wave
    for (int off = kGroup; off < kWave; off <<= 1) {
        const unsigned long long o = __shfl_xor(best, off, kWave);
        best = o < best ? o : best;
    }
    if (lane_id() == 0) {
        if (find_min) atomicMin(&out_min[blockIdx.y], best);
        else if (best != ~0ull) atomicMin(&out_arg[blockIdx.y], best);
    }
}

// out[x] = src[idx[x]]
__global__ __launch_bounds__(kBlock) void k_gather_u32(const uint32_t *__restrict__ src,
                                                       const uint32_t *__restrict__ idx, int64_t n,
                                                       uint32_t *__restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x < n) out[x] = src[idx[x]];
}

// ------------------------------------------------------------ utilities

__global__ __launch_bounds__(kBlock) void k_fill_u64(uint64_t *__restrict__ p, int64_t n,
                                                     uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
static inline unsigned gridcap(int64_t n, int64_t cap) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (unsigned)(b < cap ? b : cap);
}

void launch_select_hist(const uint64_t *P, int64_t n, int shift, int nbits, uint64_t high,
                        unsigned int *hist, hipStream_t s) {
    hipLaunchKernelGGL(k_select_hist, dim3(gridcap(n, 4096)), dim3(kBlock), 0, s, P, n, shift,
                       nbits, high, hist);
}

int64_t select_blocks(int64_t n) { return (n + kSelTile - 1) / kSelTile; }

void launch_select_count(const uint64_t *P, int64_t n, uint64_t pivot, uint32_t *cnt,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_select_count, dim3((unsigned)select_blocks(n)), dim3(kBlock), 0, s, P, n,
                       pivot, cnt);
}

void launch_select_emit(const uint64_t *P, int64_t n, uint64_t pivot, uint32_t need,
                        const uint32_t *off, uint32_t *less, uint64_t *less_val, uint32_t *nless,
                        uint32_t cap, uint32_t *eq, hipStream_t s) {
    hipLaunchKernelGGL(k_select_emit, dim3((unsigned)select_blocks(n)), dim3(kBlock), 0, s, P, n,
                       pivot, need, off, less, less_val, nless, cap, eq);
}

void launch_join_keys(const Req &q, const float *prange, int64_t N, uint32_t *jk, uint32_t *jv,
                      hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_join_keys, dim3(nblk(N)), dim3(kBlock), 0, s, q, prange, N, jk, jv);
}

void launch_join_gather(const float *jrec, const uint32_t *jperm, int64_t N, float *jsorted,
                        hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_join_gather, dim3(nblk(N)), dim3(kBlock), 0, s, jrec, jperm, N,
                           jsorted);
}

void launch_join_queries(const Req &q, const uint32_t *jinv, int64_t N, uint32_t *jq,
                         uint32_t *count, hipStream_t s) {
    if (N > 0)
        hipLaunchKernelGGL(k_join_queries, dim3(nblk(N)), dim3(kBlock), 0, s, q, jinv, N, jq, count);
}

void launch_join(int precision, const Req &q, const float *js, const uint32_t *jkey,
                 const JoinLen *jl, const uint32_t *jq, int64_t nq, int64_t N, double T,
                 hipStream_t s) {
    if (nq <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_join<double>, dim3(nblk(nq)), dim3(kBlock), 0, s, q, js, jkey, jl, jq,
                           nq, N, T);
    else
        hipLaunchKernelGGL(k_join<float>, dim3(nblk(nq)), dim3(kBlock), 0, s, q, js, jkey, jl, jq,
                           nq, N, T);
}

void launch_rows(const Req &q, const RowReq *rr, int nrows, int64_t maxN, int find_min,
                 unsigned long long *out_min, unsigned long long *out_arg, hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_rows, dim3(gridcap(maxN / 4, 1024), (unsigned)nrows), dim3(kBlock), 0, s,
                       q, rr, find_min, out_min, out_arg);
}

void launch_gather_u32(const uint32_t *src, const uint32_t *idx, int64_t n, uint32_t *out,
                       hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather_u32, dim3(nblk(n)), dim3(kBlock), 0, s, src, idx, n, out);
}

void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_u64, dim3(gridcap(n, 8192)), dim3(kBlock), 0, s, p, n, v);
}

}  // namespace pmp
