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
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    const int l = find_len_slot(q.len, q.L, s);
    const float p = q.jrec[s * 8];
    jk[s] = ((uint32_t)l << q.jkey_shift) | jquant(p, prange[l], q.jkey_shift);
    jv[s] = (uint32_t)s;
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

// One lane per sorted position.  The query's own cell is lowered through an
// atomic min (each pair is reached from both of its cells).
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_join(Req q, const float *__restrict__ js,
                                                 const uint32_t *__restrict__ jkey,
                                                 const JoinLen *__restrict__ jl, int64_t N,
                                                 double T) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t n_cand = 0, n_ver = 0;
    if (p < N) {
        const float *rq = js + p * 8;
        const uint32_t sq = __float_as_uint(rq[6]);
        const uint32_t cq = q.perm[sq];
        double Pq = bitsd(q.P[cq]);
        if (Pq > 0.0) {
            const int l = find_len_slot(q.len, q.L, sq);
            const LenInfo L = q.len[l];
            const JoinLen J = jl[l];
            const int m = L.m;
            const int kp = L.kprime;
            const float sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
            const int64_t iq = (int64_t)cq - L.cell_base;
            const double muq = q.mu[cq], isq = q.isig[cq];
            const FT *fq = (const FT *)q.F + (int64_t)sq * kRec;
            float pq[kJoinDims];
#pragma unroll
            for (int k = 0; k < kJoinDims; ++k) pq[k] = rq[k];
            const uint32_t lbase = (uint32_t)l << q.jkey_shift;
            const bool inf_r = !isfinite(J.r_key);
            const uint32_t klo = inf_r ? lbase : lbase | jquant(pq[0] - J.r_key, J.prange, q.jkey_shift);
            const uint32_t khi = inf_r ? (lbase | ((1u << q.jkey_shift) - 1u))
                                       : lbase | jquant(pq[0] + J.r_key, J.prange, q.jkey_shift);
            const float rf2 = J.r_filter * J.r_filter;
            for (int dir = 0; dir < 2; ++dir) {
                for (int64_t c = dir == 0 ? p - 1 : p + 1; c >= 0 && c < N; c += dir == 0 ? -1 : 1) {
                    const uint32_t key = jkey[c];
                    if (key < klo || key > khi) break;
                    const float *rc = js + c * 8;
                    float s2 = 0.0f;
#pragma unroll
                    for (int k = 0; k < kJoinDims; ++k) {
                        float e = rc[k] - pq[k];
                        s2 = fmaf(e, e, s2);
                    }
                    if (!(s2 <= rf2) && !inf_r) continue;
                    const uint32_t sc = __float_as_uint(rc[6]);
                    const uint32_t cc = q.perm[sc];
                    const int64_t ic = (int64_t)cc - L.cell_base;
                    const int64_t gap = ic > iq ? ic - iq : iq - ic;
                    if (gap < q.excl) continue;
                    ++n_cand;
                    const FT *fc = (const FT *)q.F + (int64_t)sc * kRec;
                    const float lb = lb_safe<FT>(fq, fc, kp, sqrt2m);
                    if ((double)lb > T || (double)lb >= Pq) continue;
                    ++n_ver;
                    const double dd = snap(zdist(q.t, iq, muq, isq, ic, q.mu[cc], q.isig[cc], m));
                    if (dd < Pq) {
                        atomicMin((unsigned long long *)&q.P[cq], (unsigned long long)dbits(dd));
                        Pq = dd;
                        if (Pq == 0.0) break;
                    }
                }
                if (Pq == 0.0) break;
            }
        }
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
// equals req[c].target.
__global__ __launch_bounds__(kBlock) void k_rows(Req q, const RowReq *__restrict__ rr, int find_min,
                                                 unsigned long long *__restrict__ out_min,
                                                 unsigned long long *__restrict__ out_arg) {
    const RowReq R = rr[blockIdx.y];
    const LenInfo L = q.len[R.l];
    const int m = L.m;
    const int64_t i = R.i;
    const int64_t ci = L.cell_base + i;
    const double mui = q.mu[ci], isi = q.isig[ci];
    __shared__ unsigned long long red[kBlock / kWave];
    unsigned long long best = find_min ? (unsigned long long)kInfBits : ~0ull;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < L.W;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t gap = j > i ? j - i : i - j;
        if (gap < q.excl) continue;
        const int64_t cj = L.cell_base + j;
        const double isj = q.isig[cj];
        if (isj == 0.0) continue;
        const double dd = snap(zdist(q.t, i, mui, isi, j, q.mu[cj], isj, m));
        if (find_min) {
            unsigned long long b = (unsigned long long)dbits(dd);
            best = b < best ? b : best;
        } else if (dbits(dd) == R.target) {
            best = (unsigned long long)j < best ? (unsigned long long)j : best;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(best, off, kWave);
        best = o < best ? o : best;
    }
    if (lane_id() == 0) red[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / kWave; ++k) best = red[k] < best ? red[k] : best;
        if (find_min) atomicMin(&out_min[blockIdx.y], best);
        else atomicMin(&out_arg[blockIdx.y], best);
    }
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

void launch_join(int precision, const Req &q, const float *js, const uint32_t *jkey,
                 const JoinLen *jl, int64_t N, double T, hipStream_t s) {
    if (N <= 0) return;
    if (precision == 0)
        hipLaunchKernelGGL(k_join<double>, dim3(nblk(N)), dim3(kBlock), 0, s, q, js, jkey, jl, N, T);
    else
        hipLaunchKernelGGL(k_join<float>, dim3(nblk(N)), dim3(kBlock), 0, s, q, js, jkey, jl, N, T);
}

void launch_rows(const Req &q, const RowReq *rr, int nrows, int64_t maxW, int find_min,
                 unsigned long long *out_min, unsigned long long *out_arg, hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_rows, dim3(gridcap(maxW, 1024), (unsigned)nrows), dim3(kBlock), 0, s, q,
                       rr, find_min, out_min, out_arg);
}

void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_u64, dim3(gridcap(n, 8192)), dim3(kBlock), 0, s, p, n, v);
}

}  // namespace pmp
