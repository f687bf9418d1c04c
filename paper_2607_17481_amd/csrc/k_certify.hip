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
// The threshold join (k_join.hip) gives every cell whose exact value is <= T
// its exact value; if the greedy's k-th acceptance is then still <= T the
// top-k is exact, otherwise T grows and the join repeats.
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

// ------------------------------------------------------------------ rows

// One pass over each requested row c: out_min[c] = min over valid j of the
// snapped distance (the certificate's check), and out_arg[c] = smallest
// valid j whose snapped distance equals req[c].target (the reported
// neighbour when the check holds).  Constant windows are not indexed and
// never scanned.
// Each lane takes every (threads)-th window of the length and evaluates the
// canonical distance on its own (lane_zdist): neighbouring lanes read
// neighbouring windows, and the row's own window is shared by all.
__global__ __launch_bounds__(kBlock) void k_rows(Req q, const RowReq *__restrict__ rr,
                                                 unsigned long long *__restrict__ out_min,
                                                 unsigned long long *__restrict__ out_arg) {
    const RowReq R = rr[blockIdx.y];
    const LenInfo L = q.len[R.l];
    const int m = L.m;
    const int64_t i = (int64_t)q.cell[R.k] - L.cell_base;
    const double mui = q.mu[R.k], isi = q.isig[R.k];
    const int64_t nt = (int64_t)gridDim.x * kBlock;
    unsigned long long best = (unsigned long long)kInfBits, arg = ~0ull;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < L.n_index; x += nt) {
        const int64_t kc = L.kbase + x;
        const int64_t j = (int64_t)q.cell[kc] - L.cell_base;
        const int64_t gap = j > i ? j - i : i - j;
        if (gap < q.excl) continue;
        const double dd = snap(lane_zdist(q.t, i, mui, isi, j, q.mu[kc], q.isig[kc], m));
        const unsigned long long b = (unsigned long long)dbits(dd);
        best = b < best ? b : best;
        if (b == R.target && (unsigned long long)j < arg) arg = (unsigned long long)j;
    }
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned long long o = __shfl_xor(best, off, kWave);
        const unsigned long long a = __shfl_xor(arg, off, kWave);
        best = o < best ? o : best;
        arg = a < arg ? a : arg;
    }
    if (lane_id() == 0) {
        atomicMin(&out_min[blockIdx.y], best);
        if (arg != ~0ull) atomicMin(&out_arg[blockIdx.y], arg);
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

void launch_rows(const Req &q, const RowReq *rr, int nrows, int64_t maxN,
                 unsigned long long *out_min, unsigned long long *out_arg, hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_rows, dim3(gridcap(maxN, 1024), (unsigned)nrows), dim3(kBlock), 0, s,
                       q, rr, out_min, out_arg);
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
