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

// The radix select runs on the device from start to end: six passes of a
// histogram over 11 (the last 9) bits of the FP64 bit pattern, each followed
// by one block that picks the bin holding the `remaining`-th smallest value
// and narrows the prefix `high`.  The state lives in a SelState; the host
// reads it once, with the selected cells.

// Start state: every finite value is a candidate, the histogram is clear.
__global__ void k_select_init(SelState *__restrict__ st, int64_t need,
                              unsigned int *__restrict__ hist) {
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) {
        st->high = 0;
        st->pivot = kInfBits;
        st->remaining = need;
        st->need_eq = 0;
        st->nless = 0;
        st->done = 0;
    }
}

// Histogram of bits [shift, shift + nbits) of P over cells whose bits above
// shift + nbits equal the state's prefix.
__global__ __launch_bounds__(kBlock) void k_select_hist(const uint64_t *__restrict__ P,
                                                        int64_t n, int shift, int nbits,
                                                        const SelState *__restrict__ st,
                                                        unsigned int *__restrict__ hist) {
    if (st->done) return;
    const uint64_t high = st->high;
    __shared__ unsigned int h[kSelBins];
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

// One block of kBlock threads: the bin of the remaining-th value, then the
// histogram is cleared for the next pass.  Pass 0 also settles two cases:
// fewer finite values than wanted (take them all), and a first bin of 0,
// whose values are exact zeros (the snap leaves nothing between 0 and 1e-6).
__global__ __launch_bounds__(kBlock) void k_select_pick(unsigned int *__restrict__ hist,
                                                        int nbits, int pass, int last,
                                                        SelState *__restrict__ st) {
    __shared__ unsigned long long part[kBlock];
    constexpr int kPer = kSelBins / kBlock;
    const int nb = 1 << nbits;
    const int done = st->done;
    unsigned long long mine = 0;
    unsigned int hv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int b = threadIdx.x * kPer + u;
        hv[u] = (!done && b < nb) ? hist[b] : 0u;
        mine += hv[u];
    }
    part[threadIdx.x] = mine;
    __syncthreads();
    // inclusive scan of the per-thread sums (Hillis-Steele)
    for (int off = 1; off < kBlock; off <<= 1) {
        const unsigned long long x = threadIdx.x >= off ? part[threadIdx.x - off] : 0ull;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    if (!done) {
        const unsigned long long total = part[kBlock - 1];
        const unsigned long long rem = (unsigned long long)st->remaining;
        if (pass == 0 && total < rem) {
            if (threadIdx.x == 0) {          // fewer finite cells than needed: take all
                st->pivot = kInfBits;
                st->need_eq = 0;
                st->done = 1;
            }
        } else {
            unsigned long long cum = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
            if (cum < rem && part[threadIdx.x] >= rem) {   // exactly one thread
                int bin = threadIdx.x * kPer;
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    if (cum + hv[u] >= rem) { bin = threadIdx.x * kPer + u; break; }
                    cum += hv[u];
                }
                const unsigned long long r2 = rem - cum;
                const uint64_t high = (st->high << nbits) | (uint64_t)bin;
                st->remaining = (int64_t)r2;
                st->high = high;
                if (pass == 0 && bin == 0) {
                    st->pivot = 0;
                    st->need_eq = (int64_t)r2;
                    st->done = 1;
                } else if (last) {
                    st->pivot = high;
                    st->need_eq = (int64_t)r2;
                    st->done = 1;
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += kBlock) hist[i] = 0;
}

// Per-block counts of cells equal to the pivot (for the ordered compaction).
constexpr int kSelTile = kBlock * 16;

__global__ __launch_bounds__(kBlock) void k_select_count(const uint64_t *__restrict__ P, int64_t n,
                                                         const SelState *__restrict__ st,
                                                         uint32_t *__restrict__ cnt) {
    __shared__ uint32_t wc[kBlock / kWave];
    const uint64_t pivot = st->pivot;
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
                                                        SelState *__restrict__ st,
                                                        const uint32_t *__restrict__ off,
                                                        uint32_t *__restrict__ less,
                                                        uint64_t *__restrict__ less_val,
                                                        uint32_t cap,
                                                        uint32_t *__restrict__ eq) {
    __shared__ uint32_t wc[kBlock / kWave];
    const uint64_t pivot = st->pivot;
    const uint32_t need = (uint32_t)st->need_eq;
    uint32_t *nless = &st->nless;
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

// Cells of the selected positions: the first min(nless, cap) of `less` and
// the first need_eq of `eq`.
__global__ __launch_bounds__(kBlock) void k_select_cells(const uint32_t *__restrict__ cell,
                                                         const SelState *__restrict__ st,
                                                         const uint32_t *__restrict__ less,
                                                         const uint32_t *__restrict__ eq,
                                                         int64_t cap, uint32_t *__restrict__ less_cell,
                                                         uint32_t *__restrict__ eq_cell) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= cap) return;
    const int64_t nl = (int64_t)st->nless < cap ? (int64_t)st->nless : cap;
    if (x < nl) less_cell[x] = cell[less[x]];
    if (x < st->need_eq) eq_cell[x] = cell[eq[x]];
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

// The number of the n values of P that are 0 (the FP64 bits of +0),
// added to *out.
__global__ __launch_bounds__(kBlock) void k_count_zero(const uint64_t *__restrict__ P, int64_t n,
                                                       unsigned long long *__restrict__ out) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        c += P[i] == 0ull;
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ p, int64_t n,
                                                     uint32_t v) {
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

int64_t select_blocks(int64_t n) { return (n + kSelTile - 1) / kSelTile; }

void launch_select(const uint64_t *P, int64_t n, int64_t need, SelState *st,
                   unsigned int *hist, uint32_t *cnt, uint32_t *scan_tmp, uint32_t *less,
                   uint64_t *less_val, uint32_t *eq, uint32_t *less_cell, uint32_t *eq_cell,
                   const uint32_t *cell, hipStream_t s) {
    static const int shifts[6] = {53, 42, 31, 20, 9, 0};
    static const int widths[6] = {11, 11, 11, 11, 11, 9};
    hipLaunchKernelGGL(k_select_init, dim3(1), dim3(kBlock), 0, s, st, need, hist);
    if (n <= 0) return;
    for (int ps = 0; ps < 6; ++ps) {
        hipLaunchKernelGGL(k_select_hist, dim3(gridcap(n, 4096)), dim3(kBlock), 0, s, P, n,
                           shifts[ps], widths[ps], (const SelState *)st, hist);
        hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(kBlock), 0, s, hist, widths[ps], ps,
                           ps == 5 ? 1 : 0, st);
    }
    const int64_t nsb = select_blocks(n);
    hipLaunchKernelGGL(k_select_count, dim3((unsigned)nsb), dim3(kBlock), 0, s, P, n,
                       (const SelState *)st, cnt);
    scan_exclusive_u32(cnt, cnt, nsb, nullptr, scan_tmp, s);
    hipLaunchKernelGGL(k_select_emit, dim3((unsigned)nsb), dim3(kBlock), 0, s, P, n, st,
                       (const uint32_t *)cnt, less, less_val, (uint32_t)need, eq);
    hipLaunchKernelGGL(k_select_cells, dim3(nblk(need)), dim3(kBlock), 0, s, cell,
                       (const SelState *)st, (const uint32_t *)less, (const uint32_t *)eq, need,
                       less_cell, eq_cell);
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

void launch_count_zero(const uint64_t *P, int64_t n, unsigned long long *out, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_count_zero, dim3(gridcap(n, 1024)), dim3(kBlock), 0, s, P, n, out);
}

void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_u64, dim3(gridcap(n, 8192)), dim3(kBlock), 0, s, p, n, v);
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_u32, dim3(gridcap(n, 8192)), dim3(kBlock), 0, s, p, n, v);
}

}  // namespace pmp
