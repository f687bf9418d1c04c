// k_scan.hip -- exclusive scan and stable LSD radix sort for gfx950.
//
// The radix sort ranks keys inside a wave with ballots (one ballot per digit
// bit gives each lane the set of lanes holding the same digit), so a block
// needs no LDS histogram per thread; each wave takes a contiguous slice of
// its block's tile, waves are chained through a small LDS table of digit
// counts (one block barrier), and blocks through a scan of per-(digit,
// block) counts.  Stability
// (equal keys keep their input order) is what keeps each bucket of the
// directory sorted by window start.
#include "pmp_dev.h"

namespace pmp {

namespace {

constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = kBlock * kScanItems;      // 2048 per block

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds /* >= 4 */, uint32_t &excl) {
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    // inclusive wave scan by shuffles
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) lds[w] = x;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        uint32_t s = lds[i];
        if (i < w) wbase += s;
        total += s;
    }
    __syncthreads();
    excl = wbase + x - v;
    return total;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                        int64_t n, uint32_t *__restrict__ sums) {
    __shared__ uint32_t lds[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) s += in[i];
    }
    uint32_t ex;
    uint32_t tot = block_exclusive_scan(s, lds, ex);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block scans the block sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *__restrict__ sums, int64_t nb,
                                                    uint32_t *__restrict__ total) {
    __shared__ uint32_t lds[1024 / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t x = v;
        for (int off = 1; off < kWave; off <<= 1) {
            uint32_t y = __shfl_up(x, off, kWave);
            if (lane >= off) x += y;
        }
        if (lane == kWave - 1) lds[w] = x;
        __syncthreads();
        uint32_t wbase = 0, tot = 0;
        for (int k = 0; k < 1024 / kWave; ++k) {
            uint32_t s = lds[k];
            if (k < w) wbase += s;
            tot += s;
        }
        uint32_t c = carry;
        if (i < nb) sums[i] = c + wbase + x - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t *__restrict__ in,
                                                       uint32_t *__restrict__ out, int64_t n,
                                                       const uint32_t *__restrict__ sums) {
    __shared__ uint32_t lds[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0u;
        s += v[k];
    }
    uint32_t ex;
    block_exclusive_scan(s, lds, ex);
    uint32_t run = sums[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// ------------------------------------------------------------ radix sort

constexpr int kSortRounds = 8;                       // items per thread
constexpr int kSortTile = kBlock * kSortRounds;      // 2048 per tile
constexpr int kSortSub = 4;                          // consecutive tiles per block
constexpr int kSortChunk = kSortTile * kSortSub;     // keys per block
constexpr int kRadix = 256;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                       int64_t n, int shift, int nbits,
                                                       uint32_t *__restrict__ counts,
                                                       int64_t nblocks) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t mask = (1u << nbits) - 1u;
    const int lane = lane_id();
    // the block's kSortSub tiles; wavefront w counts the slice [w, w + 1) *
    // kSortTile / 4 of each.  Equal digits of a round are matched by ballots
    // (one per digit bit) and counted by one lane, so a tile whose keys share
    // a digit (as they do after the lower passes) costs one LDS atomic per
    // round, not 64
    for (int sub = 0; sub < kSortSub; ++sub) {
        const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)sub * kSortTile +
                             (int64_t)(threadIdx.x / kWave) * (kSortTile / (kBlock / kWave));
        if (base >= n) break;
        uint32_t key[kSortRounds];
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            key[r] = i < n ? keys[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const bool valid = base + (int64_t)r * kWave + lane < n;
            const uint32_t dig = (key[r] >> shift) & mask;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < nbits; ++b) {
                const uint64_t bal = __ballot((dig >> b) & 1u);
                peers &= ((dig >> b) & 1u) ? bal : ~bal;
            }
            if (valid && (peers & lanemask_lt()) == 0)
                atomicAdd(&h[dig], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    // digit-major so that the exclusive scan gives each (digit, block) its
    // first output position
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// kSortSub consecutive tiles of kSortTile keys per block, in order; in each
// tile wavefront w takes the contiguous slice [w, w + 1) * kSortTile / 4 in
// kSortRounds rounds of 64.  Pass 1 ranks each key among the equal digits of
// its round (one ballot per digit bit) and counts each wavefront's digits;
// after one block barrier every (wavefront, digit) knows its first output
// position (the digit's running position in the block, which starts at the
// block's offset of the digit, plus the counts of the earlier wavefronts);
// pass 2 writes the keys.  Stable: within a digit, tiles, wavefronts, rounds
// and lanes keep their input order.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift, int nbits,
    const uint32_t *__restrict__ offs, int64_t nblocks) {
    constexpr int kW = kBlock / kWave;
    __shared__ uint32_t wcnt[kW][kRadix];
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const uint32_t mask = (1u << nbits) - 1u;
    // thread d: the next output position of digit d
    uint32_t run = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    for (int sub = 0; sub < kSortSub; ++sub) {
        const int64_t tbase = (int64_t)blockIdx.x * kSortChunk + (int64_t)sub * kSortTile;
        if (tbase >= n) break;
        for (int q = 0; q < kW; ++q) wcnt[q][threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = tbase + (int64_t)w * (kSortTile / kW);
        uint32_t key[kSortRounds], val[kSortRounds], rank[kSortRounds];
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            const bool valid = i < n;
            key[r] = valid ? kin[i] : 0u;
            val[r] = valid ? vin[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            const bool valid = i < n;
            const uint32_t dig = (key[r] >> shift) & mask;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < nbits; ++b) {
                const uint64_t bal = __ballot((dig >> b) & 1u);
                peers &= ((dig >> b) & 1u) ? bal : ~bal;
            }
            const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
            // the digit's count so far in this wavefront (earlier rounds) plus the
            // equal digits of earlier lanes; the leader then adds the round's count
            rank[r] = below + (valid ? wcnt[w][dig] : 0u);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (valid && below == 0) wcnt[w][dig] += (uint32_t)__popcll(peers);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        {
            // thread d: the first position of digit d for each wavefront
            const int d = threadIdx.x;
            for (int q = 0; q < kW; ++q) {
                const uint32_t c = wcnt[q][d];
                wcnt[q][d] = run;
                run += c;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const int64_t i = base + (int64_t)r * kWave + lane;
            if (i < n) {
                const uint32_t pos = wcnt[w][(key[r] >> shift) & mask] + rank[r];
                kout[pos] = key[r];
                vout[pos] = val[r];
            }
        }
        __syncthreads();                                 // wcnt is cleared next
    }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t scan_temp_bytes(int64_t n) {
    return (size_t)(cdiv(n, kScanTile) + 64) * sizeof(uint32_t);
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                        void *temp, hipStream_t s) {
    if (n <= 0) {
        if (total) launch_fill_u32(total, 1, 0u, s);
        return;
    }
    int64_t nb = cdiv(n, kScanTile);
    uint32_t *sums = (uint32_t *)temp;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n,
                       (const uint32_t *)sums);
}

size_t sort_temp_bytes(int64_t n) {
    int64_t nb = cdiv(n, kSortChunk);
    size_t counts = (size_t)(nb * kRadix) * sizeof(uint32_t);
    return 2 * counts + scan_temp_bytes(nb * kRadix) + 256;
}

int radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                     int lo, int hi, void *temp, hipStream_t s, bool copy_back) {
    if (n <= 1 || hi <= lo) return 0;
    int64_t nb = cdiv(n, kSortChunk);
    uint32_t *counts = (uint32_t *)temp;
    uint32_t *offs = counts + nb * kRadix;
    void *stemp = (void *)(offs + nb * kRadix);
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    int passes = 0;
    for (int shift = lo; shift < hi; shift += 8, ++passes) {
        int nbits = hi - shift < 8 ? hi - shift : 8;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, s, ka, n, shift,
                           nbits, counts, nb);
        scan_exclusive_u32(counts, offs, nb * kRadix, nullptr, stemp, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, s, ka, va, kb,
                           vb, n, shift, nbits, (const uint32_t *)offs, nb);
        uint32_t *t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    if ((passes & 1) && copy_back) {
        (void)hipMemcpyAsync(k0, ka, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(v0, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        return 0;
    }
    return passes & 1;
}

}  // namespace pmp
