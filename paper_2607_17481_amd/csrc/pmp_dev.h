// pmp_dev.h -- internal declarations shared by the HIP translation units of
// libpmp (not a public header).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmp {

// ------------------------------------------------------------ constants
constexpr int    kBlock      = 256;       // threads per block (4 waves of 64)
constexpr int    kWave       = 64;
constexpr int    kMaxK       = 16;        // largest spectral width K
constexpr int    kRec        = 32;        // feature record: 30 features + e_i + |F|
constexpr int    kSlotErr    = 30;        // record slot of the error bound e_i
constexpr int    kSlotNorm   = 31;        // record slot of ||F||
constexpr int    kMaxBits    = 24;        // SimHash bits B (Sec. 4: B = 24)
constexpr int    kProbeSlots = 8;         // Hamming-1 probes kept per key word
constexpr int    kJoinDims   = 6;         // orthonormal projections of a join record
constexpr int    kMaxM       = 4096;      // longest window supported
constexpr int    kTileW      = 256;       // windows per sketch tile
constexpr int    kSegW       = 16;        // windows per sliding-DFT segment
constexpr double kEps0       = 1e-6;      // zero snap (Sec. 3.6)
constexpr uint64_t kInfBits  = 0x7FF0000000000000ull;   // +inf as FP64 bits

// Per-length metadata, device resident.
struct LenInfo {
    int32_t m;            // window length
    int32_t kprime;       // K' = min(K-1, ceil(m/2)-1)
    int32_t depth;        // directory depth d (Prop. 4 final state)
    int32_t probes;       // Hamming-1 probes h = min(cap, d, 1 + max(0, d - d0))
    int64_t W;            // windows n - m + 1
    int64_t cell_base;    // first cell of this length in natural order
    int64_t slot_base;    // first slot of this length in bucket order
    int64_t bucket_base;  // first bucket counter of this length
    int64_t n_index;      // non-constant windows (entries of the directory)
    int64_t tile_base;    // first sketch tile of this length
};

// Everything a kernel needs to know about one request.
struct Req {
    const double *t;       // series
    int64_t n;
    int32_t L;             // number of lengths
    int32_t K;             // spectral width
    int32_t B;             // signature bits
    int32_t excl;          // exclusion zone
    int32_t budget_R;      // inspections per query (R = gamma * alpha)
    int32_t key_shift;     // bucket key: len_idx << key_shift | prefix << (key_shift - d)
    int32_t jkey_shift;    // join key: len_idx << jkey_shift | quantized p1
    int32_t precision;
    const LenInfo *len;    // [L]
    const int32_t *cpre;   // [n] inclusive prefix count of change points
    double  *mu;           // [cells] window mean
    double  *isig;         // [cells] 1 / sigma (population standard deviation)
    uint64_t *P;           // [cells] profile, FP64 bits (atomicMin)
    uint64_t *keyw_nat;    // [cells] key word (natural order), pass A
    uint32_t *skey;        // [N] sort keys (bucket)       -- sort buffers
    uint32_t *sval;        // [N] sort values (cell id)
    uint32_t *bucket_cnt;  // [buckets] population, then start slot (scan)
    uint32_t *perm;        // [N] slot -> cell
    uint32_t *inv;         // [cells] cell -> slot (valid for indexed cells)
    void    *F;            // [N][kRec] features in slot order (float or double)
    uint64_t *keyw;        // [N] key words in slot order
    const float *gproj;    // [L][B][30] SimHash projections
    const double *ujoin;   // [kJoinDims][30] orthonormal join directions
    float   *jrec;         // [N][8] join record in slot order: p1..p6, slot bits
    float   *emax;         // [L] largest e_i of each length
    unsigned long long *counters;   // stats counters
    int     *bad;          // raised on inputs the library cannot represent
};

enum Counter {
    C_PASS_CAND = 0, C_PASS_VER, C_JOIN_CAND, C_JOIN_VER, C_HOT, C_NCOUNTERS
};

// ------------------------------------------------------------- helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Snapped distance (Sec. 3.6: values below eps0 are reported as 0).
__device__ __forceinline__ double snap(double d) { return d < kEps0 ? 0.0 : d; }

__device__ __forceinline__ uint64_t dbits(double d) {
    return (uint64_t)__double_as_longlong(d);
}
__device__ __forceinline__ double bitsd(uint64_t b) {
    return __longlong_as_double((long long)b);
}

// Length index of a cell (binary search over cell_base, L is small).
__device__ __forceinline__ int find_len(const LenInfo *len, int L, int64_t cell) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (len[mid].cell_base <= cell) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_len_slot(const LenInfo *len, int L, int64_t slot) {
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (len[mid].slot_base <= slot) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Exact z-normalized distance between windows a and b of length m, FP64,
// r ascending, z = (t - mu) * (1/sigma) per sample (Sec. 2).  Symmetric bit
// for bit in (a, b): only squares of differences are summed.
// Contraction is off so that every kernel rounds this function the same way:
// the profile, the join and the exact rows must agree bit for bit.
__device__ __forceinline__ double zdist(const double *__restrict__ t, int64_t a, double mua,
                                        double ia, int64_t b, double mub, double ib, int m) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int r = 0; r < m; ++r) {
        double za = (t[a + r] - mua) * ia;
        double zb = (t[b + r] - mub) * ib;
        double e = za - zb;
        acc = fma(e, e, acc);
    }
    return sqrt(acc);
}

// Certified lower bound on d_m(q, c) from the stored features: the Parseval
// bound (Lemma 2) of the true features is at least
//   sqrt(2/m) (||F~q - F~c|| - e_q - e_c),
// and every rounding of this evaluation is absorbed by the relative slacks.
template <typename FT>
__device__ __forceinline__ float lb_safe(const FT *__restrict__ fq, const FT *__restrict__ fc,
                                         int kp, float sqrt2m) {
    FT acc = 0;
    for (int c = 0; c < 2 * kp; ++c) {
        FT e = fq[c] - fc[c];
        acc = fma(e, e, acc);
    }
    const FT nd = sqrt(acc);
    const FT es = fq[kSlotErr] + fc[kSlotErr];
    if (sizeof(FT) == 4) {
        float v = (float)nd * (1.0f - 1e-5f) - (float)es * (1.0f + 1e-5f);
        return v > 0.0f ? v * sqrt2m * (1.0f - 1e-6f) : 0.0f;
    } else {
        double v = (double)nd * (1.0 - 1e-12) - (double)es * (1.0 + 1e-12);
        // the float result is rounded down
        return v > 0.0 ? __double2float_rd(v * (double)sqrt2m * (1.0 - 1e-6)) : 0.0f;
    }
}

struct JoinLen {
    float r_filter;     // radius on the join projections
    float r_key;        // radius used for the key range
    float prange;       // quantization half-range of the first projection
    float pad;
};

struct RowReq {
    int32_t l;          // length index
    int32_t pad;
    int64_t i;          // start of the cell
    uint64_t target;    // pass 2: FP64 bits of the value whose smallest j is wanted
};

// --------------------------------------------------- host-side launchers
// (k_scan.hip)
size_t scan_temp_bytes(int64_t n);
// out[i] = sum_{j<i} in[j]; total (optional, device) = sum of all.
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                        void *temp, hipStream_t s);
size_t sort_temp_bytes(int64_t n);
// Stable LSD radix sort of (key, val) pairs on key bits [lo, hi).  Result in
// (k0, v0); (k1, v1) are scratch of the same size.
void radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                      int64_t n, int lo, int hi, void *temp, hipStream_t s);

// (k_sketch.hip)
void launch_changepoints(const double *t, int64_t n, uint32_t *flag, int *bad, hipStream_t s);
void launch_count_index(const LenInfo *len, int L, const uint32_t *E, unsigned long long *cnt,
                        int64_t maxW, hipStream_t s);
void launch_sketch(int pass, int precision, const Req &q, const uint32_t *E, uint32_t *tile_cnt,
                   int64_t ntiles, int max_m, hipStream_t s);
void launch_emit_sortin(const Req &q, const uint32_t *tile_off, int64_t ntiles, hipStream_t s);
void launch_invert(const uint32_t *perm, int64_t N, uint32_t *inv, hipStream_t s);
// (k_probe.hip)
void launch_probe(int precision, const Req &q, const uint32_t *bstart, int64_t N, hipStream_t s);
void launch_hot_buckets(const uint32_t *bstart, int64_t nb, int R, unsigned long long *cnt,
                        hipStream_t s);
// (k_certify.hip)
void launch_select_hist(const uint64_t *P, int64_t n, int shift, int nbits, uint64_t high,
                        unsigned int *hist, hipStream_t s);
int64_t select_blocks(int64_t n);
void launch_select_count(const uint64_t *P, int64_t n, uint64_t pivot, uint32_t *cnt,
                         hipStream_t s);
void launch_select_emit(const uint64_t *P, int64_t n, uint64_t pivot, uint32_t need,
                        const uint32_t *off, uint32_t *less, uint64_t *less_val, uint32_t *nless,
                        uint32_t cap, uint32_t *eq, hipStream_t s);
void launch_join_keys(const Req &q, const float *prange, int64_t N, uint32_t *jk, uint32_t *jv,
                      hipStream_t s);
void launch_join_gather(const float *jrec, const uint32_t *jperm, int64_t N, float *jsorted,
                        hipStream_t s);
void launch_join(int precision, const Req &q, const float *js, const uint32_t *jkey,
                 const JoinLen *jl, int64_t N, double T, hipStream_t s);
void launch_rows(const Req &q, const RowReq *rr, int nrows, int64_t maxW, int find_min,
                 unsigned long long *out_min, unsigned long long *out_arg, hipStream_t s);
void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);

}  // namespace pmp
