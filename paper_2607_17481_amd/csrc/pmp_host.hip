// pmp_host.hip -- orchestration of the hot path and the C ABI of libpmp.
//
// One request runs, on one HIP stream:
//   change points -> per-length index counts -> depths            (host sync)
//   one sketch pass: moments, features, SimHash keys, join records (k_sketch)
//   stable radix sort into buckets, bucket starts, slot maps
//   probe / Parseval prune / exact verification     (k_probe)      -> upper profile
//   top-k selection (radix select + greedy)                        (host sync)
//   certificate: threshold join at T, repeated while needed         (k_join)
//   exact rows of the reported cells (nearest neighbour)           (k_rows)
#include "pmp_dev.h"
#include "pmp.h"
#include "pmp_stages.h"
#include "pmp_host.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace pmp {

// ---------------------------------------------------------------- errors

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

int read_options(const pmp_options *o, Opt &out) {
    Opt d;
    if (o) {
        if (o->size != sizeof(pmp_options))
            return fail(PMP_EINVAL, "pmp_options.size mismatch (%u != %zu)", o->size,
                        sizeof(pmp_options));
        d.m_step = o->m_step;
        d.precision = o->precision;
        d.K = o->spectral_width;
        d.seed = o->seed;
        d.certify = o->certify;
        d.B = o->signature_bits;
        d.gamma = o->gamma;
        d.d0 = o->probe_ref_depth;
        d.probe_cap = o->probe_cap;
        d.stride = o->anchor_stride;
        d.sieve_w = o->sieve_width;
        d.compl_rounds = o->complete_rounds;
        d.compl_dm = o->complete_dm;
        d.compl_dp = o->complete_dp;
    }
    if (d.m_step < 1) return fail(PMP_EINVAL, "m_step must be >= 1");
    if (d.precision < 0 || d.precision > 2) return fail(PMP_EINVAL, "unknown precision");
    if (d.K != 0 && (d.K < 2 || d.K > kMaxK)) return fail(PMP_EINVAL, "spectral_width in [2,16] or 0");
    if (d.B < 1 || d.B > kMaxBits) return fail(PMP_EINVAL, "signature_bits in [1,24]");
    if (d.gamma < 1) return fail(PMP_EINVAL, "gamma must be >= 1");
    if (d.d0 < 0) return fail(PMP_EINVAL, "probe_ref_depth must be >= 0");
    if (d.probe_cap < 0 || d.probe_cap > kProbeSlots) return fail(PMP_EINVAL, "probe_cap in [0,8]");
    if (d.certify != 0 && d.certify != 1) return fail(PMP_EINVAL, "certify is 0 or 1");
    if (d.stride < 1) return fail(PMP_EINVAL, "anchor_stride must be >= 1");
    if (d.sieve_w < 0 || d.sieve_w > 64) return fail(PMP_EINVAL, "sieve_width in [0,64]");
    if (d.compl_rounds < 0 || d.compl_rounds > 64) return fail(PMP_EINVAL, "complete_rounds in [0,64]");
    if (d.compl_dm < 0 || d.compl_dp < 0 || d.compl_dp > 64)
        return fail(PMP_EINVAL, "complete_dm >= 0 and complete_dp in [0,64]");
    out = d;
    return PMP_OK;
}

// ------------------------------------------- seeded Gaussian projections

// SplitMix64 output function (Steele, Lea, Flood 2014) used as a
// counter-based generator: the c-th value of stream `seed`.
static uint64_t splitmix(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Standard normal by the Box-Muller transform of two counter values.
static double gauss(uint64_t seed, int m, int l, int c) {
    const uint64_t ctr = (((uint64_t)m * 64u + (uint64_t)l) * 64u + (uint64_t)c) * 2u;
    const uint64_t a = splitmix(seed, ctr), b = splitmix(seed, ctr + 1);
    const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(b >> 11) * 0x1.0p-53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925286766559 * u2);
}


// The SimHash projections of one length (kMaxBits x 30, a pure function of
// the seed and m) into out, from a table kept across requests: a request
// over 51 lengths needs 36,720 Gaussian draws, about 1.7 ms of host time
// while the GPU would wait.  The table is bounded (cleared past 8192
// lengths) and shared by the server's threads.
void projections(uint64_t seed, int m, float *out) {
    static std::mutex mu;
    static std::map<std::pair<uint64_t, int>, std::vector<float>> table;
    std::lock_guard<std::mutex> lock(mu);
    auto it = table.find({seed, m});
    if (it == table.end()) {
        if (table.size() >= 8192) table.clear();
        std::vector<float> v((size_t)kMaxBits * kFD);
        for (int l = 0; l < kMaxBits; ++l)
            for (int c = 0; c < kFD; ++c) v[(size_t)l * kFD + c] = (float)gauss(seed, m, l, c);
        it = table.emplace(std::make_pair(seed, m), std::move(v)).first;
    }
    std::memcpy(out, it->second.data(), it->second.size() * sizeof(float));
}

int kprime_of(int K, int m) {
    int half = (m + 1) / 2 - 1;
    int kp = std::min(K - 1, half);
    return kp < 0 ? 0 : kp;
}

// ----------------------------------------------- spectral width (Sec. 3.2)

// Smallest K in [4, 16] whose retained bins hold a fraction eta of the
// normalized spectral energy on average, and whose expected accidental
// collision count n E[(1 - theta_K / pi)^B] stays within 2 gamma alpha, at
// each of the sampled lengths.  Near-duplicate pairs (angle below 1e-3 rad at
// the full width) are left out of the collision estimate.
static int calibrate(const std::vector<std::vector<std::vector<double>>> &sets,
                     const std::vector<int> &ms, int64_t n, int alpha, int gamma, int B) {
    const double eta = 0.85;
    // per sampled window: prefix sums over the bins k = 1..K' of its energy
    // (e[k]), and per consecutive pair those of the dot product and of both
    // energies, so that each candidate K costs O(1) per window and pair
    struct Spec { double re[kMaxK], im[kMaxK]; };
    std::vector<std::vector<Spec>> spec(sets.size());
    for (size_t s = 0; s < sets.size(); ++s) {
        const int m = ms[s];
        const int kp = kprime_of(kMaxK, m);
        // twiddles cos, sin (2 pi j / m), j < m, laid out per sample r for
        // the bins 1..K' (bin k at r uses j = k r mod m)
        std::vector<double> tc(m), ts(m);
        for (int j = 0; j < m; ++j) {
            tc[j] = std::cos(6.283185307179586 * (double)j / m);
            ts[j] = std::sin(6.283185307179586 * (double)j / m);
        }
        std::vector<double> cr((size_t)m * kMaxK, 0.0), sr((size_t)m * kMaxK, 0.0);
        for (int r = 0; r < m; ++r)
            for (int k = 1; k <= kp; ++k) {
                const int j = (int)(((int64_t)k * r) % m);
                cr[(size_t)r * kMaxK + k] = tc[j];
                sr[(size_t)r * kMaxK + k] = ts[j];
            }
        std::vector<double> zw(m);
        for (const auto &w : sets[s]) {
            double mu = 0.0;
            for (double x : w) mu += x;
            mu /= m;
            double q = 0.0;
            for (double x : w) q += (x - mu) * (x - mu);
            const double sg = std::sqrt(q / m);
            if (!(sg > 0.0)) continue;
            for (int r = 0; r < m; ++r) zw[r] = (w[r] - mu) / sg;
            Spec f;
            for (int k = 0; k < kMaxK; ++k) f.re[k] = f.im[k] = 0.0;
            // every bin sums its terms in ascending r
            for (int r = 0; r < m; ++r) {
                const double z = zw[r];
                const double *c = &cr[(size_t)r * kMaxK], *sn = &sr[(size_t)r * kMaxK];
                for (int k = 1; k < kMaxK; ++k) {
                    f.re[k] += z * c[k];
                    f.im[k] -= z * sn[k];
                }
            }
            spec[s].push_back(f);
        }
    }
    struct Pre { std::vector<double> e; std::vector<double> ab, aa, bb; std::vector<char> dup; };
    std::vector<Pre> pre(sets.size());
    for (size_t s = 0; s < sets.size(); ++s) {
        const auto &v = spec[s];
        const int kpf = kprime_of(kMaxK, ms[s]);
        Pre &P = pre[s];
        P.e.assign((size_t)v.size() * (kMaxK + 1), 0.0);
        for (size_t w = 0; w < v.size(); ++w)
            for (int k = 1; k <= kMaxK; ++k)
                P.e[w * (kMaxK + 1) + k] = P.e[w * (kMaxK + 1) + k - 1] +
                    (k < kMaxK ? v[w].re[k] * v[w].re[k] + v[w].im[k] * v[w].im[k] : 0.0);
        const size_t np = v.size() > 0 ? v.size() - 1 : 0;
        P.ab.assign(np * (kMaxK + 1), 0.0);
        P.aa.assign(np * (kMaxK + 1), 0.0);
        P.bb.assign(np * (kMaxK + 1), 0.0);
        P.dup.assign(np, 0);
        for (size_t w = 0; w < np; ++w) {
            double ab = 0.0, aa = 0.0, bb = 0.0;
            for (int k = 1; k <= kMaxK; ++k) {
                if (k < kMaxK) {
                    ab += v[w].re[k] * v[w + 1].re[k] + v[w].im[k] * v[w + 1].im[k];
                    aa += v[w].re[k] * v[w].re[k] + v[w].im[k] * v[w].im[k];
                    bb += v[w + 1].re[k] * v[w + 1].re[k] + v[w + 1].im[k] * v[w + 1].im[k];
                }
                P.ab[w * (kMaxK + 1) + k] = ab;
                P.aa[w * (kMaxK + 1) + k] = aa;
                P.bb[w * (kMaxK + 1) + k] = bb;
            }
        }
        auto angle = [&](size_t w, int kk) {
            const double ab = P.ab[w * (kMaxK + 1) + kk], aa = P.aa[w * (kMaxK + 1) + kk],
                         bb = P.bb[w * (kMaxK + 1) + kk];
            if (!(aa > 0.0 && bb > 0.0)) return 0.0;
            double c = ab / std::sqrt(aa * bb);
            c = std::max(-1.0, std::min(1.0, c));
            return std::acos(c);
        };
        for (size_t w = 0; w < np; ++w) P.dup[w] = angle(w, kpf) < 1e-3;
    }
    for (int K = 4; K <= kMaxK; ++K) {
        bool ok = true;
        for (size_t s = 0; s < sets.size() && ok; ++s) {
            const int m = ms[s];
            const int kp = kprime_of(K, m);
            const auto &v = spec[s];
            const Pre &P = pre[s];
            if (v.empty()) continue;
            double e = 0.0;
            for (size_t w = 0; w < v.size(); ++w) e += 2.0 * P.e[w * (kMaxK + 1) + kp] / ((double)m * m);
            e /= (double)v.size();
            if (e < eta) { ok = false; break; }
            double coll = 0.0;
            int pairs = 0;
            for (size_t w = 0; w + 1 < v.size(); ++w) {
                if (P.dup[w]) continue;
                const double ab = P.ab[w * (kMaxK + 1) + kp], aa = P.aa[w * (kMaxK + 1) + kp],
                             bb = P.bb[w * (kMaxK + 1) + kp];
                double th = 0.0;
                if (aa > 0.0 && bb > 0.0) {
                    double c = ab / std::sqrt(aa * bb);
                    c = std::max(-1.0, std::min(1.0, c));
                    th = std::acos(c);
                }
                coll += std::pow(1.0 - th / M_PI, (double)B);
                ++pairs;
            }
            if (pairs && (double)n * coll / pairs > 2.0 * gamma * alpha) ok = false;
        }
        if (ok) return K;
    }
    return kMaxK;
}

static std::vector<int64_t> sample_starts(int64_t W) {
    std::vector<int64_t> v;
    if (W <= 256) {
        for (int64_t i = 0; i < W; ++i) v.push_back(i);
    } else {
        for (int j = 0; j < 256; ++j) v.push_back((int64_t)((double)j * (double)(W - 1) / 255.0));
    }
    return v;
}

__global__ void k_gather_windows(const double *__restrict__ t, const int64_t *__restrict__ starts,
                                 int count, int m, double *__restrict__ out) {
    const int w = blockIdx.x;
    if (w >= count) return;
    for (int r = threadIdx.x; r < m; r += blockDim.x) out[(int64_t)w * m + r] = t[starts[w] + r];
}

// ------------------------------------------------------------ workspace

struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0;
    bool sizing = false;              // only count bytes
    std::vector<void *> owned;        // blocks this arena allocated
    bool can_alloc = false;

    void *take(size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void *p = sizing ? nullptr : base + off;
        off += bytes;
        if (!sizing && off > cap) return nullptr;
        return sizing ? (void *)1 : p;
    }
    ~Arena() {
        for (void *p : owned) (void)hipFree(p);
    }
};

template <typename T>
static T *take(Arena &a, int64_t count) {
    return (T *)a.take((size_t)std::max<int64_t>(count, 1) * sizeof(T));
}

// --------------------------------------------------------------- plan

struct Plan {
    int64_t n = 0;
    int L = 0;
    std::vector<int> ms;
    std::vector<LenInfo> len;
    int64_t cells = 0, ntiles = 0, nbuckets = 0, N = 0, Na = 0, nkblocks = 0;
    int64_t nprobe_blocks = 0, nhint_blocks = 0;
    int anchors = 0;
    int max_m = 0, len_bits = 0, key_shift = 0, jkey_shift = 0, max_depth = 0;
};

static void plan_lengths(Plan &p, int64_t n, int m_min, int m_max, int step) {
    p.n = n;
    p.ms.clear();
    for (int64_t m = m_min; m <= m_max; m += step) p.ms.push_back((int)m);
    p.L = (int)p.ms.size();
    p.len.assign(p.L, LenInfo{});
    int64_t cb = 0, tb = 0;
    for (int l = 0; l < p.L; ++l) {
        LenInfo &L = p.len[l];
        L.m = p.ms[l];
        L.W = n - L.m + 1;
        L.cell_base = cb;
        L.tile_base = tb;
        cb += L.W;
        tb += (L.W + kTileW - 1) / kTileW;
    }
    p.cells = cb;
    p.ntiles = tb;
    p.max_m = p.ms.back();
    p.len_bits = 0;
    while ((1 << p.len_bits) < p.L) ++p.len_bits;
}

// depths, probes and bases from the per-length index counts
static void plan_index(Plan &p, const std::vector<int64_t> &cnt, const Opt &o, int alpha, int K) {
    const int dcap = std::min(o.B, 32 - p.len_bits - 1);
    int64_t kb = 0, bb = 0;
    p.max_depth = 0;
    p.nkblocks = 0;
    // anchor lengths (Sec. 3.3): every stride-th length of the list, and the
    // last one; each other length knows its nearest anchors
    p.anchors = 0;
    for (int l = 0; l < p.L; ++l) {
        LenInfo &L = p.len[l];
        L.anchor = (l % o.stride == 0 || l == p.L - 1) ? 1 : 0;
        p.anchors += L.anchor;
        L.a_lo = L.a_hi = -1;
        L.pad_ = 0;
    }
    for (int l = 0; l < p.L; ++l) {
        if (p.len[l].anchor) continue;
        for (int a = l - 1; a >= 0 && p.len[l].a_lo < 0; --a)
            if (p.len[a].anchor) p.len[l].a_lo = a;
        for (int a = l + 1; a < p.L && p.len[l].a_hi < 0; ++a)
            if (p.len[a].anchor) p.len[l].a_hi = a;
    }
    p.nprobe_blocks = p.nhint_blocks = 0;
    int64_t ab = 0;
    for (int l = 0; l < p.L; ++l) {
        LenInfo &L = p.len[l];
        L.kprime = kprime_of(K, L.m);
        L.n_index = cnt[l];
        // directories at the anchor lengths only: the one pass probes them
        // alone, and the lengths between take their hints
        int d = 0;
        while (L.anchor && d < dcap && L.n_index > (int64_t)alpha << d) ++d;   // Prop. 4 final depth
        L.depth = d;
        int h = d > 0 ? 1 + std::max(0, d - o.d0) : 0;
        h = std::min(h, std::min(d, o.probe_cap));
        L.probes = h;
        L.kbase = kb;
        L.abase = ab;
        L.blk_base = p.nkblocks;
        if (L.anchor) {
            p.nkblocks += (L.n_index + kBlock - 1) / kBlock;
            ab += L.n_index;
        }
        L.pblk_base = p.nprobe_blocks;
        L.hblk_base = p.nhint_blocks;
        if (L.anchor)
            p.nprobe_blocks += (L.n_index + kWave - 1) / kWave;
        else
            p.nhint_blocks += (L.n_index + kWave - 1) / kWave;
        L.bucket_base = bb;
        kb += L.n_index;
        bb += (int64_t)1 << d;
        p.max_depth = std::max(p.max_depth, d);
    }
    p.N = kb;
    p.Na = ab;
    p.nbuckets = bb;
    p.key_shift = p.max_depth;
    p.jkey_shift = 32 - p.len_bits - 1;
}

struct Bufs {
    // phase 1: sized by the series and the lengths
    LenInfo *len;
    uint32_t *flags, *E, *scan_tmp, *tile_off;
    int *bad;
    unsigned long long *counters;
    float *emax, *gproj;
    double *cov, *udir;
    GridLen *gl;
    int64_t *bbase;            // MFMA sketch basis: offsets per length, then hi / mid / lo tables
    uint16_t *bh, *bm, *bl;
    unsigned int *hist;
    RowReq *rows;
    unsigned long long *row_min, *row_arg;
    int64_t *cal_starts;
    double *cal_win;
    // phase 2: sized by the indexed windows N
    uint32_t *cell;
    double *mu, *isig;
    uint64_t *P, *keyw;
    void *F;
    uint4 *jop;
    float4 *jmeta;
    uint8_t *qf;
    float4 *gp;
    uint32_t *skey, *sval, *skey2, *sval2, *pcell, *bstart;
    void *sort_tmp;
    uint32_t *jk, *jv, *jk2, *jv2;
    uint4 *jop_s;              // join operands and coordinates in grid order
    float4 *gp_s;
    uint2 *jpairs;             // the join's kept pairs (k_q, k_c), jcap of them
    unsigned long long *jcount;
    int64_t jcap;
    // emit stage: cell -> k map, partner hints, sieve segments and
    // directions, completion seeds
    uint32_t *kmap, *hint, *scnt, *stotal, *sseg, *seeds;
    float *sdir;
    uint32_t *sel_cnt;
    // the selection's results, one contiguous block read back at once:
    // state, then less_val, less_k, less_cell, eq_k, eq_cell (need each)
    char *selblk;
    SelState *sel;
    uint64_t *less_val;
    uint32_t *less_k, *less_cell, *eq_k, *eq_cell;
};

int64_t need_select(int k, int m_max) { return (int64_t)k * (m_max + 1); }
size_t select_block_bytes(int64_t need) { return kSelHead + (size_t)need * 24; }

static void carve1(Arena &a, Bufs &b, const Plan &p, int k) {
    b.len = take<LenInfo>(a, p.L);
    b.flags = take<uint32_t>(a, p.n + 1);
    b.E = take<uint32_t>(a, p.n + 1);
    b.tile_off = take<uint32_t>(a, p.ntiles + 1);
    // the scans run over n + 1 change points, the tiles, the selection's
    // blocks and the sieve's buckets (at most 2 W + 1 per length)
    b.scan_tmp = (uint32_t *)a.take(scan_temp_bytes(std::max<int64_t>(
        {p.n + 1, p.ntiles + 1, select_blocks(p.cells) + 1, 2 * p.cells + p.L + 1})));
    b.bad = take<int>(a, 1);
    b.counters = take<unsigned long long>(a, C_NCOUNTERS);
    b.emax = take<float>(a, p.L);
    b.gproj = take<float>(a, (int64_t)p.L * kMaxBits * kFD);
    b.cov = take<double>(a, (int64_t)join_cov_doubles(p.L));
    b.udir = take<double>(a, (int64_t)p.L * kJoinDirs * 32);
    {
        std::vector<int64_t> base;
        const int64_t ne = basis_elems(p.len.data(), p.L, base);
        b.bbase = take<int64_t>(a, p.L + 1);
        b.bh = take<uint16_t>(a, ne);
        b.bm = take<uint16_t>(a, ne);
        b.bl = take<uint16_t>(a, ne);
    }
    b.gl = take<GridLen>(a, p.L);
    b.hist = take<unsigned int>(a, kSelBins);
    b.rows = take<RowReq>(a, k);
    b.row_min = take<unsigned long long>(a, k);
    b.row_arg = take<unsigned long long>(a, k);
    b.cal_starts = take<int64_t>(a, 3 * 256);
    b.cal_win = take<double>(a, (int64_t)3 * 256 * p.max_m);
    b.sdir = take<float>(a, (int64_t)p.L * kFD);
    b.seeds = take<uint32_t>(a, k);
    b.stotal = take<uint32_t>(a, 1);
}

static bool needs_kmap(const Opt &o) { return o.stride > 1; }

// Kept pairs of the join buffered between its tiles and its exact stage:
// two per indexed window (16 bytes a window), at least 2^16.
static int64_t join_pair_cap(int64_t N) { return std::max<int64_t>(int64_t(1) << 16, 2 * N); }

static void carve2(Arena &a, Bufs &b, const Plan &p, const Opt &o, int k) {
    const int precision = o.precision;
    const int64_t N = std::max<int64_t>(p.N, 1);
    const int64_t need = need_select(k, p.max_m);
    b.cell = take<uint32_t>(a, N);
    b.mu = take<double>(a, N);
    b.isig = take<double>(a, N);
    b.P = take<uint64_t>(a, N);
    b.keyw = take<uint64_t>(a, N);
    b.F = a.take((size_t)N * kRec * (precision == 0 ? 8 : 4));
    b.jop = take<uint4>(a, N * 8);
    b.jmeta = take<float4>(a, N);
    b.qf = take<uint8_t>(a, N);
    b.gp = take<float4>(a, N);
    b.skey = take<uint32_t>(a, N);
    b.sval = take<uint32_t>(a, N);
    b.skey2 = take<uint32_t>(a, N);
    b.sval2 = take<uint32_t>(a, N);
    b.pcell = take<uint32_t>(a, N);
    b.bstart = take<uint32_t>(a, p.nbuckets + 1);
    b.sort_tmp = a.take(sort_temp_bytes(N));
    b.jop_s = take<uint4>(a, N * 8);
    b.gp_s = take<float4>(a, N);
    b.jk = take<uint32_t>(a, N);
    b.jv = take<uint32_t>(a, N);
    b.jk2 = take<uint32_t>(a, N);
    b.jv2 = take<uint32_t>(a, N);
    b.jcap = join_pair_cap(N);
    b.jpairs = take<uint2>(a, b.jcap);
    b.jcount = take<unsigned long long>(a, 1);
    b.sel_cnt = take<uint32_t>(a, select_blocks(N) + 1);
    b.selblk = (char *)a.take(select_block_bytes(need));
    b.sel = (SelState *)b.selblk;
    b.less_val = (uint64_t *)(b.selblk + kSelHead);
    b.less_k = (uint32_t *)(b.less_val + need);
    b.less_cell = b.less_k + need;
    b.eq_k = b.less_cell + need;
    b.eq_cell = b.eq_k + need;
    b.kmap = needs_kmap(o) ? take<uint32_t>(a, p.cells) : nullptr;
    b.hint = take<uint32_t>(a, N);
    b.scnt = o.sieve_w > 0 ? take<uint32_t>(a, p.nbuckets + 1) : nullptr;
    b.sseg = o.sieve_w > 0 ? take<uint32_t>(a, N) : nullptr;
}

// ------------------------------------------------------------ selection

struct Cand {
    double d;
    int l;
    int64_t i;
    uint32_t k;
};

static bool cand_less(const Cand &a, const Cand &b, const Plan &p) {
    if (a.d != b.d) return a.d < b.d;
    if (p.ms[a.l] != p.ms[b.l]) return p.ms[a.l] < p.ms[b.l];
    return a.i < b.i;
}

static int len_of_cell(const Plan &p, int64_t cell) {
    int lo = 0, hi = p.L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (p.len[mid].cell_base <= cell) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The first `need` cells of the (P, m, i) order, sorted, then the greedy of
// Sec. 2 over them.  P is indexed by k, whose order is the (m, i) order of the
// non-constant windows; constant windows have no cell value.
// The selection runs on the device (launch_select); one read-back brings the
// state and the selected positions, values and cells, after any copies the
// caller has already enqueued on the stream (they complete with the same
// synchronization).
static int select_topk(const Plan &p, Bufs &b, int k, hipStream_t s, std::vector<Cand> &accepted) {
    accepted.clear();
    const int64_t N = p.N;
    const int64_t need_all = need_select(k, p.max_m);
    if (N == 0) {
        HIPCHK(hipStreamSynchronize(s));
        return PMP_OK;
    }
    launch_select(b.P, N, need_all, b.sel, b.hist, b.sel_cnt, b.scan_tmp, b.less_k, b.less_val,
                  b.eq_k, b.less_cell, b.eq_cell, b.cell, s);
    std::vector<char> host(select_block_bytes(need_all));
    HIPCHK(hipMemcpyAsync(host.data(), b.selblk, host.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    SelState st;
    memcpy(&st, host.data(), sizeof(st));
    if (!st.done) return fail(PMP_EINTERNAL, "selection did not settle");
    if (st.nless > (uint32_t)need_all) return fail(PMP_EINTERNAL, "selection overflow");
    const uint32_t nless = st.nless;
    const int64_t need_eq = st.need_eq;
    const uint64_t pivot = st.pivot;
    const uint64_t *lv = (const uint64_t *)(host.data() + kSelHead);
    const uint32_t *lk = (const uint32_t *)(lv + need_all);
    const uint32_t *lc = lk + need_all;
    const uint32_t *ek = lc + need_all;
    const uint32_t *ec = ek + need_all;
    std::vector<Cand> c;
    c.reserve(nless + need_eq);
    for (uint32_t x = 0; x < nless; ++x) {
        double d;
        memcpy(&d, &lv[x], 8);
        const int l = len_of_cell(p, lc[x]);
        c.push_back({d, l, (int64_t)lc[x] - p.len[l].cell_base, lk[x]});
    }
    std::sort(c.begin(), c.end(), [&](const Cand &a, const Cand &bb) { return cand_less(a, bb, p); });
    double pv;
    memcpy(&pv, &pivot, 8);
    for (int64_t x = 0; x < need_eq; ++x) {
        const int l = len_of_cell(p, ec[x]);
        c.push_back({pv, l, (int64_t)ec[x] - p.len[l].cell_base, ek[x]});
    }
    // greedy (Sec. 2): skip a cell within m/2 of an accepted cell of its length
    for (const Cand &x : c) {
        const int m = p.ms[x.l];
        bool skip = false;
        for (const Cand &a : accepted)
            if (a.l == x.l && 2 * std::llabs(a.i - x.i) <= m) { skip = true; break; }
        if (skip) continue;
        accepted.push_back(x);
        if ((int)accepted.size() == k) break;
    }
    return PMP_OK;
}

// Phase times from HIP events on the request's stream.  Off (no events
// created at all) for callers that must not allocate.
struct Timer {
    hipEvent_t ev[12] = {};
    bool ok = false;
    explicit Timer(bool on) {
        if (!on) return;
        ok = true;
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) ok = false;
    }
    ~Timer() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i, hipStream_t s) {
        if (ok) (void)hipEventRecord(ev[i], s);
    }
    double ms(int a, int b) {
        float x = 0.0f;
        if (ok && hipEventElapsedTime(&x, ev[a], ev[b]) == hipSuccess) return x;
        return 0.0;
    }
};

// ------------------------------------------------------------ emit stage

// The hot-class sieve (Sec. 3.6): members of the anchor lengths' buckets of
// more than R entries, sorted by one seeded Gaussian projection within their
// bucket, each verified against the w members after it.
static int run_sieve(const Plan &p, Bufs &b, const Req &q, const Opt &o, hipStream_t s) {
    launch_sieve_count(q, b.bstart, p.nbuckets, q.budget_R, b.scnt, s);
    scan_exclusive_u32(b.scnt, b.scnt, p.nbuckets, b.stotal, b.scan_tmp, s);
    uint32_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, b.stotal, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (total == 0) return PMP_OK;
    if ((int64_t)total > p.N) return fail(PMP_EINTERNAL, "sieve member count %u > %lld", total,
                                          (long long)p.N);
    launch_sieve_keys(o.precision, q, b.bstart, b.scnt, p.nbuckets, total, b.sdir, b.jk, b.jv,
                      b.sseg, s);
    radix_sort_pairs(b.jk, b.jv, b.jk2, b.jv2, total, 0, 32, b.sort_tmp, s);
    launch_sieve_regroup(b.jv, b.sseg, total, b.jk, s);
    int bits = 1;
    while (((int64_t)1 << bits) < p.nbuckets) ++bits;
    radix_sort_pairs(b.jk, b.jv, b.jk2, b.jv2, total, 0, bits, b.sort_tmp, s);
    launch_sieve_verify(o.precision, q, b.bstart, b.scnt, b.jv, b.sseg, total, o.sieve_w, s);
    return PMP_OK;
}

// Sieve, hints at the lengths between anchors, then local completion around
// the current top-k for up to P_max rounds, each round's seeds re-selected,
// until a round lowers no cell.  When the k-th cell accepted before the hints
// is at 0, only zeros ordered before it -- at shorter lengths -- can change
// the top-k, so only those lengths get hints, and no completion runs (it
// cannot lower a 0).  `selected`: `acc` holds the selection of the final upper
// profile (otherwise the caller selects); `rounds`: completion rounds run.
// The sketch of the tiles [0, ntiles) in the request's form (mode: which
// tiles get records, kSketch*).
static void launch_records(const Plan &p, Bufs &b, const Req &q, const Opt &o, int64_t ntiles,
                           int mode, hipStream_t s) {
    if (o.precision == 0)
        launch_sketch(o.precision, q, b.E, b.tile_off, ntiles, p.max_m, mode, s);
    else
        launch_sketch_mfma(o.precision, q, b.E, b.tile_off, ntiles, p.max_m, b.bbase, b.bh, b.bm,
                           b.bl, mode, s);
}

// rec_lim: with `lazy` (the first pass gave records to the anchor lengths
// only), the last length whose records exist when this returns
static int emit_stage(const Plan &p, Bufs &b, Req &q, const Opt &o, int k, hipStream_t s,
                      Timer &tm, std::vector<Cand> &acc, bool &selected, int &rounds, bool lazy,
                      int &rec_lim) {
    rounds = 0;
    tm.mark(9, s);
    tm.mark(10, s);
    if (p.N == 0) return PMP_OK;
    std::vector<float> dir((size_t)p.L * kFD);
    if (o.sieve_w > 0) {
        // one Gaussian direction per length from the projections' stream (row 32,
        // past the signature rows)
        for (int l = 0; l < p.L; ++l)
            for (int c = 0; c < kFD; ++c) dir[(size_t)l * kFD + c] = (float)gauss(o.seed, p.ms[l], 32, c);
        HIPCHK(hipMemcpyAsync(b.sdir, dir.data(), dir.size() * sizeof(float), hipMemcpyHostToDevice,
                              s));
        const int rc = run_sieve(p, b, q, o, s);
        if (rc) return rc;
    }
    tm.mark(9, s);
    if (o.stride == 1) {
        tm.mark(10, s);
        return PMP_OK;
    }
    if (!selected || o.sieve_w > 0) {
        const int rc = select_topk(p, b, k, s, acc);
        if (rc) return rc;
        selected = true;
    }
    const bool zero_kth = acc.size() == (size_t)k && acc.back().d == 0.0;
    if (lazy) {
        // the records of the lengths between anchors that the steps below
        // can read: with a k-th value of 0 those up to the k-th cell's length
        // (the hints stop before it, and the certificate's queries and
        // candidates at it, since that key can only move earlier); otherwise
        // every length.  Nothing has lowered a cell of these lengths yet.
        rec_lim = zero_kth ? acc.back().l : p.L - 1;
        const int64_t nt = rec_lim + 1 < p.L ? p.len[rec_lim + 1].tile_base : p.ntiles;
        launch_records(p, b, q, o, nt, kSketchBetween, s);
    }
    // hint blocks follow the lengths' order: those of the lengths before the
    // k-th cell's come first
    const int64_t hint_blocks = zero_kth ? p.len[acc.back().l].hblk_base : p.nhint_blocks;
    if (hint_blocks > 0) {
        launch_hints(o.precision, q, hint_blocks, s);
        selected = false;
    }
    tm.mark(10, s);
    if (o.compl_rounds == 0 || zero_kth) return PMP_OK;
    std::vector<uint32_t> seeds;
    std::vector<Cand> prev;
    unsigned long long improved = 1;
    for (int r = 0; r <= o.compl_rounds; ++r) {
        const int rc = select_topk(p, b, k, s, acc);   // also completes the copy of `improved`
        if (rc) return rc;
        selected = true;
        // stop once a round lowers no cell or leaves the selected cells and
        // their values as they were (later rounds would only re-verify), or
        // when the k-th value is already 0, which no completion can lower
        bool same = r > 0 && prev.size() == acc.size();
        for (size_t x = 0; same && x < acc.size(); ++x)
            same = prev[x].k == acc[x].k && prev[x].d == acc[x].d;
        if (r == o.compl_rounds || improved == 0 || acc.empty() || same) break;
        if (acc.size() == (size_t)k && acc.back().d == 0.0) break;
        prev = acc;
        seeds.resize(acc.size());
        for (size_t x = 0; x < acc.size(); ++x) seeds[x] = acc[x].k;
        HIPCHK(hipMemcpyAsync(b.seeds, seeds.data(), seeds.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, s));
        launch_fill_u64((uint64_t *)&b.counters[C_COMPL_IMPROVED], 1, 0ull, s);
        launch_complete(o.precision, q, b.seeds, (int)seeds.size(), o.compl_dm, o.compl_dp, s);
        HIPCHK(hipMemcpyAsync(&improved, &b.counters[C_COMPL_IMPROVED], sizeof(improved),
                              hipMemcpyDeviceToHost, s));
        selected = false;
        ++rounds;
    }
    return PMP_OK;
}

// ------------------------------------------------------------- pipeline

static int check_args(int64_t n, int m_min, int m_max, int k, int excl, int budget) {
    if (n < 3) return fail(PMP_EINVAL, "series must have at least 3 samples");
    if (!(3 <= m_min && m_min <= m_max && (int64_t)m_max <= n))
        return fail(PMP_EINVAL, "need 3 <= m_min <= m_max <= n");
    if (m_max > kMaxM) return fail(PMP_EINVAL, "window lengths above %d are not supported", kMaxM);
    if (k < 1) return fail(PMP_EINVAL, "k must be >= 1");
    if (excl < 1) return fail(PMP_EINVAL, "exclusion must be >= 1");
    if (budget < 1) return fail(PMP_EINVAL, "budget must be >= 1");
    return PMP_OK;
}

static size_t upper_bytes(int64_t n, int m_min, int m_max, const Opt &o, int k) {
    Plan p;
    plan_lengths(p, n, m_min, m_max, o.m_step);
    std::vector<int64_t> cnt(p.L);
    for (int l = 0; l < p.L; ++l) cnt[l] = p.len[l].W;
    plan_index(p, cnt, o, 1, kMaxK);   // alpha = 1 gives the deepest directories
    Arena a;
    a.sizing = true;
    Bufs b;
    carve1(a, b, p, k);
    carve2(a, b, p, o, k);
    return a.off + 4096;
}

struct Run {
    const double *t;
    int64_t n;
    int m_min, m_max, k, excl, budget;
    Opt o;
    hipStream_t s;
    pmp_motif *out;
    int32_t *n_out;
    pmp_stats *st;
    pmp_debug *dbg;
    bool timed = true;     // phase events (stats); off for the no-allocation entry
};

// debug exports: per-k arrays to per-cell arrays (constant cells keep the fill)
__global__ void k_debug_scatter(const uint32_t *__restrict__ cell, int64_t N,
                                const uint64_t *__restrict__ src, int invert,
                                uint64_t *__restrict__ dst) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    uint64_t v = src[k];
    if (invert) {       // 1/isig -> sigma
        double x = __longlong_as_double((long long)v);
        v = (uint64_t)__double_as_longlong(1.0 / x);
    }
    dst[cell[k]] = v;
}

template <typename FT>
__global__ void k_debug_features(const FT *__restrict__ F, const uint32_t *__restrict__ cell,
                                 int64_t N, FT *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * 8 + threadIdx.x / 32;
    int e = threadIdx.x % 32;
    if (k >= N) return;
    out[(int64_t)cell[k] * kRec + e] = F[k * kRec + e];
}

__global__ void k_debug_perm(const uint32_t *__restrict__ perm, const uint32_t *__restrict__ cell,
                             int64_t N, uint32_t *__restrict__ out) {
    int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < N) out[s] = cell[perm[s]];
}

static int run_pipeline(Run &R, Arena &ar) {
    const hipStream_t s = R.s;
    const Opt &o = R.o;
    Plan p;
    plan_lengths(p, R.n, R.m_min, R.m_max, o.m_step);
    // cells are numbered in uint32 and indexed windows in int32
    if (p.cells > (int64_t)INT32_MAX) return fail(PMP_EINVAL, "too many cells (%lld > 2^31 - 1)", (long long)p.cells);
    Bufs b;
    carve1(ar, b, p, R.k);
    if (ar.off > ar.cap) return fail(PMP_ENOMEM, "workspace too small (%zu < %zu)", ar.cap, ar.off);
    Timer tm(R.timed && R.st);
    tm.mark(0, s);

    // ---- validation, change points, index counts per tile
    launch_fill_u32((uint32_t *)b.bad, 1, 0u, s);
    launch_changepoints(R.t, R.n, b.flags, b.bad, s);
    scan_exclusive_u32(b.flags, b.E, R.n + 1, nullptr, b.scan_tmp, s);
    HIPCHK(hipMemcpyAsync(b.len, p.len.data(), p.L * sizeof(LenInfo), hipMemcpyHostToDevice, s));
    launch_tile_counts(b.len, p.L, b.E, p.ntiles, b.tile_off, s);
    launch_fill_u32(b.tile_off + p.ntiles, 1, 0u, s);
    scan_exclusive_u32(b.tile_off, b.tile_off, p.ntiles + 1, nullptr, b.scan_tmp, s);
    int bad = 0;
    std::vector<uint32_t> toff(p.ntiles + 1);
    HIPCHK(hipMemcpyAsync(&bad, b.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(toff.data(), b.tile_off, (p.ntiles + 1) * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, s));
    // calibration samples
    std::vector<int> cal_m;
    std::vector<std::vector<int64_t>> cal_st;
    std::vector<int64_t> cal_all(3 * 256, 0);   // lives until the sync below
    std::vector<double> cal_host;
    if (o.K == 0) {
        int idx[3] = {0, (p.L - 1) / 2, p.L - 1};
        for (int a = 0; a < 3; ++a) {
            if (a > 0 && idx[a] == idx[a - 1]) continue;
            cal_m.push_back(p.ms[idx[a]]);
            cal_st.push_back(sample_starts(p.len[idx[a]].W));
        }
        for (size_t a = 0; a < cal_m.size(); ++a)
            for (size_t w = 0; w < cal_st[a].size(); ++w) cal_all[a * 256 + w] = cal_st[a][w];
        HIPCHK(hipMemcpyAsync(b.cal_starts, cal_all.data(), cal_all.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
        for (size_t a = 0; a < cal_m.size(); ++a)
            hipLaunchKernelGGL(k_gather_windows, dim3((unsigned)cal_st[a].size()), dim3(256), 0, s,
                               R.t, (const int64_t *)b.cal_starts + a * 256,
                               (int)cal_st[a].size(), cal_m[a],
                               b.cal_win + (int64_t)a * 256 * p.max_m);
        cal_host.resize((size_t)3 * 256 * p.max_m);
        HIPCHK(hipMemcpyAsync(cal_host.data(), b.cal_win, cal_host.size() * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return fail(PMP_EINVAL, "series contains a non-finite sample");
    int K = o.K;
    if (K == 0) {
        std::vector<std::vector<std::vector<double>>> sets(cal_m.size());
        for (size_t a = 0; a < cal_m.size(); ++a)
            for (size_t w = 0; w < cal_st[a].size(); ++w) {
                const double *src = cal_host.data() + (a * 256 + w) * p.max_m;
                sets[a].emplace_back(src, src + cal_m[a]);
            }
        K = calibrate(sets, cal_m, R.n, R.budget, o.gamma, o.B);
    }
    std::vector<int64_t> cnt(p.L);
    for (int l = 0; l < p.L; ++l) {
        const int64_t t1 = l + 1 < p.L ? p.len[l + 1].tile_base : p.ntiles;
        cnt[l] = (int64_t)toff[t1] - (int64_t)toff[p.len[l].tile_base];
    }
    plan_index(p, cnt, o, R.budget, K);
    if (p.N != (int64_t)toff[p.ntiles]) return fail(PMP_EINTERNAL, "index count mismatch");
    carve2(ar, b, p, o, R.k);
    if (ar.off > ar.cap) return fail(PMP_ENOMEM, "workspace too small (%zu < %zu)", ar.cap, ar.off);
    if (R.dbg && R.dbg->join_pair_cap > 0) b.jcap = std::min(b.jcap, R.dbg->join_pair_cap);
    const int64_t N = p.N;

    // ---- per-request constants (the host vectors live until the next
    // synchronization, at the first selection)
    std::vector<float> gproj_host((size_t)p.L * o.B * kFD);
    {
        std::vector<float> one((size_t)kMaxBits * kFD);
        for (int l = 0; l < p.L; ++l) {
            projections(o.seed, p.ms[l], one.data());
            std::memcpy(gproj_host.data() + (size_t)l * o.B * kFD, one.data(),
                        (size_t)o.B * kFD * sizeof(float));
        }
    }
    HIPCHK(hipMemcpyAsync(b.gproj, gproj_host.data(), gproj_host.size() * sizeof(float),
                          hipMemcpyHostToDevice, s));
    const std::vector<LenInfo> len_host = p.len;
    HIPCHK(hipMemcpyAsync(b.len, len_host.data(), p.L * sizeof(LenInfo), hipMemcpyHostToDevice, s));
    launch_fill_u32((uint32_t *)b.emax, p.L, 0u, s);
    launch_fill_u64((uint64_t *)b.counters, C_NCOUNTERS, 0ull, s);

    Req q{};
    q.t = R.t;
    q.n = R.n;
    q.L = p.L;
    q.K = K;
    q.B = o.B;
    q.excl = R.excl;
    q.budget_R = o.gamma * R.budget;
    q.key_shift = p.key_shift;
    q.jkey_shift = p.jkey_shift;
    q.precision = o.precision;
    q.len = b.len;
    q.cell = b.cell;
    q.mu = b.mu;
    q.isig = b.isig;
    q.P = b.P;
    q.F = b.F;
    q.keyw = b.keyw;
    q.jop = b.jop;
    q.jmeta = b.jmeta;
    q.gp = b.gp;
    q.udir = o.certify ? b.udir : nullptr;
    q.skey = b.skey;
    q.sval = b.sval;
    q.perm = b.sval;
    q.pcell = b.pcell;
    q.gproj = b.gproj;
    q.emax = b.emax;
    q.counters = b.counters;
    q.bad = b.bad;
    q.kmap = b.kmap;
    q.hint = b.hint;

    // ---- one sketch pass, buckets
    std::vector<int64_t> bbase;             // lives until the call ends (async copy)
    basis_elems(p.len.data(), p.L, bbase);
    tm.mark(1, s);
    // with anchors the first pass gives records to the anchor lengths only:
    // the probe reads nothing else, and the emit stage adds those of the
    // other lengths its later steps can reach (all of them unless the k-th
    // value is 0); a debug copy of the features asks for every record here
    const bool lazy = o.stride > 1 && !(R.dbg && R.dbg->features);
    int rec_lim = p.L - 1;
    if (o.precision != 0) {
        // precision forms: the projection on the matrix cores
        HIPCHK(hipMemcpyAsync(b.bbase, bbase.data(), (p.L + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
        launch_basis(b.len, p.L, b.bbase, b.bh, b.bm, b.bl, p.max_m, s);
    }
    launch_records(p, b, q, o, p.ntiles, lazy ? kSketchAnchors : kSketchAll, s);
    tm.mark(11, s);
    // the debug copy of the key words shows all ones where no key is made
    // (the lengths between anchors)
    if (R.dbg && R.dbg->keys) launch_fill_u64(b.keyw, N, ~0ull, s);
    launch_keys(o.precision, q, p.nkblocks, s);
    tm.mark(2, s);
    if (radix_sort_pairs(b.skey, b.sval, b.skey2, b.sval2, p.Na, 0, p.key_shift + p.len_bits,
                         b.sort_tmp, s, false)) {
        // an odd number of passes leaves the sorted pairs in the scratch pair
        q.skey = b.skey2;
        q.sval = b.sval2;
        q.perm = b.sval2;
    }
    launch_bucket_bounds(q, p.Na, p.nbuckets, b.bstart, s);
    launch_hot_buckets(b.bstart, p.nbuckets, q.budget_R, &b.counters[C_HOT], s);
    launch_fill_u32(b.hint, N, kNone, s);
    tm.mark(3, s);
    tm.mark(4, s);
    // the selection after the first anchor's probe, when it settled the top-k
    std::vector<Cand> acc0;
    bool have_acc0 = false;
    // The first anchor length alone first.  When its cells already give k
    // accepted cells at 0, every cell of a longer length comes after the k-th
    // in the (P, m, i) order and can change nothing: the other anchors'
    // probes are skipped (the certificate stops at that length too).
    {
        int a1 = -1;                                   // the second anchor
        for (int l = 1; l < p.L && a1 < 0; ++l)
            if (p.len[l].anchor) a1 = l;
        const int64_t first = a1 < 0 ? p.nprobe_blocks : p.len[a1].pblk_base;
        launch_probe(o.precision, q, b.bstart, 0, first, p.max_m, s);
        bool rest = first < p.nprobe_blocks;
        if (rest && o.certify) {
            // fewer than k zeros at the first length (counted on the device,
            // in the join's pair counter, free until the certificate) cannot
            // give k accepted ones; otherwise the selection decides
            unsigned long long zeros = 0;
            launch_fill_u64((uint64_t *)b.jcount, 1, 0ull, s);
            launch_count_zero(b.P + p.len[0].kbase, p.len[0].n_index, b.jcount, s);
            HIPCHK(hipMemcpyAsync(&zeros, b.jcount, 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (zeros >= (unsigned long long)R.k) {
                const int rc = select_topk(p, b, R.k, s, acc0);
                if (rc) return rc;
                rest = !(acc0.size() == (size_t)R.k && acc0.back().d == 0.0);
                have_acc0 = !rest;
            }
        }
        if (rest)
            launch_probe(o.precision, q, b.bstart, first, p.nprobe_blocks - first, p.max_m, s);
    }
    tm.mark(5, s);
    HIPCHK(hipGetLastError());

    if (R.dbg && R.dbg->profile_pass) {
        launch_fill_u64((uint64_t *)R.dbg->profile_pass, p.cells, kInfBits, s);
        if (N)
            hipLaunchKernelGGL(k_debug_scatter, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                               b.cell, N, b.P, 0, (uint64_t *)R.dbg->profile_pass);
    }

    // ---- emit stage (Sec. 3.6, Algorithm 2); the flag of unrepresentable
    // windows and the largest feature errors come back with the first
    // selection
    std::vector<float> emax(p.L);
    HIPCHK(hipMemcpyAsync(&bad, b.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(emax.data(), b.emax, p.L * sizeof(float), hipMemcpyDeviceToHost, s));
    std::vector<Cand> acc;
    int crounds = 0;
    bool selected = false;
    // (no kernel has changed P since that selection unless the sieve runs)
    if (have_acc0 && o.sieve_w == 0) {
        acc = acc0;
        selected = true;
    }
    int rc = emit_stage(p, b, q, o, R.k, s, tm, acc, selected, crounds, lazy, rec_lim);
    if (rc) return rc;
    tm.mark(8, s);
    // the largest feature errors again, with the records the emit stage added
    if (lazy) HIPCHK(hipMemcpyAsync(emax.data(), b.emax, p.L * sizeof(float), hipMemcpyDeviceToHost, s));
    if (!selected) {
        rc = select_topk(p, b, R.k, s, acc);
        if (rc) return rc;
    } else {
        // the copies of the flag and the feature errors complete here
        HIPCHK(hipStreamSynchronize(s));
    }
    if (bad) return fail(PMP_EINVAL, "series has windows whose standard deviation underflows");
    int rounds = 0;
    double T = acc.size() == (size_t)R.k ? acc.back().d : INFINITY;
    if (R.dbg && R.dbg->t_start_scale > 0.0 && std::isfinite(T)) T *= R.dbg->t_start_scale;
    // The greedy's first k acceptances depend only on the cells whose exact
    // key (P, m, i) lies at or before the k-th accepted one: those that reach
    // it from a cell the join left inexact have upper values no lower than
    // their exact ones.  So each round makes exact every cell whose key may
    // lie at or below the bound (T, l_lim, i_lim): while T > 0 every cell at
    // or below T, whatever its start; at T = 0 only the zeros at or before the
    // k-th accepted cell in (length, start) order -- the join's queries and
    // its lengths stop there.  The round is the last once the k-th accepted
    // key after it lies within the bound.
    int l_lim = p.L - 1;
    int64_t i_lim = INT64_MAX;
    auto set_bound = [&]() {
        l_lim = p.L - 1;
        i_lim = INT64_MAX;
        if (acc.size() == (size_t)R.k && T == 0.0) {
            l_lim = acc.back().l;
            i_lim = acc.back().i;
        }
    };
    set_bound();
    int64_t nq_ops = 0;                      // windows whose join operands exist
    if (o.certify && N > 0) {
        std::vector<GridLen> gl(p.L);
        // join blocks of kJoinBlock tiles of 32 windows, each within one length
        const int64_t win_per_blk = (int64_t)kJoinTile * kJoinBlock;
        int64_t nblk = 0;
        for (int l = 0; l < p.L; ++l) {
            gl[l].blk_base = nblk;
            nblk += (p.len[l].n_index + win_per_blk - 1) / win_per_blk;
        }
        // three grid coordinates of cb3d bits each or two of cb bits, as far
        // as every length's radius resolves at that grid's cell width; else
        // one coordinate of cb_fine bits.  Each further coordinate cuts the
        // pairs the tiles form (at ECG-like data the third keeps about a
        // quarter of the pairs the first two let through)
        const int cb3d = std::min(8, (31 - p.len_bits) / 3);
        const int cb = std::min(10, (31 - p.len_bits) / 2);
        const int cb_fine = 31 - p.len_bits;
        for (;;) {
            ++rounds;
            const double Teff = std::max(T, kEps0);
            // R: radius on the join vectors G (bf16 pairs); Rf: on the FP32
            // feature copies f, which place the grid
            std::vector<double> Rl(p.L), Rf(p.L);
            bool two_d = true, three_d = true;
            for (int l = 0; l < p.L; ++l) {
                const double m = p.ms[l];
                const double nmax = m / std::sqrt(2.0) * 1.01 + 1.0;
                const double epmax = ((double)emax[l] + (5.9604644775390625e-08 + 0x1.0p-17) * nmax * 1.01) *
                                         (1.0 + 1e-6) + 1e-30;
                const double efmax = ((double)emax[l] + 5.9604644775390625e-08 * nmax * 1.01) *
                                         (1.0 + 1e-6) + 1e-30;
                const double Tr = Teff * std::sqrt(m / 2.0) * (1.0 + 1e-9);
                Rl[l] = std::isinf(Teff) ? INFINITY : Tr + 2.0 * epmax;
                Rf[l] = std::isinf(Teff) ? INFINITY : Tr + 2.0 * efmax;
                // (the lengths this round's windows belong to)
                const double cw = Rf[l] / kJoinNb;           // the cell width the radius asks for
                const bool used = p.len[l].n_index > 0 && l <= l_lim;
                if (used && cw * (double)(1u << cb) < 2.0 * (nmax * 1.001 + 1e-9)) two_d = false;
                if (used && cw * (double)(1u << cb3d) < 2.0 * (nmax * 1.001 + 1e-9)) three_d = false;
            }
            const int cb1 = three_d ? cb3d : two_d ? cb : cb_fine;
            const int cb2 = three_d ? cb3d : two_d ? cb : 0;
            const int cb3 = three_d ? cb3d : 0;
            for (int l = 0; l < p.L; ++l) {
                const double m = p.ms[l];
                const double nmax = m / std::sqrt(2.0) * 1.01 + 1.0;
                GridLen &G = gl[l];
                G.qlo = -(nmax * 1.001 + 1e-9);
                // each coordinate's cells span [qlo, -qlo] in 2^bits cells at
                // least 1/kJoinNb of the radius wide
                const double hmin = 2.0 * -G.qlo / (double)(1u << cb1) * (1.0 + 1e-9);
                const double hmin2 = 2.0 * -G.qlo / (double)(1u << std::max(cb2, 1)) * (1.0 + 1e-9);
                if (std::isinf(Rl[l])) {
                    G.R2 = INFINITY;
                    G.hinv = G.hinv2 = 0.0;
                } else {
                    G.R2 = Rl[l] * Rl[l] * (1.0 + 1e-9);
                    // coordinates are computed in FP64 from floats: 1e-12 nmax
                    // covers their rounding; cells of 1/kJoinNb of the radius
                    // put a pair within it at most kJoinNb cells apart
                    const double hr = (Rf[l] * (1.0 + 1e-9) + 1e-12 * nmax) * (1.0 + 1e-9);
                    G.hinv = 1.0 / std::max(hr / kJoinNb, hmin);
                    G.hinv2 = 1.0 / std::max(hr / kJoinNb, hmin2);
                }
                G.eps_c = 1.6e-5 * nmax;
                // per-pair test on the stored coordinates (floats, each within
                // 2^-24 nmax of its FP64 value)
                G.rp = std::isinf(Rf[l]) ? INFINITY
                                         : (float)((Rf[l] * (1.0 + 1e-6) + 0x1.0p-21 * nmax + 1e-12) * (1.0 + 1e-6));
                G.nmax2 = nmax * nmax;
                G.sqrt2m = (float)std::sqrt(2.0 / m) * (1.0f + 1e-7f);
            }
            HIPCHK(hipMemcpyAsync(b.gl, gl.data(), p.L * sizeof(GridLen), hipMemcpyHostToDevice, s));
            // windows and tiles of the lengths up to the bound (sorted by
            // length first, so they are a prefix)
            const int64_t Nq = p.len[l_lim].kbase + p.len[l_lim].n_index;
            const int64_t nbq =
                gl[l_lim].blk_base + (p.len[l_lim].n_index + win_per_blk - 1) / win_per_blk;
            // the join's operands, for the windows this round queries that
            // have none yet (the principal directions first, once)
            if (nq_ops == 0 && Nq > 0) launch_join_dirs(o.precision, q, rec_lim + 1, b.cov, b.udir, s);
            launch_join_ops(o.precision, q, nq_ops, Nq, s);
            nq_ops = std::max(nq_ops, Nq);
            launch_grid_keys(q, b.gl, Nq, cb1, cb2, cb3, l_lim, i_lim, b.jk, b.jv, b.qf, b.gp, s);
            radix_sort_pairs(b.jk, b.jv, b.jk2, b.jv2, Nq, 0, p.len_bits + cb1 + cb2 + cb3,
                             b.sort_tmp, s);
            launch_join_gather(b.jv, b.jop, b.gp, Nq, b.jop_s, b.gp_s, s);
            // the tiles in chunks of blocks, each followed by the exact stage
            // of the pairs it kept (a kernel of its own, at full occupancy).
            // A chunk is sized to fill at most half the pair buffer at the
            // largest rate of kept pairs per block seen so far in the round
            // (the first at 16 pairs per window); a wavefront that still
            // finds the buffer full verifies the rest of its pairs itself.
            launch_fill_u64((uint64_t *)b.jcount, 1, 0ull, s);
            {
                const int64_t first = std::max<int64_t>(64, b.jcap / (2 * 16 * win_per_blk));
                double rate = 0.0;                       // kept pairs per block
                for (int64_t b0 = 0; b0 < nbq;) {
                    const int64_t lim =
                        rate > 0.0 ? std::max<int64_t>(64, (int64_t)std::min(0.5 * (double)b.jcap / rate, 1e15))
                                   : first;
                    const int64_t nb = std::min(nbq - b0, lim);
                    launch_join_tiles(o.precision, q, b.gl, b.jk, b.jv, b.qf, b.jop_s, b.jmeta,
                                      b.gp_s, b0, nb, cb1, cb2, cb3, Teff, b.jpairs, b.jcount,
                                      b.jcap, s);
                    launch_join_verify(o.precision, q, b.gl, b.jpairs, b.jcount, b.jcap, Teff, s);
                    HIPCHK(hipGetLastError());
                    b0 += nb;
                    if (b0 < nbq) {
                        unsigned long long kept = 0;
                        HIPCHK(hipMemcpyAsync(&kept, b.jcount, 8, hipMemcpyDeviceToHost, s));
                        HIPCHK(hipStreamSynchronize(s));
                        rate = std::max(rate, (double)(kept + 1) / (double)nb);
                        launch_fill_u64((uint64_t *)b.jcount, 1, 0ull, s);
                    }
                }
            }
            HIPCHK(hipGetLastError());
            rc = select_topk(p, b, R.k, s, acc);   // synchronizes: gl may be rewritten next
            if (rc) return rc;
            if (std::isinf(T)) break;                               // exhaustive
            if (acc.size() == (size_t)R.k) {
                const Cand &c = acc.back();
                const bool within = c.d < T || (c.d == T && (T > 0.0 || c.l < l_lim ||
                                                             (c.l == l_lim && c.i <= i_lim)));
                if (within) break;
                T = c.d;
            } else {
                T = INFINITY;
            }
            set_bound();
            if (rounds > 64) return fail(PMP_EINTERNAL, "threshold join did not converge");
        }
    }
    tm.mark(6, s);

    // ---- exact rows of the reported cells
    const int nacc = (int)acc.size();
    std::vector<RowReq> rr(nacc);
    int64_t maxN = 1;
    for (int l = 0; l < p.L; ++l) maxN = std::max(maxN, p.len[l].n_index);
    for (int x = 0; x < nacc; ++x) {
        rr[x].l = acc[x].l;
        rr[x].pad = 0;
        rr[x].k = acc[x].k;
        double d = acc[x].d;
        memcpy(&rr[x].target, &d, 8);
    }
    std::vector<unsigned long long> rmin(nacc), rarg(nacc);
    std::vector<unsigned long long> ctr(C_NCOUNTERS);
    if (nacc) {
        HIPCHK(hipMemcpyAsync(b.rows, rr.data(), nacc * sizeof(RowReq), hipMemcpyHostToDevice, s));
        launch_fill_u64((uint64_t *)b.row_min, nacc, kInfBits, s);
        launch_fill_u64((uint64_t *)b.row_arg, nacc, ~0ull, s);
        // each reported cell's exact row: its minimum (checked against the
        // certified value) and the smallest neighbour attaining that value
        launch_rows(q, b.rows, nacc, maxN, b.row_min, b.row_arg, s);
        HIPCHK(hipMemcpyAsync(rmin.data(), b.row_min, nacc * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(rarg.data(), b.row_arg, nacc * 8, hipMemcpyDeviceToHost, s));
    }
    tm.mark(7, s);
    if (R.st)
        HIPCHK(hipMemcpyAsync(ctr.data(), b.counters, C_NCOUNTERS * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    if (nacc) {
        if (o.certify) {
            for (int x = 0; x < nacc; ++x)
                if (rmin[x] != rr[x].target) {
                    double a, bq;
                    memcpy(&a, &rmin[x], 8);
                    memcpy(&bq, &rr[x].target, 8);
                    return fail(PMP_EINTERNAL,
                                "certificate mismatch at m=%d i=%lld: row minimum %.17g, "
                                "certified value %.17g",
                                p.ms[acc[x].l], (long long)acc[x].i, a, bq);
                }
        }
    }
    for (int x = 0; x < nacc; ++x) {
        R.out[x].i = acc[x].i;
        R.out[x].j = (int64_t)rarg[x];
        R.out[x].m = p.ms[acc[x].l];
        R.out[x].flags = 0;
        R.out[x].dist = acc[x].d;
    }
    *R.n_out = nacc;

    if (R.dbg) {
        pmp_debug *d = R.dbg;
        d->K = K;
        for (int l = 0; l < p.L; ++l) {
            if (d->lengths) d->lengths[l] = p.ms[l];
            if (d->depth) d->depth[l] = p.len[l].depth;
            if (d->indexed) d->indexed[l] = p.len[l].n_index;
        }
        const unsigned gb = (unsigned)((std::max<int64_t>(N, 1) + 255) / 256);
        if (d->mu) {
            launch_fill_u64((uint64_t *)d->mu, p.cells, 0ull, s);
            if (N) hipLaunchKernelGGL(k_debug_scatter, dim3(gb), dim3(256), 0, s, b.cell, N,
                                      (const uint64_t *)b.mu, 0, (uint64_t *)d->mu);
        }
        if (d->sigma) {
            launch_fill_u64((uint64_t *)d->sigma, p.cells, 0ull, s);
            if (N) hipLaunchKernelGGL(k_debug_scatter, dim3(gb), dim3(256), 0, s, b.cell, N,
                                      (const uint64_t *)b.isig, 1, (uint64_t *)d->sigma);
        }
        if (d->profile_final) {
            launch_fill_u64((uint64_t *)d->profile_final, p.cells, kInfBits, s);
            if (N) hipLaunchKernelGGL(k_debug_scatter, dim3(gb), dim3(256), 0, s, b.cell, N, b.P, 0,
                                      (uint64_t *)d->profile_final);
        }
        if (d->keys) {
            launch_fill_u64(d->keys, p.cells, ~0ull, s);
            if (N) hipLaunchKernelGGL(k_debug_scatter, dim3(gb), dim3(256), 0, s, b.cell, N, b.keyw,
                                      0, d->keys);
        }
        if (d->perm && p.Na)
            hipLaunchKernelGGL(k_debug_perm, dim3(gb), dim3(256), 0, s, q.perm, b.cell, p.Na,
                               d->perm);
        if (d->bucket_start)
            HIPCHK(hipMemcpyAsync(d->bucket_start, b.bstart, (p.nbuckets + 1) * 4,
                                  hipMemcpyDeviceToDevice, s));
        if (d->features) {
            const size_t fb = (size_t)p.cells * kRec * (o.precision == 0 ? 8 : 4);
            launch_fill_u32((uint32_t *)d->features, (int64_t)(fb / 4), 0u, s);
            const unsigned fbk = (unsigned)((std::max<int64_t>(N, 1) + 7) / 8);
            if (N && o.precision == 0)
                hipLaunchKernelGGL(k_debug_features<double>, dim3(fbk), dim3(256), 0, s,
                                   (const double *)b.F, b.cell, N, (double *)d->features);
            else if (N)
                hipLaunchKernelGGL(k_debug_features<float>, dim3(fbk), dim3(256), 0, s,
                                   (const float *)b.F, b.cell, N, (float *)d->features);
        }
        HIPCHK(hipStreamSynchronize(s));
    }

    if (R.st) {
        pmp_stats *st = R.st;
        st->K = K;
        st->lengths = p.L;
        st->certify_rounds = rounds;
        st->cells = (uint64_t)p.cells;
        st->indexed_cells = (uint64_t)N;
        st->pass_candidates = ctr[C_PASS_CAND];
        st->pass_verified = ctr[C_PASS_VER];
        st->join_candidates = ctr[C_JOIN_CAND];
        st->join_verified = ctr[C_JOIN_VER];
        st->join_pairs = ctr[C_JOIN_PAIRS];
        st->join_windows = (uint64_t)nq_ops;
        st->probe_queries = 0;
        for (int l = 0; l < p.L; ++l)
            if (p.len[l].anchor) st->probe_queries += (uint64_t)p.len[l].n_index;
        st->sieve_verified = ctr[C_SIEVE_VER];
        st->hint_verified = ctr[C_HINT_VER];
        st->complete_verified = ctr[C_COMPL_VER];
        st->complete_rounds = crounds;
        st->anchors = p.anchors;
        st->hot_buckets = ctr[C_HOT];
        st->max_depth = p.max_depth;
        st->threshold = T;
        st->ms_total = tm.ms(0, 7);
        st->ms_onepass = tm.ms(0, 5);
        st->ms_certify = tm.ms(8, 7);
        st->ms_complete = tm.ms(5, 8);
        st->ms_sieve = tm.ms(5, 9);
        st->ms_hints = tm.ms(9, 10);
        st->ms_sketch = tm.ms(1, 11);
        st->ms_keys = tm.ms(11, 2);
        st->ms_sort = tm.ms(2, 3);
        st->ms_probe = tm.ms(4, 5);
        st->ms_join = tm.ms(8, 6);
        st->ms_rows = tm.ms(6, 7);
        st->workspace_bytes = ar.off;
    }
    return PMP_OK;
}

static int run_device(const double *d_series, int64_t n, int32_t m_min, int32_t m_max, int32_t k,
                      int32_t excl, int32_t budget, const pmp_options *opt, void *ws,
                      size_t ws_bytes, void *stream, pmp_motif *out, int32_t *n_out,
                      pmp_stats *stats, pmp_debug *dbg, bool timed = true) {
    g_err.clear();
    if (!d_series || !out || !n_out) return fail(PMP_EINVAL, "null argument");
    if (stats && stats->size != sizeof(pmp_stats)) return fail(PMP_EINVAL, "pmp_stats.size mismatch");
    if (dbg && dbg->size != sizeof(pmp_debug)) return fail(PMP_EINVAL, "pmp_debug.size mismatch");
    if (dbg && !(dbg->t_start_scale >= 0.0 && dbg->t_start_scale < 1.0))
        return fail(PMP_EINVAL, "pmp_debug.t_start_scale must lie in [0, 1)");
    if (dbg && dbg->join_pair_cap < 0)
        return fail(PMP_EINVAL, "pmp_debug.join_pair_cap must be >= 0");
    int rc = check_args(n, m_min, m_max, k, excl, budget);
    if (rc) return rc;
    Run R{};
    rc = read_options(opt, R.o);
    if (rc) return rc;
    if (!ws || ((uintptr_t)ws & 255)) return fail(PMP_EINVAL, "workspace must be 256-byte aligned");
    R.t = d_series;
    R.n = n;
    R.m_min = m_min;
    R.m_max = m_max;
    R.k = k;
    R.excl = excl;
    R.budget = budget;
    R.s = (hipStream_t)stream;
    R.out = out;
    R.n_out = n_out;
    R.st = stats;
    R.dbg = dbg;
    R.timed = timed;
    *n_out = 0;
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    try {
        return run_pipeline(R, ar);
    } catch (...) {
        return fail(PMP_EINTERNAL, "unexpected host exception");
    }
}

}  // namespace pmp

using namespace pmp;

// ------------------------------------------ fixed device scratch
// The workspace of pmp_run_device_noalloc: a device array of fixed size,
// which every GPU the library runs on holds until the process ends.  In host
// code its name is a host-side stand-in, never a device address: the address
// on each device comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is handed to kernels.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

// Address of the scratch array on the current device (looked up on the first
// call on that device).
static int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PMP_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(PMP_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PMP_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PMP_OK;
}

extern "C" {

void pmp_default_options(pmp_options *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->size = sizeof(pmp_options);
    Opt d;
    o->m_step = d.m_step;
    o->precision = d.precision;
    o->spectral_width = d.K;
    o->seed = d.seed;
    o->certify = d.certify;
    o->signature_bits = d.B;
    o->gamma = d.gamma;
    o->probe_ref_depth = d.d0;
    o->probe_cap = d.probe_cap;
    o->anchor_stride = d.stride;
    o->sieve_width = d.sieve_w;
    o->complete_rounds = d.compl_rounds;
    o->complete_dm = d.compl_dm;
    o->complete_dp = d.compl_dp;
}

const char *pmp_last_error(void) { return g_err.c_str(); }

size_t pmp_workspace_bytes(int64_t n, int32_t m_min, int32_t m_max, int32_t k,
                           const pmp_options *opt) {
    Opt o;
    if (read_options(opt, o)) return 0;
    if (check_args(n, m_min, m_max, k, 1, 1)) return 0;
    return upper_bytes(n, m_min, m_max, o, k);
}

int pmp_run_device(const double *d_series, int64_t n, int32_t m_min, int32_t m_max, int32_t k,
                   int32_t exclusion, int32_t budget, const pmp_options *opt, void *d_workspace,
                   size_t ws_bytes, void *stream, pmp_motif *out, int32_t *n_out,
                   pmp_stats *stats) {
    return run_device(d_series, n, m_min, m_max, k, exclusion, budget, opt, d_workspace, ws_bytes,
                      stream, out, n_out, stats, nullptr);
}

int pmp_run_device_noalloc(const double *d_series, int64_t n, int32_t m_min, int32_t m_max,
                           int32_t k, int32_t exclusion, int32_t budget, const pmp_options *opt,
                           void *stream, pmp_motif *out, int32_t *n_out, pmp_stats *stats) {
    g_err.clear();
    if (!d_series || !out || !n_out) return fail(PMP_EINVAL, "null argument");
    int rc = check_args(n, m_min, m_max, k, exclusion, budget);
    if (rc) return rc;
    Opt o;
    rc = read_options(opt, o);
    if (rc) return rc;
    const size_t need = upper_bytes(n, m_min, m_max, o, k);
    if (need > kScratchBytes)
        return fail(PMP_ENOMEM,
                    "request needs up to %zu bytes of scratch; pmp_run_device_noalloc holds "
                    "%zu (use pmp_run_device with a workspace)",
                    need, kScratchBytes);
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    // no phase events: creating them would allocate
    return run_device(d_series, n, m_min, m_max, k, exclusion, budget, opt, ws, kScratchBytes,
                      stream, out, n_out, stats, nullptr, false);
}

int pmp_run_device_debug(const double *d_series, int64_t n, int32_t m_min, int32_t m_max,
                         int32_t k, int32_t exclusion, int32_t budget, const pmp_options *opt,
                         void *d_workspace, size_t ws_bytes, void *stream, pmp_motif *out,
                         int32_t *n_out, pmp_stats *stats, pmp_debug *dbg) {
    return run_device(d_series, n, m_min, m_max, k, exclusion, budget, opt, d_workspace, ws_bytes,
                      stream, out, n_out, stats, dbg);
}

int pmp_open_ex(const double *series, int64_t n, int32_t m_min, int32_t m_max, int32_t k,
                int32_t exclusion, int32_t budget, const pmp_options *opt, pmp_motif *out,
                int32_t *n_out, pmp_stats *stats) {
    g_err.clear();
    if (!series || !out || !n_out) return fail(PMP_EINVAL, "null argument");
    int rc = check_args(n, m_min, m_max, k, exclusion, budget);
    if (rc) return rc;
    Opt o;
    rc = read_options(opt, o);
    if (rc) return rc;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(series[i])) return fail(PMP_EINVAL, "series contains a non-finite sample");
    const size_t ws = upper_bytes(n, m_min, m_max, o, k);
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    double *d_t = nullptr;
    void *d_ws = nullptr;
    if (hipMalloc(&d_t, (size_t)n * sizeof(double)) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return fail(PMP_ENOMEM, "device allocation of the series failed");
    }
    if (hipMalloc(&d_ws, ws) != hipSuccess) {
        (void)hipFree(d_t);
        (void)hipStreamDestroy(s);
        return fail(PMP_ENOMEM, "device allocation of %zu workspace bytes failed", ws);
    }
    rc = PMP_OK;
    if (hipMemcpyAsync(d_t, series, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        rc = fail(PMP_EDEVICE, "copy of the series failed");
    if (!rc)
        rc = run_device(d_t, n, m_min, m_max, k, exclusion, budget, opt, d_ws, ws, (void *)s, out,
                        n_out, stats, nullptr);
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_ws);
    (void)hipFree(d_t);
    (void)hipStreamDestroy(s);
    return rc;
}

int pmp_open(const double *series, int64_t n, int32_t m_min, int32_t m_max, int32_t k,
             int32_t exclusion, int32_t budget, pmp_motif *out, int32_t *n_out) {
    return pmp_open_ex(series, n, m_min, m_max, k, exclusion, budget, nullptr, out, n_out, nullptr);
}

double pmp_projection(uint64_t seed, int32_t m, int32_t l, int32_t c) { return gauss(seed, m, l, c); }

int pmp_calibrate_width(const double *series, int64_t n, int32_t m_min, int32_t m_max,
                        int32_t m_step, int32_t budget, int32_t gamma, int32_t bits, int32_t *K) {
    g_err.clear();
    if (!series || !K) return fail(PMP_EINVAL, "null argument");
    int rc = check_args(n, m_min, m_max, 1, 1, budget);
    if (rc) return rc;
    if (m_step < 1 || gamma < 1 || bits < 1 || bits > kMaxBits) return fail(PMP_EINVAL, "bad option");
    Plan p;
    plan_lengths(p, n, m_min, m_max, m_step);
    int idx[3] = {0, (p.L - 1) / 2, p.L - 1};
    std::vector<int> ms;
    std::vector<std::vector<std::vector<double>>> sets;
    for (int a = 0; a < 3; ++a) {
        if (a > 0 && idx[a] == idx[a - 1]) continue;
        const int m = p.ms[idx[a]];
        ms.push_back(m);
        std::vector<std::vector<double>> set;
        for (int64_t i : sample_starts(n - m + 1)) set.emplace_back(series + i, series + i + m);
        sets.push_back(std::move(set));
    }
    *K = calibrate(sets, ms, n, budget, gamma, bits);
    return PMP_OK;
}

}  // extern "C"
