// k_stream.hip -- the stream update (Sec. 3.1, 3.5, Algorithm 1) on the GPU.
//
// Samples arrive in batches of beta <= excl consecutive samples.  At every
// anchor length a batch completes up to beta windows (the windows ending at
// its samples, Sec. 3.1); no two of them form a valid pair, so they never
// search each other (Sec. 3.5).  One batch is:
//   windows  one wavefront per completed non-constant window: moments,
//            normalized spectral features F (Sec. 3.2) by a direct FP64 DFT
//            against a per-anchor basis table, their error bound, SimHash
//            key and projection margins (Sec. 3.4);
//   probe    one wavefront per completed window: its exact-prefix bucket and
//            the h Hamming-1 buckets of its smallest-margin prefix bits, at
//            most R candidates (the rest of the budget spent half on a
//            bucket's most recent entries, half at even intervals over it),
//            the Parseval prune against max(best_q, P[c]) (Lemma 2), exact
//            FP64 distances of the survivors; the query's own best is
//            written, the candidates' improvements are buffered;
//   apply    one block merges the buffered improvements into the profile;
//            equal distances resolve to the smallest query start, so the
//            result does not depend on the order the searches ran in
//            (Prop. 5);
//   runs     the batch's windows of each anchor become a new sorted run of
//            its directory, and the newest runs are merged as a binary
//            counter.
// The directory of an anchor is its indexed windows in arrival order, cut
// into runs sorted by (key, start).  A bucket at depth d is the d-bit key
// prefix, so it is one contiguous range of every run, found by binary
// search: when the population passes alpha 2^d the depth grows (Prop. 4)
// and nothing is rehomed.
#include "pmp_dev.h"

namespace pmp {

namespace {

// First position in keys[lo, hi) with key >= v.
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *__restrict__ keys,
                                                    uint32_t lo, uint32_t hi, uint32_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// First position in keys[lo, hi) with key > v.
__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t *__restrict__ keys,
                                                    uint32_t lo, uint32_t hi, uint32_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

constexpr int kFDs = 2 * (kMaxK - 1);          // 30 feature reals

}  // namespace

// Basis tables: anchor a, row c (bin k = c / 2 + 1; even rows cos, odd rows
// -sin), sample r: the value at the exact phase ((k r) mod m) / m.
__global__ __launch_bounds__(kBlock) void k_stream_basis(const SAnchor *__restrict__ anc, int na,
                                                         double *__restrict__ basis) {
    const int a = blockIdx.y;
    if (a >= na) return;
    const int m = anc[a].m, kp = anc[a].kprime;
    const int64_t o = anc[a].bbase;
    for (int x = blockIdx.x * kBlock + threadIdx.x; x < 2 * kp * m; x += gridDim.x * kBlock) {
        const int c = x / m, r = x % m;
        const int k = c / 2 + 1;
        const int64_t j = ((int64_t)k * r) % m;
        double sn, cs;
        sincospi(2.0 * (double)j / (double)m, &sn, &cs);
        basis[o + x] = (c & 1) ? -sn : cs;
    }
}

// One completed non-constant window per block (one wavefront).
__global__ __launch_bounds__(kWave) void k_stream_windows(StreamDev S) {
    extern __shared__ double ys[];                 // the window's samples, then y = x - mu
    __shared__ double s_mu, s_is;
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int a = S.la[j];
    const int64_t q = S.lq[j];
    const SAnchor &A = S.anc[a];
    const int m = A.m, kp = A.kprime;
    const int64_t cell = A.cbase + q;
    for (int r = lane; r < m; r += kWave) ys[r] = S.t[q + r];
    __syncthreads();
    if (lane == 0) {
        double mu;
        const double sg = window_moments(ys, m, mu);
        s_mu = mu;
        s_is = 1.0 / sg;
    }
    __syncthreads();
    const double mu = s_mu, is = s_is;
    double sabs = 0.0;
    for (int r = lane; r < m; r += kWave) {
        const double y = ys[r] - mu;
        ys[r] = y;
        sabs += fabs(y);
    }
    sabs = wave_sum(sabs);
    __syncthreads();
    // feature c = lane: X_c = sum_r y_r B[c][r], in order, then F = X / sigma
    double f = 0.0;
    if (lane < 2 * kp) {
        const double *b = S.basis + A.bbase + (int64_t)lane * m;
        double x = 0.0;
        for (int r = 0; r < m; ++r) x = fma(ys[r], b[r], x);
        f = x * is;
    }
    const double nrm = sqrt(wave_sum(lane < kFDs ? f * f : 0.0)) * (1.0 + 1e-15);
    // Error bound e >= ||F~ - F||.  With u = 2^-53: each y_r is the rounded
    // difference x_r - mu~ (u relative), and by Lemma 1 the bins k >= 1 of
    // x - mu~ are the window's own for any constant mu~; each basis value is
    // within 12u of the exact cos / sin (the phase 2 j / m rounded by up to
    // 2u, times pi, and sincospi's own error); the in-order sum of m
    // products adds gamma_m sum |y|.
    // Per component that is (13u + gamma_m) sum_r |y_r| (1 + 2u), over 2K'
    // components sqrt(2K') times as much; scaling by 1/sigma~ (within
    // (m + 8) u of 1/sigma, plus the product's u) adds (m + 10) u ||F||.
    const double u = 1.1102230246251565e-16;
    const double gm = (double)m * u / (1.0 - (double)m * u);
    const double ex = sqrt(2.0 * kp) * (13.0 * u + gm) * (1.0 + 2e-15) * sabs * (1.0 + (double)m * u);
    const double e = (ex * is * (1.0 + (m + 10.0) * u) + (m + 10.0) * u * nrm * 1.001) * (1.0 + 1e-6) +
                     1e-300;
    if (lane < kRec)
        S.F[cell * kRec + lane] = lane < kFDs ? f : lane == kSlotErr ? e : nrm;
    if (lane == 0) {
        S.mu[cell] = mu;
        S.isig[cell] = is;
        S.P[cell] = kInfBits;
        S.I[cell] = -1;
    }
    // SimHash (Sec. 3.4): bit l = [<g_l, F> >= 0], paper bit 1 at the key's
    // top; the margins |<g_l, F>| order the Hamming-1 probes
    double v = 0.0;
    const float *g = S.gproj + ((int64_t)a * kMaxBits + (lane < kMaxBits ? lane : 0)) * kFDs;
    for (int c = 0; c < kFDs; ++c) {
        const double fc = __shfl(f, c, kWave);
        if (lane < S.B) v = fma((double)g[c], fc, v);
    }
    const uint64_t bits = __ballot(lane < S.B && v >= 0.0);
    if (lane < kMaxBits) S.bmarg[(int64_t)j * kMaxBits + lane] = lane < S.B ? (float)fabs(v) : INFINITY;
    if (lane == 0) {
        uint32_t key = 0;
        for (int l = 0; l < S.B; ++l) key |= (uint32_t)((bits >> l) & 1ull) << (S.B - 1 - l);
        S.bkey[j] = key;
    }
}

// One completed window per block (one wavefront): candidates, prune, verify.
__global__ __launch_bounds__(kWave) void k_stream_probe(StreamDev S) {
    __shared__ uint32_t roff[kStreamMaxRuns];      // bucket offset of each run (exclusive scan)
    __shared__ uint32_t rlo[kStreamMaxRuns];       // the bucket's first position in each run
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int a = S.la[j];
    const int64_t q = S.lq[j];
    const SAnchor &A = S.anc[a];
    const int m = A.m, d = A.depth, nr = A.nruns;
    const int64_t cq = A.cbase + q;
    const double *Fq = S.F + cq * kRec;
    const double muq = S.mu[cq], isq = S.isig[cq];
    const float sqrt2m = (float)sqrt(2.0 / (double)m) * (1.0f + 1e-7f);
    const uint32_t key = S.bkey[j];

    // Hamming-1 probes: the h prefix bits of smallest margin, in that order
    int pbit[kProbeSlots];
    {
        float mg = lane < d ? S.bmarg[(int64_t)j * kMaxBits + lane] : INFINITY;
        for (int x = 0; x < kProbeSlots; ++x) {
            pbit[x] = -1;
            if (x >= A.probes) continue;
            // smallest (margin, bit) over the lanes still in
            float bm = mg;
            int bl = lane < d ? lane : kWave;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const float om = __shfl_xor(bm, off, kWave);
                const int ol = __shfl_xor(bl, off, kWave);
                if (om < bm || (om == bm && ol < bl)) {
                    bm = om;
                    bl = ol;
                }
            }
            if (bl >= d) break;
            pbit[x] = bl;
            if (lane == bl) mg = INFINITY;
        }
    }

    double best = INFINITY;                         // wave-uniform
    int32_t bestc = -1;
    unsigned long long n_cand = 0, n_ver = 0;
    int brem = S.R;
    const int sh = S.B - d;
    const uint32_t pfx = d > 0 ? key >> sh : 0u;

    // inspect one candidate per lane (c < 0: none)
    auto inspect = [&](int32_t c) {
        const bool valid = c >= 0 && q - (int64_t)c >= S.excl;
        int64_t cc = 0;
        double Pc = INFINITY, thr = INFINITY, muc = 0.0, isc = 0.0;
        bool prop = false;
        if (valid) {
            ++n_cand;
            cc = A.cbase + c;
            Pc = bitsd(S.P[cc]);
            thr = fmax(best, Pc);
            const float lb = lb_mem<double>(Fq, S.F + cc * kRec, sqrt2m);
            prop = (double)lb < thr;
            if (prop) {
                muc = S.mu[cc];
                isc = S.isig[cc];
            }
        }
        const uint64_t mask = __ballot(prop);
        double lb_d = INFINITY;
        int32_t lb_c = -1;
        if (mask)
            verify_proposals(mask, SeriesA{S.t}, S.t, q, muq, isq, (int64_t)c, muc, isc, m,
                             [&](double dd) {
                ++n_ver;
                if (dd < Pc) {
                    const uint32_t slot = atomicAdd(S.nupd, 1u);
                    if (slot < S.updcap)
                        S.upd[slot] = SUpdate{(uint32_t)cc, (int32_t)q, dbits(dd)};
                    else
                        atomicAdd(&S.counters[CS_DROP], 1ull);
                }
                if (dd < INFINITY) {
                    lb_d = dd;
                    lb_c = c;
                }
            }, exit_bound(thr));
        // the query's best over the round: smallest (distance, start)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double od = __shfl_xor(lb_d, off, kWave);
            const int32_t oc = __shfl_xor(lb_c, off, kWave);
            if (od < lb_d || (od == lb_d && (uint32_t)oc < (uint32_t)lb_c)) {
                lb_d = od;
                lb_c = oc;
            }
        }
        if (lb_c >= 0 && (lb_d < best || (lb_d == best && lb_c < bestc))) {
            best = lb_d;
            bestc = lb_c;
        }
        return valid;
    };

    for (int pi = 0; pi <= A.probes && brem > 0; ++pi) {
        uint32_t p = pfx;
        if (pi > 0) {
            if (pbit[pi - 1] < 0) break;
            p ^= 1u << (d - 1 - pbit[pi - 1]);
        }
        const uint32_t klo = d > 0 ? p << sh : 0u;
        const uint32_t khi = d > 0 ? (p + 1u) << sh : 1u << S.B;
        uint32_t lo = 0, sz = 0;
        if (lane < nr) {
            const uint32_t *keys = S.skey + A.cbase;
            lo = lower_bound_u32(keys, A.runs[lane], A.runs[lane + 1], klo);
            sz = lower_bound_u32(keys, lo, A.runs[lane + 1], khi) - lo;
        }
        uint32_t incl = sz;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += y;
        }
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        if (lane < nr) {
            roff[lane] = incl - sz;
            rlo[lane] = lo;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (total == 0) continue;
        // bucket position (runs oldest first) -> window start
        auto entry = [&](uint32_t pos) -> int32_t {
            int rl = 0, rh = nr - 1;
            while (rl < rh) {
                const int mid = (rl + rh + 1) >> 1;
                if (roff[mid] <= pos) rl = mid; else rh = mid - 1;
            }
            return (int32_t)S.perm[A.cbase + rlo[rl] + (pos - roff[rl])];
        };
        if (total <= (uint32_t)brem) {
            int used = 0;
            for (uint32_t base = 0; base < total; base += kWave) {
                const uint32_t pos = base + lane;
                used += __popcll(__ballot(inspect(pos < total ? entry(pos) : -1)));
            }
            brem -= used;
        } else {
            // more entries than budget: half on the most recent, half at
            // even intervals over the older rest
            const int nrec = brem / 2, nstr = brem - nrec;
            for (int base = 0; base < nrec; base += kWave) {
                const int x = base + lane;
                inspect(x < nrec ? entry(total - 1u - (uint32_t)x) : -1);
            }
            const uint64_t span = total - (uint32_t)nrec;
            for (int base = 0; base < nstr; base += kWave) {
                const int x = base + lane;
                inspect(x < nstr ? entry((uint32_t)((uint64_t)x * span / (uint64_t)nstr)) : -1);
            }
            brem = 0;
        }
    }
    if (lane == 0) {
        S.P[cq] = dbits(best);
        S.I[cq] = bestc;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        n_cand += __shfl_xor(n_cand, off, kWave);
        n_ver += __shfl_xor(n_ver, off, kWave);
    }
    if (lane == 0) {
        if (n_cand) atomicAdd(&S.counters[CS_CAND], n_cand);
        if (n_ver) atomicAdd(&S.counters[CS_VER], n_ver);
    }
}

// The batch's buffered improvements into the profile (one block).  Every
// buffered distance is below its cell's value when the searches started, so
// each touched cell drops to the smallest one; its neighbour is the smallest
// query start among those reaching that value.
__global__ __launch_bounds__(1024) void k_stream_apply(StreamDev S) {
    const uint32_t n = min(*S.nupd, S.updcap);
    for (uint32_t x = threadIdx.x; x < n; x += blockDim.x)
        __hip_atomic_store(&S.Icand[S.upd[x].cell], INT_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < n; x += blockDim.x)
        atomicMin((unsigned long long *)&S.P[S.upd[x].cell], (unsigned long long)S.upd[x].d);
    __syncthreads();
    // values other threads changed by atomics are read at device scope (not
    // from this compute unit's cache)
    for (uint32_t x = threadIdx.x; x < n; x += blockDim.x) {
        const SUpdate u = S.upd[x];
        if (__hip_atomic_load(&S.P[u.cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == u.d)
            atomicMin(&S.Icand[u.cell], u.j);
    }
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < n; x += blockDim.x) {
        const uint32_t c = S.upd[x].cell;
        S.I[c] = __hip_atomic_load(&S.Icand[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (n) atomicAdd(&S.counters[CS_UPD], (unsigned long long)n);
        *S.nupd = 0;
    }
}

// The batch's windows of each anchor as a new run, sorted by (key, start)
// (one block per anchor; the list holds an anchor's windows in start order).
__global__ __launch_bounds__(kBlock) void k_stream_newruns(StreamDev S) {
    const SAnchor &A = S.anc[blockIdx.x];
    const int nn = A.nnew;
    for (int i = threadIdx.x; i < nn; i += kBlock) {
        const uint32_t ki = S.bkey[A.j0 + i];
        int rank = 0;
        for (int x = 0; x < nn; ++x) {
            const uint32_t kx = S.bkey[A.j0 + x];
            rank += kx < ki || (kx == ki && x < i);
        }
        const int64_t pos = A.cbase + A.nidx + rank;
        S.skey[pos] = ki;
        S.perm[pos] = (uint32_t)S.lq[A.j0 + i];
    }
}

// Merges of the newest runs of an anchor into one (binary counter): each
// element's place is its rank in its own run plus, in every other run, the
// entries before it (an older run's equal keys come first).  Written to the
// scratch arrays, then copied back.
__global__ __launch_bounds__(kBlock) void k_stream_merge(StreamDev S, const SMerge *__restrict__ mg,
                                                         int nmerge, int64_t nthreads) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nthreads) return;
    int lo = 0, hi = nmerge - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mg[mid].first <= x) lo = mid; else hi = mid - 1;
    }
    const SMerge &M = mg[lo];
    const uint32_t e = M.runs[0] + (uint32_t)(x - M.first);
    if (e >= M.runs[M.nruns]) return;
    const uint32_t *keys = S.skey + M.cbase;
    int r = 0;
    while (r + 1 < M.nruns && M.runs[r + 1] <= e) ++r;
    const uint32_t k = keys[e];
    uint32_t out = M.runs[0] + (e - M.runs[r]);
    for (int o = 0; o < M.nruns; ++o) {
        if (o == r) continue;
        const uint32_t b0 = M.runs[o], b1 = M.runs[o + 1];
        out += (o < r ? upper_bound_u32(keys, b0, b1, k) : lower_bound_u32(keys, b0, b1, k)) - b0;
    }
    S.ktmp[M.cbase + out] = k;
    S.ptmp[M.cbase + out] = S.perm[M.cbase + e];
}

__global__ __launch_bounds__(kBlock) void k_stream_merge_back(StreamDev S,
                                                              const SMerge *__restrict__ mg,
                                                              int nmerge, int64_t nthreads) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= nthreads) return;
    int lo = 0, hi = nmerge - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mg[mid].first <= x) lo = mid; else hi = mid - 1;
    }
    const SMerge &M = mg[lo];
    const uint32_t e = M.runs[0] + (uint32_t)(x - M.first);
    if (e >= M.runs[M.nruns]) return;
    S.skey[M.cbase + e] = S.ktmp[M.cbase + e];
    S.perm[M.cbase + e] = S.ptmp[M.cbase + e];
}

__global__ __launch_bounds__(kBlock) void k_iota_u32(uint32_t *__restrict__ p, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x < n) p[x] = (uint32_t)x;
}

// ------------------------------------------------------------ launchers

static inline unsigned sblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_stream_basis(const SAnchor *anc, int na, int64_t max_elems, double *basis,
                         hipStream_t s) {
    if (na <= 0) return;
    const unsigned gx = (unsigned)std::min<int64_t>(64, (max_elems + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_stream_basis, dim3(gx, (unsigned)na), dim3(kBlock), 0, s, anc, na, basis);
}

void launch_stream_windows(const StreamDev &S, int max_m, hipStream_t s) {
    if (S.nlist <= 0) return;
    hipLaunchKernelGGL(k_stream_windows, dim3((unsigned)S.nlist), dim3(kWave),
                       (size_t)max_m * sizeof(double), s, S);
}

void launch_stream_probe(const StreamDev &S, hipStream_t s) {
    if (S.nlist <= 0) return;
    hipLaunchKernelGGL(k_stream_probe, dim3((unsigned)S.nlist), dim3(kWave), 0, s, S);
}

void launch_stream_apply(const StreamDev &S, hipStream_t s) {
    hipLaunchKernelGGL(k_stream_apply, dim3(1), dim3(1024), 0, s, S);
}

void launch_stream_newruns(const StreamDev &S, int na, hipStream_t s) {
    if (na <= 0) return;
    hipLaunchKernelGGL(k_stream_newruns, dim3((unsigned)na), dim3(kBlock), 0, s, S);
}

void launch_stream_merge(const StreamDev &S, const SMerge *mg, int nmerge, int64_t nthreads,
                         hipStream_t s) {
    if (nmerge <= 0 || nthreads <= 0) return;
    hipLaunchKernelGGL(k_stream_merge, dim3(sblk(nthreads)), dim3(kBlock), 0, s, S, mg, nmerge,
                       nthreads);
    hipLaunchKernelGGL(k_stream_merge_back, dim3(sblk(nthreads)), dim3(kBlock), 0, s, S, mg,
                       nmerge, nthreads);
}

void launch_iota_u32(uint32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota_u32, dim3(sblk(n)), dim3(kBlock), 0, s, p, n);
}

}  // namespace pmp
