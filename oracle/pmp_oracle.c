/*
 * pmp_oracle.c -- plain, slow CPU reference for the exact pan matrix profile.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, calls or
 * includes this file, and this file includes nothing of the library.  It is
 * loaded by the tests, by the package's smoke check and by the CPU-baseline
 * leg of the benchmark.
 *
 * Every quantity is computed in IEEE binary64 with round-to-nearest and no
 * contraction of multiply-add (build with -ffp-contract=off).  The functions
 * follow the paper's definitions directly:
 *
 *   window T_{i,m} = (t_i .. t_{i+m-1}); its z-normalized form
 *   Z = (T - mu 1)/sigma, constant windows (sigma = 0) ignored      [Sec. 2]
 *   d_m(i,j) = || Z_{i,m} - Z_{j,m} ||_2                            [Sec. 2]
 *   valid pair: |i - j| >= excl                                     [Sec. 2]
 *   P_m[i] = min over valid j of d_m(i,j), I_m[i] a minimizer      [Sec. 2, profile eq.]
 *   moments: mu = S/m, sigma^2 = Q/m - mu^2 (population)            [Sec. 3.2, update eq.]
 *   distances below eps0 = 1e-6 are reported as exactly 0           [Sec. 3.6; Sec. 4 constants]
 *   F_{i,m} = (X_1 .. X_{K'}) / sigma, K' = min(K-1, ceil(m/2)-1)   [Sec. 3.2]
 *   Parseval bound  lb^2 = (2/m) sum_{k<=K'} |F_i,k - F_j,k|^2      [Sec. 3.2, Lemma 2]
 *
 * Readings taken where the paper is silent (also listed in the design notes):
 *   - sigma is computed two-pass, (1/m) sum (t - mu)^2, which equals the
 *     paper's Q/m - mu^2 in exact arithmetic and avoids its cancellation;
 *   - a window is constant iff its m samples compare equal; constant windows
 *     have no cell (P = +inf, I = -1) and are never a neighbour;
 *   - the zero snap is strict (d < eps0) and is applied to d before the
 *     minimum and before tie decisions;
 *   - among equal (snapped) distances I_m[i] is the smallest j.
 *
 * parity: every exported function is pinned by tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EPS0 1e-6

/* ---------------------------------------------------------------- moments */

/* Two-pass population moments of one window (Sec. 3.2 running moments). */
static void win_moments(const double *w, int32_t m, double *mu, double *sig)
{
    double s = 0.0;
    for (int32_t r = 0; r < m; ++r) s += w[r];
    double mean = s / (double)m;
    double q = 0.0;
    for (int32_t r = 0; r < m; ++r) {
        double c = w[r] - mean;
        q += c * c;
    }
    *mu = mean;
    *sig = sqrt(q / (double)m);
}

/* Constant window: all m samples compare equal (Sec. 2: sigma = 0). */
static int win_const(const double *w, int32_t m)
{
    for (int32_t r = 1; r < m; ++r)
        if (w[r] != w[0]) return 0;
    return 1;
}

/* Moments and constant flags of every window of length m. */
int orc_window_stats(const double *t, int64_t n, int32_t m,
                     double *mu, double *sig, uint8_t *cst)
{
    if (m < 2 || (int64_t)m > n) return -1;
    int64_t W = n - m + 1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < W; ++i) {
        win_moments(t + i, m, &mu[i], &sig[i]);
        cst[i] = (uint8_t)win_const(t + i, m);
    }
    return 0;
}

/* -------------------------------------------------------------- distance */

/* Direct z-normalized distance from given moments, r ascending. */
static double dist_direct(const double *a, double mua, double sa,
                          const double *b, double mub, double sb, int32_t m)
{
    double acc = 0.0;
    for (int32_t r = 0; r < m; ++r) {
        double za = (a[r] - mua) / sa;
        double zb = (b[r] - mub) / sb;
        double e = za - zb;
        acc += e * e;
    }
    return sqrt(acc);
}

static double snap(double d) { return d < ORC_EPS0 ? 0.0 : d; }

/* d_m(i,j) without the snap; +inf if either window is constant. */
double orc_distance(const double *t, int64_t n, int32_t m, int64_t i, int64_t j)
{
    if (m < 2 || i < 0 || j < 0 || i + m > n || j + m > n) return NAN;
    if (win_const(t + i, m) || win_const(t + j, m)) return INFINITY;
    double mi, si, mj, sj;
    win_moments(t + i, m, &mi, &si);
    win_moments(t + j, m, &mj, &sj);
    return dist_direct(t + i, mi, si, t + j, mj, sj, m);
}

/* ---------------------------------------------------------------- profile */

/* One cell by brute force over every j, ascending; moments precomputed.
 * stop_at_zero: return at the first j whose snapped distance is 0 (that j is
 * then the smallest minimizer, since no distance is below 0). */
static void cell_scan(const double *t, int64_t W, int32_t m, int32_t excl,
                      const double *mu, const double *sig, const uint8_t *cst,
                      int64_t i, int stop_at_zero, double *P, int64_t *I)
{
    double best = INFINITY;
    int64_t arg = -1;
    if (!cst[i]) {
        for (int64_t j = 0; j < W; ++j) {
            int64_t gap = j > i ? j - i : i - j;
            if (gap < excl || cst[j]) continue;
            double d = snap(dist_direct(t + i, mu[i], sig[i], t + j, mu[j], sig[j], m));
            if (d < best) { best = d; arg = j; }
            if (stop_at_zero && best == 0.0) break;
        }
    }
    *P = best;
    *I = arg;
}

/* Full profile row pair (P_m, I_m) of one length, brute force O(W^2 m). */
int orc_profile(const double *t, int64_t n, int32_t m, int32_t excl,
                double *P, int64_t *I)
{
    if (m < 2 || (int64_t)m > n || excl < 1) return -1;
    int64_t W = n - m + 1;
    double *mu = (double *)malloc(sizeof(double) * W);
    double *sig = (double *)malloc(sizeof(double) * W);
    uint8_t *cst = (uint8_t *)malloc(W);
    if (!mu || !sig || !cst) { free(mu); free(sig); free(cst); return -2; }
    orc_window_stats(t, n, m, mu, sig, cst);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < W; ++i)
        cell_scan(t, W, m, excl, mu, sig, cst, i, 0, &P[i], &I[i]);
    free(mu); free(sig); free(cst);
    return 0;
}

/* Selected cells of one length (exact row minimum for each listed start). */
int orc_cells(const double *t, int64_t n, int32_t m, int32_t excl,
              const int64_t *starts, int64_t count, int32_t stop_at_zero,
              double *P, int64_t *I)
{
    if (m < 2 || (int64_t)m > n || excl < 1) return -1;
    int64_t W = n - m + 1;
    for (int64_t c = 0; c < count; ++c)
        if (starts[c] < 0 || starts[c] >= W) return -1;
    double *mu = (double *)malloc(sizeof(double) * W);
    double *sig = (double *)malloc(sizeof(double) * W);
    uint8_t *cst = (uint8_t *)malloc(W);
    if (!mu || !sig || !cst) { free(mu); free(sig); free(cst); return -2; }
    orc_window_stats(t, n, m, mu, sig, cst);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < count; ++c)
        cell_scan(t, W, m, excl, mu, sig, cst, starts[c], stop_at_zero, &P[c], &I[c]);
    free(mu); free(sig); free(cst);
    return 0;
}

/* ------------------------------------------------------ spectral features */

/* Aliasing-safe cap K' = min(K-1, ceil(m/2)-1)   (Sec. 3.2). */
int32_t orc_kprime(int32_t K, int32_t m)
{
    int32_t half = (m + 1) / 2 - 1;
    int32_t kp = K - 1 < half ? K - 1 : half;
    return kp < 0 ? 0 : kp;
}

/* F_{i,m}: naive DFT of the z-normalized window at bins 1..K', stored as
 * (re_1, im_1, re_2, im_2, ...), zero-padded to 2(K-1) reals (Sec. 3.2).
 * Computed from Z directly (the definition of hat X), not from X / sigma. */
int orc_features(const double *t, int64_t n, int32_t m, int64_t i, int32_t K,
                 double *F)
{
    if (m < 2 || K < 2 || i < 0 || i + m > n) return -1;
    const double *w = t + i;
    for (int32_t c = 0; c < 2 * (K - 1); ++c) F[c] = 0.0;
    if (win_const(w, m)) return 1;
    double mu, sg;
    win_moments(w, m, &mu, &sg);
    int32_t kp = orc_kprime(K, m);
    const double two_pi = 6.283185307179586476925286766559;
    for (int32_t k = 1; k <= kp; ++k) {
        double re = 0.0, im = 0.0;
        for (int32_t r = 0; r < m; ++r) {
            double z = (w[r] - mu) / sg;
            /* reduce k*r mod m before the angle so the phase is exact */
            int64_t kr = ((int64_t)k * r) % m;
            double ang = two_pi * (double)kr / (double)m;
            re += z * cos(ang);
            im -= z * sin(ang);
        }
        F[2 * (k - 1)] = re;
        F[2 * (k - 1) + 1] = im;
    }
    return 0;
}

/* Parseval lower bound (Sec. 3.2, Lemma 2) from two feature vectors. */
double orc_parseval_bound(const double *Fi, const double *Fj, int32_t K, int32_t m)
{
    int32_t kp = orc_kprime(K, m);
    double acc = 0.0;
    for (int32_t c = 0; c < 2 * kp; ++c) {
        double e = Fi[c] - Fj[c];
        acc += e * e;
    }
    return sqrt(2.0 / (double)m * acc);
}

/* --------------------------------------- seeded projections (Sec. 3.4) */

/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), used as
 * a counter-based generator: value number c of stream `seed`. */
static uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Gaussian projection g_{m,l}[c] (Sec. 3.4 SimHash: seeded Gaussian vectors
 * drawn independently per length), by Box-Muller (1958) on two uniforms of the
 * counter stream.  Counter layout: ((m * 64 + l) * 64 + c) * 2 + {0,1}. */
double orc_projection(uint64_t seed, int32_t m, int32_t l, int32_t c)
{
    uint64_t base = (((uint64_t)m * 64u + (uint64_t)l) * 64u + (uint64_t)c) * 2u;
    uint64_t a = splitmix64_at(seed, base);
    uint64_t b = splitmix64_at(seed, base + 1);
    double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;   /* (0, 1] */
    double u2 = (double)(b >> 11) * 0x1.0p-53;           /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

/* SimHash signature bits of one feature vector (Sec. 3.4): bit l (l = 0..B-1)
 * is [<g_{m,l}, F> >= 0]; bit 0 is the most significant of the B-bit word. */
uint32_t orc_signature(const double *F, int32_t K, int32_t m, int32_t B, uint64_t seed,
                       double *margins)
{
    uint32_t sig = 0;
    for (int32_t l = 0; l < B; ++l) {
        double dot = 0.0;
        for (int32_t c = 0; c < 2 * (K - 1); ++c)
            dot += orc_projection(seed, m, l, c) * F[c];
        if (margins) margins[l] = dot;
        if (dot >= 0.0) sig |= 1u << (B - 1 - l);
    }
    return sig;
}
