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
 * parity: every exported function is pinned by tests/test_oracle_pins.py;
 * the screened profile (oracle v2, at the end) by tests/test_oracle_v2.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS0 1e-6

/* OpenMP threads of the parallel loops below (1 without OpenMP). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

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

/* ============================================ oracle v2: screened profile */

/* The exact profile of one length, the same P and I as orc_profile bit for
 * bit, in O(W^2) arithmetic instead of O(W^2 m).  A cheap screen decides which
 * pairs need the direct distance; every other pair is provably not a
 * minimizer of either of its rows.
 *
 * Screen (Sec. 2, closed form).  d^2 = 2m (1 - rho) with
 * m rho = (T_i . T_j - m mu_i mu_j) / (sigma_i sigma_j).  Along a diagonal
 * j - i = k the dot product QT(i, j) = sum_r t_{i+r} t_{j+r} follows
 *     QT(i+1, j+1) = QT(i, j) - t_i t_j + t_{i+m} t_{j+m},
 * and is summed from scratch every ORC_SCREEN_REFRESH steps.  With the
 * moments mu, sigma of orc_window_stats as inputs, the screen evaluates
 *     s = 2 (m - x),  x = g QT - m (mu_i / sigma_i)(mu_j / sigma_j),
 *     g = (1 / sigma_i)(1 / sigma_j).
 *
 * Band.  Let D be the exact distance of the direct form with those same
 * moments, d_v the value dist_direct returns (the value v1 compares), u the
 * unit roundoff 2^-53 and Tmax the largest |t|.  Standard bounds for sums
 * and products give
 *   |d_v - D| <= delta = (2m + 32) u sqrt(m)
 *     (z terms rounded twice, differences once, m squares summed, a root);
 *   |s - D^2| <= Delta = g Eg + Ec, with
 *     Eg = 1.1 u Tmax^2 (6.2 m^2 + 1080 m + 1600)
 *       (the dot product: m^2 u Tmax^2 for the direct sum plus
 *        (2m + 3) u Tmax^2 per recurrence step, 255 steps at most; the
 *        products and difference forming x; and the error of the two-pass
 *        means, which enters through the mean correction), and
 *     Ec = 1.1 u (2.1 m^2 + 40 m)
 *       (the two-pass variances, which make |Z|^2 = m (1 + eta),
 *        |eta| <= (m + 5) u, and the roundings of s and of the test).
 * So d_v >= D - delta >= sqrt(max(0, s - Delta)) - delta.  A pair is
 * recomputed with dist_direct when s - Delta <= (max(best, eps0) + delta)^2
 * for either of its rows, where best is the row's smallest snapped direct
 * value so far.  Any pair that could lower a row's minimum, tie with it, or
 * snap to zero is therefore recomputed; ties go to the smallest j, as in v1.
 *
 * The tests pin the band by auditing it over every pair of small inputs with
 * large offsets and small deviations (orc_screen_audit) and by the equality
 * with orc_profile.  band_scale multiplies Eg, Ec and delta: 1 is the
 * derived band; the tests set 0 once to show that the equality depends on it.
 */
#define ORC_SCREEN_REFRESH 256    /* recurrence steps between direct sums of QT */
#define ORC_SCREEN_DIAGS   64     /* diagonals screened together by one task    */

typedef struct {
    const double *t, *mu, *sig;
    const double *is;     /* 1/sigma; NaN for windows without a cell          */
    const double *mus;    /* mu/sigma                                          */
    int64_t W;
    int32_t m, excl;
    double Eg, Ec, delta;
    double *audit;        /* non-null: every pair is also checked against the
                             band; the largest ratio is kept here (one slot per
                             thread)                                          */
} screen_ctx;

static double row_thr(double best, double delta)
{
    if (best == INFINITY) return INFINITY;
    double s = (fmax(best, ORC_EPS0) + delta) * (1.0 + 1e-12);
    return s * s;
}

/* Direct distance of a screened pair; lowers both rows' (best, arg). */
static void take_pair(const screen_ctx *c, int64_t i, int64_t j,
                      double *best, int64_t *arg, double *thr)
{
    double d = snap(dist_direct(c->t + i, c->mu[i], c->sig[i],
                                c->t + j, c->mu[j], c->sig[j], c->m));
    if (d < best[i] || (d == best[i] && j < arg[i])) {
        best[i] = d; arg[i] = j; thr[i] = row_thr(d, c->delta);
    }
    if (d < best[j] || (d == best[j] && i < arg[j])) {
        best[j] = d; arg[j] = i; thr[j] = row_thr(d, c->delta);
    }
}

/* Band audit of one pair: (s - d_v^2) / (Delta + 2 delta d_v + delta^2),
 * which the derivation above keeps within [-1, 1]. */
static double audit_pair(const screen_ctx *c, int64_t i, int64_t j, double s, double g)
{
    double dv = dist_direct(c->t + i, c->mu[i], c->sig[i],
                            c->t + j, c->mu[j], c->sig[j], c->m);
    double lim = c->Eg * g + c->Ec + 2.0 * c->delta * dv + c->delta * c->delta;
    return fabs(s - dv * dv) / lim;
}

/* Diagonals k0 .. k0+nb-1, every row; QT holds their nb dot products.  One
 * loop per row steps the dot products and tests every pair against the
 * thresholds at the start of the row.  When some pair passes, the screened
 * values are formed again (the same operations, so the same values) and the
 * passing pairs are taken smallest first, each tested again against the
 * thresholds as the pairs before it left them: a row seen for the first time
 * (threshold +inf) costs about one direct distance, not one per diagonal. */
/* Built for three instruction sets, picked when the library loads (gcc
 * function multiversioning); contraction stays off in all three, so they
 * compute the same values. */
__attribute__((target_clones("avx512f", "avx2", "default")))
static void screen_block(const screen_ctx *c, int64_t k0, int nb, double *QT,
                         double *best, int64_t *arg, double *thr, double *audit,
                         int64_t *ndirect)
{
    const int32_t m = c->m;
    const double dm = (double)m;
    const double *t = c->t;
    const int64_t W = c->W;
    const int64_t iend = W - k0;
    const double Eg = c->Eg, Ec = c->Ec;
    double w[ORC_SCREEN_DIAGS];
    for (int64_t i0 = 0; i0 < iend; i0 += ORC_SCREEN_REFRESH) {
        const int64_t i1 = i0 + ORC_SCREEN_REFRESH < iend ? i0 + ORC_SCREEN_REFRESH : iend;
        for (int64_t i = i0; i < i1; ++i) {
            const int nd = (int)(W - i - k0 < nb ? W - i - k0 : nb);
            const double *tj = t + i + k0;          /* t_j, j = i + k0 + d */
            const double gi = c->is[i], mi = dm * c->mus[i], thri = thr[i];
            const double *gj = c->is + i + k0, *uj = c->mus + i + k0, *thrj = thr + i + k0;
            int64_t any = 0;
            if (i == i0) {
                /* direct sums, r ascending for every diagonal */
                for (int d = 0; d < nd; ++d) QT[d] = 0.0;
                for (int32_t r = 0; r < m; ++r) {
                    const double a = t[i + r];
                    const double *b = tj + r;
                    for (int d = 0; d < nd; ++d) QT[d] = QT[d] + a * b[d];
                }
                for (int d = 0; d < nd; ++d) {
                    const double g = gi * gj[d];
                    const double s = 2.0 * (dm - (g * QT[d] - mi * uj[d]));
                    const double val = s - (Eg * g + Ec);
                    any |= (int64_t)((val <= thri) | (val <= thrj[d]));
                }
            } else {
                const double a0 = t[i - 1], a1 = t[i - 1 + m];
                const double *b0 = tj - 1, *b1 = tj - 1 + m;
                for (int d = 0; d < nd; ++d) {
                    const double q = (QT[d] - a0 * b0[d]) + a1 * b1[d];
                    QT[d] = q;
                    const double g = gi * gj[d];
                    const double s = 2.0 * (dm - (g * q - mi * uj[d]));
                    const double val = s - (Eg * g + Ec);
                    any |= (int64_t)((val <= thri) | (val <= thrj[d]));
                }
            }
            if (audit) {
                for (int d = 0; d < nd; ++d) {
                    const double g = gi * gj[d];
                    if (g == g) {   /* both windows have cells */
                        const double s = 2.0 * (dm - (g * QT[d] - mi * uj[d]));
                        double q = audit_pair(c, i, i + k0 + d, s, g);
                        if (q > *audit) *audit = q;
                    }
                }
            }
            if (!any) continue;
            int first = -1;
            for (int d = 0; d < nd; ++d) {
                const double g = gi * gj[d];
                const double s = 2.0 * (dm - (g * QT[d] - mi * uj[d]));
                const double val = s - (Eg * g + Ec);
                w[d] = (val <= thri) | (val <= thrj[d]) ? val : NAN;
                if (w[d] == w[d] && (first < 0 || w[d] < w[first])) first = d;
            }
            take_pair(c, i, i + k0 + first, best, arg, thr);
            ++*ndirect;
            for (int d = 0; d < nd; ++d) {
                const int64_t j = i + k0 + d;
                if (d != first && w[d] == w[d] && (w[d] <= thr[i] || w[d] <= thr[j])) {
                    take_pair(c, i, j, best, arg, thr);
                    ++*ndirect;
                }
            }
        }
    }
}

/* Screened exact profile row pair (P_m, I_m): equal to orc_profile.
 * n_direct (nullable) receives the number of direct distances computed;
 * audit (nullable) makes every pair audited and receives the largest ratio. */
int orc_profile_v2(const double *t, int64_t n, int32_t m, int32_t excl,
                   double band_scale, double *P, int64_t *I,
                   int64_t *n_direct, double *audit)
{
    if (m < 2 || (int64_t)m > n || excl < 1 || !(band_scale >= 0.0)) return -1;
    const int64_t W = n - m + 1;
    double *mu = (double *)malloc(sizeof(double) * W);
    double *sig = (double *)malloc(sizeof(double) * W);
    double *is = (double *)malloc(sizeof(double) * W);
    double *mus = (double *)malloc(sizeof(double) * W);
    uint8_t *cst = (uint8_t *)malloc(W);
    if (!mu || !sig || !is || !mus || !cst) {
        free(mu); free(sig); free(is); free(mus); free(cst);
        return -2;
    }
    orc_window_stats(t, n, m, mu, sig, cst);
    double tmax = 0.0;
    for (int64_t r = 0; r < n; ++r) tmax = fmax(tmax, fabs(t[r]));
    for (int64_t i = 0; i < W; ++i) {
        if (cst[i] || !(sig[i] > 0.0)) {   /* no cell: v1 never takes such a window */
            is[i] = NAN; mus[i] = 0.0;
        } else {
            is[i] = 1.0 / sig[i];
            mus[i] = mu[i] * is[i];
        }
    }
    const double u = 0x1.0p-53, dm = (double)m;
    screen_ctx c;
    c.t = t; c.mu = mu; c.sig = sig; c.is = is; c.mus = mus;
    c.W = W; c.m = m; c.excl = excl;
    c.Eg = band_scale * 1.1 * u * tmax * tmax * (6.2 * dm * dm + 1080.0 * dm + 1600.0);
    c.Ec = band_scale * 1.1 * u * (2.1 * dm * dm + 40.0 * dm);
    c.delta = band_scale * (2.0 * dm + 32.0) * u * sqrt(dm);

    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *best = (double *)malloc(sizeof(double) * W * nth);
    double *thr = (double *)malloc(sizeof(double) * W * nth);
    int64_t *arg = (int64_t *)malloc(sizeof(int64_t) * W * nth);
    double *aud = (double *)calloc((size_t)nth, sizeof(double));
    int64_t *ndir = (int64_t *)calloc((size_t)nth, sizeof(int64_t));
    if (!best || !thr || !arg || !aud || !ndir) {
        free(mu); free(sig); free(is); free(mus); free(cst);
        free(best); free(thr); free(arg); free(aud); free(ndir);
        return -2;
    }
    const int64_t nblk = W > excl ? (W - excl + ORC_SCREEN_DIAGS - 1) / ORC_SCREEN_DIAGS : 0;
    #pragma omp parallel num_threads(nth)
    {
        int me = 0;
#ifdef _OPENMP
        me = omp_get_thread_num();
#endif
        double *bt = best + (size_t)me * W, *th = thr + (size_t)me * W;
        int64_t *ag = arg + (size_t)me * W;
        for (int64_t i = 0; i < W; ++i) { bt[i] = INFINITY; th[i] = INFINITY; ag[i] = -1; }
        double QT[ORC_SCREEN_DIAGS];
        #pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < nblk; ++b) {
            const int64_t k0 = excl + b * ORC_SCREEN_DIAGS;
            const int nb = (int)(W - k0 < ORC_SCREEN_DIAGS ? W - k0 : ORC_SCREEN_DIAGS);
            screen_block(&c, k0, nb, QT, bt, ag, th, audit ? &aud[me] : NULL,
                         &ndir[me]);
        }
    }
    /* merge: the smallest (P, I) over the threads, per row */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < W; ++i) {
        double bp = INFINITY;
        int64_t bi = -1;
        for (int h = 0; h < nth; ++h) {
            const double p = best[(size_t)h * W + i];
            const int64_t a = arg[(size_t)h * W + i];
            if (p < bp || (p == bp && a >= 0 && (bi < 0 || a < bi))) { bp = p; bi = a; }
        }
        P[i] = bp;
        I[i] = bi;
    }
    if (audit) {
        double w = 0.0;
        for (int h = 0; h < nth; ++h) w = fmax(w, aud[h]);
        *audit = w;
    }
    if (n_direct) {
        int64_t tot = 0;
        for (int h = 0; h < nth; ++h) tot += ndir[h];
        *n_direct = tot;
    }
    free(mu); free(sig); free(is); free(mus); free(cst);
    free(best); free(thr); free(arg); free(aud); free(ndir);
    return 0;
}
