"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's formulas: each compares it with a
closed form, an identity proved in the paper, an independent library routine
(numpy FFT / corrcoef, Python's exact-rational statistics) or a brute force
written a different way.  A dropped term, a wrong sign or a transposed index
anywhere in the oracle fails at least one of them.
"""
import math
import statistics

import numpy as np
import pytest

from paper_2607_17481_amd import synth


def _series_with(*chunks, filler=37):
    rng = np.random.default_rng(123)
    parts = []
    starts = []
    pos = 0
    for c in chunks:
        starts.append(pos)
        parts.append(np.asarray(c, dtype=np.float64))
        pos += len(c)
        f = rng.standard_normal(filler)
        parts.append(f)
        pos += filler
    return np.concatenate(parts), starts


# ---------------------------------------------------------------- distance
# Section 2: d = ||Z_i - Z_j||, d^2 = 2m(1 - rho).

@pytest.mark.parametrize("m", [8, 33, 64, 101])
def test_negated_window_is_two_root_m(oracle, m):
    x = np.random.default_rng(m).standard_normal(m)
    t, (i, j) = _series_with(x, -2.5 * x + 7.0)
    d = oracle.distance(t, m, i, j)
    assert d == pytest.approx(2.0 * math.sqrt(m), rel=1e-12)


@pytest.mark.parametrize("m", [8, 50, 97])
def test_affine_copy_is_distance_zero(oracle, m):
    x = np.random.default_rng(m + 1).standard_normal(m)
    t, (i, j) = _series_with(x, 3.25 * x - 2.0)
    d = oracle.distance(t, m, i, j)
    assert d < 1e-12
    P, I = oracle.cells(t, m, 1, [i])
    assert P[0] == 0.0                   # snapped (Section 3.6)


@pytest.mark.parametrize("m", [12, 40, 77])
def test_whole_period_sine_cosine_orthogonal(oracle, m):
    r = np.arange(m)
    s = np.sin(2 * np.pi * r / m)
    c = np.cos(2 * np.pi * r / m)
    t, (i, j) = _series_with(s, c)
    assert oracle.distance(t, m, i, j) == pytest.approx(math.sqrt(2 * m), rel=1e-12)


def test_correlation_identity_and_symmetry(oracle):
    rng = np.random.default_rng(5)
    t = np.cumsum(rng.standard_normal(3000))
    for m in (10, 57, 128):
        for _ in range(20):
            i, j = rng.integers(0, len(t) - m + 1, size=2)
            d = oracle.distance(t, m, int(i), int(j))
            rho = np.corrcoef(t[i:i + m], t[j:j + m])[0, 1]
            assert d * d == pytest.approx(2 * m * (1 - rho), rel=1e-9, abs=1e-9)
            assert d == oracle.distance(t, m, int(j), int(i))      # bitwise


# ----------------------------------------------------------------- moments

def test_moments_match_exact_rational_arithmetic(oracle):
    rng = np.random.default_rng(9)
    t = 1e3 + np.cumsum(rng.standard_normal(600))        # offset stresses cancellation
    m = 45
    mu, sig, cst = oracle.window_stats(t, m)
    for i in range(0, len(t) - m + 1, 37):
        w = [float(v) for v in t[i:i + m]]
        assert mu[i] == pytest.approx(math.fsum(w) / m, rel=1e-15)
        assert sig[i] == pytest.approx(statistics.pstdev(w), rel=1e-12)
        assert not cst[i]


def test_constant_windows_have_no_cell(oracle):
    rng = np.random.default_rng(3)
    t = rng.standard_normal(400)
    t[100:160] = 0.75                      # a flat run of 60 samples
    m, excl = 20, 10
    mu, sig, cst = oracle.window_stats(t, m)
    flat = set(range(100, 160 - m + 1))
    assert set(np.nonzero(cst)[0].tolist()) == flat
    P, I = oracle.profile(t, m, excl)
    for i in flat:
        assert math.isinf(P[i]) and I[i] == -1
    assert not (set(I.tolist()) & flat)    # never anyone's neighbour


# ------------------------------------------------------ spectral features

@pytest.mark.parametrize("K", [4, 9, 16])
@pytest.mark.parametrize("m", [7, 10, 31, 64, 100])
def test_features_are_fft_of_z_window(oracle, m, K):
    rng = np.random.default_rng(m * 100 + K)
    t = np.cumsum(rng.standard_normal(400))
    i = 123
    F = oracle.features(t, m, i, K)
    w = t[i:i + m]
    z = (w - w.mean()) / w.std()
    X = np.fft.fft(z)
    kp = oracle.kprime(K, m)
    want = np.zeros(2 * (K - 1))
    want[0:2 * kp:2] = X[1:kp + 1].real
    want[1:2 * kp:2] = X[1:kp + 1].imag
    np.testing.assert_allclose(F, want, atol=1e-10 * m)
    # Lemma 1 (AC invariance): raw-window DFT divided by sigma, for k >= 1
    Xraw = np.fft.fft(w) / w.std()
    np.testing.assert_allclose(F[0:2 * kp:2], Xraw[1:kp + 1].real, atol=1e-9 * m)
    np.testing.assert_allclose(F[1:2 * kp:2], Xraw[1:kp + 1].imag, atol=1e-9 * m)


def test_kprime_aliasing_cap(oracle):
    # K' = min(K-1, ceil(m/2)-1)  (Section 3.2)
    table = {(16, 2): 0, (16, 3): 1, (16, 4): 1, (16, 10): 4, (16, 11): 5,
             (16, 30): 14, (16, 31): 15, (16, 32): 15, (16, 100): 15,
             (8, 100): 7, (4, 9): 3, (4, 5): 2}
    for (K, m), kp in table.items():
        assert oracle.kprime(K, m) == kp, (K, m)


@pytest.mark.parametrize("m", [9, 25, 63])
def test_parseval_equality_when_all_bins_kept_odd_m(oracle, m):
    # For odd m and K' = (m-1)/2 every non-DC bin is covered once by the
    # conjugate pair, so the bound equals the distance (proof of Lemma 2).
    K = (m + 1) // 2
    rng = np.random.default_rng(m)
    t = np.cumsum(rng.standard_normal(500))
    for i, j in [(0, 200), (17, 301), (250, 40)]:
        lb = oracle.parseval_bound(oracle.features(t, m, i, K),
                                   oracle.features(t, m, j, K), K, m)
        assert lb == pytest.approx(oracle.distance(t, m, i, j), rel=1e-10)


@pytest.mark.parametrize("m", [10, 48])
def test_parseval_even_m_missing_only_nyquist(oracle, m):
    K = m // 2          # K' = m/2 - 1: all bins but DC and Nyquist
    rng = np.random.default_rng(m + 7)
    t = np.cumsum(rng.standard_normal(400))
    i, j = 5, 250
    lb = oracle.parseval_bound(oracle.features(t, m, i, K),
                               oracle.features(t, m, j, K), K, m)
    d = oracle.distance(t, m, i, j)
    zi = (t[i:i + m] - t[i:i + m].mean()) / t[i:i + m].std()
    zj = (t[j:j + m] - t[j:j + m].mean()) / t[j:j + m].std()
    nyq = abs(np.fft.fft(zi)[m // 2] - np.fft.fft(zj)[m // 2]) ** 2 / m
    assert lb * lb + nyq == pytest.approx(d * d, rel=1e-10)


def test_bound_below_distance_and_monotone_in_K(oracle):
    # Lemma 2 and Proposition 2 (i)
    rng = np.random.default_rng(11)
    t = np.cumsum(rng.standard_normal(2000))
    for m in (6, 20, 50, 99):
        for _ in range(25):
            i, j = (int(v) for v in rng.integers(0, len(t) - m + 1, size=2))
            d = oracle.distance(t, m, i, j)
            prev = 0.0
            for K in (2, 3, 5, 8, 12, 16, 24):
                lb = oracle.parseval_bound(oracle.features(t, m, i, K),
                                           oracle.features(t, m, j, K), K, m)
                assert lb <= d * (1 + 1e-12) + 1e-12
                assert lb >= prev * (1 - 1e-12) - 1e-12
                prev = lb


def test_energy_of_z_window(oracle):
    # sum_k |X_k|^2 = m^2 over all bins; the stored half carries at most m^2/2
    rng = np.random.default_rng(2)
    t = np.cumsum(rng.standard_normal(300))
    for m in (11, 40):
        K = (m + 1) // 2 + 1
        F = oracle.features(t, m, 10, K)
        stored = float(np.sum(F ** 2))
        assert stored <= m * m / 2 * (1 + 1e-12)
        if m % 2 == 1:
            assert 2 * stored == pytest.approx(m * m, rel=1e-11)


# ----------------------------------------------------------------- profile

def _profile_by_corrcoef(t, m, excl):
    """Brute force written differently: Pearson matrix -> d = sqrt(2m(1-rho))."""
    W = len(t) - m + 1
    win = np.stack([t[i:i + m] for i in range(W)])
    rho = np.corrcoef(win)
    D = np.sqrt(np.maximum(0.0, 2 * m * (1 - rho)))
    idx = np.arange(W)
    D[np.abs(idx[:, None] - idx[None, :]) < excl] = np.inf
    D[D < 1e-6] = 0.0
    return D.min(axis=1), D.argmin(axis=1)


@pytest.mark.parametrize("m,excl", [(16, 8), (20, 20), (37, 5)])
def test_profile_matches_independent_brute_force(oracle, m, excl):
    t = np.cumsum(np.random.default_rng(m).standard_normal(350))
    P, I = oracle.profile(t, m, excl)
    P2, I2 = _profile_by_corrcoef(t, m, excl)
    np.testing.assert_allclose(P, P2, rtol=1e-7, atol=1e-7)
    assert np.array_equal(I, I2)
    for i in range(len(P)):
        assert abs(I[i] - i) >= excl


def test_profile_affine_invariance(oracle):
    t = np.cumsum(np.random.default_rng(17).standard_normal(400))
    for m in (16, 25):
        P, I = oracle.profile(t, m, 8)
        P2, I2 = oracle.profile(4.0 * t - 3.0, m, 8)
        np.testing.assert_allclose(P2, P, rtol=1e-9)
        assert np.array_equal(I, I2)


def test_profile_time_reversal(oracle):
    t = np.cumsum(np.random.default_rng(19).standard_normal(300))
    m, excl = 20, 10
    P, I = oracle.profile(t, m, excl)
    Pr, Ir = oracle.profile(t[::-1].copy(), m, excl)
    W = len(t) - m + 1
    np.testing.assert_allclose(Pr[::-1], P, rtol=1e-9)
    assert np.array_equal(W - 1 - Ir[::-1], I)


def test_planted_pairs_are_nearest_neighbours(oracle):
    t, info = synth.random_walk_planted()
    m = info.motif_len
    P, I = oracle.profile(t, m, m)
    med = float(np.median(P[np.isfinite(P)]))
    for p, q in info.pairs:
        assert abs(int(I[p]) - q) <= 3, (p, q, I[p])
        assert abs(int(I[q]) - p) <= 3, (p, q, I[q])
        assert P[p] < 0.25 * med


# ------------------------------------------------------------------- top-k
# Section 2: sort cells by distance; skip a cell within m/2 of an accepted
# cell at the same length.

def _rows(spec, W=60):
    rows = {}
    for m, cells in spec.items():
        P = np.full(W, np.inf)
        I = np.full(W, -1, dtype=np.int64)
        for i, (d, j) in cells.items():
            P[i], I[i] = d, j
        rows[m] = (P, I)
    return rows


def test_topk_within_half_m_is_inclusive(oracle):
    rows = _rows({10: {0: (0.1, 30), 5: (0.2, 40), 6: (0.3, 41)}})
    got = [(x.i, x.m) for x in oracle.topk(rows, 3)]
    assert got == [(0, 10), (6, 10)]       # 2*5 <= 10 skipped, 2*6 > 10 kept


def test_topk_tie_order_is_length_then_start(oracle):
    rows = _rows({12: {3: (0.5, 30)}, 10: {8: (0.5, 40), 2: (0.5, 50)}})
    got = [(x.m, x.i) for x in oracle.topk(rows, 3)]
    assert got == [(10, 2), (10, 8), (12, 3)]


def test_topk_cells_not_pairs_and_per_length_suppression(oracle):
    rows = _rows({10: {3: (0.1, 40), 40: (0.1, 3)}, 11: {3: (0.2, 40)}})
    got = [(x.i, x.j, x.m) for x in oracle.topk(rows, 5)]
    assert got == [(3, 40, 10), (40, 3, 10), (3, 40, 11)]


# ----------------------------------------------------- special-case shortcut

def test_first_zero_shortcut_equals_full_brute_force(oracle):
    t = synth.wafer_like(6000, seed=99, copies=2)
    lengths = range(50, 54)
    full = oracle.pan_topk(t, lengths, 50, 20)
    fast = oracle.first_zero_topk(t, 50, 50, 20)
    assert fast is not None
    assert full == fast
    assert all(x.dist == 0.0 and x.m == 50 for x in full)


# ------------------------------------------- projections and signatures

def test_projections_are_standard_gaussian(oracle):
    from scipy import stats
    g = np.array([oracle.projection(7, m, l, c)
                  for m in range(40, 60) for l in range(24) for c in range(30)])
    assert abs(g.mean()) < 0.03
    assert abs(g.var() - 1.0) < 0.03
    assert stats.kstest(g, "norm").pvalue > 1e-3


def test_simhash_collision_frequency_fact1(oracle):
    # Fact 1: P[sign<g,u> != sign<g,v>] = theta / pi
    K = 16
    u = np.zeros(30); u[0] = 1.0
    for theta in (0.3, 1.0, 2.0):
        v = np.zeros(30); v[0] = math.cos(theta); v[1] = math.sin(theta)
        diff = 0
        total = 0
        for m in range(20, 220):
            su, _ = oracle.signature(u, K, m, 24, 11)
            sv, _ = oracle.signature(v, K, m, 24, 11)
            diff += bin(su ^ sv).count("1")
            total += 24
        p = theta / math.pi
        assert abs(diff / total - p) < 4 * math.sqrt(p * (1 - p) / total)


def test_signature_scale_and_sign(oracle):
    rng = np.random.default_rng(4)
    F = rng.standard_normal(30)
    s, mg = oracle.signature(F, 16, 50, 24, 3)
    s2, _ = oracle.signature(3.0 * F, 16, 50, 24, 3)
    s3, _ = oracle.signature(-F, 16, 50, 24, 3)
    assert s == s2
    assert s3 == (~s) & ((1 << 24) - 1)
    # bit 0 of the paper is the most significant bit of the word
    assert ((s >> 23) & 1) == (1 if mg[0] >= 0 else 0)
