"""The rounding model behind the error bound of the MFMA sketch forms (CPU).

The precision forms project each centred window y onto the DFT basis B on
the matrix cores in bf16 with FP32 accumulation, and every stored feature
vector carries a bound e_i on its error, so that the Parseval prune
(Sec. 3.2, Lemma 1) stays a true lower bound.  The bound rests on four facts
about bf16 (8 significant bits, unit roundoff u = 2^-8, round to nearest
even) that these tests check on an exact emulation in numpy:

- a float splits exactly into three bf16 parts hi + mid + lo;
- with those splits, the six products hi.hi, hi.mid, mid.hi, hi.lo, lo.hi
  and mid.mid miss y B by less than 2^-23 |y B| (form 1);
- one bf16 product misses y B by at most (2u + u^2) |y B| (form 2), and
  values at rounding ties come within 2% of that, so a bound built on
  u = 2^-9 would fail;
- the cos and sin rows of each bin hold m units of energy together, so
  over K' bins sum_rows |B_row|^2 = K' m (the Cauchy-Schwarz step).

Products of two bf16 parts, and of two floats, are exact in float64, so
the comparisons below are exact.
"""
import numpy as np

U = 2.0 ** -8                      # bf16 unit roundoff


def bf16(x):
    """Round float32 values to bf16 (nearest, ties to even), as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b << 16).astype(np.uint32).view(np.float32)


def split3(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16(x)
    r1 = (x - hi).astype(np.float32)
    mid = bf16(r1)
    lo = bf16((r1 - mid).astype(np.float32))
    return hi, mid, lo


def _floats(rng, n):
    """Random floats over many binades, plus values at bf16 rounding ties."""
    r = (rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n))).astype(np.float32)
    ties = []
    for e in range(-8, 9):
        for k in range(1, 128, 7):
            # 1 + k/128 + 1/256 (a tie at the eighth bit), and with a lower bit set
            ties.append(np.ldexp(1.0 + k / 128.0 + 1.0 / 256.0, e))
            ties.append(np.ldexp(1.0 + k / 128.0 + 1.0 / 256.0 + 2.0 ** -20, e))
            ties.append(-np.ldexp(1.0 + 1.0 / 256.0 - 2.0 ** -23, e))
    return np.concatenate([r, np.asarray(ties, dtype=np.float32)])


def test_three_way_split_is_exact():
    rng = np.random.default_rng(1)
    x = _floats(rng, 200_000)
    hi, mid, lo = split3(x)
    total = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(total, x.astype(np.float64))
    # each part is a bf16 value, and the lower parts are as small as the
    # derivation takes them: |mid| <= (1 + u) u |x|, |lo| <= u^2 |x|
    for p in (hi, mid, lo):
        assert np.array_equal(bf16(p), p)
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(mid) <= (1 + U) * U * ax)
    assert np.all(np.abs(lo) <= U * U * ax)


def test_six_products_miss_by_less_than_2_pow_minus_23():
    rng = np.random.default_rng(2)
    y = _floats(rng, 100_000)
    b = rng.permutation(_floats(rng, 100_000))[: len(y)]
    yh, ym, yl = (v.astype(np.float64) for v in split3(y))
    bh, bm, bl = (v.astype(np.float64) for v in split3(b))
    kept = yh * bh + (yh * bm + ym * bh + yh * bl + yl * bh + ym * bm)
    dropped = ym * bl + yl * bm + yl * bl
    exact = y.astype(np.float64) * b.astype(np.float64)
    assert np.allclose(kept + dropped, exact, rtol=1e-15, atol=0)
    assert np.all(np.abs(dropped) <= 2.0 ** -23 * 1.01 * np.abs(exact))
    # the five smaller products together stay below 1.03 x 2^-7 of |y B|,
    # and hi.hi within (1 + u)^2 of it
    small = np.abs(yh * bm) + np.abs(ym * bh) + np.abs(yh * bl) + np.abs(yl * bh) + np.abs(ym * bm)
    assert np.all(small <= 1.03 * 2.0 ** -7 * np.abs(exact))
    assert np.all(np.abs(yh * bh) <= (1 + U) ** 2 * np.abs(exact))


def test_one_product_bound_and_its_tightness():
    rng = np.random.default_rng(3)
    y = _floats(rng, 100_000)
    b = rng.permutation(_floats(rng, 100_000))[: len(y)]
    exact = y.astype(np.float64) * b.astype(np.float64)
    got = bf16(y).astype(np.float64) * bf16(b).astype(np.float64)
    rel = np.abs(got - exact) / np.abs(exact)
    assert np.all(rel <= 2 * U + U * U)
    # at a tie in both operands (1 + 2^-8 + 2^-20 rounds up to 1 + 2^-7) the
    # error approaches 2u: a bound with u = 2^-9 would not hold
    t = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)
    worst = abs(float(bf16(t)) ** 2 - float(t) ** 2) / float(t) ** 2
    assert worst > 0.98 * 2 * U
    assert worst > 2.01 * 2.0 ** -9


def test_basis_rows_hold_k_m_units_of_energy():
    for m in (3, 7, 16, 31, 32, 50, 101, 400):
        for kp in (1, 4, 15, 16):
            r = np.arange(m)
            e = 0.0
            for k in range(1, kp + 1):
                ph = 2.0 * np.pi * ((k * r) % m) / m
                c = np.cos(ph).astype(np.float32).astype(np.float64)
                s = np.sin(ph).astype(np.float32).astype(np.float64)
                e += float(np.sum(c * c) + np.sum(s * s))
            assert abs(e - kp * m) <= kp * m * 2.0 ** -22, (m, kp, e)
