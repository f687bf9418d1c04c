"""Oracle v2 (the screened profile) pinned against oracle v1 and the goldens.

v2 computes the closed form of Sec. 2 (d^2 = 2m(1 - rho), rho from the
dot product and the window moments) along each diagonal by the dot-product
recurrence, with a derived rounding band, and recomputes with v1's direct
formula every pair that could reach a row's minimum.  Its rows must equal
v1's bit for bit.  These CPU tests check that on the tiny planted-motif
workload, on a reduced Wafer-like workload, on the ECG-like golden, and on
inputs built to stress the band (large offsets, small deviations, exact
repeats), where the band is also audited pair by pair and shown to matter.
"""
import json
import os

import numpy as np
import pytest

from paper_2607_17481_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        return json.load(f)


def _same_rows(oracle, t, m, excl):
    P1, I1 = oracle.profile(t, m, excl)
    P2, I2, nd, _ = oracle.profile_v2(t, m, excl)
    assert np.array_equal(P1, P2), f"m={m}: P differs at {np.nonzero(P1 != P2)[0][:5]}"
    assert np.array_equal(I1, I2), f"m={m}: I differs at {np.nonzero(I1 != I2)[0][:5]}"
    return nd


def test_v2_rows_equal_v1_tiny(oracle):
    t, _ = synth.random_walk_planted()
    for m in range(32, 83, 10):
        _same_rows(oracle, t, m, 64)


def test_v2_rows_equal_v1_wafer_reduced(oracle):
    """The Wafer-like generator at n = 12,000: most windows are constant and
    the others have exact twins, so ties at 0 decide most rows."""
    t = synth.wafer_like(12_000, synth.SEED_WAFER_100K, copies=4)
    for m in (50, 75, 100):
        _same_rows(oracle, t, m, 50)


def test_v2_topk_equals_golden_tiny_and_ecg5k(oracle):
    for name in ("tiny_top20", "ecg5k_top20"):
        g = _golden(name)
        if g["generator"] == "random_walk_planted":
            t = synth.random_walk_planted(g["n"], seed=g["seed"])[0]
        else:
            t = synth.ecg_like(g["n"], g["seed"])
        lengths = range(g["m_min"], g["m_max"] + 1, g["m_step"])
        rows = oracle.pan_profile_v2(t, lengths, g["exclusion"])
        top = oracle.topk(rows, g["k"])
        assert [[x.i, x.j, x.m, x.dist] for x in top] == g["top"], name


@pytest.mark.parametrize("offset,step,band_matters",
                         [(1e4, 1e-2, False), (1e5, 1e-3, True), (1e6, 1e-2, True)])
def test_band_audit_on_adversarial_series(oracle, offset, step, band_matters):
    """Large offsets make the dot-product form cancel badly.  Every pair's
    screened value stays inside the derived band (audit ratio < 1; the
    derivation leaves it about 25x below), v2 still equals v1, and at the two
    largest offsets, without the band (scale 0), it does not: the band is
    what keeps v2 exact."""
    rng = np.random.default_rng(11)
    t = offset + np.cumsum(rng.standard_normal(3000)) * step
    t[2000:2040] = t[100:140] + 0.5 * step          # an exact repeat (distance 0)
    for m in (16, 40):
        P1, I1 = oracle.profile(t, m, 20)
        P2, I2, _, audit = oracle.profile_v2(t, m, 20, audit=True)
        assert audit < 0.5, audit
        assert np.array_equal(P1, P2) and np.array_equal(I1, I2)
        if band_matters:
            P0, I0, _, _ = oracle.profile_v2(t, m, 20, band_scale=0.0)
            assert not (np.array_equal(P1, P0) and np.array_equal(I1, I0))


def test_band_audit_on_workload_series(oracle):
    t = synth.ecg_like(3000, 5)
    for m in (100, 250):
        _, _, _, audit = oracle.profile_v2(t, m, 100, audit=True)
        assert audit < 0.5, audit


def test_screen_recomputes_few_pairs(oracle):
    """A speed property, not a correctness one: on a random walk the screen
    sends only a small fraction of the pairs to the direct formula."""
    t = np.cumsum(np.random.default_rng(3).standard_normal(6000))
    m, excl = 64, 32
    nd = _same_rows(oracle, t, m, excl)
    W = len(t) - m + 1
    pairs = (W - excl) * (W - excl + 1) // 2
    assert nd < 0.1 * pairs, (nd, pairs)


def test_v2_degenerate_inputs(oracle):
    # constant stretches, a constant series, and fewer windows than excl
    t = np.concatenate([np.zeros(200), np.arange(50.0), np.full(100, 3.0), np.arange(50.0)])
    for m in (5, 30):
        _same_rows(oracle, t, m, 10)
    P, I, nd, _ = oracle.profile_v2(np.full(100, 1.5), 10, 5)
    assert np.all(np.isinf(P)) and np.all(I == -1) and nd == 0
    P, I, _, _ = oracle.profile_v2(np.arange(30.0) ** 2, 10, 25)
    assert np.all(np.isinf(P)) and np.all(I == -1)
