"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every test here runs libpmp on an MI355X (gfx950) and compares its output
with the oracle on the same seeded inputs.  Bars: top-k cells and neighbours
bit-exact (ties within 1e-9 relative allowed), distances within 1e-6
relative; integer outputs (flags, keys, buckets) exact.
"""
import ctypes as C
import json
import math
import os

import numpy as np
import pytest

from paper_2607_17481_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
PRECS = {"fp64": 0, "fp32": 1, "bf16": 2}


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2607_17481_amd import pmp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pmp.lib()                                   # fails loudly if libpmp.so is missing
    return pmp


@pytest.fixture(scope="module")
def ws(gpu):
    return gpu.Workspace("cuda:0")


def run(gpu, ws, t, m_min, m_max, excl, k=20, budget=16, debug=None, **opt):
    import torch
    td = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).cuda()
    o = gpu.options(**opt)
    print(f"[run] n={len(t)} m={m_min}..{m_max} excl={excl} k={k} opts={opt}", flush=True)
    return gpu.run_device(td, m_min, m_max, k, excl, budget, o, ws, debug=debug)


def golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        return json.load(f)


def golden_series(g):
    if g["generator"] == "random_walk_planted":
        return synth.random_walk_planted(g["n"], seed=g["seed"])[0]
    if g["generator"] == "wafer_like":
        return synth.wafer_like(g["n"], g["seed"])
    return synth.ecg_like(g["n"], g["seed"])


# --------------------------------------------------------------- top-k (a7, a8)

@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("name", ["tiny_top20", "wafer100k_top20", "ecg5k_top20"])
def test_golden_topk(gpu, ws, name, prec):
    g = golden(name)
    t = golden_series(g)
    res, st = run(gpu, ws, t, g["m_min"], g["m_max"], g["exclusion"], g["k"],
                  m_step=g["m_step"], precision=PRECS[prec])
    ok, msg = parity.canonical_equal(res, g["top"])
    assert ok, msg
    assert st["certify_rounds"] >= 1


def test_wafer5m_full_size(gpu, ws, oracle):
    """The benchmark workload at full size (5M samples x 51 lengths)."""
    g = golden("wafer5m_top20")
    t = golden_series(g)
    res, st = run(gpu, ws, t, 50, 100, 50, 20)
    ok, msg = parity.canonical_equal(res, g["top"])
    assert ok, msg
    for r in res:   # each reported pair recomputed directly by the oracle
        assert abs(r.i - r.j) >= 50
        assert oracle.snap(oracle.distance(t, r.m, r.i, r.j)) == r.dist


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_ecg1m_full_size(gpu, ws, prec):
    """The precision-form workload at full size (ECG-like, 1M samples, m =
    100..400 step 6, exclusion 100, top-20), as the benchmark runs it,
    against the oracle's full profile (every cell of every length, by oracle
    v2, which equals the brute force; the committed golden).  The distance
    error of each reported motif against the oracle is printed."""
    g = golden("ecg1m_top20")
    t = golden_series(g)
    res, st = run(gpu, ws, t, g["m_min"], g["m_max"], g["exclusion"], g["k"],
                  m_step=g["m_step"], precision=PRECS[prec])
    for x, (r, ref) in enumerate(zip(res, g["top"])):
        rel = abs(r.dist - ref[3]) / ref[3] if ref[3] else abs(r.dist)
        print(f"ecg1m {prec} motif {x}: gpu ({r.i}, {r.j}, {r.m}, {r.dist!r}) "
              f"oracle {tuple(ref)} rel_err={rel:.3g}")
    ok, msg = parity.canonical_equal(res, g["top"])
    assert ok, msg
    assert st["certify_rounds"] >= 1


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_random_walk_all_lengths_profile_certified(gpu, ws, oracle, prec):
    """Full oracle profile on a ragged size: every cell the certificate
    claims exact (value <= T) equals the oracle; the rest is an upper bound."""
    t = np.cumsum(np.random.default_rng(31).standard_normal(1337))
    lengths = list(range(12, 40, 3))
    rows = oracle.pan_profile(t, lengths, 9)
    cells = sum(len(t) - m + 1 for m in lengths)
    import torch
    pf = torch.empty(cells, dtype=torch.float64, device="cuda")
    pp = torch.empty(cells, dtype=torch.float64, device="cuda")
    dbg = gpu.Debug()
    dbg.size = C.sizeof(gpu.Debug)
    dbg.profile_final = pf.data_ptr()
    dbg.profile_pass = pp.data_ptr()
    res, st = run(gpu, ws, t, 12, 39, 9, 20, debug=dbg, m_step=3, precision=PRECS[prec])
    ok, msg = parity.check_topk(res, rows, 20, oracle, t, excl=9)
    assert ok, msg
    T = st["threshold"]
    P_or = np.concatenate([rows[m][0] for m in lengths])
    P_fin = pf.cpu().numpy()
    P_pass = pp.cpu().numpy()
    fin = np.isfinite(P_or)
    # soundness of the one pass (Prop. 1) and of the final profile
    assert np.all(P_pass[fin] >= P_or[fin] * (1 - 1e-9))
    assert np.all(np.isinf(P_pass[~fin])) and np.all(np.isinf(P_fin[~fin]))
    exact = fin & (P_or <= T)
    assert exact.sum() > 0
    np.testing.assert_allclose(P_fin[exact], P_or[exact], rtol=1e-9)
    assert np.all(P_fin[fin] >= P_or[fin] * (1 - 1e-9))
    # every kernel evaluates the one canonical distance (one lane or a group
    # of eight, the same bits): where the pass already holds a cell's exact
    # value, it is bit-identical to the certified one
    same = exact.copy()
    same[exact] = np.abs(P_pass[exact] - P_fin[exact]) <= 1e-9 * P_fin[exact]
    assert same.sum() > 0.5 * exact.sum()
    assert np.array_equal(P_pass[same], P_fin[same])


# ------------------------------------------------------- stages a1 .. a6

def _debug_arrays(gpu, cells, L, precision, torch, want_keys=True):
    dbg = gpu.Debug()
    dbg.size = C.sizeof(gpu.Debug)
    bufs = {
        "mu": torch.empty(cells, dtype=torch.float64, device="cuda"),
        "sigma": torch.empty(cells, dtype=torch.float64, device="cuda"),
        "features": torch.empty(cells * 32, dtype=torch.float64 if precision == 0 else torch.float32,
                                device="cuda"),
        "keys": torch.empty(cells, dtype=torch.int64, device="cuda"),
        "profile_pass": torch.empty(cells, dtype=torch.float64, device="cuda"),
    }
    for k, v in bufs.items():
        setattr(dbg, k, v.data_ptr())
    host = {"lengths": np.zeros(L, np.int32), "depth": np.zeros(L, np.int32),
            "indexed": np.zeros(L, np.int64)}
    for k, v in host.items():
        setattr(dbg, k, v.ctypes.data)
    return dbg, bufs, host


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_moments_features_keys(gpu, ws, oracle, prec):
    import torch
    t, _ = synth.random_walk_planted()
    t = t.copy()
    t[1000:1100] = t[1000]            # a flat run: constant windows
    lengths = [32, 57, 82]
    cells = sum(len(t) - m + 1 for m in lengths)
    dbg, bufs, host = _debug_arrays(gpu, cells, 51, PRECS[prec], torch)
    seed = 12345
    # every length an anchor, so every length has keys (only anchor lengths
    # are indexed, Sec. 3.3)
    res, st = run(gpu, ws, t, 32, 82, 64, debug=dbg, precision=PRECS[prec], seed=seed,
                  m_step=25, spectral_width=16, anchor_stride=1)
    mu = bufs["mu"].cpu().numpy()
    sig = bufs["sigma"].cpu().numpy()
    F = bufs["features"].cpu().numpy().astype(np.float64).reshape(cells, 32)
    keys = bufs["keys"].cpu().numpy().view(np.uint64)
    base = 0
    rng = np.random.default_rng(0)
    worst = 0.0                       # largest err / e_i over the sampled windows
    for li, m in enumerate(lengths):
        W = len(t) - m + 1
        omu, osig, ocst = oracle.window_stats(t, m)
        # a1: moments (two-pass; the kernel sums in four interleaved partial
        # sums, so agreement is to rounding, relative to the window scale)
        scale = np.max(np.abs(t))
        np.testing.assert_allclose(mu[base:base + W][~ocst], omu[~ocst], rtol=0, atol=1e-13 * scale)
        np.testing.assert_allclose(sig[base:base + W][~ocst], osig[~ocst], rtol=1e-12)
        assert np.array_equal(sig[base:base + W] == 0.0, ocst)
        assert host["indexed"][li] == int((~ocst).sum())
        gproj = np.array([[oracle.projection(seed, m, b, c) for c in range(30)]
                          for b in range(24)])
        # a2: features within the bound the library derives for them
        for i in rng.choice(np.nonzero(~ocst)[0], size=300, replace=False):
            fo = oracle.features(t, m, int(i), 16)
            fg = F[base + i, :30]
            err = float(np.linalg.norm(fg - fo))
            e_i = F[base + i, 30]
            assert err <= e_i, (m, i, err, e_i)
            worst = max(worst, err / e_i)
            # slot 31 bounds the norm of the stored features, which are
            # within e_i of the exact ones
            assert F[base + i, 31] >= np.linalg.norm(fg) * (1 - 1e-6)
            assert F[base + i, 31] >= (np.linalg.norm(fo) - e_i) * (1 - 1e-6)
            if prec == "fp64":
                assert err <= 1e-9 * m
            if prec in ("fp32", "bf16"):
                # FP32-grade features in both precision forms (form 2 differs
                # in its keys only), and a bound of the same order
                # (sqrt(K') m per, per about 18 x 2^-23)
                assert err <= 1e-5 * np.linalg.norm(fo), (m, i, err)
                assert e_i <= 2e-5 * m, (m, i, e_i)
            # a3: signature bits where the margin clears the key error: the
            # split-bf16 projection of the FP32 copy (about 2^-16 |g| |f|),
            # or in form 2 the plain bf16 one (2^-7 sum |g_c f_c|, bf16
            # rounding of both operands, plus FP32 sums)
            sig_o, marg = oracle.signature(fo, 16, m, 24, seed)
            kw = int(keys[base + i])
            for b in range(24):
                if prec == "bf16":
                    tol = (2.0 ** -7 * 1.05 * float(np.abs(gproj[b]) @ np.abs(fo))
                           + 2 * e_i * float(np.linalg.norm(gproj[b])) + 1e-6)
                else:
                    tol = 1e-5 * np.linalg.norm(fo) * 6.0 + 2 * e_i * 6.0
                if abs(marg[b]) > tol:
                    assert ((kw >> (23 - b)) & 1) == ((sig_o >> (23 - b)) & 1), (m, i, b)
        assert np.all(keys[base:base + W][ocst] == np.uint64(0xFFFFFFFFFFFFFFFF))
        base += W
    print(f"{prec}: largest feature error / bound {worst:.3g}")


def test_projections_match_oracle_generator(gpu, oracle):
    for seed in (0, 1, 0x5eed2607):
        for m in (3, 50, 400):
            for l in (0, 7, 23):
                for c in (0, 13, 29):
                    assert gpu.projection(seed, m, l, c) == oracle.projection(seed, m, l, c)


def test_buckets_occupancy_and_order(gpu, ws, oracle):
    """a4: depth is the final state of global-depth doubling (Prop. 4), each
    bucket holds the windows whose key prefix is its index, by start (every
    length an anchor, so every length has a directory)."""
    import torch
    t = synth.wafer_like(30000, seed=5, copies=4)
    lengths = list(range(50, 60))
    cells = sum(len(t) - m + 1 for m in lengths)
    dbg, bufs, host = _debug_arrays(gpu, cells, len(lengths), 0, torch)
    res, st = run(gpu, ws, t, 50, 59, 50, debug=dbg, anchor_stride=1)   # sizes from the first call
    N = int(host["indexed"].sum())
    nb = int(sum(1 << int(d) for d in host["depth"])) + 1
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    bst = torch.empty(nb, dtype=torch.int32, device="cuda")
    dbg.perm = perm.data_ptr()
    dbg.bucket_start = bst.data_ptr()
    res, st = run(gpu, ws, t, 50, 59, 50, debug=dbg, anchor_stride=1)
    perm = perm.cpu().numpy().view(np.uint32).astype(np.int64)
    bst = bst.cpu().numpy().view(np.uint32).astype(np.int64)
    keys = bufs["keys"].cpu().numpy().view(np.uint64)
    alpha = 16
    cb = 0
    bb = 0
    slot = 0
    for li, m in enumerate(lengths):
        W = len(t) - m + 1
        Nm = int(host["indexed"][li])
        d = int(host["depth"][li])
        # Prop. 4: smallest d with N <= alpha 2^d; mean occupancy in (alpha/2, alpha]
        assert Nm <= alpha << d and (d == 0 or Nm > alpha << (d - 1))
        if d > 0:
            assert alpha / 2 < Nm / (1 << d) <= alpha
        _, _, ocst = oracle.window_stats(t, m)
        assert Nm == int((~ocst).sum())
        for b in range(1 << d):
            s0, s1 = bst[bb + b], bst[bb + b + 1]
            members = perm[s0:s1] - cb
            assert np.all(np.diff(members) > 0)
            for i in members[:8]:
                pre = (int(keys[cb + i]) & 0xFFFFFF) >> (24 - d) if d else 0
                assert pre == b
        assert bst[bb] == slot
        slot += Nm
        bb += 1 << d
        cb += W
    assert bst[bb] == slot == N



def test_directories_at_anchor_lengths_only(gpu, ws, oracle):
    """Sec. 3.3: only anchor lengths are indexed.  With stride 4 over 10
    lengths (anchors 0, 4, 8, 9) the anchors get the Prop. 4 depth and keys,
    the lengths between get depth 0, no keys (all ones) and empty buckets,
    and the bucket order lists exactly the anchors' windows."""
    import torch
    t = synth.wafer_like(30000, seed=5, copies=4)
    lengths = list(range(50, 60))
    anchors = {0, 4, 8, 9}
    cells = sum(len(t) - m + 1 for m in lengths)
    dbg, bufs, host = _debug_arrays(gpu, cells, len(lengths), 0, torch)
    res, st = run(gpu, ws, t, 50, 59, 50, debug=dbg, anchor_stride=4)
    Na = int(sum(host["indexed"][li] for li in anchors))
    nb = int(sum(1 << int(d) for d in host["depth"])) + 1
    perm = torch.empty(max(Na, 1), dtype=torch.int32, device="cuda")
    bst = torch.empty(nb, dtype=torch.int32, device="cuda")
    dbg.perm = perm.data_ptr()
    dbg.bucket_start = bst.data_ptr()
    res, st = run(gpu, ws, t, 50, 59, 50, debug=dbg, anchor_stride=4)
    perm = perm.cpu().numpy().view(np.uint32).astype(np.int64)[:Na]
    bst = bst.cpu().numpy().view(np.uint32).astype(np.int64)
    keys = bufs["keys"].cpu().numpy().view(np.uint64)
    alpha = 16
    cb = bb = slot = 0
    listed = []
    for li, m in enumerate(lengths):
        W = len(t) - m + 1
        Nm = int(host["indexed"][li])
        d = int(host["depth"][li])
        _, _, ocst = oracle.window_stats(t, m)
        if li in anchors:
            assert Nm <= alpha << d and (d == 0 or Nm > alpha << (d - 1))
            assert np.all(keys[cb:cb + W][~ocst] != np.uint64(0xFFFFFFFFFFFFFFFF))
            listed.append(cb + np.nonzero(~ocst)[0])
            assert bst[bb] == slot
            slot += Nm
        else:
            assert d == 0
            assert np.all(keys[cb:cb + W] == np.uint64(0xFFFFFFFFFFFFFFFF))
            assert bst[bb] == bst[bb + 1] == slot          # one empty bucket
        bb += 1 << d
        cb += W
    assert bst[bb] == slot == Na
    assert np.array_equal(np.sort(perm), np.sort(np.concatenate(listed)))


# ------------------------------------------------ invariances, determinism

def test_result_independent_of_width_budget_seed_precision(gpu, ws, oracle):
    """Prop. 2 (any width is sound) and the certificate: the exact top-k does
    not depend on K, alpha, the seed or the feature precision."""
    t, _ = synth.random_walk_planted(2500, seed=77)
    rows = oracle.pan_profile(t, range(40, 71, 5), 40)
    ref = oracle.topk(rows, 20)
    for kw in [dict(spectral_width=4), dict(spectral_width=8), dict(spectral_width=16),
               dict(seed=1), dict(seed=99), dict(precision=1), dict(precision=2),
               dict(signature_bits=8), dict(gamma=1), dict(probe_cap=0),
               dict(anchor_stride=1), dict(anchor_stride=2), dict(anchor_stride=3),
               dict(anchor_stride=6), dict(sieve_width=8), dict(complete_rounds=0), dict(sieve_width=8, complete_rounds=0),
               dict(anchor_stride=4, sieve_width=32, complete_rounds=1, complete_dm=0,
                    complete_dp=0)]:
        for budget in (4, 16, 64):
            res, _ = run(gpu, ws, t, 40, 70, 40, budget=budget, m_step=5, **kw)
            ok, msg = parity.check_topk(res, rows, 20, oracle, t, excl=40)
            assert ok, (kw, budget, msg)
            assert [(r.i, r.m) for r in res] == [(x.i, x.m) for x in ref]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_emit_stage_does_its_work_and_keeps_the_result(gpu, ws, oracle, prec):
    """Anchors (Sec. 3.3): with stride 2 only every second length is probed,
    the lengths between are re-cut from their anchors' hints, local
    completion runs around the top cells, and the hot-class sieve (Sec. 3.6)
    verifies the over-budget buckets; the exact top-k is the golden's in
    every configuration, and dense indexing probes more."""
    g = golden("tiny_top20")
    t = golden_series(g)
    stats = {}
    for name, kw in (("dense", dict(anchor_stride=1)), ("s2", dict(anchor_stride=2, sieve_width=8)),
                     ("s6", dict(anchor_stride=6)), ("no_emit", dict(anchor_stride=2,
                                                                     sieve_width=0,
                                                                     complete_rounds=0))):
        res, st = run(gpu, ws, t, g["m_min"], g["m_max"], g["exclusion"], g["k"], gamma=1,
                      precision=PRECS[prec], **kw)
        ok, msg = parity.canonical_equal(res, g["top"])
        assert ok, (name, msg)
        stats[name] = st
    L = g["m_max"] - g["m_min"] + 1
    assert stats["dense"]["anchors"] == L and stats["dense"]["hint_verified"] == 0
    assert stats["dense"]["complete_rounds"] == 0
    assert stats["s2"]["anchors"] == (L + 1) // 2 + (0 if (L - 1) % 2 == 0 else 1)
    assert stats["s2"]["hint_verified"] > 0 and stats["s2"]["complete_rounds"] >= 1
    assert stats["s2"]["complete_verified"] > 0
    assert stats["s2"]["pass_candidates"] < stats["dense"]["pass_candidates"]
    assert stats["s6"]["pass_candidates"] < stats["s2"]["pass_candidates"]
    # gamma = 1 makes R = 16, so the planted repeats overflow their buckets
    assert stats["s2"]["hot_buckets"] > 0 and stats["s2"]["sieve_verified"] > 0
    assert stats["no_emit"]["sieve_verified"] == 0 and stats["no_emit"]["complete_verified"] == 0


def test_sieve_on_wafer_like_duplicates(gpu, ws):
    """Wafer-like data puts thousands of exact repeats in one bucket: the
    sieve verifies its members against their projection neighbours, and the
    exact top-k stays the golden's with a small budget R."""
    g = golden("wafer100k_top20")
    t = golden_series(g)
    res, st = run(gpu, ws, t, 50, 100, 50, 20, gamma=1, sieve_width=8)
    ok, msg = parity.canonical_equal(res, g["top"])
    assert ok, msg
    assert st["hot_buckets"] > 0 and st["sieve_verified"] > 0


_ZERO_ROWS: dict = {}


@pytest.mark.parametrize("prec,stride", [("fp64", 6), ("fp64", 1), ("fp32", 6), ("bf16", 3)])
def test_zero_kth_value_spanning_lengths(gpu, ws, oracle, prec, stride):
    """Exact repeats (affine copies, distance 0) short enough that the zeros
    accepted at the shortest length run out: the k-th accepted cell is a 0 at
    the third length.  With a k-th value of 0 the certificate only has to
    settle the zeros ordered before that cell, (m, i) <= (m_k, i_k), and the
    hints only the lengths before m_k; the top-k must still be the oracle's."""
    rng = np.random.default_rng(31)
    t = np.cumsum(rng.standard_normal(3000))
    pat = t[200:230].copy()
    for a, sc, off in ((900, 2.0, 5.0), (1700, 0.5, -3.0), (2500, 1.0, 10.0)):
        t[a:a + 30] = sc * pat + off
    if not _ZERO_ROWS:
        _ZERO_ROWS.update(oracle.pan_profile_v2(t, range(16, 41), 60))
    ref = oracle.topk(_ZERO_ROWS, 20)
    assert ref[-1].dist == 0.0 and ref[-1].m == 18
    res, st = run(gpu, ws, t, 16, 40, 60, 20, precision=PRECS[prec], anchor_stride=stride)
    ok, msg = parity.check_topk(res, _ZERO_ROWS, 20, oracle, t, excl=60)
    assert ok, msg


def test_bitwise_repeatable(gpu, ws):
    t = synth.wafer_like(50000, seed=8, copies=5)
    a, _ = run(gpu, ws, t, 50, 70, 50)
    b, _ = run(gpu, ws, t, 50, 70, 50)
    assert a == b


def test_affine_invariance_and_reversal(gpu, ws, oracle):
    t = np.cumsum(np.random.default_rng(5).standard_normal(1500))
    a, _ = run(gpu, ws, t, 20, 30, 15)
    b, _ = run(gpu, ws, 3.5 * t - 11.0, 20, 30, 15)
    assert [(x.i, x.j, x.m) for x in a] == [(x.i, x.j, x.m) for x in b]
    for x, y in zip(a, b):
        assert parity.dist_close(x.dist, y.dist, 1e-9)


# ------------------------------------------------------------ edge cases

def test_no_valid_pairs(gpu, ws):
    t = np.random.default_rng(1).standard_normal(120)
    res, _ = run(gpu, ws, t, 50, 60, 80)         # W <= excl at every length
    assert res == []


def test_constant_series_has_no_motif(gpu, ws):
    res, _ = run(gpu, ws, np.full(3000, 2.5), 10, 20, 10)
    assert res == []


def test_fewer_cells_than_k(gpu, ws, oracle):
    t = np.random.default_rng(2).standard_normal(140)
    rows = oracle.pan_profile(t, [30], 90)
    res, _ = run(gpu, ws, t, 30, 30, 90, k=50)
    ok, msg = parity.check_topk(res, rows, 50, oracle, t, excl=90)
    assert ok, msg
    assert 0 < len(res) < 50


def test_duplicates_and_flat_runs(gpu, ws, oracle):
    rng = np.random.default_rng(4)
    base = rng.standard_normal(60)
    t = np.concatenate([rng.standard_normal(300), base, np.zeros(90), 2 * base + 1,
                        rng.standard_normal(211), base, np.full(40, 3.0)])
    lengths = range(16, 31, 2)
    rows = oracle.pan_profile(t, lengths, 20)
    res, _ = run(gpu, ws, t, 16, 30, 20, m_step=2)
    ok, msg = parity.check_topk(res, rows, 20, oracle, t, excl=20)
    assert ok, msg
    assert res[0].dist == 0.0


@pytest.mark.parametrize("n,lo,hi,excl", [(257, 3, 3, 1), (1001, 3, 9, 2), (777, 64, 64, 64),
                                          (2049, 100, 130, 33)])
def test_ragged_and_extreme_lengths(gpu, ws, oracle, n, lo, hi, excl):
    t = np.cumsum(np.random.default_rng(n).standard_normal(n))
    rows = oracle.pan_profile(t, range(lo, hi + 1), excl)
    res, _ = run(gpu, ws, t, lo, hi, excl)
    ok, msg = parity.check_topk(res, rows, 20, oracle, t, excl=excl)
    assert ok, msg


_KSWEEP_ROWS: dict = {}


@pytest.mark.parametrize("k", [1, 3, 150])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_k_from_one_to_many(gpu, ws, oracle, prec, k):
    """k = 1, a few, and 150 motifs, whose greedy selection (Sec. 3.6) reaches
    far down the profile (the 150th distance is 1.04 against 0.72 for the
    first), so the certificate's threshold join covers far more pairs;
    against the full oracle profile."""
    n, lo, hi, excl = 3000, 20, 40, 10
    t = np.cumsum(np.random.default_rng(77).standard_normal(n))
    if not _KSWEEP_ROWS:
        _KSWEEP_ROWS.update(oracle.pan_profile(t, range(lo, hi + 1), excl))
    res, st = run(gpu, ws, t, lo, hi, excl, k=k, precision=PRECS[prec])
    assert len(res) == k
    ok, msg = parity.check_topk(res, _KSWEEP_ROWS, k, oracle, t, excl=excl)
    assert ok, msg
    print(f"k={k} {prec}: certify rounds {st['certify_rounds']}")


def test_queried_workspace_suffices_for_large_k_at_budget_one(gpu, oracle):
    """A fresh workspace of the size pmp_workspace_bytes reports for this k
    is enough at budget 1 and 8 signature bits (the deepest directories the
    query assumes, and selection buffers of k (m_max + 1) cells), with
    k = 150; against the full oracle profile."""
    n, lo, hi, excl = 3000, 20, 40, 10
    t = np.cumsum(np.random.default_rng(77).standard_normal(n))
    if not _KSWEEP_ROWS:
        _KSWEEP_ROWS.update(oracle.pan_profile(t, range(lo, hi + 1), excl))
    fresh = gpu.Workspace("cuda:0")
    res, st = run(gpu, fresh, t, lo, hi, excl, k=150, budget=1, signature_bits=8)
    need = gpu.workspace_bytes(n, lo, hi, 150, gpu.options(signature_bits=8))
    assert fresh.buf.numel() <= need + 256 and st["workspace_bytes"] <= need
    ok, msg = parity.check_topk(res, _KSWEEP_ROWS, 150, oracle, t, excl=excl)
    assert ok, msg


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_join_pair_buffer_overflow(gpu, ws, prec):
    """The threshold join's kept pairs pass through a bounded buffer to their
    own exact-stage kernel; pairs that find it full are verified by the tiles
    in place.  With the buffer capped far below what the join keeps (one
    pair, then an eighth of the uncapped count), the top-k must equal the
    uncapped run's and the stored oracle top-k (Sec. 3.6: the join verifies
    every kept pair either way)."""
    g = golden("ecg5k_top20")
    t = golden_series(g)
    args = (gpu, ws, t, g["m_min"], g["m_max"], g["exclusion"], g["k"])
    dbg = gpu.Debug()
    dbg.size = C.sizeof(gpu.Debug)
    base, st0 = run(*args, debug=dbg, m_step=g["m_step"], precision=PRECS[prec])
    print(f"{prec} uncapped: kept {st0['join_candidates']} verified {st0['join_verified']}")
    assert st0["join_candidates"] >= 64
    for cap in (1, st0["join_candidates"] // 8):
        dbg.join_pair_cap = cap
        res, st = run(*args, debug=dbg, m_step=g["m_step"], precision=PRECS[prec])
        print(f"{prec} cap {cap}: kept {st['join_candidates']} verified {st['join_verified']}")
        assert res == base
        ok, msg = parity.canonical_equal(res, g["top"])
        assert ok, msg
    dbg.join_pair_cap = -1
    with pytest.raises(gpu.PMPError) as e:
        run(*args, debug=dbg, m_step=g["m_step"], precision=PRECS[prec])
    assert e.value.code == gpu.PMP_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_threshold_loop_past_first_round(gpu, ws, oracle, prec):
    """The certificate's threshold loop (Sec. 3.6; the greedy prefix up to T
    depends only on cells at or below T) started at a quarter of the one-pass
    threshold: it must raise T over further rounds and still report the exact
    top-k, the same as the run that starts at the one-pass threshold."""
    n, lo, hi, excl = 3000, 20, 40, 10
    t = np.cumsum(np.random.default_rng(77).standard_normal(n))
    if not _KSWEEP_ROWS:
        _KSWEEP_ROWS.update(oracle.pan_profile(t, range(lo, hi + 1), excl))
    base, st0 = run(gpu, ws, t, lo, hi, excl, precision=PRECS[prec])
    dbg = gpu.Debug()
    dbg.size = C.sizeof(gpu.Debug)
    dbg.t_start_scale = 0.25
    res, st = run(gpu, ws, t, lo, hi, excl, debug=dbg, precision=PRECS[prec])
    print(f"{prec}: certify rounds {st0['certify_rounds']} -> {st['certify_rounds']}")
    assert st["certify_rounds"] >= 2
    ok, msg = parity.check_topk(res, _KSWEEP_ROWS, 20, oracle, t, excl=excl)
    assert ok, msg
    assert res == base
    dbg.t_start_scale = 1.5
    with pytest.raises(gpu.PMPError) as e:
        run(gpu, ws, t, lo, hi, excl, debug=dbg, precision=PRECS[prec])
    assert e.value.code == gpu.PMP_EINVAL


_MAXLEN_ROWS: dict = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_longest_supported_windows(gpu, ws, oracle, prec):
    """Windows of the longest supported length (2048, where the sketch and
    probe kernels hold their largest LDS tiles), against the full oracle
    profile."""
    n, lo, hi, excl = 4500, 2046, 2048, 1024
    t = np.cumsum(np.random.default_rng(n).standard_normal(n))
    if not _MAXLEN_ROWS:
        _MAXLEN_ROWS.update(oracle.pan_profile(t, range(lo, hi + 1), excl))
    res, _ = run(gpu, ws, t, lo, hi, excl, precision=PRECS[prec])
    ok, msg = parity.check_topk(res, _MAXLEN_ROWS, 20, oracle, t, excl=excl)
    assert ok, msg


def test_invalid_arguments(gpu):
    t = np.random.default_rng(0).standard_normal(100)
    with pytest.raises(gpu.PMPError) as e:
        gpu.open_host(t, 2, 10, 5, 5)
    assert e.value.code == gpu.PMP_EINVAL
    with pytest.raises(gpu.PMPError):
        gpu.open_host(t, 10, 101, 5, 5)
    bad = t.copy()
    bad[17] = np.nan
    with pytest.raises(gpu.PMPError) as e:
        gpu.open_host(bad, 10, 20, 5, 5)
    assert e.value.code == gpu.PMP_EINVAL


def test_open_host_matches_device_path(gpu, ws):
    t, _ = synth.random_walk_planted()
    g = golden("tiny_top20")
    res = gpu.open_host(t, 32, 82, 20, 64)
    ok, msg = parity.canonical_equal(res, g["top"])
    assert ok, msg
