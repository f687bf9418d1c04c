"""GPU tests of stream sessions (Sec. 3.1, 3.5, Algorithm 1) through the C ABI.

The one-pass profile a stream keeps at its anchor lengths must be a sound
upper bound whose finite values are exact distances of valid pairs (Prop. 1);
it must not depend on how the samples were split over append calls
(Prop. 5); the exact query must equal the oracle's top-k on the samples
appended so far.  Each is checked against the oracle's brute-force profile,
its distance and its top-k on the same seeded series.
"""
import numpy as np
import pytest

from paper_2607_17481_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2607_17481_amd import pmp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pmp.lib()
    return pmp


def chunks(t, seed):
    """The series cut into pieces of random sizes (1 to 700 samples)."""
    rng = np.random.default_rng(seed)
    out, x = [], 0
    while x < len(t):
        c = int(rng.integers(1, 701))
        out.append(t[x:x + c])
        x += c
    return out


def feed(gpu, t, m_min, m_max, k, excl, batch=0, seed=None, **opt):
    s = gpu.Stream(len(t), m_min, m_max, k, excl, batch=batch,
                   opts=gpu.options(**opt) if opt else None)
    print(f"[stream] n={len(t)} m={m_min}..{m_max} excl={excl} batch={batch} "
          f"chunks={'one' if seed is None else seed} opts={opt}", flush=True)
    for c in ([t] if seed is None else chunks(t, seed)):
        s.append(c)
    s.flush()
    return s


def check_upper_profile(s, t, excl, oracle, exact_rows=None, sample=None):
    """Every anchor's profile: never below the exact one, and each finite
    value the exact distance of its (valid) recorded neighbour."""
    info = s.info()
    rng = np.random.default_rng(5)
    for a, m in enumerate(info["lengths"]):
        P, I = s.profile(a)
        if exact_rows is not None and m in exact_rows:
            Pex = exact_rows[m][0]
        else:
            Pex = oracle.profile(t, m, excl)[0]
        assert len(P) == len(Pex) == len(t) - m + 1
        fin = np.isfinite(P)
        # constant windows are never indexed, and windows with a valid
        # partner are all non-constant here only where the oracle says so
        assert np.all(np.isfinite(Pex[fin]))
        assert np.all(P[fin] >= Pex[fin] * (1 - 1e-9) - 1e-12), f"m={m}: below the exact profile"
        idx = np.nonzero(fin)[0]
        if sample is not None and len(idx) > sample:
            idx = rng.choice(idx, size=sample, replace=False)
        for q in idx.tolist():
            j = int(I[q])
            assert 0 <= j < len(P) and abs(q - j) >= excl, f"m={m} q={q}: neighbour {j}"
            d = oracle.snap(oracle.distance(t, m, q, j))
            assert parity.dist_close(P[q], d), f"m={m} q={q} j={j}: {P[q]} vs {d}"
        assert np.all(I[~fin] == -1)
    return info


TINY = dict(m_min=32, m_max=82, k=20, excl=64)


def test_stream_tiny(gpu, oracle):
    t, planted = synth.random_walk_planted(4000)
    lengths = range(TINY["m_min"], TINY["m_max"] + 1)
    with feed(gpu, t, TINY["m_min"], TINY["m_max"], TINY["k"], TINY["excl"], seed=1) as s:
        info = check_upper_profile(s, t, TINY["excl"], oracle)
        assert info["processed"] == info["appended"] == len(t)
        assert info["dropped"] == 0
        assert info["verified"] > 0 and info["updates"] > 0
        # anchors (Sec. 3.3): every s-th length from m_min, and the last
        stride = gpu.options().anchor_stride
        assert info["lengths"] == sorted(set(list(lengths)[::stride]) | {TINY["m_max"]})
        assert len(info["lengths"]) >= 2
        # one-pass top-k: valid pairs at exact distances, key order
        top = s.topk()
        assert len(top) == TINY["k"]
        for x, r in enumerate(top):
            assert r.m in info["lengths"] and abs(r.i - r.j) >= TINY["excl"]
            assert parity.dist_close(r.dist, oracle.snap(oracle.distance(t, r.m, r.i, r.j)))
            if x:
                assert (top[x - 1].dist, top[x - 1].m, top[x - 1].i) < (r.dist, r.m, r.i)
        # recall at the planted occurrences: at anchor lengths up to the
        # motif's, the window starting at an occurrence has its exact
        # profile value (its planted partner, or better, was found)
        found, cases = 0, 0
        for a, m in enumerate(info["lengths"]):
            if m > planted.motif_len:
                continue
            P, _ = s.profile(a)
            Pex = oracle.profile(t, m, TINY["excl"])[0]
            for pair in planted.pairs:
                for p in pair:
                    cases += 1
                    found += bool(P[p] <= Pex[p] * (1 + 1e-9) + 1e-12)
        print(f"[stream] planted occurrences at their exact value: {found} of {cases}", flush=True)
        assert found >= 0.8 * cases, f"{found} of {cases}"
        # exact query: the oracle's top-k over every length
        rows = oracle.pan_profile(t, lengths, TINY["excl"])
        res = s.exact()
        ok, msg = parity.check_topk(res, rows, TINY["k"], oracle, t, excl=TINY["excl"])
        assert ok, msg


def test_stream_prefix_exact(gpu, oracle):
    """Updates at sample tau use samples 0..tau only: the exact query after a
    prefix is the oracle's top-k of that prefix."""
    t, _ = synth.random_walk_planted(4000)
    lengths = range(TINY["m_min"], TINY["m_max"] + 1)
    with gpu.Stream(len(t), TINY["m_min"], TINY["m_max"], TINY["k"], TINY["excl"]) as s:
        for n1 in (1500, 2731, 4000):
            s.append(t[s.info()["appended"]:n1])
            print(f"[stream] prefix {n1}", flush=True)
            rows = oracle.pan_profile(t[:n1], lengths, TINY["excl"])
            ok, msg = parity.check_topk(s.exact(), rows, TINY["k"], oracle, t[:n1],
                                        excl=TINY["excl"])
            assert ok, f"prefix {n1}: {msg}"
            # the one-pass profile covers whole batches of the prefix only
            info = s.info()
            assert info["processed"] == n1 - n1 % TINY["excl"]
            assert len(s.profile(0)[0]) == max(0, info["processed"] - TINY["m_min"] + 1)


@pytest.mark.parametrize("batch", [0, 1, 21])
def test_stream_split_invariance(gpu, oracle, batch):
    """The same samples in one append or in many pieces give the same
    profile, bit for bit, and the same one-pass top-k (Prop. 5)."""
    t, _ = synth.random_walk_planted(2500, seed=synth.SEED_TINY + 11)
    args = (TINY["m_min"], TINY["m_max"], TINY["k"], TINY["excl"])
    with feed(gpu, t, *args, batch=batch) as s1, feed(gpu, t, *args, batch=batch, seed=7) as s2:
        info = s1.info()
        for a in range(info["anchors"]):
            P1, I1 = s1.profile(a)
            P2, I2 = s2.profile(a)
            assert P1.tobytes() == P2.tobytes() and np.array_equal(I1, I2), f"anchor {a}"
        assert [(r.i, r.j, r.m, r.dist) for r in s1.topk()] == \
               [(r.i, r.j, r.m, r.dist) for r in s2.topk()]
        if batch:
            check_upper_profile(s1, t, TINY["excl"], oracle)


def test_stream_wafer100k(gpu, oracle):
    """Wafer-like series with its constant stretches: constant windows stay
    out, the exact query equals the stored oracle top-k."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "wafer100k_top20.json")))
    t = synth.wafer_like(g["n"], g["seed"])
    with feed(gpu, t, g["m_min"], g["m_max"], g["k"], g["exclusion"], seed=3) as s:
        info = s.info()
        assert info["processed"] == len(t) and info["dropped"] == 0
        for a, m in enumerate(info["lengths"]):
            P, _ = s.profile(a)
            _, _, cst = oracle.window_stats(t, m)
            assert np.all(~np.isfinite(P[cst])), f"m={m}: a constant window has a value"
        # soundness and exact values on a sample of cells at two anchors
        rows = {m: oracle.profile_v2(t, m, g["exclusion"])[:2] for m in (info["lengths"][0],
                                                                       info["lengths"][-1])}
        for a in (0, info["anchors"] - 1):
            m = info["lengths"][a]
            P, I = s.profile(a)
            Pex = rows[m][0]
            fin = np.isfinite(P)
            assert np.all(P[fin] >= Pex[fin] * (1 - 1e-9) - 1e-12)
            idx = np.nonzero(fin)[0]
            for q in np.random.default_rng(1).choice(idx, size=min(200, len(idx)), replace=False):
                d = oracle.snap(oracle.distance(t, m, int(q), int(I[q])))
                assert parity.dist_close(P[q], d) and abs(int(q) - int(I[q])) >= g["exclusion"]
        for r in s.topk():
            assert parity.dist_close(r.dist, oracle.snap(oracle.distance(t, r.m, r.i, r.j)))
        ok, msg = parity.canonical_equal(s.exact(), g["top"])
        assert ok, msg


def test_stream_errors(gpu):
    from paper_2607_17481_amd.pmp import PMPError
    with pytest.raises(PMPError):
        gpu.Stream(1000, 32, 82, 20, 64, batch=65)          # batch > exclusion
    with pytest.raises(PMPError):
        gpu.Stream(1000, 32, 82, 20, 64, opts=gpu.options(precision=1))
    with pytest.raises(PMPError):
        gpu.Stream(50, 32, 82, 20, 64)                       # capacity < m_max
    with gpu.Stream(1000, 32, 40, 5, 16) as s:
        s.append(np.arange(600, dtype=np.float64) % 7)
        bad = np.ones(10)
        bad[3] = np.nan
        with pytest.raises(PMPError):
            s.append(bad)
        assert s.info()["appended"] == 600                   # nothing was appended
        with pytest.raises(PMPError):
            s.append(np.zeros(401))                          # past the capacity
        s.append(np.zeros(400))
        assert s.info()["appended"] == 1000
