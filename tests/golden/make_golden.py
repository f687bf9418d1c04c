"""Writes the stored expected values under tests/golden/.

Calls only the CPU oracle (``oracle/``) and the seeded input generators; no
value here comes from the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_2607_17481_amd import synth              # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _dump(name, meta, motifs, seconds):
    out = dict(meta)
    out["oracle_seconds"] = round(seconds, 3)
    out["top"] = [[x.i, x.j, x.m, x.dist] for x in motifs]
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, len(motifs), "motifs in", round(seconds, 2), "s")


def tiny():
    t, _ = synth.random_walk_planted()
    t0 = time.time()
    top = O.pan_topk(t, range(32, 83), 64, 20)
    _dump("tiny_top20", dict(workload="random walk + 5 planted pairs",
                             generator="random_walk_planted", n=4000,
                             seed=synth.SEED_TINY, m_min=32, m_max=82, m_step=1,
                             exclusion=64, k=20, method="brute force, every length"),
          top, time.time() - t0)


def wafer(n, seed, name):
    t = synth.wafer_like(n, seed)
    t0 = time.time()
    top = O.first_zero_topk(t, 50, 50, 20)
    assert top is not None
    _dump(name, dict(workload="wafer-like", generator="wafer_like", n=n, seed=seed,
                     m_min=50, m_max=100, m_step=1, exclusion=50, k=20,
                     method="exact scan of length-50 cells for zero cells"),
          top, time.time() - t0)


def ecg_small():
    n, seed = 5000, synth.SEED_ECG_1M
    t = synth.ecg_like(n, seed)
    t0 = time.time()
    top = O.pan_topk(t, range(100, 401, 6), 100, 20)
    _dump("ecg5k_top20", dict(workload="ecg-like", generator="ecg_like", n=n, seed=seed,
                              m_min=100, m_max=400, m_step=6, exclusion=100, k=20,
                              method="brute force, every length"),
          top, time.time() - t0)


def ecg_1m():
    """The ECG-like workload at full size (1M samples, 51 lengths) by oracle
    v2: every row exact, equal to v1's by construction (the screen only
    chooses which pairs the direct formula recomputes)."""
    n, seed = 1_000_000, synth.SEED_ECG_1M
    t = synth.ecg_like(n, seed)
    t0 = time.time()

    def progress(m, nd):
        print(f"  m={m} done, {nd} direct distances, {time.time() - t0:.0f} s", flush=True)

    rows = O.pan_profile_v2(t, range(100, 401, 6), 100, progress=progress)
    top = O.topk(rows, 20)
    _dump("ecg1m_top20", dict(workload="ecg-like", generator="ecg_like", n=n, seed=seed,
                              m_min=100, m_max=400, m_step=6, exclusion=100, k=20,
                              method="oracle v2 (closed-form screen with a rigorous band, "
                                     "direct recomputation), every length"),
          top, time.time() - t0)


JOBS = {
    "tiny": tiny,
    "wafer100k": lambda: wafer(100_000, synth.SEED_WAFER_100K, "wafer100k_top20"),
    "wafer5m": lambda: wafer(5_000_000, synth.SEED_WAFER_5M, "wafer5m_top20"),
    "ecg5k": ecg_small,
    "ecg1m": ecg_1m,
}

if __name__ == "__main__":
    O.build(force=True)
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
