"""Comparison helpers for the GPU parity tests (test infrastructure).

Bar: top-k index sets bit-exact, ties within 1e-9 relative
allowed; distances within 1e-6 relative (values below the 1e-6 zero snap are
both 0).
"""
from __future__ import annotations

import numpy as np

REL_DIST = 1e-6
REL_TIE = 1e-9


def dist_close(a: float, b: float, rel: float = REL_DIST) -> bool:
    if a == 0.0 or b == 0.0:
        return a == b
    return abs(a - b) <= rel * max(abs(a), abs(b))


def canonical_equal(gpu, ref) -> tuple[bool, str]:
    """gpu: list of pmp.Motif; ref: list of (i, j, m, dist) or oracle Motifs."""
    ref = [(r.i, r.j, r.m, r.dist) if hasattr(r, "i") else tuple(r) for r in ref]
    if len(gpu) != len(ref):
        return False, f"length {len(gpu)} != {len(ref)}"
    for x, (g, r) in enumerate(zip(gpu, ref)):
        if (g.i, g.j, g.m) != tuple(r[:3]) or not dist_close(g.dist, r[3]):
            return False, f"rank {x}: gpu {(g.i, g.j, g.m, g.dist)} oracle {r}"
    return True, ""


def tie_aware_equal(gpu, rows, k: int, oracle, t=None, *, excl: int) -> tuple[bool, str]:
    """Accept a GPU list that differs from the canonical one only inside tie
    groups: re-run the oracle's greedy with each tie group (P within 1e-9
    relative, or both 0) reordered to put the GPU's cells first; the accepted
    list must equal the GPU's, and each GPU neighbour j that differs from the
    oracle's must be a valid partner (|i - j| >= excl, the exclusion zone of
    Sec. 2) attaining the cell's exact minimum within the distance
    tolerance."""
    P, m, i, j = oracle.sorted_cells(rows)
    gpu_cells = {(g.m, g.i): x for x, g in enumerate(gpu)}
    order = np.arange(len(P))
    s = 0
    prio = np.zeros(len(P))
    while s < len(P):
        e = s + 1
        while e < len(P) and (P[e] == P[s] or (P[s] > 0 and abs(P[e] - P[s]) <= REL_TIE * P[s])):
            e += 1
        for x in range(s, e):
            prio[x] = gpu_cells.get((int(m[x]), int(i[x])), 1e9)
        order[s:e] = s + np.argsort(prio[s:e], kind="stable")
        s = e
    acc = oracle.greedy(P[order], m[order], i[order], j[order], k)
    if [(a.i, a.m) for a in acc] != [(g.i, g.m) for g in gpu]:
        return False, f"accepted cells differ: oracle {[(a.i, a.m) for a in acc]} gpu {[(g.i, g.m) for g in gpu]}"
    for a, g in zip(acc, gpu):
        if not dist_close(g.dist, a.dist):
            return False, f"distance at {(g.i, g.m)}: gpu {g.dist} oracle {a.dist}"
        if g.j != a.j:
            if t is None:
                return False, f"neighbour at {(g.i, g.m)}: gpu {g.j} oracle {a.j}"
            if abs(g.i - g.j) < excl:
                return False, f"gpu neighbour {g.j} of {(g.i, g.m)} lies in the exclusion zone"
            dj = oracle.snap(oracle.distance(t, g.m, g.i, g.j))
            if not dist_close(dj, a.dist):
                return False, f"gpu neighbour {g.j} of {(g.i, g.m)} is not a minimizer"
    return True, ""


def check_topk(gpu, rows, k, oracle, t=None, *, excl: int):
    """Canonical equality, else the tie-aware acceptance test (excl: the
    request's exclusion zone, which every substituted neighbour must
    respect)."""
    ref = oracle.topk(rows, k)
    ok, msg = canonical_equal(gpu, ref)
    if ok:
        return True, ""
    ok2, msg2 = tie_aware_equal(gpu, rows, k, oracle, t, excl=excl)
    if not ok2:
        return False, msg + " | " + msg2
    return True, "tie-aware"
