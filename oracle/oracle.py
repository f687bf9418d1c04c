"""Python face of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  The GPU library never does, and this module imports
nothing from the library.

It wraps ``pmp_oracle.c`` (plain FP64 brute force, see the header there) and
adds the top-k selection of Section 2: sort the finite cells of the pan
profile by distance and skip any cell within m/2 of an already accepted cell
at the same length.  Readings where the paper is silent:

  * "within m/2" is inclusive: cell (m, i) is skipped iff some accepted
    (m, i') has 2|i - i'| <= m;
  * ties in "sorting cells by distance" are broken by (m, i) ascending;
  * the selection is over cells, so both endpoints of one pair may appear
    (the paper's table of rarest patterns lists such paired rows).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
EPS0 = 1e-6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no FMA contraction, OpenMP."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
            "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        d, i64, i32, u64 = C.c_double, C.c_int64, C.c_int32, C.c_uint64
        P = C.c_void_p
        L.orc_window_stats.argtypes = [P, i64, i32, P, P, P]
        L.orc_distance.argtypes = [P, i64, i32, i64, i64]
        L.orc_distance.restype = d
        L.orc_profile.argtypes = [P, i64, i32, i32, P, P]
        L.orc_cells.argtypes = [P, i64, i32, i32, P, i64, i32, P, P]
        L.orc_profile_v2.argtypes = [P, i64, i32, i32, d, P, P, P, P]
        L.orc_threads.restype = C.c_int
        L.orc_kprime.argtypes = [i32, i32]
        L.orc_kprime.restype = i32
        L.orc_features.argtypes = [P, i64, i32, i64, i32, P]
        L.orc_parseval_bound.argtypes = [P, P, i32, i32]
        L.orc_parseval_bound.restype = d
        L.orc_projection.argtypes = [u64, i32, i32, i32]
        L.orc_projection.restype = d
        L.orc_signature.argtypes = [P, i32, i32, i32, u64, P]
        L.orc_signature.restype = C.c_uint32
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def window_stats(t, m: int):
    t = _f64(t)
    W = len(t) - m + 1
    mu = np.empty(W)
    sig = np.empty(W)
    cst = np.empty(W, dtype=np.uint8)
    if lib().orc_window_stats(_ptr(t), len(t), m, _ptr(mu), _ptr(sig), _ptr(cst)) != 0:
        raise ValueError("bad window length")
    return mu, sig, cst.astype(bool)


def distance(t, m: int, i: int, j: int) -> float:
    t = _f64(t)
    return float(lib().orc_distance(_ptr(t), len(t), m, i, j))


def snap(d: float) -> float:
    return 0.0 if d < EPS0 else d


def profile(t, m: int, excl: int):
    """Exact (P_m, I_m) by brute force: P = inf, I = -1 where no cell exists."""
    t = _f64(t)
    W = len(t) - m + 1
    P = np.empty(W)
    I = np.empty(W, dtype=np.int64)
    if lib().orc_profile(_ptr(t), len(t), m, excl, _ptr(P), _ptr(I)) != 0:
        raise ValueError("bad profile arguments")
    return P, I


def profile_v2(t, m: int, excl: int, band_scale: float = 1.0, audit: bool = False):
    """Oracle v2: the same exact (P_m, I_m) as ``profile``, from the
    closed-form screen with a rigorous rounding band (see pmp_oracle.c).
    Returns (P, I, direct distances computed, largest band ratio or None);
    with ``audit`` every pair is also checked against the band (slow)."""
    t = _f64(t)
    W = len(t) - m + 1
    P = np.empty(W)
    I = np.empty(W, dtype=np.int64)
    nd = C.c_int64(0)
    aud = C.c_double(0.0)
    if lib().orc_profile_v2(_ptr(t), len(t), m, excl, float(band_scale), _ptr(P), _ptr(I),
                            C.byref(nd), C.byref(aud) if audit else None) != 0:
        raise ValueError("bad profile arguments")
    return P, I, int(nd.value), (float(aud.value) if audit else None)


def pan_profile_v2(t, lengths, excl: int, progress=None):
    """Oracle v2 rows for every listed length: {m: (P_m, I_m)}."""
    out = {}
    for m in lengths:
        P, I, nd, _ = profile_v2(t, int(m), excl)
        out[int(m)] = (P, I)
        if progress:
            progress(int(m), nd)
    return out


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def cells(t, m: int, excl: int, starts, stop_at_zero: bool = False):
    """Exact (P_m[i], I_m[i]) for selected starts i."""
    t = _f64(t)
    s = np.ascontiguousarray(starts, dtype=np.int64)
    P = np.empty(len(s))
    I = np.empty(len(s), dtype=np.int64)
    if lib().orc_cells(_ptr(t), len(t), m, excl, _ptr(s), len(s), int(stop_at_zero),
                       _ptr(P), _ptr(I)) != 0:
        raise ValueError("bad cell arguments")
    return P, I


def kprime(K: int, m: int) -> int:
    return int(lib().orc_kprime(K, m))


def features(t, m: int, i: int, K: int) -> np.ndarray:
    t = _f64(t)
    F = np.empty(2 * (K - 1))
    if lib().orc_features(_ptr(t), len(t), m, i, K, _ptr(F)) < 0:
        raise ValueError("bad feature arguments")
    return F


def parseval_bound(Fi, Fj, K: int, m: int) -> float:
    Fi, Fj = _f64(Fi), _f64(Fj)
    return float(lib().orc_parseval_bound(_ptr(Fi), _ptr(Fj), K, m))


def projection(seed: int, m: int, l: int, c: int) -> float:
    return float(lib().orc_projection(seed, m, l, c))


def signature(F, K: int, m: int, B: int, seed: int):
    F = _f64(F)
    margins = np.empty(B)
    s = int(lib().orc_signature(_ptr(F), K, m, B, seed, _ptr(margins)))
    return s, margins


# ------------------------------------------------------------------ top-k

@dataclass(frozen=True)
class Motif:
    i: int
    j: int
    m: int
    dist: float


def pan_profile(t, lengths, excl: int):
    """Exact rows for every listed length: {m: (P_m, I_m)}."""
    return {int(m): profile(t, int(m), excl) for m in lengths}


def sorted_cells(rows):
    """Finite cells as arrays (P, m, i, j) sorted by the key (P, m, i)."""
    Ps, ms, iis, js = [], [], [], []
    for m, (P, I) in rows.items():
        fin = np.isfinite(P)
        idx = np.nonzero(fin)[0]
        Ps.append(P[idx]); iis.append(idx); js.append(I[idx])
        ms.append(np.full(len(idx), m, dtype=np.int64))
    if not Ps:
        return (np.empty(0),) + (np.empty(0, dtype=np.int64),) * 3
    P = np.concatenate(Ps); m = np.concatenate(ms)
    i = np.concatenate(iis); j = np.concatenate(js)
    order = np.lexsort((i, m, P))
    return P[order], m[order], i[order], j[order]


def greedy(P, m, i, j, k: int):
    """Greedy top-k over cells already sorted by (P, m, i) (Section 2)."""
    acc: list[Motif] = []
    for d, mm, ii, jj in zip(P.tolist(), m.tolist(), i.tolist(), j.tolist()):
        if any(a.m == mm and 2 * abs(ii - a.i) <= mm for a in acc):
            continue
        acc.append(Motif(int(ii), int(jj), int(mm), float(d)))
        if len(acc) == k:
            break
    return acc


def topk(rows, k: int):
    return greedy(*sorted_cells(rows), k)


def pan_topk(t, lengths, excl: int, k: int):
    """Exact top-k pan-motifs by brute force over every length."""
    return topk(pan_profile(t, lengths, excl), k)


def first_zero_topk(t, m: int, excl: int, k: int, batch: int = 256):
    """Exact top-k when at least k greedy-accepted cells of length m have
    P = 0 and m is the smallest length of the interval.

    Every cell with P = 0 at the smallest length precedes every other cell in
    the (P, m, i) order, so scanning the cells of length m by ascending start,
    computing each exactly (stopping a row at its first zero, which is then
    the smallest minimizer), and running the greedy over the zero cells gives
    the exact answer once k of them are accepted.  Returns None if the series
    runs out before k zero cells are accepted.
    """
    t = _f64(t)
    W = len(t) - m + 1
    acc: list[Motif] = []
    start = 0
    while start < W and len(acc) < k:
        s = np.arange(start, min(W, start + batch), dtype=np.int64)
        P, I = cells(t, m, excl, s, stop_at_zero=True)
        for ii, d, jj in zip(s.tolist(), P.tolist(), I.tolist()):
            if d != 0.0:
                continue
            if any(2 * abs(ii - a.i) <= m for a in acc):
                continue
            acc.append(Motif(int(ii), int(jj), m, 0.0))
            if len(acc) == k:
                break
        start += batch
    return acc if len(acc) == k else None
