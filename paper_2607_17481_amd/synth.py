"""Seeded synthetic workloads.

These generators only produce input series (and the random draws that
describe them).  They contain none of the motif-search arithmetic, so the
CPU oracle under ``oracle/`` and the GPU library can both be fed from them
without sharing any computation.

Every generator is a pure function of its arguments: the same seed gives the
same float64 array bit for bit (numpy PCG64 stream).

Workloads (stand-ins for the paper's UCR series, which are not shipped):

* ``random_walk_planted`` -- random walk with planted motif pairs, the small
  case a brute-force oracle finishes in seconds.
* ``wafer_like`` -- noiseless piecewise-constant regimes plus noisy square
  pulses; the shape of the paper's Wafer length-scaling rows
  (Section 4, Table ``tab:master``).
* ``ecg_like`` -- quasi-periodic beats built from Gaussian bumps, with period
  and amplitude jitter, baseline wander and noise.
* ``serving_requests`` -- a Poisson stream of heterogeneous requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20261203

# Sub-seeds, one per workload family.
SEED_TINY = BASE_SEED + 1
SEED_WAFER_100K = BASE_SEED + 2
SEED_WAFER_5M = BASE_SEED + 3
SEED_ECG_1M = BASE_SEED + 4
SEED_SERVING = BASE_SEED + 5


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass
class Planted:
    """Where the planted occurrences of ``random_walk_planted`` went."""
    motif_len: int
    pairs: list = field(default_factory=list)   # [(p, q), ...]


def random_walk_planted(n: int = 4000, n_pairs: int = 5, motif_len: int = 64,
                        noise: float = 0.05, seed: int = SEED_TINY):
    """Random walk (cumulative N(0,1) steps) with ``n_pairs`` planted pairs.

    Each pair has its own ``motif_len``-step N(0,1) random-walk template.  An
    occurrence at position p is the template shifted so that it starts at the
    current level t[p], plus fresh N(0, noise) samples, written over
    t[p:p+motif_len].  Occurrence positions are uniform, redrawn until every
    occurrence starts at least ``motif_len`` samples from every other one.
    Returns (t, Planted).
    """
    rng = _rng(seed)
    t = np.cumsum(rng.standard_normal(n))
    need = 2 * n_pairs
    if need * motif_len > n:
        raise ValueError("series too short for the planted occurrences")
    pos: list[int] = []
    while len(pos) < need:
        p = int(rng.integers(0, n - motif_len + 1))
        if all(abs(p - q) >= motif_len for q in pos):
            pos.append(p)
    info = Planted(motif_len=motif_len)
    for k in range(n_pairs):
        tmpl = np.cumsum(rng.standard_normal(motif_len))
        pair = (pos[2 * k], pos[2 * k + 1])
        for p in pair:
            occ = tmpl - tmpl[0] + t[p] + noise * rng.standard_normal(motif_len)
            t[p:p + motif_len] = occ
        info.pairs.append(pair)
    return t, info


def wafer_like(n: int, seed: int, n_templates: int = 4, copies: int = 10,
               seg_lo: int = 100, seg_hi: int = 400,
               width_lo: int = 60, width_hi: int = 140,
               amp_lo: float = 2.0, amp_hi: float = 4.0,
               pulse_noise: float = 0.1) -> np.ndarray:
    """Piecewise-constant regimes plus noisy square pulses.

    Background: consecutive segments of length U{seg_lo..seg_hi}, each at a
    level drawn from N(0,1), with no noise.  ``n_templates`` square-pulse
    templates get a width U{width_lo..width_hi} and an amplitude
    U[amp_lo, amp_hi].  ``copies`` copies of each template are added to the
    background at positions that overlap no other pulse, each with fresh
    N(0, pulse_noise) samples over the pulse span.
    """
    rng = _rng(seed)
    t = np.empty(n, dtype=np.float64)
    pos = 0
    while pos < n:
        # draw segment lengths in blocks to keep the loop short at large n
        lens = rng.integers(seg_lo, seg_hi + 1, size=4096)
        levels = rng.standard_normal(4096)
        for L, lev in zip(lens, levels):
            if pos >= n:
                break
            t[pos:pos + int(L)] = lev
            pos += int(L)
    widths = rng.integers(width_lo, width_hi + 1, size=n_templates)
    amps = rng.uniform(amp_lo, amp_hi, size=n_templates)
    placed: list[tuple[int, int]] = []
    for k in range(n_templates):
        w = int(widths[k])
        if w > n:
            raise ValueError("series shorter than a pulse")
        for _ in range(copies):
            for _attempt in range(100000):
                p = int(rng.integers(0, n - w + 1))
                if all(p + w <= q or q + wq <= p for q, wq in placed):
                    break
            else:
                raise ValueError("could not place the pulses without overlap")
            placed.append((p, w))
            t[p:p + w] += amps[k] + pulse_noise * rng.standard_normal(w)
    return t


# Beat model of ``ecg_like``: bump centres as fractions of the beat period,
# bump widths (Gaussian standard deviations, in samples) and amplitudes.
ECG_CENTRES = (0.20, 0.36, 0.40, 0.44, 0.70)
ECG_WIDTHS = (10.0, 3.0, 4.0, 3.0, 16.0)
ECG_AMPS = (0.15, -0.12, 1.0, -0.25, 0.30)


def ecg_like(n: int, seed: int, period: int = 250, jitter: int = 20,
             amp_jitter: float = 0.1, wander: float = 0.2,
             wander_period: float = 2000.0, noise: float = 0.02) -> np.ndarray:
    """Quasi-periodic beats, each a sum of five Gaussian bumps.

    Beat b has period ``period`` + U{-jitter..jitter} and amplitude scale
    U[1-amp_jitter, 1+amp_jitter].  A baseline wander
    wander*sin(2*pi*t/wander_period) and N(0, noise) samples are added.
    """
    rng = _rng(seed)
    t = np.zeros(n, dtype=np.float64)
    start = 0
    while start < n:
        P = period + int(rng.integers(-jitter, jitter + 1))
        a = rng.uniform(1.0 - amp_jitter, 1.0 + amp_jitter)
        for c, w, A in zip(ECG_CENTRES, ECG_WIDTHS, ECG_AMPS):
            centre = start + c * P
            lo = max(0, int(math.floor(centre - 8 * w)))
            hi = min(n, int(math.ceil(centre + 8 * w)) + 1)
            if lo >= hi:
                continue
            x = np.arange(lo, hi, dtype=np.float64)
            t[lo:hi] += a * A * np.exp(-0.5 * ((x - centre) / w) ** 2)
        start += P
    x = np.arange(n, dtype=np.float64)
    t += wander * np.sin(2.0 * np.pi * x / wander_period)
    t += noise * rng.standard_normal(n)
    return t


@dataclass
class Request:
    index: int
    arrival_s: float
    kind: str          # "wafer" or "ecg"
    n: int
    m_min: int
    m_max: int
    exclusion: int
    k: int
    seed: int

    def series(self) -> np.ndarray:
        if self.kind == "wafer":
            return wafer_like(self.n, self.seed)
        return ecg_like(self.n, self.seed)

    @property
    def cells(self) -> int:
        return cells(self.n, range(self.m_min, self.m_max + 1))


def serving_requests(count: int = 2000, rate_per_s: float = 1.0,
                     n_lo: int = 10_000, n_hi: int = 2_000_000,
                     seed: int = SEED_SERVING) -> list[Request]:
    """Poisson arrivals of heterogeneous requests.

    Series length log-uniform on [n_lo, n_hi]; Wafer-like or ECG-like with
    probability 1/2 each; m_min ~ U{16..512}; span ~ U{8..64} contiguous
    lengths; exclusion = m_min; k = 20; request seed = BASE_SEED + index.
    """
    rng = _rng(seed)
    out = []
    now = 0.0
    for idx in range(count):
        now += float(rng.exponential(1.0 / rate_per_s))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        kind = "wafer" if rng.random() < 0.5 else "ecg"
        m_min = int(rng.integers(16, 513))
        span = int(rng.integers(8, 65))
        out.append(Request(index=idx, arrival_s=now, kind=kind, n=n,
                           m_min=m_min, m_max=m_min + span - 1,
                           exclusion=m_min, k=20, seed=BASE_SEED + idx))
    return out


def cells(n: int, lengths) -> int:
    """Number of (window, length) cells: sum over m of n - m + 1."""
    return int(sum(max(0, n - m + 1) for m in lengths))

