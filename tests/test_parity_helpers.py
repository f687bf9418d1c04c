"""The comparison helpers of the GPU parity tests, on the CPU.

A ramp makes every pair of windows an affine copy (distance 0 after the
zero snap), so every cell ties with many partners and the tie-aware check
decides.  A substituted neighbour must then still be a valid partner: one
inside the exclusion zone is rejected even though its distance is 0.
"""
import numpy as np

from tests import parity


class _M:
    def __init__(self, i, j, m, dist):
        self.i, self.j, self.m, self.dist = i, j, m, dist


def _ramp_case(oracle):
    t = np.arange(200.0)
    excl = 10
    rows = oracle.pan_profile(t, [16], excl)
    ref = oracle.topk(rows, 5)
    return t, excl, rows, ref


def test_canonical_list_passes(oracle):
    t, excl, rows, ref = _ramp_case(oracle)
    assert all(r.dist == 0.0 for r in ref)
    gpu = [_M(r.i, r.j, r.m, r.dist) for r in ref]
    ok, msg = parity.check_topk(gpu, rows, 5, oracle, t, excl=excl)
    assert ok and msg == "", msg


def test_other_valid_minimizer_passes(oracle):
    t, excl, rows, ref = _ramp_case(oracle)
    gpu = [_M(r.i, r.j, r.m, r.dist) for r in ref]
    g = gpu[0]
    gpu[0] = _M(g.i, g.i + excl + 7, g.m, 0.0)      # another partner at distance 0
    ok, msg = parity.check_topk(gpu, rows, 5, oracle, t, excl=excl)
    assert ok and msg == "tie-aware", msg


def test_neighbour_inside_exclusion_zone_fails(oracle):
    t, excl, rows, ref = _ramp_case(oracle)
    gpu = [_M(r.i, r.j, r.m, r.dist) for r in ref]
    g = gpu[0]
    gpu[0] = _M(g.i, g.i + 1, g.m, 0.0)             # distance 0, but |i - j| < excl
    assert oracle.snap(oracle.distance(t, g.m, g.i, g.i + 1)) == 0.0
    ok, msg = parity.check_topk(gpu, rows, 5, oracle, t, excl=excl)
    assert not ok and "exclusion zone" in msg, msg


def test_wrong_cell_fails(oracle):
    t, excl, rows, ref = _ramp_case(oracle)
    gpu = [_M(r.i, r.j, r.m, r.dist) for r in ref]
    g = gpu[1]
    gpu[1] = _M(g.i + 1, g.j, g.m, 0.0)             # within m/2 of an accepted cell
    ok, _ = parity.check_topk(gpu, rows, 5, oracle, t, excl=excl)
    assert not ok
