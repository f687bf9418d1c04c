"""Serving: continuous batching over libpmp's request server (pmp_server_*).

Each request's result must be the same alone and in the mix (FP64: bit for
bit; mixed precision: within the distance tolerance, same cells)."""
import time

import numpy as np
import pytest

from paper_2607_17481_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu


def _requests(count, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for x in range(count):
        n = int(np.exp(rng.uniform(np.log(8_000), np.log(60_000))))
        kind = "wafer" if x % 2 == 0 else "ecg"
        m_min = int(rng.integers(16, 129))
        span = int(rng.integers(4, 17))
        t = synth.wafer_like(n, 1000 + x, copies=2) if kind == "wafer" else synth.ecg_like(n, 1000 + x)
        out.append((t, m_min, m_min + span - 1, m_min))
    return out


_ORACLE_ROWS: dict = {}


def _oracle_rows(oracle, x, t, lo, hi, ex):
    """Exact rows of request x (oracle v2, equal to the brute force)."""
    if x not in _ORACLE_ROWS:
        _ORACLE_ROWS[x] = oracle.pan_profile_v2(t, range(lo, hi + 1), ex)
    return _ORACLE_ROWS[x]


@pytest.mark.parametrize("prec", [0, 1])
def test_alone_equals_in_the_mix(prec, oracle):
    """Every served request equals its result alone (FP64 form: bit for bit)
    and the oracle's exact top-k (every request here has n <= 1e5)."""
    import torch
    from paper_2607_17481_amd import pmp
    reqs = _requests(12)
    opts = pmp.options(precision=prec)
    alone = []
    ws = pmp.Workspace("cuda:0")
    for t, lo, hi, ex in reqs:
        td = torch.from_numpy(t).cuda()
        alone.append(pmp.run_device(td, lo, hi, 20, ex, 16, opts, ws)[0])
    del ws
    torch.cuda.empty_cache()
    with pmp.Server(0, 24 << 30, slots=4) as srv:
        ids = [srv.submit(t, lo, hi, 20, ex, 16, opts) for t, lo, hi, ex in reqs]
        got = [srv.wait(i) for i in ids]
    for x, ((res, tm), ref, (t, lo, hi, ex)) in enumerate(zip(got, alone, reqs)):
        assert tm["end_s"] >= tm["start_s"] >= tm["submit_s"] > 0
        if prec == 0:
            assert res == ref
        else:
            ok, msg = parity.canonical_equal(res, [(r.i, r.j, r.m, r.dist) for r in ref])
            assert ok, msg
        assert len(t) <= 100_000
        ok, msg = parity.check_topk(res, _oracle_rows(oracle, x, t, lo, hi, ex), 20, oracle, t,
                                    excl=ex)
        assert ok, (x, msg)


def test_requests_overlap_and_admission():
    from paper_2607_17481_amd import pmp
    reqs = _requests(8, seed=9)
    need = max(pmp.workspace_bytes(len(t), lo, hi, 20) for t, lo, hi, _ in reqs)
    budget = 2 * need + (1 << 20)
    with pmp.Server(0, budget, slots=4) as srv:
        ids = [srv.submit(t, lo, hi, 20, ex) for t, lo, hi, ex in reqs]
        tms = [srv.wait(i)[1] for i in ids]
    spans = sorted((tm["start_s"], tm["end_s"], tm["workspace_bytes"]) for tm in tms)
    # the workspaces of the requests in flight never exceed the budget
    for s, _, _ in spans:
        assert sum(w for a, b, w in spans if a <= s < b) <= budget
    # and requests did run concurrently
    assert any(sum(1 for a, b, _ in spans if a <= s < b) >= 2 for s, _, _ in spans)


def test_refuses_what_can_never_fit_and_polls():
    from paper_2607_17481_amd import pmp
    t = synth.wafer_like(20_000, 5, copies=2)
    need = pmp.workspace_bytes(len(t), 50, 60, 20)
    with pmp.Server(0, need // 2, slots=2) as srv:
        with pytest.raises(pmp.PMPError) as e:
            srv.submit(t, 50, 60, 20, 50)
        assert e.value.code == pmp.PMP_ENOMEM
    with pmp.Server(0, 4 * need, slots=1) as srv:
        rid = srv.submit(t, 50, 60, 20, 50)
        deadline = time.time() + 60
        res = None
        while res is None and time.time() < deadline:
            res = srv.poll(rid)
            time.sleep(0.01)
        assert res is not None and len(res[0]) == 20
        bad = t.copy()
        bad[3] = np.inf
        with pytest.raises(pmp.PMPError) as e:
            srv.submit(bad, 50, 60, 20, 50)
        assert e.value.code == pmp.PMP_EINVAL


def test_least_work_is_admitted_first():
    """With one slot busy, queued requests start in order of estimated work
    (cells x mean window length), not in arrival order."""
    from paper_2607_17481_amd import pmp
    busy = synth.ecg_like(300_000, 7)
    sizes = {"large": 60_000, "small": 20_000, "tiny": 6_000}
    series = {k: synth.wafer_like(v, 11, copies=2) for k, v in sizes.items()}
    with pmp.Server(0, 16 << 30, slots=1) as srv:
        first = srv.submit(busy, 100, 130, 20, 100)
        ids = {k: srv.submit(series[k], 50, 70, 20, 50) for k in ("large", "small", "tiny")}
        srv.wait(first)
        starts = {k: srv.wait(i)[1]["start_s"] for k, i in ids.items()}
    assert starts["tiny"] < starts["small"] < starts["large"], starts
