"""C ABI checks that need no GPU: the library loads, exports every entry point
its headers declare, and its host-only functions behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in ("pmp.h", "pmp_stages.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(pmp_[a-z_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2607_17481_amd import pmp
    lib = pmp.lib()
    names = declared_symbols()
    assert {"pmp_open", "pmp_run_device", "pmp_server_create", "pmp_submit"} <= names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options_are_the_paper_constants():
    from paper_2607_17481_amd import pmp
    o = pmp.options()
    assert o.size == C.sizeof(pmp.Options)
    assert (o.m_step, o.signature_bits, o.gamma, o.probe_ref_depth, o.certify) == (1, 24, 8, 12, 1)
    assert o.spectral_width == 0 and o.precision == 0
    # refinement radii (6, 4) and at most eight rounds (Sec. 4 constants); an
    # anchor stride of 16 (the paper's maximum-performance setting is 6) and
    # the sieve off, both measured faster with the same certified result
    assert (o.anchor_stride, o.sieve_width, o.complete_dm, o.complete_dp, o.complete_rounds) == \
        (16, 0, 6, 4, 8)


def test_workspace_query_and_argument_checks():
    from paper_2607_17481_amd import pmp
    assert pmp.workspace_bytes(100_000, 50, 100) > 0
    assert pmp.workspace_bytes(100_000, 50, 100, opts=pmp.options(precision=1)) < \
        pmp.workspace_bytes(100_000, 50, 100, opts=pmp.options(precision=0))
    assert pmp.workspace_bytes(100, 2, 10) == 0          # m_min < 3
    assert pmp.workspace_bytes(100, 10, 101) == 0        # m_max > n
    assert pmp.workspace_bytes(100, 20, 10) == 0
    assert pmp.workspace_bytes(10_000, 100, 2048) > 0     # the longest supported window
    assert pmp.workspace_bytes(10_000, 100, 2049) == 0
    assert pmp.workspace_bytes(10_000, 100, 200, k=0) == 0
    # the selection buffers grow with k: 24 bytes per selected cell, k (m_max + 1) cells
    w20 = pmp.workspace_bytes(10_000, 100, 2048, k=20)
    w150 = pmp.workspace_bytes(10_000, 100, 2048, k=150)
    assert w150 - w20 >= 24 * 130 * 2049
    with pytest.raises(pmp.PMPError) as e:
        pmp.open_host(np.zeros(10), 2, 5, 3, 1)
    assert e.value.code == pmp.PMP_EINVAL


def test_projection_generator_matches_oracle(oracle):
    from paper_2607_17481_amd import pmp
    for seed in (0, 7, 0x5eed2607):
        for m, l, c in [(3, 0, 0), (50, 23, 29), (4096, 11, 5), (0, 32, 3)]:
            assert pmp.projection(seed, m, l, c) == oracle.projection(seed, m, l, c)


def test_width_calibration_rules():
    """Sec. 3.2 calibration: smooth windows need few bins, white noise many."""
    from paper_2607_17481_amd import pmp, synth
    rng = np.random.default_rng(0)
    smooth = np.sin(np.arange(20000) * 2 * np.pi / 97.0) + 0.001 * rng.standard_normal(20000)
    noise = rng.standard_normal(20000)
    k_smooth = pmp.calibrate_width(smooth, 50, 100)
    k_noise = pmp.calibrate_width(noise, 50, 100)
    assert 4 <= k_smooth < k_noise <= 16
    assert k_noise == 16


def test_struct_layouts_match_the_headers(tmp_path):
    """The binding's ctypes structures have the size and field offsets that a
    C compiler gives the header's structs."""
    import subprocess
    from paper_2607_17481_amd import pmp
    pairs = [("pmp_motif", pmp.MotifC), ("pmp_options", pmp.Options), ("pmp_stats", pmp.Stats),
             ("pmp_timing", pmp.Timing), ("pmp_debug", pmp.Debug),
             ("pmp_stream_stats", pmp.StreamStats)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pmp_stages.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} (sizeof) %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict()
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, v = ln.split()
        got[(cname, field)] = int(v)
    for cname, py in pairs:
        assert got[(cname, "(sizeof)")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_stream_argument_checks():
    """pmp_stream_create rejects bad arguments before it touches a device."""
    from paper_2607_17481_amd import pmp
    L = pmp.lib()
    h = C.c_void_p()
    cases = [dict(batch=65),                       # batch > exclusion
             dict(capacity=50),                    # capacity < m_max
             dict(m_min=2),                        # m_min < 3
             dict(k=0), dict(budget=0), dict(exclusion=0),
             dict(opts=pmp.options(precision=1)),  # FP64 form only
             dict(opts=pmp.options(anchor_stride=0))]
    for kw in cases:
        a = dict(capacity=1000, m_min=32, m_max=82, k=20, exclusion=64, budget=16, batch=0,
                 opts=None)
        a.update(kw)
        rc = L.pmp_stream_create(0, a["capacity"], a["m_min"], a["m_max"], a["k"], a["exclusion"],
                                 a["budget"], a["batch"],
                                 C.byref(a["opts"]) if a["opts"] is not None else None, C.byref(h))
        assert rc == pmp.PMP_EINVAL, kw
        assert not h.value
        assert L.pmp_last_error()
