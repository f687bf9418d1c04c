"""ctypes binding of libpmp (argument marshalling only).

Every step of the computation runs in the HIP library; this module only
converts arguments.  It raises if ``libpmp.so`` is missing: there is no CPU
fallback.  PyTorch provides device memory and streams for the device-resident
entry points.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpmp.so")

PMP_OK, PMP_EINVAL, PMP_ENOMEM, PMP_EDEVICE, PMP_EBUSY, PMP_ENOTFOUND, PMP_EINTERNAL = (
    0, -1, -2, -3, -4, -5, -6)
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2


class MotifC(C.Structure):
    _fields_ = [("i", C.c_int64), ("j", C.c_int64), ("m", C.c_int32), ("flags", C.c_int32),
                ("dist", C.c_double)]


class Options(C.Structure):
    _fields_ = [("size", C.c_uint32), ("m_step", C.c_int32), ("precision", C.c_int32),
                ("spectral_width", C.c_int32), ("seed", C.c_uint64), ("certify", C.c_int32),
                ("signature_bits", C.c_int32), ("gamma", C.c_int32),
                ("probe_ref_depth", C.c_int32), ("probe_cap", C.c_int32),
                ("anchor_stride", C.c_int32), ("sieve_width", C.c_int32),
                ("complete_rounds", C.c_int32), ("complete_dm", C.c_int32),
                ("complete_dp", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("size", C.c_uint32), ("K", C.c_int32), ("lengths", C.c_int32),
                ("certify_rounds", C.c_int32), ("cells", C.c_uint64),
                ("indexed_cells", C.c_uint64), ("pass_candidates", C.c_uint64),
                ("pass_verified", C.c_uint64), ("join_candidates", C.c_uint64),
                ("join_verified", C.c_uint64), ("hot_buckets", C.c_uint64),
                ("max_depth", C.c_int32), ("reserved", C.c_int32), ("threshold", C.c_double),
                ("ms_total", C.c_double), ("ms_onepass", C.c_double), ("ms_certify", C.c_double),
                ("ms_sketch", C.c_double), ("ms_sort", C.c_double), ("ms_probe", C.c_double),
                ("ms_join", C.c_double), ("ms_rows", C.c_double),
                ("workspace_bytes", C.c_uint64), ("join_pairs", C.c_uint64),
                ("sieve_verified", C.c_uint64), ("hint_verified", C.c_uint64),
                ("complete_verified", C.c_uint64), ("ms_complete", C.c_double),
                ("complete_rounds", C.c_int32), ("anchors", C.c_int32),
                ("ms_sieve", C.c_double), ("ms_hints", C.c_double),
                ("ms_keys", C.c_double), ("join_windows", C.c_uint64),
                ("probe_queries", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f not in ("size", "reserved")}


class Debug(C.Structure):
    _fields_ = [("size", C.c_uint32), ("K", C.c_int32),
                ("lengths", C.c_void_p), ("depth", C.c_void_p), ("indexed", C.c_void_p),
                ("mu", C.c_void_p), ("sigma", C.c_void_p), ("profile_pass", C.c_void_p),
                ("profile_final", C.c_void_p), ("features", C.c_void_p), ("keys", C.c_void_p),
                ("perm", C.c_void_p), ("bucket_start", C.c_void_p), ("t_start_scale", C.c_double),
                ("join_pair_cap", C.c_int64)]


class Timing(C.Structure):
    _fields_ = [("submit_s", C.c_double), ("start_s", C.c_double), ("end_s", C.c_double),
                ("cells", C.c_uint64), ("workspace_bytes", C.c_uint64)]


class StreamStats(C.Structure):
    _fields_ = [("appended", C.c_uint64), ("processed", C.c_uint64), ("batches", C.c_uint64),
                ("windows", C.c_uint64), ("candidates", C.c_uint64), ("verified", C.c_uint64),
                ("updates", C.c_uint64), ("dropped", C.c_uint64), ("anchors", C.c_int32),
                ("K", C.c_int32), ("batch", C.c_int32), ("reserved", C.c_int32),
                ("ms_ingest", C.c_double), ("device_bytes", C.c_uint64)]


@dataclass(frozen=True)
class Motif:
    i: int
    j: int
    m: int
    dist: float


class PMPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpmp error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libpmp.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2607_17481_amd.build` "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, u64, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_size_t
        L.pmp_default_options.argtypes = [vp]
        L.pmp_default_options.restype = None
        L.pmp_last_error.restype = C.c_char_p
        L.pmp_workspace_bytes.argtypes = [i64, i32, i32, i32, vp]
        L.pmp_workspace_bytes.restype = sz
        L.pmp_open.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp]
        L.pmp_open_ex.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, vp, vp]
        L.pmp_run_device.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, sz, vp, vp, vp, vp]
        L.pmp_run_device_debug.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, sz, vp, vp,
                                           vp, vp, vp]
        L.pmp_run_device_noalloc.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.pmp_projection.argtypes = [u64, i32, i32, i32]
        L.pmp_projection.restype = C.c_double
        L.pmp_calibrate_width.argtypes = [vp, i64, i32, i32, i32, i32, i32, i32, vp]
        if hasattr(L, "pmp_server_create"):
            L.pmp_server_create.argtypes = [C.c_int, sz, i32]
            L.pmp_server_create.restype = vp
            L.pmp_submit.argtypes = [vp, vp, i64, i32, i32, i32, i32, i32, vp, vp]
            L.pmp_poll.argtypes = [vp, u64, vp, vp, vp]
            L.pmp_wait.argtypes = [vp, u64, vp, vp, vp]
            L.pmp_server_destroy.argtypes = [vp]
            L.pmp_server_destroy.restype = None
        L.pmp_stream_create.argtypes = [C.c_int, i64, i32, i32, i32, i32, i32, i32, vp, vp]
        L.pmp_stream_append.argtypes = [vp, vp, i64]
        L.pmp_stream_flush.argtypes = [vp]
        L.pmp_stream_topk.argtypes = [vp, vp, vp]
        L.pmp_stream_exact.argtypes = [vp, vp, vp, vp]
        L.pmp_stream_profile.argtypes = [vp, i32, vp, vp, vp]
        L.pmp_stream_info.argtypes = [vp, vp, vp, i32]
        L.pmp_stream_destroy.argtypes = [vp]
        L.pmp_stream_destroy.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc != PMP_OK:
        raise PMPError(rc, lib().pmp_last_error().decode(errors="replace"))


def options(**kw) -> Options:
    o = Options()
    lib().pmp_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _motifs(buf, n):
    return [Motif(int(buf[x].i), int(buf[x].j), int(buf[x].m), float(buf[x].dist))
            for x in range(n)]


def open_host(series, m_min: int, m_max: int, k: int, exclusion: int, budget: int = 16,
              opts: Options | None = None, stats: bool = False):
    """pmp_open_ex on a host float64 series."""
    t = np.ascontiguousarray(series, dtype=np.float64)
    out = (MotifC * max(k, 1))()
    n_out = C.c_int32(0)
    st = Stats()
    st.size = C.sizeof(Stats)
    rc = lib().pmp_open_ex(t.ctypes.data_as(C.c_void_p), len(t), m_min, m_max, k, exclusion,
                           budget, C.byref(opts) if opts is not None else None, out,
                           C.byref(n_out), C.byref(st))
    _check(rc)
    res = _motifs(out, n_out.value)
    return (res, st.as_dict()) if stats else res


def workspace_bytes(n: int, m_min: int, m_max: int, k: int = 20,
                    opts: Options | None = None) -> int:
    return int(lib().pmp_workspace_bytes(n, m_min, m_max, k,
                                         C.byref(opts) if opts is not None else None))


class Workspace:
    """A torch-owned device workspace for pmp_run_device (grows on demand)."""

    def __init__(self, device="cuda:0"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            torch.cuda.empty_cache()
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.buf.data_ptr()
        off = (-ptr) % 256
        return ptr + off, self.buf.numel() - off


def run_device(t_dev, m_min: int, m_max: int, k: int, exclusion: int, budget: int = 16,
               opts: Options | None = None, workspace: Workspace | None = None, stream=None,
               debug: Debug | None = None):
    """pmp_run_device on a torch float64 CUDA tensor; returns (motifs, stats dict)."""
    import torch
    assert t_dev.dtype == torch.float64 and t_dev.is_cuda and t_dev.is_contiguous()
    n = t_dev.numel()
    ws = workspace or Workspace(t_dev.device)
    need = workspace_bytes(n, m_min, m_max, k, opts)
    if need == 0:
        raise PMPError(PMP_EINVAL, "invalid arguments for the workspace query")
    wptr, wbytes = ws.get(need)
    s = stream if stream is not None else torch.cuda.current_stream(t_dev.device)
    out = (MotifC * max(k, 1))()
    n_out = C.c_int32(0)
    st = Stats()
    st.size = C.sizeof(Stats)
    args = [C.c_void_p(t_dev.data_ptr()), n, m_min, m_max, k, exclusion, budget,
            C.byref(opts) if opts is not None else None, C.c_void_p(wptr), wbytes,
            C.c_void_p(s.cuda_stream), out, C.byref(n_out), C.byref(st)]
    if debug is not None:
        rc = lib().pmp_run_device_debug(*args, C.byref(debug))
    else:
        rc = lib().pmp_run_device(*args)
    _check(rc)
    return _motifs(out, n_out.value), st.as_dict()


def run_device_noalloc(t_dev, m_min: int, m_max: int, k: int, exclusion: int, budget: int = 16,
                       opts: Options | None = None, stream=None):
    """pmp_run_device_noalloc on a torch float64 CUDA tensor (the library's
    fixed scratch, no workspace); returns (motifs, stats dict)."""
    import torch
    assert t_dev.dtype == torch.float64 and t_dev.is_cuda and t_dev.is_contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(t_dev.device)
    out = (MotifC * max(k, 1))()
    n_out = C.c_int32(0)
    st = Stats()
    st.size = C.sizeof(Stats)
    rc = lib().pmp_run_device_noalloc(C.c_void_p(t_dev.data_ptr()), t_dev.numel(), m_min, m_max,
                                      k, exclusion, budget,
                                      C.byref(opts) if opts is not None else None,
                                      C.c_void_p(s.cuda_stream), out, C.byref(n_out), C.byref(st))
    _check(rc)
    return _motifs(out, n_out.value), st.as_dict()


def projection(seed: int, m: int, l: int, c: int) -> float:
    return float(lib().pmp_projection(seed, m, l, c))


def calibrate_width(series, m_min, m_max, m_step=1, budget=16, gamma=8, bits=24) -> int:
    t = np.ascontiguousarray(series, dtype=np.float64)
    K = C.c_int32(0)
    _check(lib().pmp_calibrate_width(t.ctypes.data_as(C.c_void_p), len(t), m_min, m_max, m_step,
                                     budget, gamma, bits, C.byref(K)))
    return K.value


class Server:
    """pmp_server_*: continuous-batching request server (see include/pmp.h)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 64 << 30, slots: int = 4):
        self.h = lib().pmp_server_create(device, hbm_budget_bytes, slots)
        if not self.h:
            raise PMPError(PMP_EINVAL, "pmp_server_create failed")
        self._k = {}

    def submit(self, series, m_min, m_max, k, exclusion, budget=16, opts=None) -> int:
        t = np.ascontiguousarray(series, dtype=np.float64)
        rid = C.c_uint64(0)
        _check(lib().pmp_submit(self.h, t.ctypes.data_as(C.c_void_p), len(t), m_min, m_max, k,
                                exclusion, budget, C.byref(opts) if opts is not None else None,
                                C.byref(rid)))
        self._k[rid.value] = k
        return rid.value

    def _result(self, fn, rid):
        k = self._k[rid]
        out = (MotifC * k)()
        n_out = C.c_int32(0)
        tm = Timing()
        rc = fn(self.h, rid, out, C.byref(n_out), C.byref(tm))
        if rc == PMP_EBUSY:
            return None
        self._k.pop(rid, None)
        _check(rc)
        timing = {f: getattr(tm, f) for f, _ in Timing._fields_}
        return _motifs(out, n_out.value), timing

    def poll(self, rid):
        return self._result(lib().pmp_poll, rid)

    def wait(self, rid):
        return self._result(lib().pmp_wait, rid)

    def close(self):
        if self.h:
            lib().pmp_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Stream:
    """pmp_stream_*: a stream session (see include/pmp.h)."""

    def __init__(self, capacity: int, m_min: int, m_max: int, k: int, exclusion: int,
                 budget: int = 16, batch: int = 0, opts: Options | None = None, device: int = 0):
        h = C.c_void_p()
        _check(lib().pmp_stream_create(device, capacity, m_min, m_max, k, exclusion, budget, batch,
                                       C.byref(opts) if opts is not None else None, C.byref(h)))
        self.h = h
        self.k = k

    def append(self, samples):
        t = np.ascontiguousarray(samples, dtype=np.float64)
        _check(lib().pmp_stream_append(self.h, t.ctypes.data_as(C.c_void_p), len(t)))

    def flush(self):
        _check(lib().pmp_stream_flush(self.h))

    def topk(self):
        out = (MotifC * self.k)()
        n_out = C.c_int32(0)
        _check(lib().pmp_stream_topk(self.h, out, C.byref(n_out)))
        return _motifs(out, n_out.value)

    def exact(self, stats: bool = False):
        out = (MotifC * self.k)()
        n_out = C.c_int32(0)
        st = Stats()
        st.size = C.sizeof(Stats)
        _check(lib().pmp_stream_exact(self.h, out, C.byref(n_out), C.byref(st)))
        res = _motifs(out, n_out.value)
        return (res, st.as_dict()) if stats else res

    def info(self):
        st = StreamStats()
        lengths = (C.c_int32 * 64)()
        _check(lib().pmp_stream_info(self.h, C.byref(st), lengths, 64))
        d = {f: getattr(st, f) for f, _ in StreamStats._fields_}
        d["lengths"] = [int(lengths[a]) for a in range(min(st.anchors, 64))]
        return d

    def profile(self, anchor: int):
        """(P, I) of anchor `anchor` over the windows processed so far."""
        W = C.c_int64(0)
        _check(lib().pmp_stream_profile(self.h, anchor, None, None, C.byref(W)))
        P = np.empty(W.value, dtype=np.float64)
        I = np.empty(W.value, dtype=np.int64)
        _check(lib().pmp_stream_profile(self.h, anchor, P.ctypes.data_as(C.c_void_p),
                                        I.ctypes.data_as(C.c_void_p), C.byref(W)))
        return P, I

    def close(self):
        if self.h:
            lib().pmp_stream_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
