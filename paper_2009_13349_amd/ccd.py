"""Python binding of the C ABI in include/ccd.h (argument marshalling only).

Every step of the root finder runs in the HIP library ``libccd.so`` next to
this file; PyTorch is used only for device memory and streams.  Importing this
module does not touch the GPU; the library is loaded on first use and a missing
library raises an error (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccd.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ETIMEDOUT, ECANCELED = 0, -1, -2, -3, -4, -5, -6
KIND_VF, KIND_EE = 0, 1
ST_CAP, ST_CARRY, ST_DEPTH, ST_OVERFLOW, ST_INVALID = 0x01, 0x02, 0x04, 0x08, 0x80
FLAG_LITERAL = 0x1
ENGINE_PERSISTENT, ENGINE_PLAIN = 0, 1

EXPORTED = [
    "ccd_vf", "ccd_ee", "ccd_params_default", "ccd_context_create", "ccd_context_destroy",
    "ccd_context_set_engine", "ccd_context_get_tuning", "ccd_context_set_tuning", "ccd_batch",
    "ccd_context_enable_timing", "ccd_context_last_stats", "ccd_strerror", "ccd_last_error",
    "ccd_context_enable_graphs", "ccd_context_graph_counts", "ccd_autotune",
    "ccd_tuning_cache_store", "ccd_tuning_cache_load", "ccd_min_toi", "ccd_batch_indexed",
    "ccd_scene_gamma", "ccd_plan_scratch", "ccd_batch_noalloc",
]


class CCDError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib().ccd_strerror(code).decode() if _LIB is not None else str(code)
        detail = _lib().ccd_last_error().decode() if _LIB is not None else ""
        if detail:
            msg = f"{msg} [{detail}]"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class Params(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("min_sep", ctypes.c_double), ("t_max", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("toi", ctypes.c_double), ("t_width", ctypes.c_double),
                ("n_checks", ctypes.c_uint64), ("hit", ctypes.c_uint8),
                ("status", ctypes.c_uint8), ("reserved", ctypes.c_uint8 * 6)]


class Tuning(ctypes.Structure):
    _fields_ = [("lane_waves_per_cu", ctypes.c_int32), ("lane_capacity", ctypes.c_int32),
                ("lane_budget", ctypes.c_int64), ("group_waves", ctypes.c_int32),
                ("group_count", ctypes.c_int32), ("group_capacity", ctypes.c_int64),
                ("block_count", ctypes.c_int32), ("group_occupancy", ctypes.c_int32),
                ("block_capacity", ctypes.c_int64), ("handoff_words", ctypes.c_int64),
                ("group_lds_words", ctypes.c_int32), ("block_lds_words", ctypes.c_int32)]


class ScratchPlan(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_uint64), ("lane_lds_bytes", ctypes.c_uint64),
                ("lane_blocks", ctypes.c_int64), ("group_count", ctypes.c_int64),
                ("group_capacity", ctypes.c_int64), ("block_count", ctypes.c_int64),
                ("block_capacity", ctypes.c_int64), ("handoff_words", ctypes.c_int64)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("pos", ctypes.c_void_p), ("kind", ctypes.c_void_p),
                ("default_kind", ctypes.c_uint8), ("reserved", ctypes.c_uint8 * 7),
                ("delta_q", ctypes.c_void_p), ("max_iter_q", ctypes.c_void_p),
                ("min_sep_q", ctypes.c_void_p), ("params", Params),
                ("on_device", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class IndexedDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_vertices", ctypes.c_int64), ("v0", ctypes.c_void_p),
                ("v1", ctypes.c_void_p), ("ids", ctypes.c_void_p), ("kind", ctypes.c_void_p),
                ("gamma", ctypes.c_void_p), ("default_kind", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8 * 7), ("params", Params),
                ("on_device", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class ResultSoA(ctypes.Structure):
    _fields_ = [("toi", ctypes.c_void_p), ("t_width", ctypes.c_void_p), ("hit", ctypes.c_void_p),
                ("n_checks", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("checks", (ctypes.c_uint64 * 2) * 3), ("promoted", ctypes.c_uint64 * 2),
                ("lane_slots", ctypes.c_uint64 * 3), ("kernel_ms", ctypes.c_float * 4),
                ("reserved", ctypes.c_uint32), ("overflowed", ctypes.c_uint64),
                ("restarted", ctypes.c_uint64), ("deep", ctypes.c_uint64),
                ("handoff_words", ctypes.c_uint64), ("probes", ctypes.c_uint64 * 2)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        # One HIP runtime per process: PyTorch-ROCm ships its own copy of
        # libamdhip64.so.7.  Loading torch first makes the library bind to that
        # copy (same soname) instead of starting a second runtime that would
        # then find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        V, P = ctypes.c_void_p, ctypes.POINTER
        D43 = P(ctypes.c_double * 3)
        L.ccd_vf.argtypes = [D43, D43, P(Params), P(Result)]
        L.ccd_ee.argtypes = [D43, D43, P(Params), P(Result)]
        L.ccd_params_default.argtypes = [P(Params)]
        L.ccd_params_default.restype = None
        L.ccd_context_create.argtypes = [ctypes.c_int, ctypes.c_size_t, P(V)]
        L.ccd_context_destroy.argtypes = [V]
        L.ccd_context_destroy.restype = None
        L.ccd_context_set_engine.argtypes = [V, ctypes.c_int]
        L.ccd_context_get_tuning.argtypes = [V, P(Tuning)]
        L.ccd_context_set_tuning.argtypes = [V, P(Tuning)]
        L.ccd_batch.argtypes = [V, P(BatchDesc), P(ResultSoA), V]
        L.ccd_batch_noalloc.argtypes = [V, P(BatchDesc), P(ResultSoA), V]
        L.ccd_context_enable_timing.argtypes = [V, ctypes.c_int]
        L.ccd_context_enable_graphs.argtypes = [V, ctypes.c_int]
        L.ccd_autotune.argtypes = [V, P(BatchDesc), P(ResultSoA), V, ctypes.c_int, P(Tuning),
                                   P(ctypes.c_float)]
        L.ccd_tuning_cache_store.argtypes = [V, ctypes.c_char_p, ctypes.c_char_p]
        L.ccd_tuning_cache_load.argtypes = [V, ctypes.c_char_p, ctypes.c_char_p]
        L.ccd_context_graph_counts.argtypes = [V, P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.ccd_context_last_stats.argtypes = [V, P(Stats)]
        L.ccd_min_toi.argtypes = [V, V, ctypes.c_int64, V, V]
        L.ccd_batch_indexed.argtypes = [V, P(IndexedDesc), P(ResultSoA), V]
        L.ccd_scene_gamma.argtypes = [V, V, V, ctypes.c_int64, V, V]
        L.ccd_plan_scratch.argtypes = [P(Tuning), ctypes.c_int, ctypes.c_size_t, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int, P(ScratchPlan)]
        L.ccd_strerror.argtypes = [ctypes.c_int]
        L.ccd_strerror.restype = ctypes.c_char_p
        L.ccd_last_error.argtypes = []
        L.ccd_last_error.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def load():
    """Loads the HIP library (raises if it is missing)."""
    return _lib()


def plan_scratch(n: int, max_iter: int, num_cu: int = 256, mem_budget_bytes: int = 0,
                 engine: int = ENGINE_PERSISTENT, **tuning) -> dict:
    """The scratch plan of a batch (ccd_plan_scratch; host only, no GPU)."""
    t = Tuning()
    for k, v in tuning.items():
        setattr(t, k, int(v))
    out = ScratchPlan()
    rc = _lib().ccd_plan_scratch(ctypes.byref(t), int(num_cu), int(mem_budget_bytes), int(n),
                                 int(max_iter), int(engine), ctypes.byref(out))
    if rc != OK:
        raise CCDError(rc, "ccd_plan_scratch")
    return {f: int(getattr(out, f)) for f, _ in ScratchPlan._fields_}


def params(delta=1e-6, max_iter=1_000_000, min_sep=0.0, literal=False, t_max=1.0) -> Params:
    p = Params()
    _lib().ccd_params_default(ctypes.byref(p))
    p.delta, p.max_iter, p.min_sep = float(delta), int(max_iter), float(min_sep)
    p.t_max = float(t_max)
    p.flags = FLAG_LITERAL if literal else 0
    return p


def _single(fn, X, delta, max_iter, min_sep, literal, t_max):
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(8, 3))
    a = ((ctypes.c_double * 3) * 4)(*[(ctypes.c_double * 3)(*X[k]) for k in range(4)])
    b = ((ctypes.c_double * 3) * 4)(*[(ctypes.c_double * 3)(*X[k]) for k in range(4, 8)])
    p = params(delta, max_iter, min_sep, literal, t_max)
    r = Result()
    D43 = ctypes.POINTER(ctypes.c_double * 3)
    rc = fn(ctypes.cast(a, D43), ctypes.cast(b, D43), ctypes.byref(p), ctypes.byref(r))
    if rc != OK:
        raise CCDError(rc, "ccd single query")
    return r


def vf(X, delta=1e-6, max_iter=1_000_000, min_sep=0.0, literal=False, t_max=1.0) -> Result:
    """One vertex-face query (24 doubles: p, v1, v2, v3 at t0 then at t1) on the GPU."""
    return _single(_lib().ccd_vf, X, delta, max_iter, min_sep, literal, t_max)


def ee(X, delta=1e-6, max_iter=1_000_000, min_sep=0.0, literal=False, t_max=1.0) -> Result:
    """One edge-edge query (24 doubles: p1, p2, p3, p4 at t0 then at t1) on the GPU."""
    return _single(_lib().ccd_ee, X, delta, max_iter, min_sep, literal, t_max)


@dataclass
class BatchResult:
    toi: object
    t_width: object
    hit: object
    n_checks: object
    status: object


class Context:
    """A device context owning the library's scratch memory."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        rc = _lib().ccd_context_create(device, mem_budget_bytes, ctypes.byref(h))
        if rc != OK:
            raise CCDError(rc, "ccd_context_create")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            _lib().ccd_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_engine(self, engine: int):
        rc = _lib().ccd_context_set_engine(self._h, engine)
        if rc != OK:
            raise CCDError(rc, "ccd_context_set_engine")

    def tuning(self) -> dict:
        t = Tuning()
        _lib().ccd_context_get_tuning(self._h, ctypes.byref(t))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def set_tuning(self, **kw):
        t = Tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        rc = _lib().ccd_context_set_tuning(self._h, ctypes.byref(t))
        if rc != OK:
            raise CCDError(rc, "ccd_context_set_tuning")

    def enable_graphs(self, on: bool = True):
        _lib().ccd_context_enable_graphs(self._h, 1 if on else 0)

    def graph_counts(self):
        b, r = ctypes.c_uint64(), ctypes.c_uint64()
        _lib().ccd_context_graph_counts(self._h, ctypes.byref(b), ctypes.byref(r))
        return int(b.value), int(r.value)

    def enable_timing(self, on: bool = True):
        _lib().ccd_context_enable_timing(self._h, 1 if on else 0)

    def last_stats(self) -> dict:
        s = Stats()
        rc = _lib().ccd_context_last_stats(self._h, ctypes.byref(s))
        out = {"checks": [[int(s.checks[t][k]) for k in range(2)] for t in range(3)],
               "promoted": [int(s.promoted[0]), int(s.promoted[1])],
               "lane_slots": [int(x) for x in s.lane_slots],
               "kernel_ms": [float(x) for x in s.kernel_ms], "overflowed": int(s.overflowed),
               "restarted": int(s.restarted), "deep": int(s.deep),
               "handoff_words": int(s.handoff_words),
               "probes": [int(s.probes[0]), int(s.probes[1])], "rc": rc}
        if rc not in (OK,):
            raise CCDError(rc, "ccd batch counters")
        return out

    # -- batches -------------------------------------------------------------
    def autotune(self, pos, kind=None, max_trials=0, stream=None, **kw) -> tuple[dict, float]:
        """Runs ccd_autotune on a device batch (same arguments as batch_device);
        returns (best tuning, its time in ms) and leaves it on the context."""
        import torch
        d, o, out, keep, stream = self._device_desc(pos, kind, stream=stream, **kw)
        t = Tuning()
        ms = ctypes.c_float()
        rc = _lib().ccd_autotune(self._h, ctypes.byref(d), ctypes.byref(o),
                                 ctypes.c_void_p(stream.cuda_stream), int(max_trials),
                                 ctypes.byref(t), ctypes.byref(ms))
        if rc != OK:
            raise CCDError(rc, "ccd_autotune")
        return {f: getattr(t, f) for f, _ in Tuning._fields_}, float(ms.value)

    def tuning_cache_store(self, path: str, key: str):
        rc = _lib().ccd_tuning_cache_store(self._h, path.encode(), key.encode())
        if rc != OK:
            raise CCDError(rc, "ccd_tuning_cache_store")

    def tuning_cache_load(self, path: str, key: str) -> bool:
        rc = _lib().ccd_tuning_cache_load(self._h, path.encode(), key.encode())
        if rc not in (OK, EAGAIN):
            raise CCDError(rc, "ccd_tuning_cache_load")
        return rc == OK

    def _device_desc(self, pos, kind=None, default_kind=0, delta=1e-6, max_iter=1_000_000,
                     min_sep=0.0, literal=False, delta_q=None, max_iter_q=None, min_sep_q=None,
                     out: BatchResult | None = None, stream=None, t_max=1.0):
        import torch
        assert pos.is_cuda and pos.dtype == torch.float64 and pos.dim() == 2 and pos.shape[0] == 24
        pos = pos.contiguous()
        n = pos.shape[1]
        dev = pos.device
        if out is None:
            out = BatchResult(
                toi=torch.empty(n, dtype=torch.float64, device=dev),
                t_width=torch.empty(n, dtype=torch.float64, device=dev),
                hit=torch.empty(n, dtype=torch.uint8, device=dev),
                n_checks=torch.empty(n, dtype=torch.int64, device=dev),
                status=torch.empty(n, dtype=torch.uint8, device=dev))
        d = BatchDesc()
        d.n = n
        d.pos = pos.data_ptr()
        keep = [pos]
        if kind is not None:
            kind = kind.contiguous()
            assert kind.dtype == torch.uint8 and kind.is_cuda and kind.numel() == n
            keep.append(kind)
            d.kind = kind.data_ptr()
        d.default_kind = default_kind
        for name, arr, dt in (("delta_q", delta_q, torch.float64), ("max_iter_q", max_iter_q, torch.int64),
                              ("min_sep_q", min_sep_q, torch.float64)):
            if arr is not None:
                arr = arr.contiguous()
                assert arr.dtype == dt and arr.is_cuda and arr.numel() == n
                keep.append(arr)
                setattr(d, name, arr.data_ptr())
        d.params = params(delta, max_iter, min_sep, literal, t_max)
        d.on_device = 1
        o = ResultSoA(out.toi.data_ptr(), out.t_width.data_ptr(), out.hit.data_ptr(),
                      out.n_checks.data_ptr(), out.status.data_ptr())
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        return d, o, out, keep, stream

    def batch_device(self, pos, kind=None, default_kind=0, delta=1e-6, max_iter=1_000_000,
                     min_sep=0.0, literal=False, delta_q=None, max_iter_q=None, min_sep_q=None,
                     out: BatchResult | None = None, stream=None, t_max=1.0) -> BatchResult:
        """Asynchronous batch on device tensors (torch): pos float64 [24, n],
        kind uint8 [n].  Results are torch tensors on the same device."""
        d, o, out, keep, stream = self._device_desc(
            pos, kind, default_kind, delta, max_iter, min_sep, literal, delta_q, max_iter_q,
            min_sep_q, out, stream, t_max)
        rc = _lib().ccd_batch(self._h, ctypes.byref(d), ctypes.byref(o),
                              ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise CCDError(rc, "ccd_batch")
        self._keep = keep
        return out

    def batch_noalloc(self, pos, kind=None, default_kind=0, delta=1e-6, max_iter=1_000_000,
                      min_sep=0.0, literal=False, delta_q=None, max_iter_q=None, min_sep_q=None,
                      out: BatchResult | None = None, stream=None, t_max=1.0) -> BatchResult:
        """ccd_batch_noalloc on device tensors (same arguments as batch_device;
        the library allocates no device memory for it).  Pass `out` to keep the
        call itself free of allocations on the Python side too."""
        d, o, out, keep, stream = self._device_desc(
            pos, kind, default_kind, delta, max_iter, min_sep, literal, delta_q, max_iter_q,
            min_sep_q, out, stream, t_max)
        rc = _lib().ccd_batch_noalloc(self._h, ctypes.byref(d), ctypes.byref(o),
                                      ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise CCDError(rc, "ccd_batch_noalloc")
        self._keep = keep
        return out

    def scene_gamma(self, v0, v1, out=None, stream=None):
        """Scene-wide gamma per axis of vertex arrays v0, v1 (device float64
        [nv, 3]) into a 3-element device tensor, asynchronously."""
        import torch
        assert v0.is_cuda and v0.dtype == torch.float64 and v0.shape == v1.shape
        v0, v1 = v0.contiguous(), v1.contiguous()
        if out is None:
            out = torch.empty(3, dtype=torch.float64, device=v0.device)
        if stream is None:
            stream = torch.cuda.current_stream(v0.device)
        rc = _lib().ccd_scene_gamma(self._h, ctypes.c_void_p(v0.data_ptr()),
                                    ctypes.c_void_p(v1.data_ptr()), v0.shape[0],
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise CCDError(rc, "ccd_scene_gamma")
        self._keep_gamma = (v0, v1, out)
        return out

    def batch_indexed(self, v0, v1, ids, kind=None, default_kind=0, gamma=None, delta=1e-6,
                      max_iter=1_000_000, min_sep=0.0, literal=False, t_max=1.0,
                      out: BatchResult | None = None, stream=None) -> BatchResult:
        """Asynchronous batch of candidate pairs over shared vertex arrays (device
        tensors): v0, v1 float64 [nv, 3]; ids int32 [n, 4]; kind uint8 [n];
        gamma: float64 [3] scene-wide gamma or None."""
        import torch
        assert v0.is_cuda and v0.dtype == torch.float64 and v0.shape == v1.shape and v0.shape[-1] == 3
        assert ids.is_cuda and ids.dtype == torch.int32 and ids.dim() == 2 and ids.shape[1] == 4
        v0, v1, ids = v0.contiguous(), v1.contiguous(), ids.contiguous()
        n = ids.shape[0]
        dev = ids.device
        if out is None:
            out = BatchResult(
                toi=torch.empty(n, dtype=torch.float64, device=dev),
                t_width=torch.empty(n, dtype=torch.float64, device=dev),
                hit=torch.empty(n, dtype=torch.uint8, device=dev),
                n_checks=torch.empty(n, dtype=torch.int64, device=dev),
                status=torch.empty(n, dtype=torch.uint8, device=dev))
        keep = [v0, v1, ids]
        d = IndexedDesc()
        d.n, d.n_vertices = n, v0.shape[0]
        d.v0, d.v1, d.ids = v0.data_ptr(), v1.data_ptr(), ids.data_ptr()
        if kind is not None:
            kind = kind.contiguous()
            assert kind.dtype == torch.uint8 and kind.is_cuda and kind.numel() == n
            keep.append(kind)
            d.kind = kind.data_ptr()
        if gamma is not None:
            gamma = gamma.contiguous()
            assert gamma.dtype == torch.float64 and gamma.is_cuda and gamma.numel() == 3
            keep.append(gamma)
            d.gamma = gamma.data_ptr()
        d.default_kind = default_kind
        d.params = params(delta, max_iter, min_sep, literal, t_max)
        d.on_device = 1
        o = ResultSoA(out.toi.data_ptr(), out.t_width.data_ptr(), out.hit.data_ptr(),
                      out.n_checks.data_ptr(), out.status.data_ptr())
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        rc = _lib().ccd_batch_indexed(self._h, ctypes.byref(d), ctypes.byref(o),
                                      ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise CCDError(rc, "ccd_batch_indexed")
        self._keep = keep
        return out

    def min_toi(self, toi, out=None, stream=None):
        """Smallest toi of a device tensor (NaN entries skipped, +inf if none) into a
        one-element device tensor, asynchronously (the line search's step bound)."""
        import torch
        assert toi.is_cuda and toi.dtype == torch.float64 and toi.dim() == 1
        toi = toi.contiguous()
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=toi.device)
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= 1
        if stream is None:
            stream = torch.cuda.current_stream(toi.device)
        rc = _lib().ccd_min_toi(self._h, ctypes.c_void_p(toi.data_ptr()), toi.numel(),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise CCDError(rc, "ccd_min_toi")
        self._keep_min = (toi, out)
        return out

    def batch_host(self, pos, kind=None, default_kind=0, delta=1e-6, max_iter=1_000_000,
                   min_sep=0.0, literal=False, delta_q=None, max_iter_q=None,
                   min_sep_q=None, t_max=1.0) -> BatchResult:
        """Blocking batch on host numpy arrays; validates on the host first."""
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64))
        assert pos.ndim == 2 and pos.shape[0] == 24
        n = pos.shape[1]
        res = BatchResult(toi=np.empty(n), t_width=np.empty(n), hit=np.empty(n, np.uint8),
                          n_checks=np.empty(n, np.uint64), status=np.empty(n, np.uint8))
        d = BatchDesc()
        d.n = n
        d.pos = pos.ctypes.data
        keep = [pos]
        if kind is not None:
            kind = np.ascontiguousarray(np.asarray(kind, dtype=np.uint8))
            keep.append(kind)
            d.kind = kind.ctypes.data
        d.default_kind = default_kind
        for name, arr, dt in (("delta_q", delta_q, np.float64), ("max_iter_q", max_iter_q, np.int64),
                              ("min_sep_q", min_sep_q, np.float64)):
            if arr is not None:
                arr = np.ascontiguousarray(np.asarray(arr, dtype=dt))
                keep.append(arr)
                setattr(d, name, arr.ctypes.data)
        d.params = params(delta, max_iter, min_sep, literal, t_max)
        d.on_device = 0
        o = ResultSoA(res.toi.ctypes.data, res.t_width.ctypes.data, res.hit.ctypes.data,
                      res.n_checks.ctypes.data, res.status.ctypes.data)
        rc = _lib().ccd_batch(self._h, ctypes.byref(d), ctypes.byref(o), None)
        if rc != OK:
            raise CCDError(rc, "ccd_batch")
        return res


# ---------------------------------------------------------------------------
# Serving

class ServeConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("max_requests", ctypes.c_int32), ("launch_target_us", ctypes.c_int32),
                ("max_queries_per_launch", ctypes.c_int64), ("pool_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t)]


class ServeInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("rc", ctypes.c_int32), ("n", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("submitted", "admitted", "completed", "rejected", "launches", "queries_completed",
                 "queued", "pool_bytes", "pool_in_use", "pool_peak")]


SERVE_NONBLOCKING = 0x1
EXPORTED += ["ccd_serve_config_default", "ccd_serve_open", "ccd_serve_submit", "ccd_serve_poll",
             "ccd_serve_wait", "ccd_serve_query", "ccd_serve_release", "ccd_serve_stats_get",
             "ccd_serve_close"]


def _serve_lib():
    L = _lib()
    if not getattr(L, "_serve_ready", False):
        V, P = ctypes.c_void_p, ctypes.POINTER
        L.ccd_serve_config_default.argtypes = [P(ServeConfig)]
        L.ccd_serve_config_default.restype = None
        L.ccd_serve_open.argtypes = [P(ServeConfig), P(V)]
        L.ccd_serve_submit.argtypes = [V, P(BatchDesc), P(ResultSoA), ctypes.c_int, P(ctypes.c_int64)]
        L.ccd_serve_poll.argtypes = [V, ctypes.c_int64]
        L.ccd_serve_wait.argtypes = [V, ctypes.c_int64, ctypes.c_int]
        L.ccd_serve_query.argtypes = [V, ctypes.c_int64, P(ServeInfo)]
        L.ccd_serve_release.argtypes = [V, ctypes.c_int64]
        L.ccd_serve_stats_get.argtypes = [V, P(ServeStats)]
        L.ccd_serve_close.argtypes = [V]
        L._serve_ready = True
    return L


class Ticket:
    """A submitted request: its id, and the arrays it reads and writes."""

    def __init__(self, tid, keep, result: BatchResult):
        self.id = tid
        self._keep = keep
        self.result = result


class Server:
    """Continuous-batching server (ccd_serve_*) on one GPU."""

    def __init__(self, device=0, streams=2, pool_bytes=8 << 30, scratch_bytes=12 << 30,
                 max_queries_per_launch=4_000_000, max_requests=1024, launch_target_us=None):
        L = _serve_lib()
        c = ServeConfig()
        L.ccd_serve_config_default(ctypes.byref(c))
        c.device, c.streams, c.max_requests = device, streams, max_requests
        c.max_queries_per_launch, c.pool_bytes, c.scratch_bytes = (
            max_queries_per_launch, pool_bytes, scratch_bytes)
        if launch_target_us is not None:
            c.launch_target_us = int(launch_target_us)
        h = ctypes.c_void_p()
        rc = L.ccd_serve_open(ctypes.byref(c), ctypes.byref(h))
        if rc != OK:
            raise CCDError(rc, "ccd_serve_open")
        self._h = h
        # The server reads the inputs and writes the outputs of a request until
        # it is done: keep every submitted ticket (and its arrays) alive until
        # release() or close(), whatever the caller does with its references.
        self._live = {}

    def submit(self, pos, kind=None, default_kind=0, delta=1e-6, max_iter=1_000_000, min_sep=0.0,
               literal=False, nonblocking=False, out: BatchResult | None = None,
               t_max=1.0) -> Ticket:
        """pos: host array float64 [24, n] (numpy, or a pinned torch CPU tensor)."""
        def host(a, dt):
            if hasattr(a, "data_ptr"):
                return a, a.data_ptr()
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            return a, a.ctypes.data
        pos, pos_ptr = host(pos, np.float64)
        n = pos.shape[1]
        keep = [pos]
        d = BatchDesc()
        d.n, d.pos, d.default_kind = n, pos_ptr, default_kind
        if kind is not None:
            kind, kptr = host(kind, np.uint8)
            keep.append(kind)
            d.kind = kptr
        d.params = params(delta, max_iter, min_sep, literal, t_max)
        d.on_device = 0
        if out is None:
            out = BatchResult(toi=np.empty(n), t_width=np.empty(n), hit=np.empty(n, np.uint8),
                              n_checks=np.empty(n, np.uint64), status=np.empty(n, np.uint8))
        o = ResultSoA(*(getattr(out, k).ctypes.data for k in ("toi", "t_width", "hit", "n_checks",
                                                             "status")))
        t = ctypes.c_int64()
        rc = _serve_lib().ccd_serve_submit(self._h, ctypes.byref(d), ctypes.byref(o),
                                           SERVE_NONBLOCKING if nonblocking else 0, ctypes.byref(t))
        if rc != OK:
            raise CCDError(rc, "ccd_serve_submit")
        tk = Ticket(int(t.value), keep, out)
        self._live[tk.id] = tk
        return tk

    def poll(self, t: Ticket) -> int:
        return _serve_lib().ccd_serve_poll(self._h, t.id)

    def wait(self, t: Ticket, timeout_ms: int = -1) -> BatchResult:
        rc = _serve_lib().ccd_serve_wait(self._h, t.id, int(timeout_ms))
        if rc != OK:
            raise CCDError(rc, "ccd_serve_wait")
        return t.result

    def info(self, t: Ticket) -> dict:
        i = ServeInfo()
        rc = _serve_lib().ccd_serve_query(self._h, t.id, ctypes.byref(i))
        if rc != OK:
            raise CCDError(rc, "ccd_serve_query")
        return {f: getattr(i, f) for f, _ in ServeInfo._fields_}

    def release(self, t: Ticket):
        rc = _serve_lib().ccd_serve_release(self._h, t.id)
        if rc == OK:
            self._live.pop(t.id, None)
        return rc

    def stats(self) -> dict:
        s = ServeStats()
        _serve_lib().ccd_serve_stats_get(self._h, ctypes.byref(s))
        return {f: int(getattr(s, f)) for f, _ in ServeStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _serve_lib().ccd_serve_close(self._h)  # finishes every submitted request
            self._h = None
            self._live = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
