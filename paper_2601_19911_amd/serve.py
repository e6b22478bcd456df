"""Binding of the served form (tk_server_*): continuous batching of Top-K
requests over device-resident key columns with the paper's cost gate.
Argument marshalling only; the request loop runs in C++ threads."""

from __future__ import annotations

import ctypes
import sys

import numpy as np

from . import TK_KEY_F32, TK_KEY_F64, TK_KEY_I32, TK_KEY_I64, TopKError, check, key_code, lib

GATE_GPU, GATE_COST, GATE_CPU = 0, 1, 2


COST_FIELDS = ("cpu_a", "cpu_b", "cpu_c", "gpu_a", "gpu_b", "gpu_c")
KEY_NAMES = {TK_KEY_I32: "int32", TK_KEY_I64: "int64", TK_KEY_F32: "float32", TK_KEY_F64: "float64"}


class tk_cost_model(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in COST_FIELDS]


class tk_server_cfg(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("window_us", ctypes.c_double), ("gate", ctypes.c_int32),
                ("margin_ms", ctypes.c_double), ("cpu_threads", ctypes.c_int32),
                ("cost", tk_cost_model * 4), ("h2d_bytes_per_s", ctypes.c_double)]


class tk_req_info(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("route", ctypes.c_int32),
                ("status", ctypes.c_int32), ("count", ctypes.c_uint64)]


class tk_server_counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "routed_gpu",
                                               "routed_cpu", "batches", "batched_requests",
                                               "live", "failed")]


def cost_models(cost):
    """The four per-key-type models of tk_server_cfg from ``cost``: None (the
    library's defaults), one dict of the six coefficients (every key type), or
    a dict from key-type name ("int32", "int64", "float32", "float64") to such
    a dict (missing types take the default)."""
    arr = (tk_cost_model * 4)()
    if not cost:
        return arr
    per_type = all(isinstance(v, dict) for v in cost.values())
    for code, name in KEY_NAMES.items():
        c = cost.get(name) if per_type else cost
        if c:
            arr[code] = tk_cost_model(*[float(c.get(f, 0.0)) for f in COST_FIELDS])
    return arr


_bound = False


def _bind():
    global _bound
    L = lib()
    if _bound:
        return L
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.tk_server_create.argtypes = [ctypes.POINTER(tk_server_cfg), vp, ctypes.c_size_t,
                                   ctypes.POINTER(vp)]
    L.tk_server_create.restype = i32
    L.tk_server_add_column.argtypes = [vp, vp, vp, u64, i32, ctypes.POINTER(u32)]
    L.tk_server_add_column.restype = i32
    L.tk_server_submit.argtypes = [vp, u32, u64, u64, u32, i32, ctypes.POINTER(u64)]
    L.tk_server_submit.restype = i32
    L.tk_server_result.argtypes = [vp, u64, vp, vp, ctypes.POINTER(tk_req_info)]
    L.tk_server_result.restype = i32
    L.tk_server_replay.argtypes = [vp, u64, vp, vp, vp, vp, vp, vp, vp]
    L.tk_server_replay.restype = i32
    L.tk_server_drain.argtypes = [vp]
    L.tk_server_drain.restype = i32
    L.tk_server_stats.argtypes = [vp, ctypes.POINTER(tk_server_counters)]
    L.tk_server_stats.restype = i32
    L.tk_server_destroy.argtypes = [vp]
    L.tk_server_destroy.restype = None
    _bound = True
    return L


class Server:
    """A request server over device-resident columns (torch tensors) with
    optional host mirrors (numpy arrays) for the CPU route."""

    def __init__(self, arena_bytes=1 << 30, max_batch=256, slots=2, window_us=0.0, gate=GATE_GPU,
                 margin_ms=0.0, cpu_threads=4, cost=None, h2d_bytes_per_s=0.0, device="cuda"):
        import torch
        L = _bind()
        self.cfg = tk_server_cfg(max_batch, slots, window_us, gate, margin_ms, cpu_threads,
                                 cost_models(cost), h2d_bytes_per_s)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.tk_server_create(ctypes.byref(self.cfg), self.arena.data_ptr(), arena_bytes,
                                 ctypes.byref(h)), "tk_server_create")
        self._h = h
        self.cols = []

    def add_column(self, d_keys=None, h_keys=None):
        """A column from a device tensor and/or a host array (numpy, or a
        pinned torch CPU tensor); either may be None, not both."""
        c = ctypes.c_uint32()
        if d_keys is None and h_keys is None:
            raise ValueError("a column needs a device or a host copy")
        hptr = None
        if h_keys is not None:
            if not isinstance(h_keys, np.ndarray):  # a torch CPU tensor (pinned for async copies)
                hptr = h_keys.data_ptr()
                kc, n = key_code(h_keys.dtype), h_keys.shape[0]
            else:
                h_keys = np.ascontiguousarray(h_keys)
                hptr = h_keys.ctypes.data
                kc, n = key_code(h_keys.dtype), len(h_keys)
        if d_keys is not None:
            kc, n = key_code(d_keys.dtype), d_keys.shape[0]
            if h_keys is not None:
                assert key_code(h_keys.dtype) == kc and h_keys.shape[0] == n
        check(_bind().tk_server_add_column(self._h, None if d_keys is None else d_keys.data_ptr(),
                                           hptr, n, kc, ctypes.byref(c)), "tk_server_add_column")
        self.cols.append((d_keys, h_keys, kc))
        return c.value

    def submit(self, col, offset, n, k, order=0):
        r = ctypes.c_uint64()
        check(_bind().tk_server_submit(self._h, col, offset, n, k, order, ctypes.byref(r)),
              "tk_server_submit")
        return r.value

    def replay(self, t_arrival, cols, offsets, ns, ks, orders):
        cnt = len(t_arrival)
        arrs = [np.ascontiguousarray(t_arrival, dtype=np.float64),
                np.ascontiguousarray(cols, dtype=np.uint32),
                np.ascontiguousarray(offsets, dtype=np.uint64),
                np.ascontiguousarray(ns, dtype=np.uint64),
                np.ascontiguousarray(ks, dtype=np.uint32),
                np.ascontiguousarray(orders, dtype=np.uint8)]
        ids = np.zeros(cnt, dtype=np.uint64)
        check(_bind().tk_server_replay(self._h, cnt, *[a.ctypes.data for a in arrs],
                                       ids.ctypes.data), "tk_server_replay")
        return ids

    def drain(self):
        check(_bind().tk_server_drain(self._h), "tk_server_drain")

    def result(self, req, col, k_eff):
        kdt = {TK_KEY_I32: np.int32, TK_KEY_I64: np.int64, TK_KEY_F32: np.float32,
               TK_KEY_F64: np.float64}[self.cols[col][2]]
        ok = np.empty(k_eff, dtype=kdt)
        orr = np.empty(k_eff, dtype=np.uint64)
        info = tk_req_info()
        rc = _bind().tk_server_result(self._h, req, ok.ctypes.data if k_eff else None,
                                      orr.ctypes.data if k_eff else None, ctypes.byref(info))
        if rc == 1:
            return None
        check(rc, "tk_server_result")
        return ok[:info.count], orr[:info.count], info

    def result_status(self, req, col, k_eff):
        """(status, info) of a finished request without raising on its error
        status; None while it runs.  Takes (releases) the request."""
        kdt = {TK_KEY_I32: np.int32, TK_KEY_I64: np.int64, TK_KEY_F32: np.float32,
               TK_KEY_F64: np.float64}[self.cols[col][2]]
        ok = np.empty(max(k_eff, 1), dtype=kdt)
        orr = np.empty(max(k_eff, 1), dtype=np.uint64)
        info = tk_req_info()
        rc = _bind().tk_server_result(self._h, req, ok.ctypes.data, orr.ctypes.data,
                                      ctypes.byref(info))
        if rc == 1:
            return None
        return rc, info

    def stats(self):
        st = tk_server_counters()
        check(_bind().tk_server_stats(self._h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in tk_server_counters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _bind().tk_server_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down: the runtime (or a
        # profiler attached to it) may already be finalized; close() explicitly.
        # The check is bound at definition time: imports fail during shutdown.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
