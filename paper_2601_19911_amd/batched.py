"""Binding of the batched form (tk_plan_*): many Top-K queries over one packed
device key buffer in one engine launch.  Argument marshalling only."""

from __future__ import annotations

import ctypes
import sys

import numpy as np

from . import TopKError, check, key_code, lib, order_code, rid_code


class tk_plan_params(ctypes.Structure):
    _fields_ = [("tile_keys", ctypes.c_uint32), ("filter_grid", ctypes.c_uint32),
                ("min_sample_log2", ctypes.c_uint32), ("max_sample_log2", ctypes.c_uint32),
                ("sample_sigma", ctypes.c_double), ("use_graph", ctypes.c_int32),
                ("cap_sigma", ctypes.c_double)]


_bound = False


def _bind():
    global _bound
    if _bound:
        return lib()
    L = lib()
    vp, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
    P = ctypes.POINTER(tk_plan_params)
    L.tk_plan_workspace_size.argtypes = [vp, vp, vp, u32, i32, i32, P]
    L.tk_plan_workspace_size.restype = ctypes.c_size_t
    L.tk_plan_create.argtypes = [vp, vp, vp, u32, i32, i32, P, vp, ctypes.c_size_t,
                                 ctypes.POINTER(vp)]
    L.tk_plan_create.restype = i32
    L.tk_plan_output_offsets.argtypes = [vp, vp]
    L.tk_plan_output_offsets.restype = i32
    L.tk_plan_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]
    L.tk_plan_info.restype = i32
    L.tk_plan_launch.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tk_plan_launch.restype = i32
    L.tk_plan_query_times.argtypes = [vp, vp]
    L.tk_plan_query_times.restype = i32
    L.tk_plan_stats.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32)]
    L.tk_plan_stats.restype = i32
    L.tk_plan_destroy.argtypes = [vp]
    L.tk_plan_destroy.restype = None
    L.tk_topk_each_workspace_size.argtypes = [vp, vp, u32, i32, i32]
    L.tk_topk_each_workspace_size.restype = ctypes.c_size_t
    L.tk_topk_each.argtypes = [vp, vp, vp, vp, vp, u32, i32, i32, vp, vp, vp, ctypes.c_size_t, vp,
                               u32, vp]
    L.tk_topk_each.restype = i32
    _bound = True
    return L


class Plan:
    """A batched Top-K plan over queries offsets[i]..offsets[i+1] of a packed key buffer.

    ``tuned=True`` takes the autotuner's cached parameters for this device and
    key type when there are any (explicit keyword parameters still win)."""

    def __init__(self, offsets, ks, orders, key_dtype, rid_dtype, device="cuda", stream=None,
                 tile_keys=0, min_sample_log2=0, max_sample_log2=0, sample_sigma=0.0,
                 use_graph=True, filter_grid=0, cap_sigma=0.0, tuned=False,
                 tune_cache=None):
        import torch
        L = _bind()
        if tuned:
            from . import autotune
            c = autotune.cached_params(torch.cuda.get_device_name(),
                                       str(key_dtype).replace("torch.", ""),
                                       tune_cache or autotune.DEFAULT_CACHE) or {}
            tile_keys = tile_keys or c.get("tile_keys", 0)
            max_sample_log2 = max_sample_log2 or c.get("max_sample_log2", 0)
            sample_sigma = sample_sigma or c.get("sample_sigma", 0.0)
            filter_grid = filter_grid or c.get("filter_grid", 0)
            cap_sigma = cap_sigma or c.get("cap_sigma", 0.0)
            self.tuned_params = c
        self.offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.ks = np.ascontiguousarray(ks, dtype=np.uint32)
        orders = np.asarray([order_code(o) if not isinstance(o, (int, np.integer)) else int(o)
                             for o in orders], dtype=np.uint8)
        self.orders = np.ascontiguousarray(orders)
        self.q = len(self.ks)
        assert len(self.offsets) == self.q + 1 and len(self.orders) == self.q
        self.key_dtype = key_dtype
        self.rid_dtype = rid_dtype
        self.kc, self.rc = key_code(key_dtype), rid_code(rid_dtype)
        self.params = tk_plan_params(tile_keys, filter_grid, min_sample_log2, max_sample_log2,
                                     sample_sigma, 0 if use_graph else -1, cap_sigma)
        nbytes = L.tk_plan_workspace_size(self.offsets.ctypes.data, self.ks.ctypes.data,
                                          self.orders.ctypes.data, self.q, self.kc, self.rc,
                                          ctypes.byref(self.params))
        if nbytes == 0:
            raise TopKError("invalid batched query description")
        self.workspace = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.tk_plan_create(self.offsets.ctypes.data, self.ks.ctypes.data,
                               self.orders.ctypes.data, self.q, self.kc, self.rc,
                               ctypes.byref(self.params), self.workspace.data_ptr(), nbytes,
                               ctypes.byref(h)), "tk_plan_create")
        self._h = h
        self.out_offsets = np.zeros(self.q + 1, dtype=np.uint64)
        check(L.tk_plan_output_offsets(h, self.out_offsets.ctypes.data), "tk_plan_output_offsets")

    def info(self):
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        check(_bind().tk_plan_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"sampled": a.value, "exact": b.value, "items": c.value}

    def alloc_outputs(self, device="cuda"):
        import torch
        total = int(self.out_offsets[-1])
        return (torch.empty(total, dtype=self.key_dtype, device=device),
                torch.empty(total, dtype=self.rid_dtype, device=device))

    def launch(self, keys, out_keys, out_rowids, rowids=None, stream=None):
        import torch
        st = (stream or torch.cuda.current_stream()).cuda_stream
        check(_bind().tk_plan_launch(self._h, keys.data_ptr(),
                                     None if rowids is None else rowids.data_ptr(),
                                     None if out_keys is None else out_keys.data_ptr(),
                                     out_rowids.data_ptr(), st), "tk_plan_launch")

    def query_times(self):
        """Per-query completion times (seconds from the launch's start) of the
        last launch, from the device's clock; call after synchronizing."""
        out = np.zeros(self.q, dtype=np.float64)
        check(_bind().tk_plan_query_times(self._h, out.ctypes.data), "tk_plan_query_times")
        return out

    def stats(self):
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        check(_bind().tk_plan_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return {"fallbacks": a.value, "unfinished": b.value}

    def close(self):
        if getattr(self, "_h", None):
            _bind().tk_plan_destroy(self._h)
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


def topk_each(offsets, ks, orders, keys, out_keys, out_rowids, streams, rowids=None,
              workspace=None, timed=True):
    """The per-query baseline (tk_topk_each): each query its own tk_topk,
    enqueued from C round robin over ``streams``.  Returns per-query completion
    times (seconds from the common start) when ``timed``, else None."""
    import torch
    L = _bind()
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    ks = np.ascontiguousarray(ks, dtype=np.uint32)
    orders = np.ascontiguousarray(orders, dtype=np.uint8)
    q = len(ks)
    kc, rc = key_code(keys.dtype), rid_code(out_rowids.dtype)
    per = int(L.tk_topk_each_workspace_size(offsets.ctypes.data, ks.ctypes.data, q, kc, rc))
    if per == 0:
        raise TopKError("invalid query description")
    if workspace is None or workspace.numel() < per * len(streams):
        workspace = torch.empty(per * len(streams), dtype=torch.uint8, device=keys.device)
    hs = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
    secs = np.zeros(q, dtype=np.float64) if timed else None
    check(L.tk_topk_each(keys.data_ptr(), None if rowids is None else rowids.data_ptr(),
                         offsets.ctypes.data, ks.ctypes.data, orders.ctypes.data, q, kc, rc,
                         None if out_keys is None else out_keys.data_ptr(), out_rowids.data_ptr(),
                         workspace.data_ptr(), workspace.numel(), hs, len(streams),
                         None if secs is None else secs.ctypes.data), "tk_topk_each")
    return secs
