"""Python binding of libmitopk.so: key-only Top-K on MI355X.

Argument marshalling only: every step of the selection runs in the HIP
kernels behind the C ABI declared in include/mitopk.h.  PyTorch supplies
device memory and streams.  There is no fallback: if the library is missing
or no GPU is present, the GPU entry points raise.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmitopk.so")

TK_KEY_I32, TK_KEY_I64, TK_KEY_F32, TK_KEY_F64 = 0, 1, 2, 3
TK_RID_U32, TK_RID_U64 = 0, 1
TK_DESC, TK_ASC = 0, 1
TK_OK, TK_EINVAL, TK_ENOMEM, TK_EHIP, TK_EUNSUPPORTED, TK_EDEVICE, TK_EAGAIN = 0, -1, -2, -3, -4, -5, 1

_lib = None


class TopKError(RuntimeError):
    pass


class tk_info(ctypes.Structure):
    _fields_ = [("path", ctypes.c_uint32), ("status", ctypes.c_uint32),
                ("survivors", ctypes.c_uint64), ("threshold_key", ctypes.c_uint64)]


class tk_tuning(ctypes.Structure):
    _fields_ = [("sample_sigma", ctypes.c_double), ("cap_sigma", ctypes.c_double),
                ("max_sample_log2", ctypes.c_int32), ("filter_grid", ctypes.c_int32),
                ("force_cap", ctypes.c_int64), ("force_exact", ctypes.c_int32),
                ("tail_mode", ctypes.c_int32), ("filter_unroll", ctypes.c_int32),
                ("recover_min_log2", ctypes.c_int32), ("join_bloom", ctypes.c_int32)]


def lib():
    """The loaded libmitopk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TopKError(f"{LIB_PATH} is missing: build it with python -m paper_2601_19911_amd.build")
        # torch first: its wheel bundles a HIP runtime with the soname the
        # library links (libamdhip64.so.7), and whichever loads first serves
        # the whole process; the library must run on the runtime that owns
        # torch's device memory and streams
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        L.tk_workspace_size.argtypes = [u64, u64, i32, i32]
        L.tk_workspace_size.restype = ctypes.c_size_t
        L.tk_workspace_min_size.argtypes = [u64, u64, i32, i32]
        L.tk_workspace_min_size.restype = ctypes.c_size_t
        L.tk_topk.argtypes = [vp, vp, u64, u64, i32, i32, i32, vp, vp, ctypes.POINTER(u64), vp,
                              ctypes.c_size_t, vp]
        L.tk_topk.restype = i32
        L.tk_topk_noalloc.argtypes = [vp, vp, u64, u64, i32, i32, i32, vp, vp, ctypes.POINTER(u64),
                                      vp]
        L.tk_topk_noalloc.restype = i32
        L.tk_query_info.argtypes = [vp, ctypes.POINTER(tk_info)]
        L.tk_query_info.restype = i32
        L.tk_set_tuning.argtypes = [ctypes.POINTER(tk_tuning)]
        L.tk_set_tuning.restype = i32
        L.tk_cpu_topk.argtypes = [vp, vp, u64, u64, i32, i32, i32, vp, vp, ctypes.POINTER(u64), i32]
        L.tk_cpu_topk.restype = i32
        L.tk_gather_f64_host.argtypes = [vp, ctypes.c_uint32, u64, vp, i32, u64, vp, i32]
        L.tk_gather_f64_host.restype = i32
        L.tk_gather_f64_device.argtypes = [vp, ctypes.c_uint32, u64, vp, i32, u64, vp, vp]
        L.tk_gather_f64_device.restype = i32
        L.tk_profile_begin.argtypes = [ctypes.c_uint32]
        L.tk_profile_begin.restype = i32
        L.tk_profile_end.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]
        L.tk_profile_end.restype = i32
        L.tk_read_probe.argtypes = [vp, u64, ctypes.c_uint32, vp, vp]
        L.tk_read_probe.restype = i32
        L.tk_stream_workspace_size.argtypes = [u64, u64, u64, i32, i32, i32]
        L.tk_stream_workspace_size.restype = ctypes.c_size_t
        L.tk_topk_stream.argtypes = [vp, vp, u64, u64, i32, i32, i32, u64, vp, vp,
                                     ctypes.POINTER(u64), vp, ctypes.c_size_t, vp, vp]
        L.tk_topk_stream.restype = i32
        L.tk_sort_workspace_size.argtypes = [u64, i32, i32]
        L.tk_sort_workspace_size.restype = ctypes.c_size_t
        L.tk_sort.argtypes = [vp, vp, u64, i32, i32, i32, vp, vp, vp, ctypes.c_size_t, vp]
        L.tk_sort.restype = i32
        L.tk_status_string.argtypes = [i32]
        L.tk_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(rc: int, what: str = "call"):
    if rc != 0:
        msg = lib().tk_status_string(rc).decode()
        raise TopKError(f"{what} failed: {msg} ({rc})")


# ---- dtype codes -------------------------------------------------------------------------------

def key_code(dtype) -> int:
    import torch
    m = {torch.int32: TK_KEY_I32, torch.int64: TK_KEY_I64, torch.float32: TK_KEY_F32,
         torch.float64: TK_KEY_F64, np.dtype(np.int32): TK_KEY_I32, np.dtype(np.int64): TK_KEY_I64,
         np.dtype(np.float32): TK_KEY_F32, np.dtype(np.float64): TK_KEY_F64}
    if dtype not in m:
        raise TypeError(f"unsupported key dtype {dtype}")
    return m[dtype]


def rid_code(dtype) -> int:
    import torch
    m = {torch.int32: TK_RID_U32, torch.uint32: TK_RID_U32, torch.int64: TK_RID_U64,
         torch.uint64: TK_RID_U64, np.dtype(np.uint32): TK_RID_U32,
         np.dtype(np.uint64): TK_RID_U64}
    if dtype not in m:
        raise TypeError(f"unsupported row-id dtype {dtype}")
    return m[dtype]


def order_code(order) -> int:
    if order in (TK_DESC, "desc", "DESC"):
        return TK_DESC
    if order in (TK_ASC, "asc", "ASC"):
        return TK_ASC
    raise ValueError(f"order must be 'desc' or 'asc', not {order!r}")


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# ---- single query ---------------------------------------------------------------------------

def workspace_size(n: int, k: int, key_type: int, rid_type: int) -> int:
    return int(lib().tk_workspace_size(n, k, key_type, rid_type))


def workspace_min_size(n: int, k: int, key_type: int, rid_type: int) -> int:
    """The least workspace tk_topk accepts (without the full sort's scratch)."""
    return int(lib().tk_workspace_min_size(n, k, key_type, rid_type))


def new_workspace(n: int, k: int, key_type: int, rid_type: int, device="cuda", least=False):
    """A workspace for tk_topk (zero-filled here only for reproducible contents;
    the library needs no initialization); least=True: the smallest one accepted."""
    import torch
    size = (workspace_min_size if least else workspace_size)(n, k, key_type, rid_type)
    return torch.zeros(size, dtype=torch.uint8, device=device)


def topk(keys, k: int, rowids=None, order="desc", out_keys=None, out_rowids=None,
         rid_dtype=None, workspace=None, stream=None, want_keys: bool = True):
    """Top-K of device tensor ``keys`` (int32, int64, float32 or float64), best first.

    ``rowids``: device tensor of uint32/uint64 row-ids, or None for the index.
    Returns ``(out_keys, out_rowids)``; tensors are allocated when not given.
    """
    import torch
    if not keys.is_cuda:
        raise TopKError("keys must be a device tensor")
    keys = keys.contiguous()
    n = keys.shape[0]
    kc = key_code(keys.dtype)
    if rowids is not None:
        rowids = rowids.contiguous()
        assert rowids.shape[0] == n and rowids.is_cuda
        rc_ = rid_code(rowids.dtype)
        rdt = rowids.dtype
    else:
        rdt = rid_dtype if rid_dtype is not None else (torch.uint32 if n <= (1 << 32) else torch.uint64)
        rc_ = rid_code(rdt)
    oc = order_code(order)
    k_eff = min(int(k), n)
    dev = keys.device
    if out_keys is None and want_keys:
        out_keys = torch.empty(k_eff, dtype=keys.dtype, device=dev)
    if out_rowids is None:
        out_rowids = torch.empty(k_eff, dtype=rdt, device=dev)
    if workspace is None:
        workspace = torch.zeros(workspace_size(n, k, kc, rc_), dtype=torch.uint8, device=dev)
    elif workspace.numel() < workspace_min_size(n, k, kc, rc_):
        raise TopKError("workspace smaller than tk_workspace_min_size")
    cnt = ctypes.c_uint64(0)
    rc = lib().tk_topk(_ptr(keys) if n else None, _ptr(rowids), n, int(k), kc, rc_, oc,
                       _ptr(out_keys), _ptr(out_rowids), ctypes.byref(cnt),
                       workspace.data_ptr(), workspace.numel(), _stream_handle(stream))
    check(rc, "tk_topk")
    return out_keys, out_rowids


# Bytes of the library's own device array behind topk_noalloc (TK_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 32 << 20


def topk_noalloc(keys, k: int, out_keys, out_rowids, rowids=None, order="desc", stream=None):
    """``topk`` through tk_topk_noalloc: no workspace, nothing allocated by the
    call (the caller passes the outputs).  Queries whose workspace would exceed
    NOALLOC_SCRATCH_BYTES raise (TK_EUNSUPPORTED).  Calls that may overlap on
    one device race on the library's shared array: keep them on one stream."""
    if not keys.is_cuda:
        raise TopKError("keys must be a device tensor")
    if not keys.is_contiguous() or (rowids is not None and not rowids.is_contiguous()):
        raise TopKError("keys and rowids must be contiguous")
    n = keys.shape[0]
    k_eff = min(int(k), n)
    if out_rowids is None or out_rowids.numel() < k_eff:
        raise TopKError("out_rowids must hold min(k, n) row-ids")
    if out_keys is not None and out_keys.numel() < k_eff:
        raise TopKError("out_keys must hold min(k, n) keys")
    if rowids is not None and rowids.shape[0] != n:
        raise TopKError("rowids must have one entry per key")
    rc_ = rid_code(out_rowids.dtype if rowids is None else rowids.dtype)
    cnt = ctypes.c_uint64(0)
    rc = lib().tk_topk_noalloc(_ptr(keys) if n else None, _ptr(rowids), n, int(k),
                               key_code(keys.dtype), rc_, order_code(order), _ptr(out_keys),
                               _ptr(out_rowids), ctypes.byref(cnt), _stream_handle(stream))
    check(rc, "tk_topk_noalloc")
    return out_keys, out_rowids


def _host_ptr(a) -> int | None:
    """Address of a host array: a CPU torch tensor (pinned or not) or a numpy array."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise TopKError("host arrays must be contiguous")
        return a.ctypes.data
    if a.is_cuda or not a.is_contiguous():
        raise TopKError("host arrays must be contiguous CPU tensors or numpy arrays")
    return a.data_ptr()


def topk_stream(h_keys, k: int, h_rowids=None, order="desc", chunk: int = 0, rid_dtype=None,
                out_keys=None, out_rowids=None, workspace=None, stream=None, copy_stream=None,
                device="cuda"):
    """Top-K of a host key column (tk_topk_stream): copied in chunks through two
    device staging buffers, the copies on ``copy_stream`` overlapping the
    chunk queries on ``stream``.  ``h_keys``/``h_rowids``: CPU tensors (pinned
    for overlap) or numpy arrays, unchanged until the stream passes the call.
    Returns device ``(out_keys, out_rowids)``."""
    import torch
    n = int(h_keys.shape[0])
    kc = key_code(h_keys.dtype)
    if h_rowids is not None:
        if int(h_rowids.shape[0]) != n:
            raise TopKError("h_rowids must have one entry per key")
        rdt_code = rid_code(h_rowids.dtype)
    else:
        rdt_code = rid_code(rid_dtype if rid_dtype is not None else
                            (torch.uint32 if n <= (1 << 32) else torch.uint64))
    tdt = torch.uint32 if rdt_code == TK_RID_U32 else torch.uint64
    kdt = {TK_KEY_I32: torch.int32, TK_KEY_I64: torch.int64, TK_KEY_F32: torch.float32,
           TK_KEY_F64: torch.float64}[kc]
    k_eff = min(int(k), n)
    if out_keys is None:
        out_keys = torch.empty(k_eff, dtype=kdt, device=device)
    if out_rowids is None:
        out_rowids = torch.empty(k_eff, dtype=tdt, device=device)
    ws_bytes = int(lib().tk_stream_workspace_size(n, int(k), int(chunk), kc, rdt_code,
                                                  int(h_rowids is not None)))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    cnt = ctypes.c_uint64(0)
    cs = None if copy_stream is None else _stream_handle(copy_stream)
    rc = lib().tk_topk_stream(_host_ptr(h_keys) if n else None, _host_ptr(h_rowids), n, int(k), kc,
                              rdt_code, order_code(order), int(chunk), _ptr(out_keys),
                              _ptr(out_rowids), ctypes.byref(cnt), workspace.data_ptr(),
                              workspace.numel(), _stream_handle(stream), cs)
    check(rc, "tk_topk_stream")
    return out_keys, out_rowids


def sort(keys, rowids=None, order="desc", out_keys=None, out_rowids=None, rid_dtype=None,
         workspace=None, stream=None, want_keys: bool = True):
    """ORDER BY key without LIMIT: every pair of device tensor ``keys``, best
    first (equal to ``topk`` with k = n).  Returns ``(out_keys, out_rowids)``."""
    import torch
    if not keys.is_cuda:
        raise TopKError("keys must be a device tensor")
    keys = keys.contiguous()
    n = keys.shape[0]
    kc = key_code(keys.dtype)
    if rowids is not None:
        rowids = rowids.contiguous()
        assert rowids.shape[0] == n and rowids.is_cuda
        rdt = rowids.dtype
    else:
        rdt = rid_dtype if rid_dtype is not None else (torch.uint32 if n <= (1 << 32) else torch.uint64)
    rc_ = rid_code(rdt)
    dev = keys.device
    if out_keys is None and want_keys:
        out_keys = torch.empty(n, dtype=keys.dtype, device=dev)
    if out_rowids is None:
        out_rowids = torch.empty(n, dtype=rdt, device=dev)
    ws_bytes = int(lib().tk_sort_workspace_size(n, kc, rc_))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    rc = lib().tk_sort(_ptr(keys) if n else None, _ptr(rowids), n, kc, rc_, order_code(order),
                       _ptr(out_keys), _ptr(out_rowids), workspace.data_ptr(), workspace.numel(),
                       _stream_handle(stream))
    check(rc, "tk_sort")
    return out_keys, out_rowids


def query_info(workspace) -> dict:
    info = tk_info()
    rc = lib().tk_query_info(workspace.data_ptr(), ctypes.byref(info))
    return {"rc": rc, "path": info.path, "status": info.status, "survivors": info.survivors,
            "threshold_key": info.threshold_key}


def set_tuning(sample_sigma=0.0, cap_sigma=0.0, max_sample_log2=0, filter_grid=0, force_cap=0,
               force_exact=0, tail_mode=0, filter_unroll=0, recover_min_log2=0, join_bloom=0):
    """Process-wide knobs; 0 leaves a field unchanged (force_cap=-1,
    force_exact=2, tail_mode=1, filter_grid=-1, recover_min_log2=29 and
    join_bloom=1 restore the defaults; tail_mode=2 makes one workgroup select
    and sort the survivors; filter_unroll is 4 or 8; recover_min_log2=-1
    leaves every misjudged sample to one workgroup; join_bloom=2 builds join
    tables without the bloom prefilter)."""
    t = tk_tuning(sample_sigma, cap_sigma, max_sample_log2, filter_grid, force_cap, force_exact,
                  tail_mode, filter_unroll, recover_min_log2, join_bloom)
    check(lib().tk_set_tuning(ctypes.byref(t)), "tk_set_tuning")


def profile_begin(max_launches: int = 4096):
    check(lib().tk_profile_begin(max_launches), "tk_profile_begin")


def profile_end():
    """(total_ms, launches) of the streaming passes timed since profile_begin."""
    ms = ctypes.c_double(0)
    n = ctypes.c_uint64(0)
    check(lib().tk_profile_end(ctypes.byref(ms), ctypes.byref(n)), "tk_profile_end")
    return ms.value, n.value


def read_probe(buf, wg_per_cu: int, sink, stream=None):
    """Enqueues one read-only pass over device tensor ``buf`` (tk_read_probe);
    ``sink`` is a device int32/uint32 tensor of at least one element."""
    check(lib().tk_read_probe(_ptr(buf), buf.numel() * buf.element_size(), int(wg_per_cu), _ptr(sink),
                              _stream_handle(stream)), "tk_read_probe")


# ---- CPU route ------------------------------------------------------------------------------

def cpu_topk(keys: np.ndarray, k: int, rowids: np.ndarray | None = None, order="desc",
             rid_dtype=np.uint32, nthreads: int = 0):
    """Multithreaded host Top-K (the CPU route of the gate) over numpy arrays."""
    keys = np.ascontiguousarray(keys)
    n = keys.shape[0]
    if rowids is not None:
        rowids = np.ascontiguousarray(rowids)
        rid_dtype = rowids.dtype
    k_eff = min(int(k), n)
    ok = np.empty(k_eff, dtype=keys.dtype)
    orr = np.empty(k_eff, dtype=rid_dtype)
    cnt = ctypes.c_uint64(0)
    rc = lib().tk_cpu_topk(keys.ctypes.data if n else None,
                           None if rowids is None else rowids.ctypes.data, n, int(k),
                           key_code(keys.dtype), rid_code(np.dtype(rid_dtype)), order_code(order),
                           ok.ctypes.data if k_eff else None, orr.ctypes.data if k_eff else None,
                           ctypes.byref(cnt), int(nthreads))
    check(rc, "tk_cpu_topk")
    return ok, orr


# ---- late materialization ---------------------------------------------------------------------

def gather_rows_host(payload: np.ndarray, rowids: np.ndarray, nthreads: int = 8) -> np.ndarray:
    """payload[:, rowids] for a [ncols, n] float64 host array (C threads)."""
    payload = np.ascontiguousarray(payload, dtype=np.float64)
    rowids = np.ascontiguousarray(rowids)
    if payload.ndim != 2:
        raise ValueError("payload must be [ncols, n]")
    ncols, n = payload.shape
    out = np.empty((ncols, len(rowids)), dtype=np.float64)
    check(lib().tk_gather_f64_host(payload.ctypes.data, ncols, n, rowids.ctypes.data,
                                   rid_code(rowids.dtype), len(rowids), out.ctypes.data, nthreads),
          "tk_gather_f64_host")
    return out


def gather_rows_device(payload, rowids, out, stream=None):
    """out[:, j] = payload[:, rowids[j]] on the device (stream-ordered)."""
    if payload.dim() != 2 or out.dim() != 2 or out.shape[0] != payload.shape[0]:
        raise ValueError("payload [ncols, n] and out [ncols, k] required")
    if out.shape[1] != rowids.shape[0]:
        raise ValueError("out must have one column per row-id")
    check(lib().tk_gather_f64_device(payload.data_ptr(), payload.shape[0], payload.shape[1],
                                     rowids.data_ptr(), rid_code(rowids.dtype), rowids.shape[0],
                                     out.data_ptr(), _stream_handle(stream)),
          "tk_gather_f64_device")
