"""Binding of the key-only hash-join probe (matching primitive, paper sec.
III-B): ``tk_join_table_size``, ``tk_join_build`` and ``tk_join_probe`` of
libmitopk.so.  Argument marshalling only; the build and the probe run in the
library's HIP kernels.
"""

from __future__ import annotations

import ctypes

from . import _ptr, _stream_handle, check, lib, rid_code, TK_KEY_I32, TK_KEY_I64


class tk_join_table(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("table_bytes", ctypes.c_uint64),
                ("n_build", ctypes.c_uint64), ("slots", ctypes.c_uint64),
                ("key_type", ctypes.c_int32), ("rid_type", ctypes.c_int32),
                ("bloom_words", ctypes.c_uint64)]


_bound = None


def _bind():
    global _bound
    L = lib()
    if _bound is not L:
        vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        L.tk_join_table_size.argtypes = [u64, i32, i32]
        L.tk_join_table_size.restype = ctypes.c_size_t
        L.tk_join_build.argtypes = [vp, vp, u64, i32, i32, vp, ctypes.c_size_t,
                                    ctypes.POINTER(tk_join_table), vp]
        L.tk_join_build.restype = i32
        L.tk_join_probe.argtypes = [ctypes.POINTER(tk_join_table), vp, vp, u64, i32, vp, vp, u64,
                                    vp, vp]
        L.tk_join_probe.restype = i32
        _bound = L
    return L


def _key_code(dtype) -> int:
    import torch
    if dtype == torch.int32:
        return TK_KEY_I32
    if dtype == torch.int64:
        return TK_KEY_I64
    raise TypeError(f"join keys must be int32 or int64, not {dtype}")


def join_table_size(n_build: int, key_type: int, rid_type: int) -> int:
    return int(_bind().tk_join_table_size(n_build, key_type, rid_type))


class JoinTable:
    """A built hash table: the device buffer and its descriptor."""

    def __init__(self, buf, desc: tk_join_table, rid_dtype):
        self.buf = buf
        self.desc = desc
        self.rid_dtype = rid_dtype

    @property
    def n_build(self) -> int:
        return int(self.desc.n_build)

    @property
    def slots(self) -> int:
        return int(self.desc.slots)


def join_build(keys, rowids=None, rid_dtype=None, table=None, stream=None) -> JoinTable:
    """Builds the table from device tensors ``keys`` (int32/int64) and
    ``rowids`` (uint32/uint64, or None for row-id = position; ``rid_dtype``
    then sets the row-id type, default uint32).  ``table`` may be a uint8
    device tensor of at least join_table_size bytes."""
    import torch
    kt = _key_code(keys.dtype)
    if rowids is not None:
        rid_dtype = rowids.dtype
    if rid_dtype is None:
        rid_dtype = torch.uint32
    rt = rid_code(rid_dtype)
    n = keys.numel()
    need = join_table_size(n, kt, rt)
    if need == 0:
        check(-4, "tk_join_table_size")
    if table is None:
        table = torch.empty(need, dtype=torch.uint8, device=keys.device)
    desc = tk_join_table()
    check(_bind().tk_join_build(_ptr(keys), _ptr(rowids), n, kt, rt, table.data_ptr(),
                                table.numel(), ctypes.byref(desc), _stream_handle(stream)),
          "tk_join_build")
    return JoinTable(table, desc, rid_dtype)


def join_probe(table: JoinTable, keys, rowids=None, rid_dtype=None, capacity: int | None = None,
               out_probe=None, out_build=None, count=None, stream=None):
    """Probes ``table`` with device tensor ``keys``; returns (out_probe,
    out_build, count) where ``count`` is a one-element uint64 device tensor
    holding the number of matches once the stream has passed the call (the
    first min(count, capacity) entries of the outputs are valid).  Default
    capacity: the number of probe keys."""
    import torch
    if _key_code(keys.dtype) != table.desc.key_type:
        raise TypeError("probe keys must have the build keys' type")
    if rowids is not None:
        rid_dtype = rowids.dtype
    if rid_dtype is None:
        rid_dtype = torch.uint32
    n = keys.numel()
    if capacity is None:
        capacity = n if out_probe is None else out_probe.numel()
    dev = keys.device
    if out_probe is None:
        out_probe = torch.empty(max(capacity, 1), dtype=rid_dtype, device=dev)
    if out_build is None:
        out_build = torch.empty(max(capacity, 1), dtype=table.rid_dtype, device=dev)
    if count is None:
        count = torch.empty(1, dtype=torch.uint64, device=dev)
    assert out_probe.numel() >= capacity and out_build.numel() >= capacity
    check(_bind().tk_join_probe(ctypes.byref(table.desc), _ptr(keys), _ptr(rowids), n,
                                rid_code(rid_dtype), out_probe.data_ptr(), out_build.data_ptr(),
                                capacity, count.data_ptr(), _stream_handle(stream)),
          "tk_join_probe")
    return out_probe, out_build, count


def join(build_keys, probe_keys, build_rowids=None, probe_rowids=None, stream=None):
    """Build + probe, sized to the exact match count (synchronizes once to read
    the count, and probes a second time only when it exceeds the probe count).
    Returns (probe_rowids, build_rowids) of all matches, in no particular order."""
    import torch
    t = join_build(build_keys, build_rowids, stream=stream)
    op, ob, cnt = join_probe(t, probe_keys, probe_rowids, stream=stream)
    torch.cuda.synchronize()
    m = int(cnt.view(torch.int64).item())
    if m > op.numel():
        op, ob, cnt = join_probe(t, probe_keys, probe_rowids, capacity=m, stream=stream)
        torch.cuda.synchronize()
    return op[:m], ob[:m]
