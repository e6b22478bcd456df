"""ORACLE — test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and the library never imports it.

* :func:`topk` / :func:`topk_batched` call ``liboracle.so`` (oracle.cpp), the
  plain definition of the ordering primitive (paper sec. III-A with the query
  template of sec. V-B): sort the (key, row-id) pairs by key (descending or
  ascending), ties by ascending row-id, keep the first min(K, N).
* :func:`brute_topk` is a pure-Python ``sorted`` of the same definition for
  tiny inputs; it orders float keys through the classic sign-flip map of the
  bit pattern, an independent formulation of IEEE 754 totalOrder.
* :func:`check_invariants` tests the properties every correct result has at
  any size.
* :func:`join` calls ``oracle_join`` (join.cpp), the plain definition of the
  matching primitive (paper sec. III-B): every (probe row-id, build row-id)
  pair whose keys are equal, sorted by (probe row-id, build row-id);
  :func:`brute_join` is the nested loop over all pairs, for tiny inputs.
"""

from __future__ import annotations

import ctypes
import os
import struct
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
SRCS = [SRC, os.path.join(HERE, "join.cpp")]
LIB = os.path.join(HERE, "liboracle.so")

KEY_CODE = {np.dtype(np.int32): 0, np.dtype(np.int64): 1, np.dtype(np.float32): 2,
            np.dtype(np.float64): 3}
RID_CODE = {np.dtype(np.uint32): 0, np.dtype(np.uint64): 1}
DESC, ASC = 0, 1

_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", *SRCS, "-o", LIB + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building liboracle.so failed:\n" + r.stderr)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(" ".join(cmd))
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in SRCS):
            build()
        L = ctypes.CDLL(LIB)
        vp, u64 = ctypes.c_void_p, ctypes.c_uint64
        L.oracle_topk.argtypes = [vp, vp, u64, u64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                  vp, ctypes.POINTER(u64)]
        L.oracle_topk.restype = ctypes.c_int
        L.oracle_topk_batched.argtypes = [vp, vp, vp, vp, vp, ctypes.c_uint32, ctypes.c_int,
                                          ctypes.c_int, vp, vp]
        L.oracle_topk_batched.restype = ctypes.c_int
        L.oracle_join.argtypes = [vp, vp, u64, ctypes.c_int, vp, vp, u64, ctypes.c_int, ctypes.c_int]
        L.oracle_join.restype = ctypes.c_int64
        L.oracle_join_fetch.argtypes = [vp, vp]
        L.oracle_join_fetch.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def topk(keys: np.ndarray, rowids: np.ndarray | None, k: int, order: int = DESC,
         rid_dtype=np.uint32):
    """Returns (out_keys, out_rowids) of the first min(k, n) pairs, best first.

    ``rowids=None`` means row-id = index; then ``rid_dtype`` sets the output type.
    """
    keys = np.ascontiguousarray(keys)
    n = keys.shape[0]
    if rowids is not None:
        rowids = np.ascontiguousarray(rowids)
        assert rowids.shape[0] == n
        rid_dtype = rowids.dtype
    kc = KEY_CODE[keys.dtype]
    rc_ = RID_CODE[np.dtype(rid_dtype)]
    k_eff = min(int(k), n)
    ok = np.empty(k_eff, dtype=keys.dtype)
    orr = np.empty(k_eff, dtype=rid_dtype)
    cnt = ctypes.c_uint64(0)
    rc = _load().oracle_topk(_ptr(keys), _ptr(rowids), n, int(k), kc, rc_, int(order), _ptr(ok),
                             _ptr(orr), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_topk rejected its arguments")
    assert cnt.value == k_eff
    return ok, orr


def topk_batched(keys: np.ndarray, rowids: np.ndarray | None, offsets: np.ndarray,
                 ks: np.ndarray, orders: np.ndarray, rid_dtype=np.uint32):
    """Per-query results packed at the exclusive prefix sum of min(k_q, n_q)."""
    keys = np.ascontiguousarray(keys)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    ks = np.ascontiguousarray(ks, dtype=np.uint32)
    orders = np.ascontiguousarray(orders, dtype=np.uint8)
    if rowids is not None:
        rowids = np.ascontiguousarray(rowids)
        rid_dtype = rowids.dtype
    n = np.diff(offsets.astype(np.int64))
    total = int(np.minimum(ks.astype(np.int64), n).sum())
    ok = np.empty(total, dtype=keys.dtype)
    orr = np.empty(total, dtype=rid_dtype)
    rc = _load().oracle_topk_batched(_ptr(keys), _ptr(rowids), offsets.ctypes.data,
                                     ks.ctypes.data, orders.ctypes.data, len(ks),
                                     KEY_CODE[keys.dtype], RID_CODE[np.dtype(rid_dtype)],
                                     _ptr(ok), _ptr(orr))
    if rc != 0:
        raise ValueError("oracle_topk_batched rejected its arguments")
    return ok, orr


JOIN_KEY_CODE = {np.dtype(np.int32): 0, np.dtype(np.int64): 1}
_join_lock = threading.Lock()


def join(build_keys: np.ndarray, build_rowids: np.ndarray | None, probe_keys: np.ndarray,
         probe_rowids: np.ndarray | None):
    """Inner equi-join matches: (probe_rowids, build_rowids), both uint64,
    sorted by (probe row-id, build row-id).  ``None`` row-ids mean position."""
    bk = np.ascontiguousarray(build_keys)
    pk = np.ascontiguousarray(probe_keys)
    assert bk.dtype == pk.dtype
    kc = JOIN_KEY_CODE[bk.dtype]
    br = None if build_rowids is None else np.ascontiguousarray(build_rowids)
    pr = None if probe_rowids is None else np.ascontiguousarray(probe_rowids)
    brc = 0 if br is None else RID_CODE[br.dtype]
    prc = 0 if pr is None else RID_CODE[pr.dtype]
    L = _load()
    with _join_lock:
        m = L.oracle_join(_ptr(bk), _ptr(br), bk.shape[0], brc, _ptr(pk), _ptr(pr), pk.shape[0],
                          prc, kc)
        if m < 0:
            raise ValueError("oracle_join rejected its arguments")
        op = np.empty(m, dtype=np.uint64)
        ob = np.empty(m, dtype=np.uint64)
        L.oracle_join_fetch(op.ctypes.data, ob.ctypes.data)
    return op, ob


def brute_join(build_keys, build_rowids, probe_keys, probe_rowids):
    """Nested loop over every (probe, build) pair: the definition itself."""
    nb, np_ = len(build_keys), len(probe_keys)
    brid = list(range(nb)) if build_rowids is None else [int(r) for r in build_rowids]
    prid = list(range(np_)) if probe_rowids is None else [int(r) for r in probe_rowids]
    out = []
    for j in range(np_):
        for i in range(nb):
            if int(probe_keys[j]) == int(build_keys[i]):
                out.append((prid[j], brid[i]))
    out.sort()
    return [p for p, _ in out], [b for _, b in out]


# ---- pure-Python brute force (tiny inputs) --------------------------------------------------

def _f32_total_rank(bits: int) -> int:
    """Integer whose natural order is IEEE totalOrder on a float32 bit pattern."""
    return (bits ^ 0xFFFFFFFF) if bits & 0x80000000 else (bits | 0x80000000)


def _f64_total_rank(bits: int) -> int:
    """Integer whose natural order is IEEE totalOrder on a float64 bit pattern."""
    return (bits ^ 0xFFFFFFFFFFFFFFFF) if bits >> 63 else (bits | (1 << 63))


def brute_topk(keys, rowids, k, order=DESC):
    """sorted() of all pairs by the definition, first min(k, n) kept."""
    keys = np.asarray(keys)
    n = len(keys)
    rids = list(range(n)) if rowids is None else [int(r) for r in rowids]
    if keys.dtype == np.float32:
        ranks = [_f32_total_rank(int(b)) for b in keys.view(np.uint32)]
    elif keys.dtype == np.float64:
        ranks = [_f64_total_rank(int(b)) for b in keys.view(np.uint64)]
    else:
        ranks = [int(x) for x in keys]
    sign = -1 if order == DESC else 1
    idx = sorted(range(n), key=lambda i: (sign * ranks[i], rids[i]))
    idx = idx[: min(int(k), n)]
    return [keys[i] for i in idx], [rids[i] for i in idx]


# ---- invariants ----------------------------------------------------------------------------

def order_rank(keys: np.ndarray, order: int) -> np.ndarray:
    """uint64 array whose ascending order is 'best first' for the key part.

    Integer keys are offset into the unsigned range; float32 keys go through
    the sign-flip map (totalOrder).  Used only by the invariant checks below.
    """
    if keys.dtype == np.int32:
        u = (keys.astype(np.int64) + (1 << 31)).astype(np.uint64)
        top = np.uint64((1 << 32) - 1)
    elif keys.dtype == np.int64:
        u = keys.view(np.uint64) ^ np.uint64(1 << 63)
        top = np.uint64((1 << 64) - 1)
    elif keys.dtype == np.float32:
        b = keys.view(np.uint32).astype(np.uint64)
        neg = (b >> np.uint64(31)) == 1
        u = np.where(neg, b ^ np.uint64(0xFFFFFFFF), b | np.uint64(0x80000000))
        top = np.uint64((1 << 32) - 1)
    elif keys.dtype == np.float64:
        b = keys.view(np.uint64)
        neg = (b >> np.uint64(63)) == 1
        u = np.where(neg, ~b, b | np.uint64(1 << 63))
        top = np.uint64((1 << 64) - 1)
    else:
        raise TypeError(keys.dtype)
    return (top - u) if order == DESC else u


def check_invariants(keys, rowids, k, order, out_keys, out_rowids, full_check=True):
    """Raises AssertionError unless (out_keys, out_rowids) is a valid Top-K.

    Checks, at any size: |out| = min(k, n); best-first order under (key,
    row-id); the inputs better than the last output are exactly the outputs
    before it (as a multiset of (key bits, row-id) pairs), and the input holds
    enough copies of the last pair.  ``rowids=None`` means row-id = index.
    With ``full_check=False`` only the length and the order are checked.
    """
    keys = np.asarray(keys)
    n = keys.shape[0]
    k_eff = min(int(k), n)
    out_keys = np.asarray(out_keys).astype(keys.dtype)
    out_rowids = np.asarray(out_rowids).astype(np.uint64)
    assert out_keys.shape[0] == k_eff, "wrong output length"
    assert out_rowids.shape[0] == k_eff, "wrong output length"
    if k_eff == 0:
        return
    ro = order_rank(out_keys, order)
    if k_eff > 1:
        ok = (ro[:-1] < ro[1:]) | ((ro[:-1] == ro[1:]) & (out_rowids[:-1] <= out_rowids[1:]))
        assert bool(np.all(ok)), "output not sorted best-first"
    if not full_check:
        return
    rid = (np.arange(n, dtype=np.uint64) if rowids is None
           else np.asarray(rowids).astype(np.uint64))
    ri = order_rank(keys, order)
    last_r, last_id = ro[-1], out_rowids[-1]
    better = (ri < last_r) | ((ri == last_r) & (rid < last_id))
    same = (ri == last_r) & (rid == last_id)
    nb, ns = int(better.sum()), int(same.sum())
    assert nb <= k_eff - 1, "more inputs are better than the K-th output than K-1"
    assert k_eff <= nb + ns, "the input lacks copies of the K-th output pair"
    bits = np.uint32 if keys.dtype.itemsize == 4 else np.uint64
    sel_r, sel_id = ri[better], rid[better]
    sel_b = keys.view(bits)[better]
    o = np.lexsort((sel_id, sel_r))
    exp_b = np.concatenate([sel_b[o], np.repeat(out_keys.view(bits)[-1:], k_eff - nb)])
    exp_id = np.concatenate([sel_id[o], np.repeat(out_rowids[-1:], k_eff - nb)])
    assert np.array_equal(exp_b, out_keys.view(bits)), "output keys are not the best keys"
    assert np.array_equal(exp_id, out_rowids), "output row-ids are not the best row-ids"
