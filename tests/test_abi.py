"""The C-ABI library loads on a machine without a GPU, exports every entry
point its headers declare, and rejects bad arguments before touching the
device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_2601_19911_amd as tk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(tk_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("tk_topk", "tk_workspace_size", "tk_query_info", "tk_cpu_topk", "tk_status_string"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports(name):
    L = ctypes.CDLL(tk.LIB_PATH)
    assert hasattr(L, name), f"{name} declared in include/ but not exported"


def test_status_strings():
    L = tk.lib()
    for code in (0, -1, -2, -3, -4, -5, 1):
        assert len(L.tk_status_string(code)) > 0


def test_argument_errors_before_device_work():
    L = tk.lib()
    cnt = ctypes.c_uint64(99)
    # bad key type, bad row-id type, bad order
    assert L.tk_topk(None, None, 0, 1, 7, 0, 0, None, None, ctypes.byref(cnt), None, 0, None) == -1
    assert L.tk_topk(None, None, 0, 1, 0, 5, 0, None, None, ctypes.byref(cnt), None, 0, None) == -1
    assert L.tk_topk(None, None, 0, 1, 0, 0, 3, None, None, ctypes.byref(cnt), None, 0, None) == -1
    # null keys with n > 0
    assert L.tk_topk(None, None, 10, 1, 0, 0, 0, None, None, ctypes.byref(cnt), None, 0, None) == -1
    # n = 0 and k = 0 are valid and enqueue nothing
    assert L.tk_topk(None, None, 0, 5, 0, 0, 0, None, None, ctypes.byref(cnt), None, 0, None) == 0
    assert cnt.value == 0
    assert L.tk_topk(ctypes.c_void_p(16), None, 100, 0, 0, 0, 0, None, None, ctypes.byref(cnt),
                     None, 0, None) == 0
    assert cnt.value == 0
    # implicit uint32 row-ids cannot index more than 2^32 keys
    assert L.tk_topk(ctypes.c_void_p(16), None, (1 << 32) + 1, 5, 0, 0, 0, None, None,
                     ctypes.byref(cnt), None, 0, None) == -1


def test_workspace_size_is_pure_arithmetic():
    for (n, k) in [(0, 0), (1, 1), (1 << 20, 100), (1 << 28, 1000), (1 << 28, 100000), (1 << 24, 1 << 23)]:
        for kt in (0, 1, 2):
            for rt in (0, 1):
                s = tk.workspace_size(n, k, kt, rt)
                assert s >= 8192 and s % 256 == 0
    # grows with k
    assert tk.workspace_size(1 << 28, 100000, 2, 0) > tk.workspace_size(1 << 28, 1000, 2, 0)


def test_noalloc_argument_errors_before_device_work():
    L = tk.lib()
    cnt = ctypes.c_uint64(99)
    assert L.tk_topk_noalloc(None, None, 0, 1, 9, 0, 0, None, None, ctypes.byref(cnt), None) == -1
    assert L.tk_topk_noalloc(None, None, 10, 1, 0, 0, 0, None, None, ctypes.byref(cnt), None) == -1
    assert L.tk_topk_noalloc(None, None, 0, 5, 0, 0, 0, None, None, ctypes.byref(cnt), None) == 0
    assert cnt.value == 0
    # a workspace beyond the library's array is refused before any device call
    n, k = 1 << 24, 1 << 22
    assert tk.workspace_size(n, k, 1, 1) > tk.NOALLOC_SCRATCH_BYTES
    assert L.tk_topk_noalloc(ctypes.c_void_p(256), None, n, k, 1, 1, 0, None, None,
                             ctypes.byref(cnt), None) == -4


def test_noalloc_array_size_matches_header():
    text = open(os.path.join(ROOT, "include", "mitopk.h")).read()
    m = re.search(r"#define TK_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and (int(m.group(1)) << int(m.group(2))) == tk.NOALLOC_SCRATCH_BYTES
    # every K up to 100000 runs in the array at any N up to 2^30, all key and
    # row-id types (a query with no usable sample may do so without the sort's scratch)
    for lg in range(1, 31):
        for n in ((1 << lg) - 1, 1 << lg, 3 << (lg - 1)):
            for kt in range(4):
                for rt in range(2):
                    assert tk.workspace_min_size(n, 100000, kt, rt) <= tk.NOALLOC_SCRATCH_BYTES


def test_workspace_min_size():
    """The least workspace differs from tk_workspace_size only by the full
    sort's scratch, only for queries without a usable sample from 2^16 keys
    (K above N / 2, or K above N / 16 past 2^20 keys)."""
    kb, rb = {0: 4, 1: 8, 2: 4, 3: 8}, {0: 4, 1: 8}
    for n, k, sorts in [(1000, 900, False), (65535, 40000, False), (65536, 40000, True),
                        (1 << 20, 1000, False), (1 << 20, 1 << 17, False), (1 << 22, 1 << 19, True),
                        (1 << 28, 1000, False), ((1 << 21) + 1, 1 << 20, True)]:
        for kt in range(4):
            for rt in range(2):
                full = tk.workspace_size(n, k, kt, rt)
                least = tk.workspace_min_size(n, k, kt, rt)
                assert 0 < least <= full
                if sorts:
                    # two ping-pong copies of every pair, plus digit counts
                    assert full - least >= 2 * n * (kb[kt] + rb[rt])
                else:
                    assert full == least, (n, k, kt, rt)


def test_sort_argument_errors_before_device_work():
    """tk_sort refuses bad arguments and sizes beyond its 32-bit digit counts
    before touching the device (no GPU here; fake aligned pointers).  A handle
    of its own, so that the argument types set here stay local."""
    L = ctypes.CDLL(tk.LIB_PATH)
    L.tk_sort_workspace_size.restype = ctypes.c_size_t
    L.tk_sort_workspace_size.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
    L.tk_sort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                          ctypes.c_void_p]
    p = ctypes.c_void_p(1 << 20)
    assert L.tk_sort_workspace_size(1000, 9, 0) == 0                       # bad key type
    assert L.tk_sort(p, None, 1000, 0, 0, 2, p, p, p, 1 << 30, None) == -1  # bad order
    assert L.tk_sort(None, None, 0, 0, 0, 0, None, None, None, 0, None) == 0  # n = 0: nothing
    assert L.tk_sort(p, None, 1000, 0, 0, 0, p, None, p, 1 << 30, None) == -1  # out_rowids required
    need = L.tk_sort_workspace_size(1000, 0, 0)
    assert L.tk_sort(p, None, 1000, 0, 0, 0, p, p, p, need - 256, None) == -1  # small workspace
    assert L.tk_sort(p, None, 1000, 0, 0, 0, p, p, ctypes.c_void_p((1 << 20) + 64), need, None) == -1
    n = 1 << 32
    big = L.tk_sort_workspace_size(n, 0, 1)
    assert big >= 2 * n * 12
    assert L.tk_sort(p, p, n, 0, 1, 0, p, p, p, big, None) == -4  # 2^32 pairs: TK_EUNSUPPORTED
