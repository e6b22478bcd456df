"""The allocation-free entry point (tk_topk_noalloc) against tk_topk.

tk_topk_noalloc runs the same kernels as tk_topk with the workspace in the
library's own per-device array.  Two calls in a row (the second on a smaller
input, so that it runs over what the first left in the array) must equal
tk_topk with a caller workspace bit for bit, and the oracle; a query whose
workspace exceeds the array is refused before anything is enqueued.
"""
import numpy as np
import pytest

import inputgen
import oracle
from tests.gpu_util import assert_same, order_code, say, to_dev, to_np

pytestmark = pytest.mark.gpu

import paper_2601_19911_amd as tk


def _both(keys, rids, k, order, rid_dtype):
    import torch
    tdt = torch.uint32 if np.dtype(rid_dtype) == np.uint32 else torch.uint64
    kd = to_dev(keys)
    rd = None if rids is None else to_dev(rids)
    k_eff = min(k, len(keys))
    ok = torch.empty(k_eff, dtype=kd.dtype, device=kd.device)
    orr = torch.empty(k_eff, dtype=tdt, device=kd.device)
    say(f"noalloc case n={len(keys)} dtype={keys.dtype} k={k} order={order}")
    tk.topk_noalloc(kd, k, ok, orr, rowids=rd, order=order)
    torch.cuda.synchronize()
    got = (to_np(ok), to_np(orr))
    ek, er = tk.topk(kd, k, rowids=rd, order=order, rid_dtype=tdt)
    torch.cuda.synchronize()
    ref = (to_np(ek), to_np(er))
    assert_same(got[0], got[1], ref[0], ref[1], what=f"noalloc vs tk_topk n={len(keys)} k={k}")
    exp = oracle.topk(keys, rids, k, order_code(order), rid_dtype=rid_dtype)
    assert_same(got[0], got[1], exp[0], exp[1], what=f"noalloc vs oracle n={len(keys)} k={k}")


def test_noalloc_two_calls_second_smaller():
    # first: a large query on the sampled path with the bucketed tail (K > 2048)
    n1 = (1 << 24) + 12345
    keys1 = inputgen.generate(inputgen.KIND_U_F32, inputgen.config_seed(2, 50), n1)
    _both(keys1, None, 20000, "desc", np.uint32)
    # second: smaller, other key and row-id types, explicit row-ids, ranked tail
    n2 = (1 << 20) + 7
    keys2 = inputgen.generate(inputgen.KIND_U_I64, inputgen.config_seed(2, 51), n2)
    rids2 = np.random.default_rng(51).permutation(n2).astype(np.uint64)
    _both(keys2, rids2, 1000, "asc", np.uint64)


def test_noalloc_exact_and_small_paths():
    # no usable sample (K above N / 2): the full sort keeping K pairs, then a one-tile query
    n = 300_001
    keys = inputgen.generate(inputgen.KIND_U_I32, inputgen.config_seed(2, 52), n)
    _both(keys, None, 200_000, "desc", np.uint32)
    keys = inputgen.generate(inputgen.KIND_U_F32, inputgen.config_seed(2, 53), 5000)
    _both(keys, None, 300, "asc", np.uint32)


def test_noalloc_sort_scratch_beyond_the_array():
    # no usable sample, the sort's scratch (64 MiB) beyond the array: the grid-wide
    # exact select (8 MiB) runs instead and equals tk_topk's sort route
    n = 1 << 22
    keys = inputgen.generate(inputgen.KIND_U_F32, inputgen.config_seed(2, 54), n)
    assert tk.workspace_size(n, 1 << 19, tk.TK_KEY_F32, tk.TK_RID_U32) > tk.NOALLOC_SCRATCH_BYTES
    _both(keys, None, 1 << 19, "desc", np.uint32)


def test_noalloc_refuses_beyond_the_array():
    import torch
    n, k = 1 << 24, 1 << 22
    need = tk.workspace_size(n, k, tk.TK_KEY_I64, tk.TK_RID_U64)
    assert need > tk.NOALLOC_SCRATCH_BYTES
    kd = torch.zeros(n, dtype=torch.int64, device="cuda")
    ok = torch.empty(k, dtype=torch.int64, device="cuda")
    orr = torch.empty(k, dtype=torch.uint64, device="cuda")
    with pytest.raises(tk.TopKError, match="unsupported"):
        tk.topk_noalloc(kd, k, ok, orr, order="desc")
