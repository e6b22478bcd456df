"""Parity of the full sort (ORDER BY key without LIMIT, paper sec. V-B with
K = N) with the oracle at K = N, bit for bit: all four key types, both orders,
implicit and explicit row-ids of both widths (explicit ones permuted, so ties
are decided by row-id digits), heavy ties (Zipf), the IEEE totalOrder specials,
ragged tails around the 4096-pair tile, and 2^24 pairs per key type (the
oracle's K = N result, which the oracle pins tie to numpy.lexsort)."""
from __future__ import annotations

import numpy as np
import pytest

import inputgen
import oracle
import paper_2601_19911_amd as tk
from inputgen import native as gen
from tests.gpu_util import assert_same, order_code, say, to_dev, to_np

pytestmark = pytest.mark.gpu

KINDS = {"int32": inputgen.KIND_U_I32, "int64": inputgen.KIND_U_I64,
         "float32": inputgen.KIND_U_F32, "float64": inputgen.KIND_U_F64}


def _run(keys, rids, order, rid_dtype=np.uint32):
    import torch
    kd = to_dev(keys)
    rd = None if rids is None else to_dev(rids)
    tdt = torch.uint32 if rid_dtype == np.uint32 else torch.uint64
    ok, orr = tk.sort(kd, rowids=rd, order=order, rid_dtype=None if rd is not None else tdt)
    torch.cuda.synchronize()
    return to_np(ok), to_np(orr)


@pytest.mark.parametrize("dtype", list(KINDS))
@pytest.mark.parametrize("order", ["desc", "asc"])
@pytest.mark.parametrize("rids", ["implicit", "u32", "u64"])
def test_sort_small_ragged(dtype, order, rids):
    rng = np.random.default_rng(17)
    for n in (1, 2, 63, 4095, 4096, 4097, 12289, 100003):
        keys = inputgen.generate(KINDS[dtype], 40 + n, n)
        if dtype in ("int32", "int64"):
            keys = keys % np.array(997, dtype=keys.dtype)  # many ties
        if rids == "implicit":
            r = None
            rdt = np.uint32
        else:
            rdt = np.uint32 if rids == "u32" else np.uint64
            r = (rng.permutation(n).astype(np.uint64) * 7 + (1 << 33 if rids == "u64" else 3)).astype(rdt)
        gk, gr = _run(keys, r, order, rdt)
        ek, er = oracle.topk(keys, r, n, order_code(order), rid_dtype=rdt)
        assert_same(gk, gr, ek, er, what=f"sort {dtype} {order} {rids} n={n}")


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_sort_total_order_specials(dtype):
    ft, it = (np.float32, np.uint32) if dtype == "float32" else (np.float64, np.uint64)
    vals = np.array([np.nan, -np.nan, np.inf, -np.inf, 0.0, -0.0, 1.0, -1.0,
                     np.finfo(ft).tiny, -np.finfo(ft).tiny, np.finfo(ft).max], dtype=ft)
    bitsv = vals.view(it).copy()
    extra = np.array([bitsv[0] | 1, bitsv[1] | 3], dtype=it)  # NaN payloads
    pool = np.concatenate([bitsv, extra]).view(ft)
    rng = np.random.default_rng(2)
    keys = pool[rng.integers(0, pool.shape[0], 30000)]
    for order in ("desc", "asc"):
        gk, gr = _run(keys, None, order)
        ek, er = oracle.topk(keys, None, keys.shape[0], order_code(order))
        assert_same(gk, gr, ek, er, what=f"specials {dtype} {order}")


@pytest.mark.parametrize("dtype", list(KINDS))
def test_sort_full_size(dtype):
    """2^24 pairs per key type, uniform, descending, implicit row-ids; plus
    Zipf (heavy ties) ascending for int64 with explicit permuted row-ids."""
    n = 1 << 24
    keys = gen.host_fill(KINDS[dtype], inputgen.config_seed(7, 1), n)
    say(f"sort {dtype} n=2^24 desc")
    gk, gr = _run(keys, None, "desc")
    ek, er = oracle.topk(keys, None, n, oracle.DESC)
    assert_same(gk, gr, ek, er, what=f"sort {dtype} 2^24")
    if dtype == "int64":
        cdf = inputgen.zipf_cdf(1.1, 10 ** 6)
        zk = gen.host_fill(inputgen.KIND_ZIPF_I64, inputgen.config_seed(7, 2), n, cdf=cdf)
        r = np.random.default_rng(5).permutation(n).astype(np.uint64)
        gk, gr = _run(zk, r, "asc", np.uint64)
        ek, er = oracle.topk(zk, r, n, oracle.ASC)
        assert_same(gk, gr, ek, er, what="sort zipf int64 asc explicit row-ids 2^24")
