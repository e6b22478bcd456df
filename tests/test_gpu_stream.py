"""Parity of the chunk-pipelined key-only streaming path (tk_topk_stream)
with the oracle: a key column in host memory copied to the device in chunks
through two staging buffers, each chunk's Top-K merged into the running
result.  Columns larger than a chunk (ragged last chunk), K larger than a
chunk, explicit and implicit row-ids (implicit ones become column positions
across chunks), pinned and pageable host memory, with and without a separate
copy stream, and a 2^26-row column at the default chunk size."""
import numpy as np
import pytest

import inputgen
import oracle
from tests.gpu_util import assert_same, order_code, say, to_np

pytestmark = pytest.mark.gpu

import paper_2601_19911_amd as tk


def _pinned(a: np.ndarray):
    import torch
    t = torch.empty(a.shape[0], dtype={np.dtype(np.float32): torch.float32,
                                       np.dtype(np.float64): torch.float64,
                                       np.dtype(np.int32): torch.int32,
                                       np.dtype(np.int64): torch.int64,
                                       np.dtype(np.uint32): torch.int32,
                                       np.dtype(np.uint64): torch.int64}[a.dtype], pin_memory=True)
    t.numpy().view(a.dtype)[:] = a
    if a.dtype == np.uint32:
        return t.view(torch.uint32)
    if a.dtype == np.uint64:
        return t.view(torch.uint64)
    return t


def _run(keys, rids, k, order, chunk, pinned, copy_stream, rid_dtype=np.uint32):
    import torch
    say(f"stream case n={len(keys)} {keys.dtype} k={k} {order} chunk={chunk} "
        f"rids={'none' if rids is None else rids.dtype} pinned={pinned} copy_stream={copy_stream}")
    hk = _pinned(keys) if pinned else keys
    hr = None if rids is None else (_pinned(rids) if pinned else rids)
    cs = torch.cuda.Stream() if copy_stream else None
    tdt = torch.uint32 if np.dtype(rid_dtype) == np.uint32 else torch.uint64
    ok, orr = tk.topk_stream(hk, k, h_rowids=hr, order=order, chunk=chunk, rid_dtype=tdt,
                             copy_stream=cs)
    torch.cuda.synchronize()
    exp = oracle.topk(keys, rids, k, order_code(order), rid_dtype=rid_dtype)
    assert_same(to_np(ok), to_np(orr), exp[0], exp[1],
                what=f"stream n={len(keys)} k={k} chunk={chunk}")


def test_stream_ragged_chunks_pinned_copy_stream():
    n = (1 << 24) + 12345
    keys = inputgen.generate(inputgen.KIND_U_F32, inputgen.config_seed(4, 70), n)
    _run(keys, None, 1000, "desc", (1 << 20) + 3, pinned=True, copy_stream=True)


def test_stream_explicit_rowids_pageable_zipf_ascending():
    n = (1 << 22) + 77
    cdf = inputgen.zipf_cdf(1.05, 10 ** 6)
    keys = inputgen.generate(inputgen.KIND_ZIPF_I64, inputgen.config_seed(4, 71), n, cdf=cdf)
    rids = np.random.default_rng(71).permutation(n).astype(np.uint64)
    _run(keys, rids, 5000, "asc", 3 * (1 << 18) + 7, pinned=False, copy_stream=False,
         rid_dtype=np.uint64)


@pytest.mark.parametrize("dtype,kind", [("int32", inputgen.KIND_U_I32), ("float64", inputgen.KIND_U_F64)])
def test_stream_k_larger_than_a_chunk(dtype, kind):
    n = 100_003
    keys = inputgen.generate(kind, inputgen.config_seed(4, 72), n)
    _run(keys, None, 10_000, "desc", 4096, pinned=True, copy_stream=True)
    _run(keys, None, 10_000, "asc", 4096, pinned=False, copy_stream=False)


def test_stream_single_chunk_and_empty():
    import torch
    keys = inputgen.generate(inputgen.KIND_U_F32, inputgen.config_seed(4, 73), 5000)
    _run(keys, None, 100, "desc", 0, pinned=True, copy_stream=False)
    ok, orr = tk.topk_stream(np.zeros(0, dtype=np.float32), 10)
    torch.cuda.synchronize()
    assert ok.numel() == 0 and orr.numel() == 0


def test_stream_full_size_default_chunk():
    """2^26 float32 keys in pinned host memory, K = 1000, default 2^24-key chunks."""
    from inputgen import native as gen
    n = 1 << 26
    keys = gen.host_fill(inputgen.KIND_U_F32, inputgen.config_seed(4, 74), n)
    _run(keys, None, 1000, "desc", 0, pinned=True, copy_stream=True)
