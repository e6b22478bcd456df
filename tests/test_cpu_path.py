"""The multithreaded CPU route of the gate (tk_cpu_topk) against the oracle."""
import numpy as np
import pytest

import inputgen
import oracle
import paper_2601_19911_amd as tk


def _same(a, b):
    assert np.array_equal(a[0].view(np.uint8), b[0].view(np.uint8))
    assert np.array_equal(a[1].astype(np.uint64), b[1].astype(np.uint64))


@pytest.mark.parametrize("kind", [inputgen.KIND_U_I32, inputgen.KIND_U_F32, inputgen.KIND_U_I64,
                                  inputgen.KIND_ZIPF_F32, inputgen.KIND_SORTED_F32, inputgen.KIND_U_F64])
@pytest.mark.parametrize("n,k", [(1, 1), (1000, 0), (1000, 999), (1000, 5000), (70001, 100),
                                 (300000, 1000), (300000, 40000)])
@pytest.mark.parametrize("order", ["desc", "asc"])
def test_cpu_matches_oracle(kind, n, k, order):
    cdf = inputgen.zipf_cdf(1.1, 10 ** 6) if kind == inputgen.KIND_ZIPF_F32 else None
    keys = inputgen.generate(kind, 17, n, cdf=cdf)
    o = oracle.DESC if order == "desc" else oracle.ASC
    for rids in (None, np.random.default_rng(n).permutation(n).astype(np.uint32)):
        got = tk.cpu_topk(keys, k, rowids=rids, order=order, nthreads=4)
        exp = oracle.topk(keys, rids, k, o)
        _same(got, exp)


def test_cpu_u64_rowids_and_specials():
    bits = np.array([0xFFC00000, 0xFF800000, 0x80000000, 0, 0x3F800000, 0x7F800000, 0x7FC00000] * 5000,
                    dtype=np.uint32)
    keys = bits.view(np.float32)
    rids = np.arange(len(keys), dtype=np.uint64)[::-1].copy()
    for order, o in (("desc", oracle.DESC), ("asc", oracle.ASC)):
        _same(tk.cpu_topk(keys, 12345, rowids=rids, order=order), oracle.topk(keys, rids, 12345, o))


def test_cpu_float64_specials():
    bits = np.array([0xFFF8000000000000, 0xFFF0000000000000, 0x8000000000000000, 0, 0x0000000000000001,
                     0x3FF0000000000000, 0x7FF0000000000000, 0x7FF8000000000000] * 4000, dtype=np.uint64)
    keys = bits.view(np.float64)
    rids = np.arange(len(keys), dtype=np.uint64)[::-1].copy()
    for order, o in (("desc", oracle.DESC), ("asc", oracle.ASC)):
        _same(tk.cpu_topk(keys, 9999, rowids=rids, order=order), oracle.topk(keys, rids, 9999, o))


def test_gather_rows_host_is_numpy_take():
    """Late materialization: gathered rows equal numpy's take on the payload."""
    import paper_2601_19911_amd as tk
    rng = np.random.default_rng(5)
    pay = rng.random((8, 50000))
    for dt in (np.uint32, np.uint64):
        r = rng.integers(0, 50000, 3000).astype(dt)
        assert np.array_equal(tk.gather_rows_host(pay, r).view(np.uint64),
                              pay[:, r.astype(np.int64)].view(np.uint64))
    assert tk.gather_rows_host(pay, np.zeros(0, dtype=np.uint32)).shape == (8, 0)
    with pytest.raises(tk.TopKError):
        tk.gather_rows_host(pay, np.array([50000], dtype=np.uint32))
