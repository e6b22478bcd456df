"""Parity of the key-only hash-join probe (matching primitive, paper sec.
III-B) with the join oracle: every (probe row-id, build row-id) pair whose keys
are equal.  The device returns the pairs in no particular order, so both sides
are compared as sequences sorted by (probe row-id, build row-id): the match
multiset is what the definition fixes.

Cases: unique and duplicated build keys, the empty-slot marker value (INT_MIN)
on both sides, all keys equal (the cross product), no match, empty sides,
explicit and implicit row-ids of both widths, int32 and int64 keys, a count-only
probe and an output smaller than the match count; and the full-size workload:
2^24 unique int64 build keys probed by 2^26 foreign keys with a 1/2 hit rate.
Every case runs on tables built with the bloom prefilter and without it.
"""
from __future__ import annotations

import numpy as np
import pytest

import inputgen
import oracle
from inputgen import native as gen
from tests.gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=["bloom", "no_bloom"])
def bloom_mode(request):
    """Every case runs on tables built with and without the bloom prefilter."""
    import paper_2601_19911_amd as tk
    tk.set_tuning(join_bloom=1 if request.param == "bloom" else 2)
    yield request.param
    tk.set_tuning(join_bloom=1)


def _sorted_pairs(p, b):
    p = np.asarray(p).astype(np.uint64)
    b = np.asarray(b).astype(np.uint64)
    o = np.lexsort((b, p))
    return p[o], b[o]


def _gpu_join(bk, br, pk, pr, rid_dtype=None):
    import torch
    from paper_2601_19911_amd.join import join
    op, ob = join(to_dev(bk), to_dev(pk), None if br is None else to_dev(br),
                  None if pr is None else to_dev(pr))
    torch.cuda.synchronize()
    return _sorted_pairs(to_np(op), to_np(ob))


def _check(bk, br, pk, pr, what):
    gp, gb = _gpu_join(bk, br, pk, pr)
    ep, eb = oracle.join(bk, br, pk, pr)
    assert gp.shape == ep.shape, f"{what}: {gp.shape[0]} matches, oracle {ep.shape[0]}"
    bad = np.flatnonzero((gp != ep) | (gb != eb))
    assert bad.size == 0, f"{what}: {bad.size} mismatching pairs, first at {int(bad[0])}"
    return ep.shape[0]


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("rids", ["implicit", "u32", "u64"])
def test_join_small_random_with_duplicates(dtype, rids):
    rng = np.random.default_rng(3)
    for nb, np_, span in [(1, 1, 2), (100, 257, 50), (5000, 20011, 3000), (70001, 65537, 1 << 20),
                          (3, 100003, 5)]:
        bk = rng.integers(-span, span, nb).astype(dtype)
        pk = rng.integers(-span, span, np_).astype(dtype)
        if rids == "implicit":
            br = pr = None
        else:
            rt = np.uint32 if rids == "u32" else np.uint64
            br = (rng.permutation(nb).astype(np.uint64) * 3 + 11).astype(rt)
            pr = (rng.permutation(np_).astype(np.uint64) * 5 + 2).astype(rt)
        m = _check(bk, br, pk, pr, f"{np.dtype(dtype).name} nb={nb} np={np_} span={span} {rids}")
        say(f"join {np.dtype(dtype).name} nb={nb} np={np_} rids={rids}: {m} matches equal the oracle")


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_join_empty_marker_and_extremes(dtype):
    info = np.iinfo(dtype)
    rng = np.random.default_rng(8)
    vals = np.array([info.min, info.min + 1, -1, 0, 1, info.max - 1, info.max], dtype=dtype)
    bk = vals[rng.integers(0, len(vals), 3000)]
    pk = vals[rng.integers(0, len(vals), 4000)]
    _check(bk, None, pk, None, "extremes with duplicates")
    # INT_MIN on the probe side only, and on the build side only
    _check(np.array([1, 2, 3], dtype=dtype), None, np.array([info.min, 2], dtype=dtype), None,
           "INT_MIN probe only")
    _check(np.array([info.min, info.min, 5], dtype=dtype), None, np.array([5, 6], dtype=dtype), None,
           "INT_MIN build only")


def test_join_all_equal_is_cross_product():
    nb, np_ = 300, 2000
    bk = np.full(nb, 77, dtype=np.int64)
    pk = np.full(np_, 77, dtype=np.int64)
    m = _check(bk, None, pk, None, "all equal")
    assert m == nb * np_


def test_join_unique_build_stops_at_first_hit():
    # unique build keys: every probe of a build key gets exactly its row
    rng = np.random.default_rng(21)
    n = 1 << 18
    bk = (rng.choice(1 << 40, n, replace=False).astype(np.int64) << 3) - (1 << 42)
    perm = rng.permutation(n)
    gp, gb = _gpu_join(bk, None, bk[perm], None)
    assert np.array_equal(gp, np.arange(n, dtype=np.uint64))
    assert np.array_equal(gb, perm.astype(np.uint64))


def test_join_no_match_and_empty_sides():
    import torch
    from paper_2601_19911_amd.join import join_build, join_probe
    bk = np.arange(0, 20000, 2, dtype=np.int32)
    pk = np.arange(1, 20000, 2, dtype=np.int32)
    assert _check(bk, None, pk, None, "disjoint") == 0
    assert _check(bk[:0], None, pk, None, "empty build") == 0
    t = join_build(to_dev(bk))
    _, _, cnt = join_probe(t, to_dev(pk[:0]))
    torch.cuda.synchronize()
    assert int(cnt.view(torch.int64).item()) == 0


def test_join_count_only_and_short_output():
    import torch
    from paper_2601_19911_amd.join import join_build, join_probe
    rng = np.random.default_rng(4)
    bk = rng.integers(0, 1000, 5000).astype(np.int64)
    pk = rng.integers(0, 1000, 7000).astype(np.int64)
    ep, eb = oracle.join(bk, None, pk, None)
    t = join_build(to_dev(bk))
    _, _, cnt = join_probe(t, to_dev(pk), capacity=0)
    torch.cuda.synchronize()
    assert int(cnt.view(torch.int64).item()) == ep.shape[0]
    cap = ep.shape[0] // 3
    op, ob, cnt = join_probe(t, to_dev(pk), capacity=cap)
    torch.cuda.synchronize()
    assert int(cnt.view(torch.int64).item()) == ep.shape[0]
    gp, gb = to_np(op)[:cap].astype(np.uint64), to_np(ob)[:cap].astype(np.uint64)
    # the written pairs are a sub-multiset of the matches
    e = ep * np.uint64(1 << 32) + eb
    g = gp * np.uint64(1 << 32) + gb
    ev, ec = np.unique(e, return_counts=True)
    gv, gc = np.unique(g, return_counts=True)
    pos = np.searchsorted(ev, gv)
    assert np.all(pos < ev.shape[0]) and np.array_equal(ev[pos], gv) and np.all(gc <= ec[pos])


def test_join_rejects_bad_arguments():
    import ctypes
    import torch
    from paper_2601_19911_amd.join import _bind, tk_join_table
    L = _bind()
    d = tk_join_table()
    buf = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    keys = torch.zeros(16, dtype=torch.float32, device="cuda")
    assert L.tk_join_build(keys.data_ptr(), None, 16, 2, 0, buf.data_ptr(), buf.numel(),
                           ctypes.byref(d), None) == -4  # float keys: TK_EUNSUPPORTED
    assert L.tk_join_build(keys.data_ptr(), None, 16, 1, 0, buf.data_ptr(), 100,
                           ctypes.byref(d), None) == -1  # table too small
    assert L.tk_join_build(keys.data_ptr(), None, 16, 1, 0, buf.data_ptr() + 8, buf.numel() - 8,
                           ctypes.byref(d), None) == -1  # misaligned table


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_join_few_repeated_keys_among_unique(dtype):
    """A handful of build keys occur 2-5 times among 2^17 unique ones: probes of
    the repeated keys return every copy, probes of the others their one match
    (the filter of repeated keys decides which walks go on past a hit)."""
    rng = np.random.default_rng(11)
    uniq = rng.permutation(1 << 18)[: 1 << 17].astype(dtype) - dtype(1 << 17)
    reps = rng.choice(uniq, 40, replace=False)
    extra = np.concatenate([np.repeat(r, 1 + (i % 4)) for i, r in enumerate(reps)]).astype(dtype)
    bk = rng.permutation(np.concatenate([uniq, extra]))
    pk = np.concatenate([rng.integers(-(1 << 17), 1 << 17, 200003).astype(dtype), reps])
    m = _check(bk, None, pk, None, f"few repeated {np.dtype(dtype).name}")
    assert m > 0


def test_join_descriptor_bloom_words(bloom_mode):
    import ctypes
    import torch
    from paper_2601_19911_amd.join import _bind, join_build, join_probe
    bk = torch.arange(1000, dtype=torch.int64, device="cuda")
    t = join_build(bk)
    assert t.desc.bloom_words == (t.slots // 16 if bloom_mode == "bloom" else 0)
    op, ob, cnt = join_probe(t, bk)
    torch.cuda.synchronize()
    assert int(cnt.view(torch.int64).item()) == 1000
    t.desc.bloom_words = 7  # not slots / 16: rejected before any device work
    assert _bind().tk_join_probe(ctypes.byref(t.desc), bk.data_ptr(), None, 1000, 0,
                                 op.data_ptr(), ob.data_ptr(), 1000, cnt.data_ptr(), None) == -1


@pytest.mark.parametrize("dtype,log2b", [(np.int64, 24), (np.int32, 22)])
def test_join_full_size(dtype, log2b):
    """2^log2b uniform build keys (int64: all distinct) probed by 2^26 foreign
    keys drawn uniformly from twice the build's index range (1/2 hit rate),
    row-ids implicit (uint32); every matched pair equals the oracle's."""
    import torch
    from paper_2601_19911_amd.join import join_build, join_probe
    nb, np_ = 1 << log2b, 1 << 26
    seed = inputgen.config_seed(6, log2b)
    bkind = inputgen.KIND_U_I64 if dtype == np.int64 else inputgen.KIND_U_I32
    pkind = inputgen.KIND_JOIN_FK_I64 if dtype == np.int64 else inputgen.KIND_JOIN_FK_I32
    bk = gen.host_fill(bkind, seed, nb)
    pk = gen.host_fill(pkind, seed, np_, n_total=2 * nb)
    say(f"join full size: build {nb} {np.dtype(dtype).name}, probe {np_}")
    t = join_build(to_dev(bk))
    op, ob, cnt = join_probe(t, to_dev(pk))
    torch.cuda.synchronize()
    m = int(cnt.view(torch.int64).item())
    assert m <= np_ or dtype == np.int32
    if m > op.numel():
        op, ob, cnt = join_probe(t, to_dev(pk), capacity=m)
        torch.cuda.synchronize()
    gp, gb = _sorted_pairs(to_np(op)[:m], to_np(ob)[:m])
    ep, eb = oracle.join(bk, None, pk, None)
    say(f"join full size: {m} matches on the device, {ep.shape[0]} in the oracle")
    assert gp.shape == ep.shape
    assert np.array_equal(gp, ep) and np.array_equal(gb, eb)
