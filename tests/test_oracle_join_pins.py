"""Pins of the join oracle (matching primitive, paper sec. III-B) against what
the definition and independent routines fix:

* hand-derived fixtures (tests/golden/join_probe.json);
* exhaustive brute force: every key vector over a small alphabet on both sides,
  with identity and permuted row-ids, against the nested loop over all pairs;
* pandas.merge (an independent inner-join implementation) on mid-size inputs
  with heavy duplicates, and the count identity sum_v n_build(v) * n_probe(v);
* closed forms: unique build keys probed by a permutation of them; all keys
  equal (the cross product); disjoint key sets (no pair).
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "join_probe.json")))


def _arr(v, dt):
    return None if v is None else np.array(v, dtype=dt)


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=lambda c: c["name"])
def test_join_golden_fixture(case):
    dt = np.dtype(case["dtype"])
    op, ob = oracle.join(_arr(case["build_keys"], dt), _arr(case["build_rowids"], np.uint32),
                         _arr(case["probe_keys"], dt), _arr(case["probe_rowids"], np.uint64))
    assert op.tolist() == case["expected_probe"]
    assert ob.tolist() == case["expected_build"]


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_join_exhaustive_alphabet(dtype):
    info = np.iinfo(dtype)
    alphabet = [int(info.min), -1, 0, int(info.max)]
    rng = np.random.default_rng(11)
    cases = 0
    for nb in range(0, 4):
        for np_ in range(0, 4):
            for bk in itertools.product(alphabet, repeat=nb):
                for pk in itertools.product(alphabet, repeat=np_):
                    bka = np.array(bk, dtype=dtype)
                    pka = np.array(pk, dtype=dtype)
                    for perm in (False, True):
                        br = rng.permutation(nb).astype(np.uint32) + 50 if perm else None
                        pr = rng.permutation(np_).astype(np.uint64) + 7 if perm else None
                        op, ob = oracle.join(bka, br, pka, pr)
                        ep, eb = oracle.brute_join(bk, br, pk, pr)
                        assert op.tolist() == ep and ob.tolist() == eb, (bk, pk, perm)
                        cases += 1
    assert cases > 10000


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_join_matches_pandas_merge(dtype):
    pd = pytest.importorskip("pandas")
    rng = np.random.default_rng(5)
    for nb, np_, span in [(2000, 5000, 300), (5000, 3000, 20000), (1, 4000, 3), (3000, 1, 2)]:
        bk = rng.integers(-span, span, nb).astype(dtype)
        pk = rng.integers(-span, span, np_).astype(dtype)
        br = rng.permutation(nb).astype(np.uint32)
        pr = rng.permutation(np_).astype(np.uint64)
        op, ob = oracle.join(bk, br, pk, pr)
        m = pd.merge(pd.DataFrame({"k": pk, "p": pr}), pd.DataFrame({"k": bk, "b": br}),
                     on="k", how="inner")
        e = m[["p", "b"]].to_numpy(dtype=np.uint64)
        o = np.lexsort((e[:, 1], e[:, 0]))
        assert np.array_equal(op, e[o, 0]) and np.array_equal(ob, e[o, 1])
        # count identity from the key histograms of both sides
        vb, cb = np.unique(bk, return_counts=True)
        vp, cp = np.unique(pk, return_counts=True)
        common, ib, ip = np.intersect1d(vb, vp, return_indices=True)
        assert op.shape[0] == int((cb[ib].astype(np.int64) * cp[ip]).sum())


def test_join_unique_build_probed_by_permutation():
    rng = np.random.default_rng(9)
    n = 50000
    bk = rng.choice(np.iinfo(np.int64).max, n, replace=False).astype(np.int64) - (1 << 62)
    perm = rng.permutation(n)
    pk = bk[perm]
    op, ob = oracle.join(bk, None, pk, None)
    # probe row j holds build row perm[j]: exactly one pair per probe row
    assert np.array_equal(op, np.arange(n, dtype=np.uint64))
    assert np.array_equal(ob, perm.astype(np.uint64))


def test_join_all_equal_is_cross_product():
    nb, np_ = 37, 53
    bk = np.full(nb, 123456789012, dtype=np.int64)
    pk = np.full(np_, 123456789012, dtype=np.int64)
    op, ob = oracle.join(bk, None, pk, None)
    assert np.array_equal(op, np.repeat(np.arange(np_, dtype=np.uint64), nb))
    assert np.array_equal(ob, np.tile(np.arange(nb, dtype=np.uint64), np_))


def test_join_disjoint_and_empty():
    bk = np.arange(0, 1000, 2, dtype=np.int32)
    pk = np.arange(1, 1000, 2, dtype=np.int32)
    assert oracle.join(bk, None, pk, None)[0].shape[0] == 0
    assert oracle.join(bk[:0], None, pk, None)[0].shape[0] == 0
    assert oracle.join(bk, None, pk[:0], None)[0].shape[0] == 0


def test_join_key_width_matters():
    # int64 keys that agree in their low 32 bits are different keys
    bk = np.array([1, 1 + (1 << 32), -(1 << 40)], dtype=np.int64)
    pk = np.array([1 + (1 << 32), 1, 0], dtype=np.int64)
    op, ob = oracle.join(bk, None, pk, None)
    assert op.tolist() == [0, 1] and ob.tolist() == [1, 0]
