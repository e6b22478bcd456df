"""Pins of the CPU oracle against facts fixed outside it.

The paper prints no worked example, so the oracle is pinned by:
hand-derived fixtures of the ORDER BY ... LIMIT K definition (tests/golden),
exhaustive brute force over small alphabets, the IEEE 754 totalOrder ladder,
library special cases (numpy lexsort for K = N, argmax/argmin for K = 1,
numpy sort for the key multiset), closed forms of presorted and Zipf inputs,
permutation invariance, and mutation tests of the invariant checker.
"""
import itertools
import json
import os

import numpy as np
import pytest

import inputgen
import oracle
from oracle import ASC, DESC

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "order_by_limit.json")


def _bits(a):
    a = np.asarray(a)
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def _same(a_keys, a_ids, b_keys, b_ids):
    a_keys, b_keys = np.asarray(a_keys), np.asarray(b_keys)
    assert np.array_equal(_bits(a_keys), _bits(b_keys.astype(a_keys.dtype)))
    assert [int(x) for x in a_ids] == [int(x) for x in b_ids]


# ---- hand-derived fixtures ---------------------------------------------------------------

def _fixture_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _fixture_cases(), ids=lambda c: c["name"])
def test_golden_fixture(case):
    dt = np.dtype(case["dtype"])
    if "keys_hex" in case:
        keys = np.array([int(h, 16) for h in case["keys_hex"]], dtype=np.uint32).view(dt)
        exp_keys = np.array([int(h, 16) for h in case["expected_keys_hex"]], dtype=np.uint32).view(dt)
    else:
        keys = np.array(case["keys"], dtype=dt)
        exp_keys = np.array(case["expected_keys"], dtype=dt)
    rids = np.array(case["rowids"], dtype=np.uint64 if dt == np.int64 else np.uint32)
    order = DESC if case["order"] == "desc" else ASC
    ok, orr = oracle.topk(keys, rids, case["k"], order)
    _same(ok, orr, exp_keys, case["expected_rowids"])
    bk, bi = oracle.brute_topk(keys, rids, case["k"], order)
    _same(ok, orr, np.array(bk, dtype=dt), bi)


# ---- exhaustive brute force --------------------------------------------------------------

INT_ALPHABET = np.array([-(2 ** 31), -1, 0, 1, 2 ** 31 - 1], dtype=np.int32)
F32_ALPHABET = np.array([0xFFC00000, 0xFF800000, 0x80000000, 0x00000000, 0x3F800000, 0x7F800000,
                         0x7FC00000], dtype=np.uint32).view(np.float32)


def _exhaustive(alphabet, max_n):
    count = 0
    for n in range(0, max_n + 1):
        perm = np.array(list(reversed(range(n))), dtype=np.uint32)
        for combo in itertools.product(range(len(alphabet)), repeat=n):
            keys = alphabet[list(combo)] if n else alphabet[:0]
            for rids in (None, perm):
                for order in (DESC, ASC):
                    for k in range(0, n + 2):
                        ok, orr = oracle.topk(keys, rids, k, order)
                        bk, bi = oracle.brute_topk(keys, rids, k, order)
                        _same(ok, orr, np.array(bk, dtype=keys.dtype), bi)
                        count += 1
    return count


def test_exhaustive_int32_alphabet():
    assert _exhaustive(INT_ALPHABET, 4) > 1000


def test_exhaustive_float32_specials():
    assert _exhaustive(F32_ALPHABET, 3) > 1000


F64_ALPHABET = np.array([0xFFF8000000000000, 0xFFF0000000000000, 0x8000000000000000, 0x0000000000000000,
                         0x3FF0000000000000, 0x7FF0000000000000, 0x7FF8000000000000],
                        dtype=np.uint64).view(np.float64)


def test_exhaustive_float64_specials():
    assert _exhaustive(F64_ALPHABET, 3) > 1000


def test_exhaustive_int64_alphabet():
    assert _exhaustive(np.array([-(2 ** 63), -5, 0, 2 ** 63 - 1], dtype=np.int64), 4) > 1000


# ---- IEEE 754 totalOrder ladder ------------------------------------------------------------

LADDER = np.array([
    0xFFFFFFFF,  # -NaN, largest significand: lowest of all
    0xFFC00001,  # -NaN (quiet)
    0xFF800001,  # -NaN (signalling)
    0xFF800000,  # -inf
    0xFF7FFFFF,  # -max finite
    0xBF800000,  # -1
    0x80800000,  # -min normal
    0x80000001,  # -min subnormal
    0x80000000,  # -0
    0x00000000,  # +0
    0x00000001,  # +min subnormal
    0x00800000,  # +min normal
    0x3F800000,  # +1
    0x7F7FFFFF,  # +max finite
    0x7F800000,  # +inf
    0x7F800001,  # +NaN (signalling)
    0x7FC00000,  # +NaN (quiet)
    0x7FFFFFFF,  # +NaN, largest significand: highest of all
], dtype=np.uint32)


def test_total_order_ladder():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = rng.permutation(len(LADDER))
        keys = LADDER[p].view(np.float32)
        ok, orr = oracle.topk(keys, None, len(LADDER), ASC)
        assert np.array_equal(ok.view(np.uint32), LADDER)
        ok, orr = oracle.topk(keys, None, len(LADDER), DESC)
        assert np.array_equal(ok.view(np.uint32), LADDER[::-1])
        # the row-ids follow their keys
        assert np.array_equal(keys.view(np.uint32)[orr.astype(np.int64)], ok.view(np.uint32))


LADDER64 = np.array([
    0xFFFFFFFFFFFFFFFF,  # -NaN, largest significand: lowest of all
    0xFFF8000000000001,  # -NaN (quiet)
    0xFFF0000000000001,  # -NaN (signalling)
    0xFFF0000000000000,  # -inf
    0xFFEFFFFFFFFFFFFF,  # -max finite
    0xBFF0000000000000,  # -1
    0x8010000000000000,  # -min normal
    0x8000000000000001,  # -min subnormal
    0x8000000000000000,  # -0
    0x0000000000000000,  # +0
    0x0000000000000001,  # +min subnormal
    0x0010000000000000,  # +min normal
    0x3FF0000000000000,  # +1
    0x7FEFFFFFFFFFFFFF,  # +max finite
    0x7FF0000000000000,  # +inf
    0x7FF0000000000001,  # +NaN (signalling)
    0x7FF8000000000000,  # +NaN (quiet)
    0x7FFFFFFFFFFFFFFF,  # +NaN, largest significand: highest of all
], dtype=np.uint64)


def test_total_order_ladder_float64():
    rng = np.random.default_rng(2)
    for _ in range(20):
        p = rng.permutation(len(LADDER64))
        keys = LADDER64[p].view(np.float64)
        ok, orr = oracle.topk(keys, None, len(LADDER64), ASC)
        assert np.array_equal(ok.view(np.uint64), LADDER64)
        ok, orr = oracle.topk(keys, None, len(LADDER64), DESC)
        assert np.array_equal(ok.view(np.uint64), LADDER64[::-1])
        assert np.array_equal(keys.view(np.uint64)[orr.astype(np.int64)], ok.view(np.uint64))


def test_float64_finite_order_is_numeric():
    # away from zeros and NaNs, totalOrder is the numeric order: numpy's sort
    rng = np.random.default_rng(4)
    keys = rng.standard_normal(5000) * 10.0 ** rng.integers(-300, 300, 5000)
    keys[keys == 0] = 1.0
    for k in (1, 17, 5000):
        ok, _ = oracle.topk(keys, None, k, DESC)
        assert np.array_equal(ok, np.sort(keys)[::-1][:k])
        ok, _ = oracle.topk(keys, None, k, ASC)
        assert np.array_equal(ok, np.sort(keys)[:k])


# ---- library special cases ---------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 7, 1000, 1 << 16])
@pytest.mark.parametrize("dtype", ["int32", "int64", "float32", "float64"])
def test_k_equals_n_is_lexsort(n, dtype):
    rng = np.random.default_rng(n)
    if dtype in ("float32", "float64"):
        keys = (rng.integers(0, 50, n).astype(dtype) * 0.25) - 3.0
        keys = keys.astype(dtype)
        keys[keys == 0] = 0.5  # keep -0/+0 out: numpy sorts them as equal
    else:
        keys = rng.integers(-40, 40, n).astype(dtype)
    rids = rng.permutation(n).astype(np.uint32)
    ok, orr = oracle.topk(keys, rids, n, DESC)
    neg = -keys if dtype in ("float32", "float64") else ~keys
    o = np.lexsort((rids, neg))
    assert np.array_equal(_bits(ok), _bits(keys[o])) and np.array_equal(orr, rids[o])
    ok, orr = oracle.topk(keys, rids, n, ASC)
    o = np.lexsort((rids, keys))
    assert np.array_equal(_bits(ok), _bits(keys[o])) and np.array_equal(orr, rids[o])


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32", "float64"])
def test_k1_is_first_argmax(dtype):
    rng = np.random.default_rng(7)
    for _ in range(50):
        n = int(rng.integers(1, 500))
        keys = rng.integers(-5, 5, n).astype(dtype)
        ok, orr = oracle.topk(keys, None, 1, DESC)
        assert int(orr[0]) == int(np.argmax(keys))
        ok, orr = oracle.topk(keys, None, 1, ASC)
        assert int(orr[0]) == int(np.argmin(keys))


@pytest.mark.parametrize("kind", [inputgen.KIND_U_I32, inputgen.KIND_U_F32, inputgen.KIND_U_I64,
                                  inputgen.KIND_PAYLOAD_F64])
def test_key_multiset_is_numpy_sort(kind):
    keys = inputgen.generate(kind, 11, 1 << 18)
    for k in (1, 100, 5000):
        ok, _ = oracle.topk(keys, None, k, DESC)
        assert np.array_equal(ok, np.sort(keys)[::-1][:k])
        ok, _ = oracle.topk(keys, None, k, ASC)
        assert np.array_equal(ok, np.sort(keys)[:k])


def test_python_brute_force_midsize():
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 300, 4096).astype(np.int32)
    rids = rng.permutation(4096).astype(np.uint32)
    for order in (DESC, ASC):
        ok, orr = oracle.topk(keys, rids, 333, order)
        bk, bi = oracle.brute_topk(keys, rids, 333, order)
        _same(ok, orr, np.array(bk, dtype=np.int32), bi)


# ---- closed forms ----------------------------------------------------------------------------

def test_presorted_closed_form():
    n, copies = 1 << 16, 16
    g = n // copies
    keys = (np.arange(n) >> 4).astype(np.float32) * np.float32(2 ** -24)
    rids = np.arange(n, dtype=np.uint32)
    k = 1000
    ok, orr = oracle.topk(keys, rids, k, DESC)
    j = np.arange(k)
    assert np.array_equal(orr, 16 * (g - 1 - j // 16) + (j % 16))
    assert np.array_equal(ok, ((g - 1 - j // 16)).astype(np.float32) * np.float32(2 ** -24))
    ok, orr = oracle.topk(keys, rids, k, ASC)
    assert np.array_equal(orr, j)


def test_presorted_generator_closed_form():
    n = 1 << 20
    keys = inputgen.generate(inputgen.KIND_SORTED_I64, 0, n)
    ok, orr = oracle.topk(keys, None, 100, ASC, rid_dtype=np.uint64)
    assert np.array_equal(orr, np.arange(100))
    ok, orr = oracle.topk(keys, None, 100, DESC, rid_dtype=np.uint64)
    assert np.array_equal(orr, np.arange(n - 1, n - 101, -1))  # one copy per value here


def test_zipf_ascending_closed_form():
    cdf = inputgen.zipf_cdf(1.1, 10 ** 6)
    keys = inputgen.generate(inputgen.KIND_ZIPF_F32, 5, 1 << 18, cdf=cdf)
    ones = np.flatnonzero(keys == 1.0)
    for k in (10, 1000, 10000):
        assert len(ones) >= k
        ok, orr = oracle.topk(keys, np.arange(len(keys), dtype=np.uint32), k, ASC)
        assert np.all(ok == 1.0)
        assert np.array_equal(orr, ones[:k])


# ---- invariances ---------------------------------------------------------------------------

def test_permutation_invariance():
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 100, 20000).astype(np.int64)
    rids = rng.permutation(20000).astype(np.uint64)
    ref = oracle.topk(keys, rids, 777, DESC)
    for _ in range(3):
        p = rng.permutation(20000)
        got = oracle.topk(keys[p], rids[p], 777, DESC)
        _same(*ref, *got)


def test_int_desc_is_asc_of_complement():
    rng = np.random.default_rng(9)
    keys = rng.integers(-2 ** 31, 2 ** 31, 50000).astype(np.int32)
    a = oracle.topk(keys, None, 500, DESC)
    b = oracle.topk(~keys, None, 500, ASC)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], ~b[0])


def test_batched_equals_per_query():
    off, ks, orders = inputgen.batched_queries(64, n_lo_log2=4, n_hi_log2=12, k_max=300)
    keys = inputgen.generate(inputgen.KIND_U_I64, 1, int(off[-1]))
    bk, bi = oracle.topk_batched(keys, None, off, ks, orders)
    pos = 0
    for q in range(64):
        lo, hi = int(off[q]), int(off[q + 1])
        ok, orr = oracle.topk(keys[lo:hi], None, int(ks[q]), int(orders[q]))
        m = len(ok)
        _same(bk[pos:pos + m], bi[pos:pos + m], ok, orr)
        pos += m
    assert pos == len(bk)


# ---- the invariant checker catches planted mistakes -------------------------------------------

def test_invariant_checker_accepts_oracle():
    keys = inputgen.generate(inputgen.KIND_U_F32, 2, 1 << 16)
    for order in (DESC, ASC):
        ok, orr = oracle.topk(keys, None, 300, order)
        oracle.check_invariants(keys, None, 300, order, ok, orr)


@pytest.mark.parametrize("mutation", ["drop", "swap", "replace_key", "replace_id", "tie_id", "dup"])
def test_invariant_checker_rejects_mutations(mutation):
    n = 1 << 14
    keys = (np.arange(n) % 997).astype(np.int32)  # ties of ~16 copies
    rids = np.arange(n, dtype=np.uint32)
    ok, orr = oracle.topk(keys, rids, 100, DESC)
    ok, orr = ok.copy(), orr.copy()
    if mutation == "drop":
        ok, orr = ok[:-1], orr[:-1]
    elif mutation == "swap":
        ok[[3, 40]] = ok[[40, 3]]
        orr[[3, 40]] = orr[[40, 3]]
    elif mutation == "replace_key":
        ok[50] = ok[50] - 1
    elif mutation == "replace_id":
        orr[50] = (orr[50] + 1) % n
    elif mutation == "tie_id":
        # the last output replaced by a tied key with a larger row-id
        same = np.flatnonzero(keys == ok[-1])
        orr[-1] = same[-1]
    elif mutation == "dup":
        ok[-1], orr[-1] = ok[-2], orr[-2]
    with pytest.raises(AssertionError):
        oracle.check_invariants(keys, rids, 100, DESC, ok, orr)
