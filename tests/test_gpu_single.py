"""Parity of the single-query HIP path (tk_topk) with the CPU oracle.

Every case runs the library through its C ABI on the GPU and compares keys
and row-ids bit for bit with the oracle on the same seeded input, at sizes
that span several tiles, ragged tails, all three key types, both row-id
widths, implicit row-ids, both orders, every execution path (one workgroup,
sample+filter+LDS tail, exact select on survivors, forced fallback, exact
select over the input) and the tie-heavy and special-value inputs.
"""
import numpy as np
import pytest

import inputgen
import oracle
from tests.gpu_util import assert_same, order_code, say, to_dev, to_np

pytestmark = pytest.mark.gpu

import paper_2601_19911_amd as tk

KINDS = {"int32": inputgen.KIND_U_I32, "float32": inputgen.KIND_U_F32, "int64": inputgen.KIND_U_I64,
         "float64": inputgen.KIND_U_F64}


def run(keys, rids, k, order, rid_dtype=np.uint32, workspace=None, offset=0):
    import torch
    say(f"case n={len(keys)} dtype={keys.dtype} k={k} order={order} "
        f"rids={'none' if rids is None else rids.dtype} offset={offset}")
    kd = to_dev(keys)
    if offset:
        base = to_dev(np.concatenate([np.zeros(offset, dtype=keys.dtype), keys]))
        kd = base[offset:]
    rd = None if rids is None else to_dev(rids)
    tdt = torch.uint32 if np.dtype(rid_dtype) == np.uint32 else torch.uint64
    ok, orr = tk.topk(kd, k, rowids=rd, order=order, rid_dtype=tdt, workspace=workspace)
    torch.cuda.synchronize()
    got = (to_np(ok), to_np(orr))
    exp = oracle.topk(keys, rids, k, order_code(order), rid_dtype=rid_dtype)
    assert_same(got[0], got[1], exp[0], exp[1], what=f"n={len(keys)} k={k} {order}")
    return got


def test_config_c1_uniform_int32():
    """N = 2^20 int32 uniform in [0, 2^31), row-ids 0..N-1, K = 100."""
    n = 1 << 20
    keys = inputgen.generate(inputgen.KIND_U_I32, inputgen.config_seed(1), n)
    rids = np.arange(n, dtype=np.uint32)
    for order in ("desc", "asc"):
        run(keys, rids, 100, order)


@pytest.mark.parametrize("dtype", ["int32", "float32", "int64"])
@pytest.mark.parametrize("n", [1, 777, 16384, 16385, 100_003, (1 << 18) + 1, (1 << 20) + 7])
@pytest.mark.parametrize("k", [1, 100, 1000, 5000])
def test_sweep(dtype, n, k):
    keys = inputgen.generate(KINDS[dtype], 1000 + n, n)
    rids = np.random.default_rng(n).permutation(n).astype(np.uint32)
    run(keys, rids, k, "desc")
    run(keys, None, k, "asc")


@pytest.mark.parametrize("dtype", ["int32", "float32", "int64"])
def test_u64_rowids(dtype):
    n = (1 << 20) + 3
    keys = inputgen.generate(KINDS[dtype], 5, n)
    rids = (np.random.default_rng(1).permutation(n).astype(np.uint64) << np.uint64(20)) + np.uint64(7)
    for order in ("desc", "asc"):
        run(keys, rids, 1000, order, rid_dtype=np.uint64)
    run(keys, None, 1000, "desc", rid_dtype=np.uint64)


def test_all_equal_keys():
    n = 1 << 20
    keys = np.full(n, 5, dtype=np.int32)
    rids = np.random.default_rng(2).permutation(n).astype(np.uint32)
    for k in (1, 1000, 20000):
        for order in ("desc", "asc"):
            run(keys, rids, k, order)


def test_presorted_closed_form():
    n = 1 << 20
    keys = (np.arange(n) >> 4).astype(np.float32) * np.float32(2 ** -24)
    rids = np.arange(n, dtype=np.uint32)
    got = run(keys, rids, 1000, "desc")
    j = np.arange(1000)
    g = n // 16
    assert np.array_equal(got[1], 16 * (g - 1 - j // 16) + (j % 16))
    got = run(keys, rids, 1000, "asc")
    assert np.array_equal(got[1], j)


@pytest.mark.parametrize("k", [10, 1000, 10000])
def test_zipf_both_orders(k):
    cdf = inputgen.zipf_cdf(1.1, 10 ** 6)
    n = 1 << 21
    keys = inputgen.generate(inputgen.KIND_ZIPF_F32, 8, n, cdf=cdf)
    rids = np.arange(n, dtype=np.uint32)
    run(keys, rids, k, "desc")
    got = run(keys, rids, k, "asc")
    assert np.array_equal(got[1], np.flatnonzero(keys == 1.0)[:k])


def test_float_special_values():
    specials = np.array([0xFFFFFFFF, 0xFFC00001, 0xFF800001, 0xFF800000, 0xFF7FFFFF, 0xBF800000,
                         0x80000001, 0x80000000, 0x00000000, 0x00000001, 0x3F800000, 0x7F7FFFFF,
                         0x7F800000, 0x7F800001, 0x7FC00000, 0x7FFFFFFF], dtype=np.uint32)
    rng = np.random.default_rng(4)
    for n in (5000, 1 << 19):
        keys = specials[rng.integers(0, len(specials), n)].view(np.float32)
        rids = rng.permutation(n).astype(np.uint32)
        for k in (1, 17, 3000):
            run(keys, rids, k, "desc")
            run(keys, rids, k, "asc")


def test_k_at_least_n():
    for n in (1000, 50_000):
        keys = inputgen.generate(inputgen.KIND_U_F32, 3, n)
        run(keys, None, n, "desc")
        run(keys, None, n + 5, "asc")


def test_large_k_paths():
    # survivors beyond one workgroup's LDS, and K beyond one LDS tile
    n = 1 << 22
    keys = inputgen.generate(inputgen.KIND_U_I32, 9, n)
    rids = np.arange(n, dtype=np.uint32)
    run(keys, rids, 20000, "desc")
    run(keys, rids, 100_000, "asc")
    keys64 = inputgen.generate(inputgen.KIND_U_I64, 9, n)
    run(keys64, None, 100_000, "desc", rid_dtype=np.uint64)


def test_unaligned_keys():
    n = (1 << 20) + 1
    keys = inputgen.generate(inputgen.KIND_U_F32, 12, n)
    run(keys, None, 1000, "desc", offset=1)
    keys64 = inputgen.generate(inputgen.KIND_U_I64, 12, n)
    run(keys64, None, 1000, "asc", offset=1, rid_dtype=np.uint64)


def test_paths_are_taken_and_exact():
    import torch
    n = 1 << 20
    keys = inputgen.generate(inputgen.KIND_U_F32, 21, n)
    kd = to_dev(keys)
    exp = oracle.topk(keys, None, 1000, oracle.DESC)

    def go(expect_path):
        ws = tk.new_workspace(n, 1000, tk.TK_KEY_F32, tk.TK_RID_U32)
        ok, orr = tk.topk(kd, 1000, workspace=ws)
        torch.cuda.synchronize()
        info = tk.query_info(ws)
        say(f"path {info}")
        assert info["status"] == 0
        assert info["path"] == expect_path
        assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"path {expect_path}")

    go(3)                                # survivors ranked across workgroups
    try:
        tk.set_tuning(tail_mode=2)       # one workgroup selects and sorts the survivors
        go(2)
        tk.set_tuning(tail_mode=1, force_cap=64)  # survivors overflow: exact select over the input
        go(4)
        tk.set_tuning(force_cap=-1, force_exact=1)
        go(5)
    finally:
        tk.set_tuning(force_cap=-1, force_exact=2, tail_mode=1)
    go(3)


def test_garbage_workspace_is_still_exact():
    """A workspace that was never zeroed: the first query may take the exact
    path, every result is exact, and the second query is back on the fast path."""
    import torch
    n = 1 << 20
    keys = inputgen.generate(inputgen.KIND_U_I32, 31, n)
    exp = oracle.topk(keys, None, 500, oracle.DESC)
    kd = to_dev(keys)
    ws = torch.full((tk.workspace_size(n, 500, tk.TK_KEY_I32, tk.TK_RID_U32),), 0xA5,
                    dtype=torch.uint8, device="cuda")
    for i in range(2):
        ok, orr = tk.topk(kd, 500, workspace=ws)
        torch.cuda.synchronize()
        assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"garbage workspace call {i}")
        info = tk.query_info(ws)
        say(f"call {i}: {info}")
        if i == 1:
            assert info["path"] == 3


def test_workspace_reuse_across_queries():
    import torch
    ws = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(5)
    for i in range(6):
        n = int(rng.integers(1 << 18, 1 << 21))
        keys = inputgen.generate(inputgen.KIND_U_I64, 50 + i, n)
        run(keys, None, int(rng.integers(1, 3000)), "desc" if i % 2 else "asc",
            rid_dtype=np.uint64, workspace=ws)


def test_repeatable():
    import torch
    n = 1 << 21
    keys = inputgen.generate(inputgen.KIND_U_F32, 77, n)
    a = run(keys, None, 777, "desc")
    for _ in range(3):
        b = run(keys, None, 777, "desc")
        assert np.array_equal(a[1], b[1])


def test_gather_rows_device_matches_take():
    import torch
    rng = np.random.default_rng(9)
    pay = rng.random((8, 70000))
    r = rng.integers(0, 70000, 1000).astype(np.uint32)
    dp = torch.from_numpy(pay).cuda()
    dr = to_dev(r)
    out = torch.empty((8, 1000), dtype=torch.float64, device="cuda")
    tk.gather_rows_device(dp, dr, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), pay[:, r].view(np.uint64))


def test_bucketed_tail_path():
    """K above the ranked tail's reach takes the bucketed tail (path 6); the
    one-workgroup tail (tail_mode=2) gives the same exact result."""
    import torch
    n = 1 << 22
    for dtype, k, order in (("float32", 5000, "desc"), ("int64", 30000, "asc"), ("int32", 2049, "desc")):
        keys = inputgen.generate(KINDS[dtype], 41, n)
        kd = to_dev(keys)
        rdt = np.uint64 if dtype == "int64" else np.uint32
        exp = oracle.topk(keys, None, k, order_code(order), rid_dtype=rdt)
        for mode, expect in ((1, 6), (2, 2)):
            try:
                tk.set_tuning(tail_mode=mode)
                ws = tk.new_workspace(n, k, tk.key_code(keys.dtype),
                                      tk.TK_RID_U64 if rdt == np.uint64 else tk.TK_RID_U32)
                ok, orr = tk.topk(kd, k, order=order, workspace=ws,
                                  rid_dtype=torch.uint64 if rdt == np.uint64 else torch.uint32)
                torch.cuda.synchronize()
                info = tk.query_info(ws)
                say(f"{dtype} k={k} {order} tail_mode={mode}: {info}")
                assert info["status"] == 0 and info["path"] == expect
                assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"{dtype} k={k} mode={mode}")
            finally:
                tk.set_tuning(tail_mode=1)


def test_repeated_rowids_identical_pairs():
    """Row-ids may repeat: groups of four identical (key, row-id) pairs, so the
    tails must order equal composites without dropping or doubling one
    (ranked tail K <= 2048, bucketed tail, one-workgroup tail)."""
    import torch
    n = 1 << 21
    i = np.arange(n, dtype=np.int64)
    rids = (i // 4).astype(np.uint32)
    keys = ((i // 4) * 2654435761 % 50021).astype(np.int32)  # many equal keys, in groups of 4
    kd, rd = to_dev(keys), to_dev(rids)
    for k, mode in ((777, 1), (6000, 1), (777, 2)):
        for order in ("desc", "asc"):
            try:
                tk.set_tuning(tail_mode=mode)
                ws = tk.new_workspace(n, k, tk.TK_KEY_I32, tk.TK_RID_U32)
                ok, orr = tk.topk(kd, k, rowids=rd, order=order, workspace=ws)
                torch.cuda.synchronize()
                info = tk.query_info(ws)
                say(f"k={k} mode={mode} {order}: {info}")
                assert info["status"] == 0
                exp = oracle.topk(keys, rids, k, order_code(order))
                assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"k={k} mode={mode} {order}")
            finally:
                tk.set_tuning(tail_mode=1)


def test_small_query_paths():
    """Queries within one LDS tile are ranked across workgroups over the input
    (path 7); tail_mode=2 keeps them in one workgroup; both equal the oracle,
    including ties and the smallest sizes."""
    import torch
    rng = np.random.default_rng(77)
    cases = [("float32", 5000, 1000, "desc"), ("int32", 16384, 2048, "asc"), ("int64", 8192, 300, "desc"),
             ("float32", 3, 2, "asc"), ("int32", 1000, 1000, "desc"), ("int64", 100, 1, "asc"),
             # K past the ranked form's reach: one workgroup in either mode
             ("int32", 8192, 10000, "desc"), ("float32", 16384, 2049, "asc"), ("int64", 8192, 5000, "desc")]
    for dtype, n, k, order in cases:
        keys = inputgen.generate(KINDS[dtype], 90 + n, n)
        if dtype == "int32":
            keys = (keys % 97).astype(np.int32)  # heavy ties
        kd = to_dev(keys)
        rdt = np.uint64 if dtype == "int64" else np.uint32
        rids = rng.permutation(n).astype(rdt)
        exp = oracle.topk(keys, rids, k, order_code(order))
        for mode in (1, 2):
            try:
                tk.set_tuning(tail_mode=mode)
                ws = tk.new_workspace(n, k, tk.key_code(keys.dtype), tk.rid_code(np.dtype(rdt)))
                ok, orr = tk.topk(kd, k, rowids=to_dev(rids), order=order, workspace=ws)
                torch.cuda.synchronize()
                info = tk.query_info(ws)
                say(f"{dtype} n={n} k={k} {order} tail_mode={mode}: {info}")
                if mode == 1 and min(k, n) <= 2048:
                    assert info["path"] == 7
                assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"{dtype} n={n} k={k} mode={mode}")
            finally:
                tk.set_tuning(tail_mode=1)


def _run_path_cases(cases, want_path, seed):
    import torch
    rng = np.random.default_rng(seed)
    for dtype, n, k, order in cases:
        keys = inputgen.generate(KINDS[dtype], seed + n, n)
        if dtype == "int32" and order == "desc":
            keys = (keys % 1009).astype(np.int32)  # ties across the boundary
        rdt = np.uint64 if dtype == "int64" else np.uint32
        rids = rng.permutation(n).astype(rdt)
        exp = oracle.topk(keys, rids, k, order_code(order))
        ws = tk.new_workspace(n, k, tk.key_code(keys.dtype), tk.rid_code(np.dtype(rdt)))
        ok, orr = tk.topk(to_dev(keys), k, rowids=to_dev(rids), order=order, workspace=ws)
        torch.cuda.synchronize()
        info = tk.query_info(ws)
        say(f"{dtype} n={n} k={k} {order}: {info}")
        assert info["path"] == want_path and info["status"] == 0
        assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"{dtype} n={n} k={k} {order}")


_NO_SAMPLE_LARGE = [("int32", 65536, 40000, "desc"), ("float32", 1 << 22, 1 << 19, "desc"),
                    ("int64", 1 << 21, 1 << 20, "asc"), ("float64", 100_003, 60_000, "desc"),
                    ("int32", (1 << 20) + 4097, 600_000, "asc")]


def test_no_sample_paths():
    """Inputs past one LDS tile that the sample cannot serve (N below 16 sample
    chunks of 2048 keys, K above N / 2, or K above N / 16 at N past 2^20): from
    2^16 keys the full radix sort keeping its first K pairs (path 9), below it
    one workgroup's select over the input (path 8)."""
    _run_path_cases(_NO_SAMPLE_LARGE, 9, seed=300)
    _run_path_cases([("int32", 23170, 10, "desc"), ("float32", 30048, 1000, "asc"),
                     ("int64", 20000, 3000, "asc"), ("int64", 16385, 10, "desc"),
                     ("float32", 65535, 40000, "asc"), ("int32", 40000, 20001, "desc")], 8, seed=301)


def test_exact_select_grid():
    """The same queries by the exact radix select over the input on a grid
    sized by N (path 5, taken here with force_exact; the sort route's queries
    take it when their workspace has no room for the sort's scratch)."""
    try:
        tk.set_tuning(force_exact=1)
        _run_path_cases(_NO_SAMPLE_LARGE, 5, seed=300)
    finally:
        tk.set_tuning(force_exact=2)


def test_least_workspace_takes_the_grid_select():
    """With tk_workspace_min_size bytes (no room for the sort's scratch) a query
    without a usable sample takes path 5, with the full size path 9; both
    equal the oracle."""
    import torch
    rng = np.random.default_rng(310)
    for dtype, n, k, order in [("float32", 1 << 20, 600_000, "asc"), ("int64", 100_000, 70_000, "desc")]:
        keys = inputgen.generate(KINDS[dtype], 310 + n, n)
        rdt = np.uint64 if dtype == "int64" else np.uint32
        rids = rng.permutation(n).astype(rdt)
        exp = oracle.topk(keys, rids, k, order_code(order))
        kc, rc = tk.key_code(keys.dtype), tk.rid_code(np.dtype(rdt))
        assert tk.workspace_min_size(n, k, kc, rc) < tk.workspace_size(n, k, kc, rc)
        for least, want in ((True, 5), (False, 9)):
            ws = tk.new_workspace(n, k, kc, rc, least=least)
            ok, orr = tk.topk(to_dev(keys), k, rowids=to_dev(rids), order=order, workspace=ws)
            torch.cuda.synchronize()
            info = tk.query_info(ws)
            say(f"{dtype} n={n} k={k} {order} least={least}: {info}")
            assert info["path"] == want and info["status"] == 0
            assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"{dtype} n={n} least={least}")
        with pytest.raises(tk.TopKError):
            small = torch.zeros(tk.workspace_min_size(n, k, kc, rc) - 256, dtype=torch.uint8, device="cuda")
            tk.topk(to_dev(keys), k, rowids=to_dev(rids), order=order, workspace=small)


def test_wide_k_sampled():
    """K between N / 16 and N / 2 at N up to 2^20: the sampled path with the
    bucketed tail (path 6), equal to the oracle."""
    _run_path_cases([("int32", 65536, 10000, "desc"), ("float32", 131072, 10000, "asc"),
                     ("int64", 100000, 7000, "desc"), ("float32", 1 << 20, 1 << 17, "desc"),
                     ("int64", 1 << 20, 1 << 19, "asc")], 6, seed=400)


def _f64_keys(n, seed):
    """float64 keys of mixed sign and magnitude with IEEE specials and ties:
    +-0, +-inf, NaNs of both signs, subnormals and repeated values."""
    rng = np.random.default_rng(seed)
    keys = rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, n)
    specials = np.array([0x0000000000000000, 0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
                         0x7FF8000000000000, 0xFFF8000000000001, 0x0000000000000001, 0x800000000000000F],
                        dtype=np.uint64).view(np.float64)
    m = max(n // 50, 1)
    keys[rng.integers(0, n, m)] = specials[rng.integers(0, len(specials), m)]
    keys[rng.integers(0, n, m)] = keys[rng.integers(0, n, m)]  # repeats
    return keys


@pytest.mark.parametrize("n,k", [(1, 1), (3000, 1000), (16384, 5000), (23170, 300), (1 << 20, 100),
                                 (1 << 20, 10000), (1 << 20, 300000)])
def test_float64_keys(n, k):
    """float64 keys (the paper's key type) through every route: ranked and
    one-workgroup small paths, the exact select, the sampled ranked and
    bucketed tails; totalOrder on the specials; both orders, row-ids given and
    implicit (u64 and u32)."""
    import torch
    keys = _f64_keys(n, seed=n + k)
    kd = to_dev(keys)
    rng = np.random.default_rng(k)
    for order in ("desc", "asc"):
        for rdt in (None, np.uint64, np.uint32):
            rids = None if rdt is None else rng.permutation(n).astype(rdt)
            exp = oracle.topk(keys, rids, k, order_code(order),
                              rid_dtype=np.uint32 if rdt is None else rdt)
            rc = tk.TK_RID_U32 if rdt in (None, np.uint32) else tk.TK_RID_U64
            ws = tk.new_workspace(n, k, tk.TK_KEY_F64, rc)
            ok, orr = tk.topk(kd, k, rowids=None if rids is None else to_dev(rids), order=order,
                              workspace=ws, rid_dtype=torch.uint32 if rdt is None else None)
            torch.cuda.synchronize()
            info = tk.query_info(ws)
            say(f"float64 n={n} k={k} {order} rids={rdt}: {info}")
            assert info["status"] == 0
            assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"float64 n={n} k={k} {order} {rdt}")


def test_read_probe():
    """The read-ceiling probe writes nothing but its zero count and rejects bad
    arguments before launching."""
    import torch
    buf = torch.full((1 << 20,), -1, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    tk.read_probe(buf, 3, sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == 0 and bool((buf == -1).all().item())
    L = tk.lib()
    assert L.tk_read_probe(buf.data_ptr() + 4, 1 << 20, 3, sink.data_ptr(), None) == -1  # TK_EINVAL
    assert L.tk_read_probe(buf.data_ptr(), 1 << 20, 0, sink.data_ptr(), None) == -1  # TK_EINVAL
    assert L.tk_read_probe(buf.data_ptr(), 1 << 20, 3, None, None) == -1  # TK_EINVAL


# ---- the sampled threshold, checked from the outside -------------------------------------------

def _plan_sample(n, k, sigma=4.0):
    """(S, r1) of the sampled path at the default tuning: the largest sample of
    2^11..2^20 keys (at least 16 keys per sampled key) whose rank r1 =
    ceil(m + sigma sqrt(m) + 3), m = K S / N, sigma = 4, keeps r1 x S / 2048
    candidates within 2048 for the final select."""
    import math
    for lg in range(20, 10, -1):
        s = 1 << lg
        if s * 16 > n:
            continue
        m = float(k) * float(s) / float(n)
        r1 = math.ceil(m + sigma * math.sqrt(m) + 3.0)
        if r1 <= 2048 and r1 * (s // 2048) <= 2048:
            return s, r1
    return None


def _sample_positions(n, s):
    """Chunk c of 16 consecutive keys starts at c x stride plus the high word of
    (SplitMix64 finalizer of c + 1 times its increment) x (stride - 15)."""
    m64 = (1 << 64) - 1
    nch = s // 16
    stride = n // nch
    span = stride - 15
    pos = np.empty(s, dtype=np.int64)
    for c in range(nch):
        z = ((c + 1) * 0x9E3779B97F4A7C15) & m64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m64
        z ^= z >> 31
        pos[16 * c:16 * c + 16] = c * stride + ((z * span) >> 64) + np.arange(16)
    return pos


def _images(keys, order):
    """Order-preserving unsigned images (totalOrder for floats), flipped for ascending."""
    if keys.dtype in (np.float32, np.float64):
        bits = 8 * keys.dtype.itemsize
        ut = np.uint32 if bits == 32 else np.uint64
        b = keys.view(ut)
        sign = ut(1) << ut(bits - 1)
        img = np.where(b & sign, ~b, b | sign).astype(np.uint64)
    else:
        bits = 8 * keys.dtype.itemsize
        ut = np.uint32 if bits == 32 else np.uint64
        img = (keys.view(ut) ^ (ut(1) << ut(bits - 1))).astype(np.uint64)
    if order == "asc":
        img = ~img & np.uint64((1 << bits) - 1 if bits < 64 else (1 << 64) - 1)
    return img


@pytest.mark.parametrize("dtype,n,k,order,explicit", [
    ("float32", (1 << 24) + 12345, 100, "desc", False),   # r1 = 10: the tournament
    ("float32", (1 << 24) + 12345, 5000, "asc", True),    # r1 = 41: the radix select
    ("int64", (1 << 22) + 7, 10, "desc", False),          # r1 = 7, 16-byte composites
    ("float64", 1 << 22, 1000, "asc", False),             # r1 = 35
    ("int32", 1 << 22, 1, "desc", True),                  # r1 = 5, heavy ties
])
def test_sampled_threshold_is_the_samples_rank(dtype, n, k, order, explicit):
    """The threshold is the r1-th best composite of the stratified sample and the
    survivor count is the number of input composites at or above it: both
    recomputed on the host from the sample's definition."""
    import torch
    kind = {"float32": inputgen.KIND_U_F32, "int64": inputgen.KIND_U_I64,
            "float64": inputgen.KIND_U_F64, "int32": inputgen.KIND_U_I32}[dtype]
    keys = inputgen.generate(kind, 900 + k, n)
    if dtype == "int32":
        keys = (keys % 1009).astype(np.int32)
    rdt = np.uint64 if dtype in ("int64", "float64") else np.uint32
    rb = 8 * np.dtype(rdt).itemsize
    rids = np.random.default_rng(k).permutation(n).astype(rdt) if explicit else np.arange(n, dtype=rdt)
    s, r1 = _plan_sample(n, k)
    img = _images(keys, order)
    flip = ~rids
    pos = _sample_positions(n, s)
    comp = sorted(((int(img[p]) << rb) | int(flip[p]) for p in pos), reverse=True)
    t = comp[r1 - 1]
    tk_, tf_ = t >> rb, t & ((1 << rb) - 1)
    surv = int(np.count_nonzero(img > np.uint64(tk_)) +
               np.count_nonzero((img == np.uint64(tk_)) & (flip.astype(np.uint64) >= np.uint64(tf_))))
    ws = tk.new_workspace(n, k, tk.key_code(keys.dtype), tk.rid_code(np.dtype(rdt)))
    ok, orr = tk.topk(to_dev(keys), k, rowids=to_dev(rids) if explicit else None, order=order,
                      rid_dtype=torch.uint64 if rdt == np.uint64 else torch.uint32, workspace=ws)
    torch.cuda.synchronize()
    info = tk.query_info(ws)
    say(f"{dtype} n={n} k={k} {order}: S={s} r1={r1} threshold {tk_:#x} survivors {surv}: {info}")
    assert info["status"] == 0 and info["path"] in (3, 6)
    assert info["threshold_key"] == tk_
    assert info["survivors"] == surv
    exp = oracle.topk(keys, rids if explicit else None, k, order_code(order), rid_dtype=rdt)
    assert_same(to_np(ok), to_np(orr), exp[0], exp[1], what=f"{dtype} n={n} k={k}")
