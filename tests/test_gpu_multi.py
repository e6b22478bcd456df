"""Parity of the batched form (tk_plan_*, multi-query launches) with the CPU
oracle: every query of a plan equals the oracle on that query alone, across
eager launches and hipGraph replays, and equals tk_topk on the same query."""
import numpy as np
import pytest

import inputgen
import oracle
from tests.gpu_util import assert_same, say, to_dev, to_np

pytestmark = pytest.mark.gpu

import paper_2601_19911_amd as tk
from paper_2601_19911_amd.batched import Plan


def _check(keys, rids, off, ks, orders, ok, orr, plan, what):
    for q in range(len(ks)):
        lo, hi = int(off[q]), int(off[q + 1])
        a, b = int(plan.out_offsets[q]), int(plan.out_offsets[q + 1])
        ek, er = oracle.topk(keys[lo:hi], None if rids is None else rids[lo:hi], int(ks[q]),
                             int(orders[q]), rid_dtype=orr.dtype)
        assert_same(ok[a:b], orr[a:b], ek, er, what=f"{what} query {q} n={hi - lo} k={ks[q]}")


def _plan_run(kind, q, n_lo, n_hi, k_max, seed, rid=np.uint32, with_rids=False, graph=True,
              launches=1, **params):
    import torch
    off, ks, orders = inputgen.batched_queries(q, seed=seed, n_lo_log2=n_lo, n_hi_log2=n_hi,
                                               k_max=k_max)
    zipf = kind in (inputgen.KIND_ZIPF_I64, inputgen.KIND_ZIPF_F32, inputgen.KIND_ZIPF_I32)
    keys = inputgen.generate(kind, seed, int(off[-1]),
                             cdf=inputgen.zipf_cdf(1.1, 10 ** 6) if zipf else None)
    rids = (np.random.default_rng(seed).permutation(int(off[-1])).astype(rid)
            if with_rids else None)
    tdt = torch.uint32 if rid == np.uint32 else torch.uint64
    stream = torch.cuda.Stream() if graph else None
    plan = Plan(off, ks, orders, key_dtype=torch.from_numpy(keys[:1]).dtype, rid_dtype=tdt,
                stream=stream, use_graph=graph, **params)
    say(f"multi q={q} n=2^{n_lo}..2^{n_hi} k<={k_max} total={int(off[-1])} {keys.dtype} "
        f"rids={'given' if with_rids else 'index'} graph={graph} plan={plan.info()}")
    kd = to_dev(keys)
    rd = None if rids is None else to_dev(rids)
    ok, orr = plan.alloc_outputs()
    torch.cuda.synchronize()
    for it in range(launches):
        ok.fill_(0)
        orr.fill_(0)
        torch.cuda.synchronize()
        say(f"launch {it}")
        plan.launch(kd, ok, orr, rowids=rd, stream=stream)
        torch.cuda.synchronize()
        st = plan.stats()
        say(f"launch {it} done, stats {st}")
        assert st["unfinished"] == 0
        _ = torch.ones(8, device="cuda").sum().item()  # eager work between replays
        _check(keys, rids, off, ks, orders, to_np(ok), to_np(orr), plan, f"launch {it}")
    return plan, keys, off, ks, orders, kd, ok, orr


def test_multi_int64_mixed_sizes_eager_then_graph_replays():
    _plan_run(inputgen.KIND_U_I64, 160, 9, 21, 4096, seed=41, launches=4)


def test_multi_float32_given_rowids():
    _plan_run(inputgen.KIND_U_F32, 96, 8, 21, 3000, seed=43, with_rids=True, launches=2)


def test_multi_int32_u64_index_rowids_large_k_no_graph():
    _plan_run(inputgen.KIND_U_I32, 80, 6, 20, 9000, seed=45, rid=np.uint64, graph=False, launches=2)


def test_multi_zipf_int64_ties():
    _plan_run(inputgen.KIND_ZIPF_I64, 24, 14, 20, 4096, seed=47)


def test_multi_ties_and_empty_queries():
    import torch
    off = np.array([0, 0, 5, 5 + 40000, 5 + 40000 + 300000, 5 + 40000 + 300000 + 3,
                    5 + 40000 + 300000 + 3 + 70001], dtype=np.uint64)
    ks = np.array([10, 3, 500, 2000, 7, 777], dtype=np.uint32)
    orders = np.array([0, 1, 0, 1, 0, 1], dtype=np.uint8)
    keys = (np.arange(int(off[-1])) % 11).astype(np.int64)
    plan = Plan(off, ks, orders, key_dtype=torch.int64, rid_dtype=torch.uint32)
    say(f"ties plan {plan.info()}")
    ok, orr = plan.alloc_outputs()
    plan.launch(to_dev(keys), ok, orr)
    torch.cuda.synchronize()
    assert plan.stats()["unfinished"] == 0
    _check(keys, None, off, ks, orders, to_np(ok), to_np(orr), plan, "ties")


def test_multi_matches_single_query_calls():
    import torch
    plan, keys, off, ks, orders, kd, ok, orr = _plan_run(inputgen.KIND_U_F32, 40, 10, 21, 2048,
                                                         seed=49, launches=1)
    okn, orn = to_np(ok), to_np(orr)
    for q in range(0, 40, 3):
        lo, hi = int(off[q]), int(off[q + 1])
        sk, sr = tk.topk(kd[lo:hi], int(ks[q]), order=int(orders[q]))
        torch.cuda.synchronize()
        a, b = int(plan.out_offsets[q]), int(plan.out_offsets[q + 1])
        assert_same(okn[a:b], orn[a:b], to_np(sk), to_np(sr), what=f"alone q={q}")


def test_multi_plan_argument_errors():
    import torch
    off = np.array([0, 10, 20], dtype=np.uint64)
    ks = np.array([1, 2], dtype=np.uint32)
    orders = np.array([0, 1], dtype=np.uint8)
    with pytest.raises(tk.TopKError):
        Plan(off, ks, orders, key_dtype=torch.int64, rid_dtype=torch.uint32, tile_keys=100)


def test_multi_float64_given_rowids():
    _plan_run(inputgen.KIND_U_F64, 64, 8, 21, 5000, seed=49, with_rids=True, launches=2)


def test_multi_query_times_from_the_device_clock():
    """tk_plan_query_times: every non-empty query has a completion time after
    the launch's start and no later than the launch's end (events around it),
    on an eager launch and on graph replays; empty queries report 0."""
    import torch
    off, ks, orders = inputgen.batched_queries(200, seed=51, n_lo_log2=8, n_hi_log2=21, k_max=4096)
    ks[7] = 0  # an empty query
    keys = inputgen.generate(inputgen.KIND_U_I64, 51, int(off[-1]))
    kd = to_dev(keys)
    s = torch.cuda.Stream()
    plan = Plan(off, ks, orders, key_dtype=torch.int64, rid_dtype=torch.uint32, stream=s)
    ok, orr = plan.alloc_outputs()
    for it in range(3):  # eager, capture, replay
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        plan.launch(kd, ok, orr, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        span = e0.elapsed_time(e1) * 1e-3
        t = plan.query_times()
        say(f"launch {it}: span {span * 1e3:.3f} ms, query times {t.min() * 1e3:.3f}.."
            f"{t.max() * 1e3:.3f} ms, p50 {np.median(t) * 1e3:.3f} ms")
        assert t[7] == 0.0
        live = np.delete(t, 7)
        assert np.all(live > 0)
        # the device clock ticks at 100 MHz: allow a few ticks and the event granularity
        assert np.all(live <= span + 5e-5)
        _check(keys, None, off, ks, orders, to_np(ok), to_np(orr), plan, f"timed launch {it}")
    plan.close()


def test_topk_each_matches_the_plan():
    """The C per-query launcher (tk_topk_each) on 1 and 3 streams writes the same
    packed results as the plan, and reports increasing completion times."""
    import torch
    from paper_2601_19911_amd.batched import topk_each
    off, ks, orders = inputgen.batched_queries(64, seed=53, n_lo_log2=8, n_hi_log2=20, k_max=3000)
    keys = inputgen.generate(inputgen.KIND_U_F32, 53, int(off[-1]))
    kd = to_dev(keys)
    plan = Plan(off, ks, orders, key_dtype=torch.float32, rid_dtype=torch.uint32)
    pk, pr = plan.alloc_outputs()
    plan.launch(kd, pk, pr)
    torch.cuda.synchronize()
    for ns in (1, 3):
        ok, orr = plan.alloc_outputs()
        streams = [torch.cuda.Stream() for _ in range(ns)]
        t = topk_each(off, ks, orders, kd, ok, orr, streams)
        torch.cuda.synchronize()
        say(f"topk_each {ns} streams: completion {t.min() * 1e3:.3f}..{t.max() * 1e3:.3f} ms")
        assert np.all(t > 0)
        if ns == 1:
            assert np.all(np.diff(t) >= 0)
        assert_same(to_np(ok), to_np(orr), to_np(pk), to_np(pr), what=f"topk_each {ns} streams")
    plan.close()
