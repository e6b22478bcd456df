"""Parity at the full size of the batched, late-materialization and served
workloads.

* Batched: 4096 queries with N log-uniform in [2^10, 2^24] (6.8e9 int64 keys,
  54 GB in one device buffer), K log-uniform in [1, 4096] capped at N, half
  ascending, row-id = index within the query.  Every query's result from the
  batched plan equals the same query run alone through tk_topk and equals the
  oracle (all 4096).
* Key-only transfer + late materialization: 2^26 rows in pinned host memory,
  an int64 Zipf(1.05) key column and 8 float64 payload columns; key + row-id
  go to the device, the Top-1000 comes back and the payload rows are gathered
  on the host (and, for the full-row variant, on the device).  Keys and row-ids
  equal the oracle, the gathered rows equal numpy.take.
* Served: the serving request mixture over device-resident columns of 2^28
  rows, through continuous batching and the cost gate; every request equals
  the oracle.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import inputgen
import oracle
import paper_2601_19911_amd as tk
from inputgen import native as gen
from tests.gpu_util import assert_same, say, to_np

pytestmark = pytest.mark.gpu


def test_batched_4096_queries_full_size():
    import torch
    from paper_2601_19911_amd.batched import Plan
    dev = torch.device("cuda:0")
    off, ks, orders = inputgen.batched_queries(4096, seed=inputgen.config_seed(3), n_lo_log2=10,
                                               n_hi_log2=24, k_max=4096)
    q = len(ks)
    total = int(off[-1])
    ns = np.diff(off).astype(np.int64)
    kef = np.minimum(ks.astype(np.int64), ns)
    oo = np.zeros(q + 1, dtype=np.int64)
    oo[1:] = np.cumsum(kef)
    say(f"batched: Q={q} sum N={total} sum K={int(oo[-1])}")
    keys = torch.empty(total, dtype=torch.int64, device=dev)
    gen.device_fill(inputgen.KIND_U_I64, inputgen.config_seed(3), total, keys.data_ptr(),
                    stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    plan = Plan(off, ks, orders, key_dtype=torch.int64, rid_dtype=torch.uint32, stream=s)
    bk, br = plan.alloc_outputs()
    plan.launch(keys, bk, br, stream=s)
    torch.cuda.synchronize()
    bk_h, br_h = to_np(bk), to_np(br)
    # every query alone, one tk_topk each, into a second output buffer
    L = tk.lib()
    wsb = max(tk.workspace_size(int(n), int(k), tk.TK_KEY_I64, tk.TK_RID_U32) for n, k in zip(ns, kef))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    ak = torch.empty(int(oo[-1]), dtype=torch.int64, device=dev)
    ar = torch.empty(int(oo[-1]), dtype=torch.uint32, device=dev)
    cnt = ctypes.c_uint64()
    st = torch.cuda.current_stream()
    for i in range(q):
        rc = L.tk_topk(keys.data_ptr() + int(off[i]) * 8, None, int(ns[i]), int(ks[i]), tk.TK_KEY_I64,
                       tk.TK_RID_U32, int(orders[i]), ak.data_ptr() + int(oo[i]) * 8,
                       ar.data_ptr() + int(oo[i]) * 4, ctypes.byref(cnt), ws.data_ptr(), wsb,
                       st.cuda_stream)
        tk.check(rc, "tk_topk")
    torch.cuda.synchronize()
    assert np.array_equal(to_np(ak), bk_h) and np.array_equal(to_np(ar), br_h), \
        "batched plan differs from the queries run alone"
    # every query against the oracle: keys copied back query by query, the
    # oracle run on a pool of host threads (its ctypes calls release the GIL)
    import concurrent.futures as cf
    import os

    def check(i, host):
        ek, er = oracle.topk(host, None, int(ks[i]), int(orders[i]), rid_dtype=np.uint32)
        a, b = int(oo[i]), int(oo[i + 1])
        assert_same(bk_h[a:b], br_h[a:b], ek, er,
                    what=f"query {i} n={host.shape[0]} k={int(ks[i])} order={int(orders[i])}")
        return i

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    done = 0
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        pending = set()
        for i in np.argsort(-ns, kind="stable"):
            i = int(i)
            host = keys[int(off[i]):int(off[i + 1])].cpu().numpy()
            pending.add(ex.submit(check, i, host))
            if len(pending) >= 2 * workers:
                fin, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
                for f in fin:
                    f.result()
                    done += 1
        for f in cf.as_completed(pending):
            f.result()
            done += 1
    assert done == q
    say(f"batched: all {q} queries equal alone and equal the oracle")
    plan.close()


def test_key_only_late_materialization_full_size():
    import torch
    dev = torch.device("cuda:0")
    n, k, ncols = 1 << 26, 1000, 8
    seed = inputgen.config_seed(4)
    cdf = inputgen.zipf_cdf(1.05, 10 ** 6)
    hk = gen.host_fill(inputgen.KIND_ZIPF_I64, seed, n, cdf=cdf)
    payload = np.empty((ncols, n), dtype=np.float64)
    for c in range(ncols):
        payload[c] = gen.host_fill(inputgen.KIND_PAYLOAD_F64, seed + 1 + c, n)
    hr = np.arange(n, dtype=np.uint32)
    pk = torch.from_numpy(hk).pin_memory()
    pr = torch.from_numpy(hr.view(np.int32)).pin_memory()
    say("late materialization: 2^26 rows, int64 Zipf(1.05) keys, 8 float64 payload columns")
    dk = pk.to(dev, non_blocking=True)
    dr = pr.to(dev, non_blocking=True).view(torch.uint32)
    ws = tk.new_workspace(n, k, tk.TK_KEY_I64, tk.TK_RID_U32, device=dev)
    ok, orr = tk.topk(dk, k, rowids=dr, workspace=ws)
    torch.cuda.synchronize()
    gk, gr = to_np(ok), to_np(orr)
    ek, er = oracle.topk(hk, hr, k, oracle.DESC)
    assert_same(gk, gr, ek, er, what="key-only Top-1000")
    rows_host = tk.gather_rows_host(payload, gr)
    expect = np.take(payload, er.astype(np.int64), axis=1)
    assert np.array_equal(rows_host.view(np.uint64), expect.view(np.uint64))
    dpay = torch.from_numpy(payload).to(dev)
    rows_dev = torch.empty((ncols, k), dtype=torch.float64, device=dev)
    tk.gather_rows_device(dpay, orr, rows_dev)
    torch.cuda.synchronize()
    assert np.array_equal(rows_dev.cpu().numpy().view(np.uint64), expect.view(np.uint64))


def test_served_mixture_on_full_columns():
    """Served form on columns of 2^28 rows (one per key type, with host mirrors):
    600 requests of the serving mixture (N 70 % in [2^12, 2^16], 25 % in
    [2^18, 2^22], 5 % = 2^26; K in {10, 100, 1000, 10000}), Poisson arrivals,
    continuous batching with the default cost gate; every request equals the
    oracle on its rows."""
    import torch
    from paper_2601_19911_amd.serve import GATE_COST, Server
    dev = torch.device("cuda:0")
    col_len = 1 << 28
    kinds = [(inputgen.KIND_U_I32, torch.int32), (inputgen.KIND_U_I64, torch.int64),
             (inputgen.KIND_U_F32, torch.float32)]
    cols = []
    for c, (kind, dt) in enumerate(kinds):
        seed = inputgen.config_seed(5) + 10 + c
        d = torch.empty(col_len, dtype=dt, device=dev)
        gen.device_fill(kind, seed, col_len, d.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
        cols.append((d, gen.host_fill(kind, seed, col_len)))
    torch.cuda.synchronize()
    count = 600
    req = inputgen.serving_requests(count, col_len=col_len)
    col_of = np.minimum((req["u_col"] * len(cols)).astype(np.int64), len(cols) - 1)
    n, k, off = req["n"], req["k"], req["offset"]
    srv = Server(arena_bytes=4 << 30, max_batch=256, slots=2, window_us=50.0, gate=GATE_COST)
    ids = [srv.add_column(d, h) for d, h in cols]
    gaps = -np.log1p(-req["u_arr"]) / 20000.0
    rids = srv.replay(np.cumsum(gaps) - gaps[0], np.array(ids)[col_of], off, n, k,
                      np.zeros(count, dtype=np.uint8))
    srv.drain()
    st = srv.stats()
    say(f"served: {st}")
    import concurrent.futures as cf
    import os

    def check(i):
        gk, gr, info = srv.result(int(rids[i]), int(col_of[i]), int(min(k[i], n[i])))
        h = cols[int(col_of[i])][1][int(off[i]):int(off[i] + n[i])]
        ek, er = oracle.topk(h, None, int(k[i]), oracle.DESC, rid_dtype=np.uint64)
        assert_same(gk, gr, ek, er + np.uint64(off[i]),
                    what=f"request {i} n={int(n[i])} k={int(k[i])} route={info.route}")
        return 1

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        checked = sum(ex.map(check, range(count)))
    say(f"served: all {checked} requests equal the oracle")
    assert st["completed"] == count
    srv.close()
