#!/usr/bin/env python3
"""Measurement suites beside the headline line of bench.py.

    python bench_suites.py c2 [--quick]      single-query variants (dtype, distribution, K, order)
    python bench_suites.py c3 [--q 4096]     batched plan vs per-query launches (1 and 4 streams)
    python bench_suites.py c4                key-only vs full-row transfer with late materialization
    python bench_suites.py c5                served form: Poisson arrivals, gate on vs always-GPU
    python bench_suites.py crossover         CPU vs GPU time over N (host- and device-resident keys)
    python bench_suites.py gate              cost-model fit, predicted vs measured break-even N,
                                             margin sweep of the gate on the serving mixture
    python bench_suites.py e2e               headline query with pinned H2D and D2H included
    python bench_suites.py join              key-only hash-join probe (matching primitive):
                                             build and probe times, probes/s, bytes per probe
    python bench_suites.py sort --log2n 24   ORDER BY without LIMIT: LSD radix sort per key type
    python bench_suites.py stream --log2n 26 chunk-pipelined key-only streaming from pinned host
                                             memory vs the pure copy of the key bytes

Each suite prints one JSON object per measurement on stdout.  Every input is
synthetic and seeded (inputgen); every GPU result that a suite reports is
checked against the CPU oracle on the same rows (all of them, or a stated
sample of queries).
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

from paper_2601_19911_amd.gate import (break_even, crossover_n, fit_costs, measured_break_even,
                                       route_gpu)

HBM_PEAK_GBS = 8000.0


def emit(d):
    print(json.dumps(d), flush=True)


def pct(a, p):
    return float(np.percentile(np.asarray(a, dtype=np.float64), p)) if len(a) else None


def _torch():
    import torch
    return torch


def key_dtype_np(kc):
    import paper_2601_19911_amd as tk
    return {tk.TK_KEY_I32: np.int32, tk.TK_KEY_I64: np.int64, tk.TK_KEY_F32: np.float32}[kc]


def dev_view_np(t):
    """Host numpy copy of a device tensor, unsigned types included."""
    torch = _torch()
    if t.dtype == torch.uint32:
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    if t.dtype == torch.uint64:
        return t.view(torch.int64).cpu().numpy().view(np.uint64)
    return t.cpu().numpy()


def same(gk, gr, ek, er):
    bits = (lambda a: a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64))
    return (gk.shape == ek.shape and np.array_equal(bits(gk), bits(ek)) and
            np.array_equal(gr.astype(np.uint64), er.astype(np.uint64)))


# ---- C2: single-query variants -------------------------------------------------------------------

def suite_c2(a):
    import bench
    variants = []
    for dt in ("float32", "int64"):
        for dist in ("uniform", "zipf", "sorted"):
            for k in ((1000,) if a.quick else (10, 1000, 100000)):
                variants.append((dt, dist, k, "desc"))
            if dist == "zipf":
                variants.append((dt, dist, 1000, "asc"))
    for dt, dist, k, order in variants:
        args = bench.parse([f"--dtype={dt}", f"--dist={dist}", f"--k={k}", f"--order={order}",
                            "--steps=31", "--warmup=5", "--no-cpu"])
        r = bench.measure(args)
        r["suite"] = "c2"
        emit(r)


# ---- C3: batched vs per-query --------------------------------------------------------------------

def suite_c3(a):
    torch = _torch()
    import inputgen
    import oracle
    import paper_2601_19911_amd as tk
    from inputgen import native as gen
    from paper_2601_19911_amd.batched import Plan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    off, ks, orders = inputgen.batched_queries(a.q, seed=inputgen.config_seed(3),
                                               n_lo_log2=10, n_hi_log2=a.n_hi_log2, k_max=4096)
    Q = len(ks)
    total = int(off[-1])
    ns = np.diff(off).astype(np.int64)
    kef = np.minimum(ks.astype(np.int64), ns)
    oo = np.zeros(Q + 1, dtype=np.uint64)
    oo[1:] = np.cumsum(kef)
    print(f"c3: Q={Q} sum N={total} ({total * 8 / 1e9:.2f} GB int64) sum K={int(oo[-1])}",
          file=sys.stderr, flush=True)
    keys = torch.empty(total, dtype=torch.int64, device=dev)
    gen.device_fill(inputgen.KIND_U_I64, inputgen.config_seed(3), total, keys.data_ptr(),
                    stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    kp = keys.data_ptr()
    L = tk.lib()
    reps = a.reps

    # (i)/(ii) per-query tk_topk launches from C (tk_topk_each) on S streams, all
    # queries released at t0 (a start event every stream waits for); per-query
    # completion times from an event after each query
    def per_query(nstreams):
        from paper_2601_19911_amd.batched import topk_each
        streams = [torch.cuda.Stream() for _ in range(nstreams)]
        ok = torch.empty(int(oo[-1]), dtype=torch.int64, device=dev)
        orr = torch.empty(int(oo[-1]), dtype=torch.uint32, device=dev)
        best = None
        for rep in range(reps + 1):
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            lat = topk_each(off, ks, orders, keys, ok, orr, streams)
            wall = time.perf_counter() - w0
            total_s = float(lat.max())
            if rep and (best is None or total_s < best[0]):
                best = (total_s, lat, wall)
        return best, ok, orr

    def plan_run(params, label):
        s = torch.cuda.Stream()
        plan = Plan(off, ks, orders, key_dtype=torch.int64, rid_dtype=torch.uint32, stream=s,
                    **params)
        ok, orr = plan.alloc_outputs()
        torch.cuda.synchronize()
        plan.launch(keys, ok, orr, stream=s)  # eager first launch
        plan.launch(keys, ok, orr, stream=s)  # captured
        torch.cuda.synchronize()
        best = None
        for rep in range(reps):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0.record(s)
            plan.launch(keys, ok, orr, stream=s)
            t1.record(s)
            torch.cuda.synchronize()
            total_s = t0.elapsed_time(t1) * 1e-3
            # per-query completion from the device clock: each query's tail
            # stamps its end, the launch's first kernel its start
            lat = plan.query_times()
            st = plan.stats()
            if best is None or total_s < best[0]:
                best = (total_s, lat, st)
        info = plan.info()
        return best, ok, orr, info, plan

    def report(mode, total_s, lat, extra):
        bytes_alg = total * 8
        emit({"suite": "c3", "mode": mode, "queries": Q, "sum_n": total, "sum_k": int(oo[-1]),
              "seconds": total_s, "keys_per_s": total / total_s, "qps": Q / total_s,
              "gbs": bytes_alg / total_s / 1e9, "frac_of_peak": bytes_alg / total_s / 1e9 / HBM_PEAK_GBS,
              "lat_p50_ms": pct(lat, 50) * 1e3, "lat_p95_ms": pct(lat, 95) * 1e3,
              "lat_p99_ms": pct(lat, 99) * 1e3, "lat_max_ms": float(np.max(lat)) * 1e3, **extra})

    from paper_2601_19911_amd import autotune
    (pb, pok, porr, pinfo, plan) = plan_run({}, "default")
    report("batched_plan", pb[0], pb[1], {"plan": pinfo, "stats": pb[2], "reps": reps,
                                          "params": "default"})
    pk, pr = dev_view_np(pok), dev_view_np(porr)
    if a.tune:
        cache = os.path.join(a.tune_cache_dir, "tuned_plans.json") if a.tune_cache_dir else None
        best, secs, table = autotune.tune(off, ks, orders, keys, quick=a.quick, reps=2,
                                          cache_path=cache)
        for row in table:
            emit({"suite": "c3", "tune_candidate": row})
        (tb, tok, torr, tinfo, tplan) = plan_run(best, "tuned")
        report("batched_plan_tuned", tb[0], tb[1], {"plan": tinfo, "stats": tb[2], "reps": reps,
                                                    "params": best})
        tuned_same = bool(np.array_equal(dev_view_np(tok), pk) and np.array_equal(dev_view_np(torr), pr))
        emit({"suite": "c3", "check": "tuned_equals_default", "equal": tuned_same})
        tplan.close()
    results = {}
    for S in (1, 4):
        (b, ok, orr) = per_query(S)
        report(f"per_query_{S}_stream", b[0], b[1], {"host_call_s": b[2], "reps": reps,
                                                       "launched_from": "C (tk_topk_each)"})
        results[S] = (dev_view_np(ok), dev_view_np(orr))
    # parity: per-query == batched everywhere; a sample of queries == oracle
    agree = all(np.array_equal(results[S][0], pk) and np.array_equal(results[S][1], pr)
                for S in results)
    order_idx = np.argsort(ns)
    pick = sorted(set(list(order_idx[:: max(1, Q // a.check_queries)]) + [int(order_idx[-1])]))
    bad = 0
    for q in pick:
        lo, hi = int(off[q]), int(off[q + 1])
        host = dev_view_np(keys[lo:hi])
        ek, er = oracle.topk(host, None, int(ks[q]), int(orders[q]), rid_dtype=np.uint32)
        a0, a1 = int(oo[q]), int(oo[q + 1])
        bad += not same(pk[a0:a1], pr[a0:a1], ek, er)
    emit({"suite": "c3", "check": "parity", "batched_equals_per_query": bool(agree),
          "oracle_checked_queries": len(pick), "oracle_mismatches": bad})
    plan.close()


# ---- E2E: pinned host keys, H2D + query + D2H ------------------------------------------------------

def _pinned_copy(np_arr):
    torch = _torch()
    t = torch.from_numpy(np_arr.view(np.int32) if np_arr.dtype == np.uint32 else np_arr)
    p = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    p.copy_(t)
    return p


def suite_e2e(a):
    torch = _torch()
    import inputgen
    import oracle
    import paper_2601_19911_amd as tk
    from inputgen import native as gen

    dev = torch.device("cuda:0")
    n, k = 1 << a.log2n, 1000
    seed = inputgen.config_seed(2)
    hk = gen.host_fill(inputgen.KIND_U_F32, seed, n)
    hr = np.arange(n, dtype=np.uint32)
    pk, pr = _pinned_copy(hk), _pinned_copy(hr)
    dk = torch.empty(n, dtype=torch.float32, device=dev)
    dr = torch.empty(n, dtype=torch.int32, device=dev)
    ok = torch.empty(k, dtype=torch.float32, device=dev)
    orr = torch.empty(k, dtype=torch.int32, device=dev)
    hok = torch.empty(k, dtype=torch.float32, pin_memory=True)
    hor = torch.empty(k, dtype=torch.int32, pin_memory=True)
    ws = tk.new_workspace(n, k, tk.TK_KEY_F32, tk.TK_RID_U32, device=dev)
    s = torch.cuda.current_stream()

    def one():
        dk.copy_(pk, non_blocking=True)
        dr.copy_(pr, non_blocking=True)
        tk.topk(dk, k, rowids=dr.view(torch.uint32), out_keys=ok, out_rowids=orr.view(torch.uint32),
                workspace=ws, stream=s)
        hok.copy_(ok, non_blocking=True)
        hor.copy_(orr, non_blocking=True)

    for _ in range(2):
        one()
    torch.cuda.synchronize()
    times, h2d = [], []
    for _ in range(a.reps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(s)
        dk.copy_(pk, non_blocking=True)
        dr.copy_(pr, non_blocking=True)
        e1.record(s)
        tk.topk(dk, k, rowids=dr.view(torch.uint32), out_keys=ok, out_rowids=orr.view(torch.uint32),
                workspace=ws, stream=s)
        hok.copy_(ok, non_blocking=True)
        hor.copy_(orr, non_blocking=True)
        e2.record(s)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e2) * 1e-3)
        h2d.append(e0.elapsed_time(e1) * 1e-3)
    ek, er = oracle.topk(hk, hr, k, oracle.DESC)
    match = same(hok.numpy(), hor.numpy().view(np.uint32), ek, er)
    t = float(np.median(times))
    emit({"suite": "e2e", "workload": f"N=2^{a.log2n} float32 + uint32 row-ids in pinned host "
          "memory, K=1000 desc: H2D of keys and row-ids, Top-K, D2H of the results",
          "median_s": t, "p95_s": pct(times, 95), "keys_per_s": n / t,
          "h2d_median_s": float(np.median(h2d)), "h2d_gbs": n * 8 / float(np.median(h2d)) / 1e9,
          "reps": a.reps, "oracle_match": bool(match)})


def suite_sort(a):
    """ORDER BY key without LIMIT (tk_sort, LSD radix): 2^log2n pairs per key
    type, uniform keys, implicit row-ids (uint32), descending.  Times the sort
    with events on the launch stream; the first result is compared with the
    oracle (Top-K with K = N).  Bytes: the minimum a sort moves (one read of
    the keys, one write of keys and row-ids) and what this design moves (per
    digit pass two reads and one write of every pair; the first pass reads the
    keys only, the last writes the outputs)."""
    torch = _torch()
    import inputgen
    import oracle
    import paper_2601_19911_amd as tk
    from inputgen import native as gen

    dev = torch.device("cuda:0")
    n = 1 << a.log2n
    s = torch.cuda.current_stream()
    for name, kind, tdt in [("int32", inputgen.KIND_U_I32, torch.int32),
                            ("float32", inputgen.KIND_U_F32, torch.float32),
                            ("int64", inputgen.KIND_U_I64, torch.int64),
                            ("float64", inputgen.KIND_U_F64, torch.float64)]:
        hk = gen.host_fill(kind, inputgen.config_seed(5, 90), n)
        dk = torch.from_numpy(hk).to(dev)
        kb, rb = hk.dtype.itemsize, 4
        ok, orr = tk.sort(dk, order="desc")
        ws = torch.empty(int(tk.lib().tk_sort_workspace_size(n, tk.key_code(tdt), tk.TK_RID_U32)),
                         dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        match = None
        if not a.no_check:
            ek, er = oracle.topk(hk, None, n, oracle.DESC)
            match = same(dev_view_np(ok), dev_view_np(orr), ek, er)
        ts = []
        for r in range(a.reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            tk.sort(dk, order="desc", out_keys=ok, out_rowids=orr, workspace=ws, stream=s)
            e1.record(s)
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1) * 1e-3)
        t = float(np.median(ts))
        passes = kb
        min_bytes = n * kb + n * (kb + rb)
        design_bytes = (passes * 3 * n * (kb + rb)) - 2 * n * rb  # first pass reads keys only
        emit({"suite": "sort", "workload": f"ORDER BY key without LIMIT, N=2^{a.log2n} {name} "
              "uniform keys, implicit uint32 row-ids, desc", "key_dtype": name, "n": n,
              "digit_passes": passes, "median_s": t, "p95_s": pct(ts, 95), "keys_per_s": n / t,
              "min_bytes": min_bytes, "min_bytes_gbs": min_bytes / t / 1e9,
              "design_bytes": design_bytes, "design_bytes_gbs": design_bytes / t / 1e9,
              "design_frac_of_peak": design_bytes / t / 1e9 / HBM_PEAK_GBS,
              "oracle_match": match, "reps": a.reps})
        del dk, ok, orr, ws


def suite_stream(a):
    """Chunk-pipelined key-only streaming (tk_topk_stream): a key column in
    pinned host memory, K = 1000 desc, implicit row-ids.  Times (events on the
    compute stream) the pure host-to-device copy of the key bytes, the copy
    followed by a device-resident query, and the pipelined call at several
    chunk sizes; every pipelined result is compared with the oracle."""
    torch = _torch()
    import inputgen
    import oracle
    import paper_2601_19911_amd as tk
    from inputgen import native as gen

    dev = torch.device("cuda:0")
    n, k = 1 << a.log2n, 1000
    s = torch.cuda.current_stream()
    cs = torch.cuda.Stream()
    for name, kind, tdt in [("float32", inputgen.KIND_U_F32, torch.float32),
                            ("int64", inputgen.KIND_U_I64, torch.int64)]:
        hk = gen.host_fill(kind, inputgen.config_seed(4, 80), n)
        pk = _pinned_copy(hk)
        kb = hk.dtype.itemsize
        dk = torch.empty(n, dtype=tdt, device=dev)
        ws = tk.new_workspace(n, k, tk.key_code(tdt), tk.TK_RID_U32, device=dev)
        ok = torch.empty(k, dtype=tdt, device=dev)
        orr = torch.empty(k, dtype=torch.uint32, device=dev)
        ek, er = oracle.topk(hk, None, k, oracle.DESC)

        def timed(fn):
            out = []
            for r in range(a.reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                fn()
                e1.record(s)
                torch.cuda.synchronize()
                if r:
                    out.append(e0.elapsed_time(e1) * 1e-3)
            return out

        copy_t = timed(lambda: dk.copy_(pk, non_blocking=True))

        def serial():
            dk.copy_(pk, non_blocking=True)
            tk.topk(dk, k, out_keys=ok, out_rowids=orr, workspace=ws, stream=s)

        serial_t = timed(serial)
        tcopy = float(np.median(copy_t))
        for chunk_log2 in a.chunks_log2:
            chunk = 1 << chunk_log2
            sws = torch.empty(tk.lib().tk_stream_workspace_size(n, k, chunk, tk.key_code(tdt),
                                                                 tk.TK_RID_U32, 0),
                              dtype=torch.uint8, device=dev)
            tk.topk_stream(pk, k, chunk=chunk, out_keys=ok, out_rowids=orr, workspace=sws,
                           stream=s, copy_stream=cs)
            torch.cuda.synchronize()
            match = same(dev_view_np(ok), dev_view_np(orr), ek, er)
            st = timed(lambda: tk.topk_stream(pk, k, chunk=chunk, out_keys=ok, out_rowids=orr,
                                              workspace=sws, stream=s, copy_stream=cs))
            t = float(np.median(st))
            emit({"suite": "stream", "workload": f"N=2^{a.log2n} {name} keys in pinned host memory, "
                  "implicit row-ids, K=1000 desc", "key_dtype": name, "chunk": chunk,
                  "workspace_bytes": int(sws.numel()), "copy_only_s": tcopy,
                  "copy_gbs": n * kb / tcopy / 1e9, "serial_copy_then_query_s": float(np.median(serial_t)),
                  "stream_s": t, "stream_p95_s": pct(st, 95), "stream_over_copy": t / tcopy,
                  "keys_per_s": n / t, "oracle_match": bool(match), "reps": a.reps})
        del dk, ws, pk


# ---- C4: key-only vs full-row with late materialization ----------------------------------------

def suite_c4(a):
    torch = _torch()
    import inputgen
    import oracle
    import paper_2601_19911_amd as tk
    from inputgen import native as gen

    dev = torch.device("cuda:0")
    n, k, ncols = 1 << a.log2n, 1000, 8
    seed = inputgen.config_seed(4)
    cdf = inputgen.zipf_cdf(1.05, 10 ** 6)
    hk = gen.host_fill(inputgen.KIND_ZIPF_I64, seed, n, cdf=cdf)
    payload = np.empty((ncols, n), dtype=np.float64)
    for c in range(ncols):
        payload[c] = gen.host_fill(inputgen.KIND_PAYLOAD_F64, seed + 1 + c, n)
    hr = np.arange(n, dtype=np.uint32)
    pk, pr = _pinned_copy(hk), _pinned_copy(hr)
    ppay = _pinned_copy(payload)
    s = torch.cuda.current_stream()
    dk = torch.empty(n, dtype=torch.int64, device=dev)
    dr = torch.empty(n, dtype=torch.int32, device=dev)
    dpay = torch.empty((ncols, n), dtype=torch.float64, device=dev)
    ok = torch.empty(k, dtype=torch.int64, device=dev)
    orr = torch.empty(k, dtype=torch.int32, device=dev)
    hok = torch.empty(k, dtype=torch.int64, pin_memory=True)
    hor = torch.empty(k, dtype=torch.int32, pin_memory=True)
    rows_dev = torch.empty((ncols, k), dtype=torch.float64, device=dev)
    hrows = torch.empty((ncols, k), dtype=torch.float64, pin_memory=True)
    ws = tk.new_workspace(n, k, tk.TK_KEY_I64, tk.TK_RID_U32, device=dev)
    L = tk.lib()

    def key_only():
        dk.copy_(pk, non_blocking=True)
        dr.copy_(pr, non_blocking=True)
        tk.topk(dk, k, rowids=dr.view(torch.uint32), out_keys=ok, out_rowids=orr.view(torch.uint32),
                workspace=ws, stream=s)
        hok.copy_(ok, non_blocking=True)
        hor.copy_(orr, non_blocking=True)
        torch.cuda.synchronize()
        # late materialization on the host: gather the payload rows at the row-ids
        return tk.gather_rows_host(payload, hor.numpy().view(np.uint32))

    def full_row():
        dk.copy_(pk, non_blocking=True)
        dr.copy_(pr, non_blocking=True)
        dpay.copy_(ppay, non_blocking=True)
        tk.topk(dk, k, rowids=dr.view(torch.uint32), out_keys=ok, out_rowids=orr.view(torch.uint32),
                workspace=ws, stream=s)
        tk.gather_rows_device(dpay, orr.view(torch.uint32), rows_dev, stream=s)
        hrows.copy_(rows_dev, non_blocking=True)
        hok.copy_(ok, non_blocking=True)
        hor.copy_(orr, non_blocking=True)
        torch.cuda.synchronize()
        return hrows.numpy().copy()

    ek, er = oracle.topk(hk, hr, k, oracle.DESC)
    expect_rows = payload[:, er.astype(np.int64)]
    for name, fn in (("key_only", key_only), ("full_row", full_row)):
        fn()
        ts = []
        for _ in range(a.reps):
            t0 = time.perf_counter()
            rows = fn()
            ts.append(time.perf_counter() - t0)
        ok_match = same(hok.numpy(), hor.numpy().view(np.uint32), ek, er)
        rows_match = bool(np.array_equal(rows.view(np.uint64), expect_rows.view(np.uint64)))
        h2d_bytes = n * (8 + 4) + (n * ncols * 8 if name == "full_row" else 0)
        emit({"suite": "c4", "mode": name, "n": n, "k": k, "payload_cols": ncols,
              "h2d_bytes": h2d_bytes, "median_s": float(np.median(ts)), "p95_s": pct(ts, 95),
              "reps": a.reps, "oracle_match": bool(ok_match), "rows_match": rows_match})


# ---- C5: served form ----------------------------------------------------------------------------

def suite_c5(a):
    torch = _torch()
    import inputgen
    import oracle
    import paper_2601_19911_amd as tk
    from inputgen import native as gen
    from paper_2601_19911_amd.serve import GATE_COST, GATE_GPU, Server

    dev = torch.device("cuda:0")
    col_len = 1 << a.col_log2
    kinds = [(inputgen.KIND_U_I32, torch.int32), (inputgen.KIND_U_I64, torch.int64),
             (inputgen.KIND_U_F32, torch.float32)]
    cols = []
    for c in range(a.columns):
        kind, dt = kinds[c % 3]
        seed = inputgen.config_seed(5) + 10 + c
        d = torch.empty(col_len, dtype=dt, device=dev)
        gen.device_fill(kind, seed, col_len, d.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
        h = gen.host_fill(kind, seed, col_len)
        cols.append((d, h))
    torch.cuda.synchronize()
    req = inputgen.serving_requests(a.requests, col_len=col_len)
    cnt = a.requests
    col_of = np.minimum((req["u_col"] * a.columns).astype(np.int64), a.columns - 1)
    n, k, off = req["n"], req["k"], req["offset"]
    cost = json.loads(a.cost) if a.cost else None

    def run(gate, rate, max_batch, slots, window_us, margin_us=0.0):
        srv = Server(arena_bytes=a.arena_mb << 20, max_batch=max_batch, slots=slots,
                     window_us=window_us, gate=gate, margin_ms=margin_us * 1e-3,
                     cpu_threads=a.cpu_threads, cost=cost)
        ids = [srv.add_column(d, h) for d, h in cols]
        # Poisson arrivals: exponential gaps from the recipe's uniforms
        gaps = -np.log1p(-req["u_arr"]) / rate
        t_arr = np.cumsum(gaps) - gaps[0]
        rids = srv.replay(t_arr, np.array(ids)[col_of], off, n, k, np.zeros(cnt, dtype=np.uint8))
        srv.drain()
        lat, routes, sub, done = [], [], [], []
        bad = 0
        for i in range(cnt):
            res = srv.result(int(rids[i]), int(col_of[i]), int(min(k[i], n[i])))
            gk, gr, info = res
            lat.append((info.t_done_ns - info.t_submit_ns) * 1e-9)
            sub.append(info.t_submit_ns)
            done.append(info.t_done_ns)
            routes.append(info.route)
            if i % a.check_every == 0:
                h = cols[int(col_of[i])][1][int(off[i]):int(off[i] + n[i])]
                ek, er = oracle.topk(h, None, int(k[i]), oracle.DESC, rid_dtype=np.uint64)
                bad += not same(gk, gr, ek, er + np.uint64(off[i]))
        st = srv.stats()
        srv.close()
        span = (max(done) - min(sub)) * 1e-9
        return np.array(lat), np.array(routes), st, bad, span

    # per_query: the same request loop, one request per launch and one slot (no
    # batching, no overlap); always_gpu: continuous batching; cost_gate: batching
    # with small requests routed to the CPU
    modes = (("per_query", GATE_GPU, 1, 1, 0.0), ("always_gpu", GATE_GPU, a.max_batch, a.slots, a.window_us),
             ("cost_gate", GATE_COST, a.max_batch, a.slots, a.window_us))
    for name, gate, mb, sl, win in modes:
        if a.modes and name not in a.modes:
            continue
        for lam in a.rates:
            for m in (a.margins_us if gate == GATE_COST else [0.0]):
                lat, routes, st, bad, span = run(gate, lam, mb, sl, win, m)
                emit({"suite": "c5", "mode": name, "rate_qps": lam, "margin_us": m, "requests": cnt,
                      "columns": a.columns, "col_rows": col_len,
                      "achieved_qps": cnt / span, "makespan_s": span,
                      "lat_p50_ms": pct(lat, 50) * 1e3, "lat_p95_ms": pct(lat, 95) * 1e3,
                      "lat_p99_ms": pct(lat, 99) * 1e3, "cpu_routed": float(np.mean(routes == 1)),
                      "stats": st, "oracle_checked": (cnt + a.check_every - 1) // a.check_every,
                      "oracle_mismatches": bad})


# ---- crossover ---------------------------------------------------------------------------------

class _Point:
    """CPU and GPU times of one Top-K (N, K) over the first N keys of a seeded
    column of one dtype: GPU with keys resident in HBM and with keys copied from
    pinned host memory (launch to results on the host), CPU route on every core
    of the affinity mask; both results checked against the oracle."""

    def __init__(self, dt, nmax, ks):
        torch = _torch()
        import inputgen
        import paper_2601_19911_amd as tk
        from inputgen import native as gen
        kinds = {"int32": (inputgen.KIND_U_I32, torch.int32), "int64": (inputgen.KIND_U_I64, torch.int64),
                 "float32": (inputgen.KIND_U_F32, torch.float32),
                 "float64": (inputgen.KIND_U_F64, torch.float64)}
        kind, tdt = kinds[dt]
        self.dt, self.tdt, self.torch, self.tk = dt, tdt, torch, tk
        self.dev = torch.device("cuda:0")
        self.cores = len(os.sched_getaffinity(0))
        self.hk = gen.host_fill(kind, inputgen.config_seed(6), nmax)
        self.pk = _pinned_copy(self.hk)
        self.dk = torch.empty(nmax, dtype=tdt, device=self.dev)
        self.dk.copy_(self.pk)
        kmax = max(ks)
        self.ws = tk.new_workspace(nmax, kmax, tk.key_code(tdt), tk.TK_RID_U32, device=self.dev)
        self.ok = torch.empty(kmax, dtype=tdt, device=self.dev)
        self.orr = torch.empty(kmax, dtype=torch.uint32, device=self.dev)
        self.hok = torch.empty(kmax, dtype=tdt, pin_memory=True)
        self.hor = torch.empty(kmax, dtype=torch.int32, pin_memory=True)
        self.s = torch.cuda.current_stream()

    def __call__(self, N, K):
        import oracle
        torch, tk = self.torch, self.tk
        ke = min(K, N)
        reps = 31 if N <= (1 << 22) else 5

        def gpu(resident):
            ts = []
            for r in range(reps + 2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if not resident:
                    self.dk[:N].copy_(self.pk[:N], non_blocking=True)
                tk.topk(self.dk[:N], K, out_keys=self.ok[:ke], out_rowids=self.orr[:ke],
                        workspace=self.ws, stream=self.s)
                self.hok[:ke].copy_(self.ok[:ke], non_blocking=True)
                self.hor[:ke].copy_(self.orr[:ke].view(torch.int32), non_blocking=True)
                torch.cuda.synchronize()
                if r >= 2:
                    ts.append(time.perf_counter() - t0)
            return float(np.median(ts))

        g_res, g_host = gpu(True), gpu(False)
        ek, er = oracle.topk(self.hk[:N], None, K, oracle.DESC, rid_dtype=np.uint32)
        match = same(self.hok[:ke].numpy(), self.hor[:ke].numpy().view(np.uint32), ek, er)
        cts = []
        for r in range(reps + 1):
            t0 = time.perf_counter()
            ck, cr = tk.cpu_topk(self.hk[:N], K, nthreads=self.cores)
            if r:
                cts.append(time.perf_counter() - t0)
        cpu_match = same(ck, cr, ek, er)
        return {"dtype": self.dt, "k": K, "n": N, "gpu_resident_s": g_res, "gpu_host_keys_s": g_host,
                "cpu_all_cores_s": float(np.median(cts)), "cpu_threads": self.cores, "reps": reps,
                "oracle_match": bool(match), "cpu_match": bool(cpu_match)}


def suite_crossover(a):
    for dt in a.dtypes:
        pt = _Point(dt, 1 << a.max_log2, a.ks)
        rows = []
        for K in a.ks:
            for lg in range(a.min_log2, a.max_log2 + 1):
                row = dict(suite="crossover", **pt(1 << lg, K))
                rows.append(row)
                emit(row)
            ks_rows = [r for r in rows if r["k"] == K]
            emit({"suite": "crossover", "dtype": dt, "k": K,
                  "crossover_n_resident": crossover_n(ks_rows, "gpu_resident_s"),
                  "crossover_n_host_keys": crossover_n(ks_rows, "gpu_host_keys_s")})
        emit({"suite": "crossover", "dtype": dt, "fit": fit_costs(rows)})
        del pt


# ---- gate: break-even prediction and margin sensitivity -------------------------------------

def suite_gate(a):
    """Break-even validation (paper sec. V-D, in kind): fit the gate's cost
    models per key type on the power-of-two sweep of every K
    (2^fit_lo_log2 <= N <= 2^fit_log2, relative residuals), predict each
    break-even N from that key type's models, measure it by bisection, and
    report the relative error.  Then the margin sweep: the serving mixture at
    one arrival rate under the fitted per-type gate, one run per margin
    (offload share predicted from the models and observed, latency,
    throughput)."""
    be, costs = [], {}
    for dt in a.dtypes:
        pt = _Point(dt, 1 << a.max_log2, a.ks)
        fit_rows = []
        for K in a.ks:
            rows = []
            for lg in range(a.min_log2, a.max_log2 + 1):
                row = dict(suite="gate", **pt(1 << lg, K))
                rows.append(row)
                emit(row)
            meas, extra = measured_break_even(pt, K, rows, a.bisect)
            for r in extra:
                emit(dict(suite="gate", bisect=True, **r))
            fit_rows += [r for r in rows if (1 << a.fit_lo_log2) <= r["n"] <= (1 << a.fit_log2)]
            be.append({"dtype": dt, "k": K, "measured": meas})
        del pt
        costs[dt] = fit_costs(fit_rows, relative=True)
        emit({"suite": "gate", "dtype": dt, "fit": costs[dt], "fit_points": len(fit_rows)})
    for b in be:
        pred = break_even(costs[b["dtype"]], b["k"])
        err = None if (pred is None or b["measured"] is None) else abs(pred - b["measured"]) / b["measured"]
        emit({"suite": "gate", "dtype": b["dtype"], "k": b["k"], "break_even_measured": b["measured"],
              "break_even_predicted": pred, "rel_error": err})
    # margin sweep on the serving mixture, under the fitted per-type gate
    import inputgen
    req = inputgen.serving_requests(a.requests, col_len=1 << a.col_log2)
    types = ["int32", "int64", "float32"]
    col_type = np.array([types[c % 3] for c in range(a.columns)])
    req_type = col_type[np.minimum((req["u_col"] * a.columns).astype(np.int64), a.columns - 1)]
    for m in a.margins_us:
        share = np.zeros(len(req["n"]), dtype=bool)
        for t in types:
            sel = req_type == t
            if t in costs and sel.any():
                share[sel] = route_gpu(costs[t], req["n"][sel], req["k"][sel], m * 1e-6)
        emit({"suite": "gate", "margin_us": m, "predicted_gpu_share": float(np.mean(share)),
              "break_even_by_k": {t: {str(k): break_even(costs[t], k, m * 1e-6)
                                      for k in (10, 100, 1000, 10000)} for t in costs}})
    a.cost = json.dumps(costs)
    a.modes = ["cost_gate"]
    suite_c5(a)


# ---- matching primitive: key-only hash-join probe ----------------------------------------------

def suite_join(a):
    """Build 2^b int32/int64 keys (uniform; int64 all distinct), probe 2^26
    foreign keys drawn from twice the build's index range (hit rate 1/2),
    row-ids implicit (uint32).  Times the build and the probe with events on
    the launch stream, with and without the bloom prefilter; the first probe's
    pairs are compared with the oracle."""
    torch = _torch()
    import inputgen
    import oracle
    from inputgen import native as gen
    import paper_2601_19911_amd as tk
    from paper_2601_19911_amd.join import join_build, join_probe
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    cases = [(np.int64, 24), (np.int64, 20), (np.int32, 22)] if not a.quick else [(np.int64, 20)]
    np_ = 1 << a.join_probe_log2
    for dt, lb in cases:
        nb = 1 << lb
        seed = inputgen.config_seed(6, lb)
        bkind = inputgen.KIND_U_I64 if dt == np.int64 else inputgen.KIND_U_I32
        pkind = inputgen.KIND_JOIN_FK_I64 if dt == np.int64 else inputgen.KIND_JOIN_FK_I32
        bk_h = gen.host_fill(bkind, seed, nb)
        pk_h = gen.host_fill(pkind, seed, np_, n_total=2 * nb)
        bk, pk = torch.from_numpy(bk_h).to(dev), torch.from_numpy(pk_h).to(dev)
        expect = None
        for bloom in (True, False) if a.join_bloom == 0 else (a.join_bloom == 1,):
            tk.set_tuning(join_bloom=1 if bloom else 2)
            t = join_build(bk)
            op, ob, cnt = join_probe(t, pk)
            torch.cuda.synchronize()
            m = int(cnt.view(torch.int64).item())
            if m > op.numel():
                op, ob, cnt = join_probe(t, pk, capacity=m)
                torch.cuda.synchronize()
            ok = None
            if not a.no_check:
                gp = dev_view_np(op)[:m].astype(np.uint64)
                gb = dev_view_np(ob)[:m].astype(np.uint64)
                o = np.lexsort((gb, gp))
                if expect is None:
                    expect = oracle.join(bk_h, None, pk_h, None)
                ep, eb = expect
                ok = bool(gp.shape == ep.shape and np.array_equal(gp[o], ep) and
                          np.array_equal(gb[o], eb))
            bt, pt = [], []
            for _ in range(a.reps):
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                e0.record(st)
                t = join_build(bk, table=t.buf)
                e1.record(st)
                join_probe(t, pk, capacity=op.numel(), out_probe=op, out_build=ob, count=cnt)
                e2.record(st)
                torch.cuda.synchronize()
                bt.append(e0.elapsed_time(e1))
                pt.append(e1.elapsed_time(e2))
            kb = np.dtype(dt).itemsize
            slot_b = 16 if dt == np.int64 else 8
            probe_ms = float(np.median(pt))
            # bytes per probe: the key, one slot, and the matched pairs written
            alg = np_ * (kb + slot_b) + m * 8
            emit({"suite": "join", "key_dtype": np.dtype(dt).name, "n_build": nb, "n_probe": np_,
                  "bloom": bloom, "hit_rate_expected": 0.5, "matches": m,
                  "table_bytes": int(t.buf.numel()), "slots": t.slots,
                  "build_ms": float(np.median(bt)), "probe_ms": probe_ms,
                  "probe_ms_p95": pct(pt, 95), "probes_per_s": np_ / (probe_ms * 1e-3),
                  "build_keys_per_s": nb / (float(np.median(bt)) * 1e-3),
                  "alg_bytes_per_probe": alg / np_,
                  "probe_alg_gbs": alg / (probe_ms * 1e-3) / 1e9,
                  "probe_frac_of_peak": alg / (probe_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "equal_to_oracle": ok, "reps": a.reps})
        tk.set_tuning(join_bloom=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("suite", choices=["c2", "c3", "c4", "c5", "crossover", "gate", "e2e", "join",
                                      "stream", "sort"])
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--q", type=int, default=4096)
    ap.add_argument("--n-hi-log2", type=float, default=24.0)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--check-queries", type=int, default=24)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--columns", type=int, default=6)
    ap.add_argument("--col-log2", type=int, default=28)
    ap.add_argument("--requests", type=int, default=4000)
    ap.add_argument("--rates", type=float, nargs="+", default=[2000.0])
    ap.add_argument("--modes", nargs="+", default=[],
                    help="c5: per_query, always_gpu, cost_gate (default: all)")
    ap.add_argument("--arena-mb", type=int, default=4096)
    ap.add_argument("--max-batch", type=int, default=256)
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--window-us", type=float, default=50.0)
    ap.add_argument("--cpu-threads", type=int, default=8)
    ap.add_argument("--cost", type=str, default="")
    ap.add_argument("--check-every", type=int, default=20)
    ap.add_argument("--dtypes", nargs="+", default=["int32", "int64", "float32"])
    ap.add_argument("--ks", type=int, nargs="+", default=[10, 100, 1000])
    ap.add_argument("--min-log2", type=int, default=8)
    ap.add_argument("--max-log2", type=int, default=26)
    ap.add_argument("--margins-us", type=float, nargs="+", default=[0.0],
                    help="c5, gate: margins of the cost gate, microseconds")
    ap.add_argument("--bisect", type=int, default=4, help="gate: bisections of each break-even")
    ap.add_argument("--fit-log2", type=int, default=20, help="gate: largest N of the model fit")
    ap.add_argument("--fit-lo-log2", type=int, default=10, help="gate: smallest N of the model fit")
    ap.add_argument("--join-probe-log2", type=int, default=26, help="join: probe keys (log2)")
    ap.add_argument("--join-bloom", type=int, default=0, choices=[0, 1, 2],
                    help="join: 1 with the bloom prefilter, 2 without, 0 both")
    ap.add_argument("--tune", action="store_true", help="c3: also autotune the plan and time it")
    ap.add_argument("--tune-cache-dir", type=str, default="",
                    help="c3: where the tuned parameters are stored (default: the package's cache)")
    ap.add_argument("--no-check", action="store_true",
                    help="join, sort: skip the oracle comparison (profiling runs)")
    ap.add_argument("--chunks-log2", type=int, nargs="+", default=[22, 24],
                    help="stream: chunk sizes (log2 keys)")
    a = ap.parse_args()
    {"join": suite_join, "c2": suite_c2, "c3": suite_c3, "c4": suite_c4, "c5": suite_c5, "crossover": suite_crossover,
     "gate": suite_gate, "e2e": suite_e2e, "stream": suite_stream, "sort": suite_sort}[a.suite](a)


if __name__ == "__main__":
    main()
