#!/usr/bin/env python3
"""Benchmark of key-only Top-K on one MI355X.

One step = one tk_topk call (sample, streaming filter, tail select + sort)
over the whole workload with keys and row-ids already resident in HBM:
N = 2^28 float32 keys uniform in [0, 1) with uint32 row-ids 0..N-1, K = 1000,
descending.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--k", type=int, default=1000)
    ap.add_argument("--dtype", choices=["float32", "int32", "int64", "float64"], default="float32")
    ap.add_argument("--dist", choices=["uniform", "zipf", "sorted"], default="uniform")
    ap.add_argument("--order", choices=["desc", "asc"], default="desc")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU budget of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle check of the result")
    ap.add_argument("--no-f64", action="store_true",
                    help="skip the float64 record measured beside a float32 run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--read-ceiling", action="store_true",
                    help="only measure the read ceiling: tk_read_probe over 1 GiB")
    return ap.parse_args(argv)


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_traffic.txt, a line "hbm_bytes_per_launch: B"), if any."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{kernel}_traffic.txt")
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("hbm_bytes_per_launch:"):
                    return float(line.split(":", 1)[1])
    except (OSError, ValueError):
        return None
    return None


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, five times: the reference
    against which the FETCH_SIZE / WRITE_SIZE counters are scaled."""
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n,
                      "bytes_written_per_copy": n, "copies": 5}), flush=True)


def read_ceiling():
    """The HBM read ceiling the streaming pass is compared against: the read
    probe of the library over 1 GiB, 20 timed passes per launch shape (event
    pairs on the launch stream), median and best in GB/s."""
    import numpy as np
    import torch
    import paper_2601_19911_amd as tk
    n = 1 << 30
    buf = torch.full((n // 4,), 0x11111111, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    rows = []
    for wg in (2, 3, 4, 8):
        for _ in range(3):
            tk.read_probe(buf, wg, sink, stream=s)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        for a, b in ev:
            a.record(s)
            tk.read_probe(buf, wg, sink, stream=s)
            b.record(s)
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        rows.append({"wg_per_cu": wg, "median_gbs": n / (np.median(ms) * 1e-3) / 1e9,
                     "best_gbs": n / (ms.min() * 1e-3) / 1e9})
    assert int(sink.item()) == 0
    print(json.dumps({"read_ceiling": rows, "bytes": n, "peak_gbs": HBM_PEAK_GBS}), flush=True)


def measure(args) -> dict:
    """Times `args.steps` whole queries of one configuration; returns the JSON record."""
    import numpy as np
    import torch

    import inputgen
    from inputgen import native as gen
    import paper_2601_19911_amd as tk

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 1 << args.log2n
    k = args.k
    dt = {"float32": torch.float32, "int32": torch.int32, "int64": torch.int64,
          "float64": torch.float64}[args.dtype]
    kind = {("float32", "uniform"): inputgen.KIND_U_F32, ("int32", "uniform"): inputgen.KIND_U_I32,
            ("int64", "uniform"): inputgen.KIND_U_I64, ("float32", "zipf"): inputgen.KIND_ZIPF_F32,
            ("int64", "zipf"): inputgen.KIND_ZIPF_I64, ("int32", "zipf"): inputgen.KIND_ZIPF_I32,
            ("float32", "sorted"): inputgen.KIND_SORTED_F32,
            ("int64", "sorted"): inputgen.KIND_SORTED_I64,
            ("float64", "uniform"): inputgen.KIND_U_F64}[(args.dtype, args.dist)]
    seed = inputgen.config_seed(2)
    stream = torch.cuda.current_stream()
    keys = torch.empty(n, dtype=dt, device=dev)
    rid_t = torch.uint64 if args.dtype == "int64" else torch.uint32
    rids = torch.empty(n, dtype=rid_t, device=dev)
    cdf = None
    cdf_dev = None
    if args.dist == "zipf":
        cdf = inputgen.zipf_cdf(1.1, 10 ** 6)
        cdf_dev = torch.from_numpy(cdf).to(dev)
    gen.device_fill(kind, seed, n, keys.data_ptr(), n_total=n,
                    cdf_dev_ptr=None if cdf_dev is None else cdf_dev.data_ptr(),
                    m=0 if cdf is None else len(cdf), stream=stream.cuda_stream)
    gen.device_fill(inputgen.KIND_IOTA_U64 if rid_t == torch.uint64 else inputgen.KIND_IOTA_U32,
                    0, n, rids.data_ptr(), stream=stream.cuda_stream)
    kc, rc = tk.key_code(dt), tk.rid_code(rid_t)
    k_eff = min(k, n)
    out_k = torch.empty(k_eff, dtype=dt, device=dev)
    out_r = torch.empty(k_eff, dtype=rid_t, device=dev)
    ws = tk.new_workspace(n, k, kc, rc, device=dev)
    torch.cuda.synchronize()

    def step():
        tk.topk(keys, k, rowids=rids, order=args.order, out_keys=out_k, out_rowids=out_r,
                workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    info = tk.query_info(ws)

    # timed region: exactly `steps` whole queries
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    ms_step = ms_total / args.steps

    # per-query latency distribution (each query bracketed by its own events)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    per_q = np.array([a.elapsed_time(b) for a, b in evs])

    # dominant kernel (the streaming filter), timed with event pairs on its stream
    tk.profile_begin(args.steps)
    for _ in range(args.steps):
        step()
    filt_ms, launches = tk.profile_end()
    filt_avg_ms = filt_ms / max(launches, 1)

    key_bytes = keys.element_size()
    alg_bytes = n * key_bytes  # one read of every key; survivors and outputs are < 0.01 %
    achieved = alg_bytes / (filt_avg_ms * 1e-3) / 1e9 if launches else None

    # correctness of the timed configuration, against the oracle (sampled check)
    check = None
    if not args.no_check:
        import oracle
        host_keys = keys.cpu().numpy()
        ok, orr = out_k.cpu(), out_r.view(torch.int64 if rid_t == torch.uint64 else torch.int32).cpu()
        exp_k, exp_r = oracle.topk(host_keys, None, k, oracle.DESC if args.order == "desc" else oracle.ASC,
                                   rid_dtype=np.uint64 if rid_t == torch.uint64 else np.uint32)
        check = bool(np.array_equal(ok.numpy().view(exp_k.dtype), exp_k) and
                     np.array_equal(orr.numpy().view(exp_r.dtype), exp_r))

    # CPU oracle baseline on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu:
        import oracle
        ns = 1 << min(args.log2n, 24)
        sample = inputgen.generate(kind, seed, ns, n_total=n, cdf=cdf)
        srids = np.arange(ns, dtype=np.uint64 if rid_t == torch.uint64 else np.uint32)
        reps, spent = 0, 0.0
        while spent < args.cpu_seconds and reps < 50:
            c0 = time.perf_counter()
            oracle.topk(sample, srids, k, oracle.DESC if args.order == "desc" else oracle.ASC)
            spent += time.perf_counter() - c0
            reps += 1
        cpu = {"value": ns * reps / spent, "unit": "keys/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} x oracle Top-{k} over the first 2^{int(np.log2(ns))} keys of the "
                         f"same {args.dist} {args.dtype} stream, single thread"}

    value = n / (ms_step * 1e-3)
    result = {
        "metric": "Top-K keys/s & % HBM peak at N=2^28,K=1000",
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"float32": "f32", "int32": "i32", "int64": "i64", "float64": "f64"}[args.dtype],
        "data": "synthetic",
        "config": {"workload": f"single Top-K query, N=2^{args.log2n} {args.dtype} keys "
                               f"({args.dist}) + {'uint64' if rid_t == torch.uint64 else 'uint32'} "
                               f"row-ids resident in HBM, K={k}, {args.order}",
                   "n": n, "k": k, "key_dtype": args.dtype, "distribution": args.dist,
                   "order": args.order},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic_from_profiles("k_filter"),
                     "kernel": "k_filter", "kernel_avg_ms": filt_avg_ms,
                     "alg_bytes_per_launch": alg_bytes},
        "whole_query_gbs": alg_bytes / (ms_step * 1e-3) / 1e9,
        "whole_query_frac_of_peak": alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "path": info["path"], "survivors": info["survivors"],
        "oracle_match": check,
        "query_ms_median": float(np.median(per_q)),
        "query_ms_p95": float(np.percentile(per_q, 95)),
        "wall_s_timed": wall,
        "cpu_baseline": cpu,
    }
    return result


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.read_ceiling:
        read_ceiling()
        return
    rec = measure(args)
    if args.dtype == "float32" and not args.no_f64:
        # the paper's own key type (double, sec. V-A) on the same workload, as
        # a second record inside the line
        a2 = parse([f"--log2n={args.log2n}", f"--k={args.k}", "--dtype=float64", f"--dist={args.dist}",
                    f"--order={args.order}", f"--steps={args.steps}", f"--warmup={args.warmup}",
                    "--no-cpu"] + (["--no-check"] if args.no_check else []))
        r2 = measure(a2)
        rec["float64_headline"] = {
            "workload": r2["config"]["workload"], "value": r2["value"], "unit": "keys/s",
            "ms_per_step": r2["ms_per_step"], "whole_query_frac_of_peak": r2["whole_query_frac_of_peak"],
            "kernel_frac_of_peak": r2["roofline"]["frac"], "kernel_avg_ms": r2["roofline"]["kernel_avg_ms"],
            "alg_bytes_per_launch": r2["roofline"]["alg_bytes_per_launch"], "path": r2["path"],
            "oracle_match": r2["oracle_match"]}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
