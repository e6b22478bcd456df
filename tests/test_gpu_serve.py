"""Served form: every request's result equals the oracle (and tk_topk) on the
same rows, alone or in the mix, through either route of the gate."""
import numpy as np
import pytest

import inputgen
import oracle
from tests.gpu_util import assert_same, say, to_dev

pytestmark = pytest.mark.gpu

ENGINE_STALL = ("these cases ran the served form's GPU route on the persistent batch engine, which "
                "did not complete on the GPU (cause not shown) and was removed; they stay "
                "skipped, and the route on multi-query launches is covered by the *_multi tests")

import paper_2601_19911_amd as tk
from paper_2601_19911_amd.serve import GATE_COST, GATE_CPU, GATE_GPU, Server


def _columns(n):
    cols = []
    for kind, seed in ((inputgen.KIND_U_I32, 1), (inputgen.KIND_U_I64, 2), (inputgen.KIND_U_F32, 3)):
        h = inputgen.generate(kind, seed, n)
        cols.append((to_dev(h), h))
    return cols


def _requests(rng, count, n_col):
    reqs = []
    for _ in range(count):
        col = int(rng.integers(0, 3))
        n = int(2 ** rng.uniform(10, 20))
        off = int(rng.integers(0, n_col - n))
        k = int(rng.choice([1, 10, 100, 1000, 10000]))
        reqs.append((col, off, n, k, int(rng.integers(0, 2))))
    return reqs


def _expect(host_cols, col, off, n, k, order):
    keys = host_cols[col][off:off + n]
    ek, er = oracle.topk(keys, None, k, order, rid_dtype=np.uint64)
    return ek, er + np.uint64(off)


@pytest.mark.parametrize("gate", [pytest.param(GATE_GPU, marks=pytest.mark.skip(reason=ENGINE_STALL)),
                                  pytest.param(GATE_COST, marks=pytest.mark.skip(reason=ENGINE_STALL)),
                                  GATE_CPU])
def test_served_results_match_oracle(gate):
    _served_vs_oracle(gate, seed=gate + 7)


def _served_vs_oracle(gate, seed, count=120, slots=2, max_batch=64):
    import torch
    ncol = 1 << 21
    cols = _columns(ncol)
    host = [h for _, h in cols]
    cost = {"cpu_a": 2e-9, "cpu_b": 5e-9, "cpu_c": 5e-6, "gpu_a": 2e-10, "gpu_b": 1e-9,
            "gpu_c": 60e-6}
    srv = Server(arena_bytes=512 << 20, max_batch=max_batch, slots=slots, gate=gate, cost=cost)
    ids = [srv.add_column(d, h) for d, h in cols]
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    reqs = _requests(rng, count, ncol)
    say(f"serving {len(reqs)} requests, gate={gate}")
    rid = [srv.submit(ids[c], off, n, k, o) for (c, off, n, k, o) in reqs]
    srv.drain()
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(reqs)
    routes = []
    for (c, off, n, k, o), r in zip(reqs, rid):
        got = srv.result(r, c, min(k, n))
        assert got is not None
        ok, orr, info = got
        routes.append(info.route)
        ek, er = _expect(host, c, off, n, k, o)
        assert_same(ok, orr, ek, er, what=f"served col={c} off={off} n={n} k={k} o={o} route={info.route}")
    if gate == GATE_CPU:
        assert all(r == 1 for r in routes)
    if gate == GATE_GPU:
        assert all(r == 0 for r in routes)
    srv.close()


@pytest.mark.skip(reason=ENGINE_STALL)
def test_served_same_alone_and_in_mix():
    """A request gives the same result submitted alone and inside a busy mix."""
    _alone_and_in_mix(seed=3)


def test_served_gpu_route_multi():
    _served_vs_oracle(GATE_GPU, seed=101, count=150, slots=2, max_batch=48)


def test_served_cost_gate_multi():
    _served_vs_oracle(GATE_COST, seed=103, count=150, slots=3, max_batch=32)


def test_served_same_alone_and_in_mix_multi():
    """A request gives the same result submitted alone and inside a busy mix."""
    _alone_and_in_mix(seed=105)


def _alone_and_in_mix(seed):
    import torch
    ncol = 1 << 22
    cols = _columns(ncol)
    host = [h for _, h in cols]
    srv = Server(arena_bytes=512 << 20, max_batch=32, slots=3, gate=GATE_GPU)
    ids = [srv.add_column(d, h) for d, h in cols]
    probe = (1, 12345, 1 << 21, 1000, 0)
    alone = srv.submit(ids[probe[0]], *probe[1:])
    srv.drain()
    a = srv.result(alone, probe[0], 1000)
    rng = np.random.default_rng(seed)
    mix = _requests(rng, 200, ncol)
    rids = [srv.submit(ids[c], off, n, k, o) for (c, off, n, k, o) in mix[:100]]
    inmix = srv.submit(ids[probe[0]], *probe[1:])
    rids += [srv.submit(ids[c], off, n, k, o) for (c, off, n, k, o) in mix[100:]]
    srv.drain()
    b = srv.result(inmix, probe[0], 1000)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ek, er = _expect(host, *probe)
    assert_same(a[0], a[1], ek, er, what="alone")
    assert srv.stats()["batches"] >= 2
    srv.close()


@pytest.mark.parametrize("margin_us", [0.0, 40.0])
def test_gate_routes_follow_cost_model(margin_us):
    """The gate offloads exactly the requests whose modelled saving,
    C_cpu - C_gpu at K = min(k, N), exceeds the margin (paper sec. II-B), and
    either route returns the oracle's result."""
    import torch
    from paper_2601_19911_amd.gate import route_gpu as gate_route_gpu
    ncol = 1 << 20
    cols = _columns(ncol)
    host = [h for _, h in cols]
    cost = {"cpu_a": 1.8e-10, "cpu_b": 1.3e-8, "cpu_c": 4.4e-5, "gpu_a": 0.0, "gpu_b": 1.5e-8,
            "gpu_c": 5.3e-5}
    srv = Server(arena_bytes=256 << 20, max_batch=32, slots=2, gate=GATE_COST, margin_ms=margin_us * 1e-3,
                 cost=cost)
    ids = [srv.add_column(d, h) for d, h in cols]
    torch.cuda.synchronize()
    rng = np.random.default_rng(11 + int(margin_us))
    reqs = []
    for _ in range(160):
        n = int(2 ** rng.uniform(8, 20))
        reqs.append((int(rng.integers(0, 3)), int(rng.integers(0, ncol - n + 1)), n,
                     int(rng.choice([1, 10, 100, 1000, 10000])), int(rng.integers(0, 2))))
    want_gpu = gate_route_gpu(cost, [r[2] for r in reqs], [r[3] for r in reqs], margin_us * 1e-6)
    say(f"gate margin {margin_us} us: {int(want_gpu.sum())} of {len(reqs)} requests modelled to offload")
    rid = [srv.submit(ids[c], off, n, k, o) for (c, off, n, k, o) in reqs]
    srv.drain()
    for i, ((c, off, n, k, o), r) in enumerate(zip(reqs, rid)):
        ok, orr, info = srv.result(r, c, min(k, n))
        assert info.route == (0 if want_gpu[i] else 1), f"request n={n} k={k} routed {info.route}"
        ek, er = _expect(host, c, off, n, k, o)
        assert_same(ok, orr, ek, er, what=f"gated n={n} k={k} o={o} route={info.route}")
    assert 0 < int(want_gpu.sum()) < len(reqs)
    srv.close()


@pytest.mark.parametrize("gate", [GATE_GPU, GATE_CPU])
def test_served_float64_column(gate):
    """A float64 column (the paper's key type) through either route of the
    served form; every request equals the oracle on its rows."""
    import torch
    ncol = 1 << 20
    h = inputgen.generate(inputgen.KIND_U_F64, 21, ncol)
    h[::997] = -h[::997]  # both signs
    srv = Server(arena_bytes=256 << 20, max_batch=32, slots=2, gate=gate)
    cid = srv.add_column(to_dev(h), h)
    torch.cuda.synchronize()
    rng = np.random.default_rng(23)
    reqs = []
    for _ in range(60):
        n = int(2 ** rng.uniform(8, 20))
        reqs.append((int(rng.integers(0, ncol - n + 1)), n, int(rng.choice([1, 10, 100, 1000, 10000])),
                     int(rng.integers(0, 2))))
    rid = [srv.submit(cid, off, n, k, o) for (off, n, k, o) in reqs]
    srv.drain()
    for (off, n, k, o), r in zip(reqs, rid):
        ok, orr, info = srv.result(r, 0, min(k, n))
        assert info.route == (0 if gate == GATE_GPU else 1)
        ek, er = oracle.topk(h[off:off + n], None, k, o, rid_dtype=np.uint64)
        assert_same(ok, orr, ek, er + np.uint64(off), what=f"float64 served n={n} k={k} o={o}")
    srv.close()


def test_oversize_request_on_gpu_only_column_fails_cleanly():
    """A request larger than a slot, on a column with no host copy and at an
    offset > 0 (where a CPU route would read an invalid host address), comes
    back with TK_ENOMEM and no results; the requests around it are served and
    equal the oracle; every request is released once taken."""
    import torch
    ncol = 1 << 22
    h = inputgen.generate(inputgen.KIND_U_I32, 5, ncol)
    srv = Server(arena_bytes=8 << 20, max_batch=8, slots=2, gate=GATE_GPU)  # 4 MiB per slot
    cid = srv.add_column(to_dev(h))  # device copy only
    torch.cuda.synchronize()
    # K = 10^6 of 3 * 2^20 rows: 12 MB of results alone, past the slot's 4 MiB
    big = (12345, 3 << 20, 1_000_000, 0)
    small = [(int(o), 1 << 16, 10, int(o) & 1) for o in np.linspace(7, ncol - (1 << 16), 12)]
    ids = [srv.submit(cid, *small[i]) for i in range(6)]
    bid = srv.submit(cid, *big)
    ids += [srv.submit(cid, *small[i]) for i in range(6, 12)]
    srv.drain()
    st = srv.stats()
    say(f"oversize: {st}")
    assert st["failed"] == 1 and st["completed"] == 13 and st["live"] == 13
    rc, info = srv.result_status(bid, cid, big[2])
    assert rc == tk.TK_ENOMEM and info.status == tk.TK_ENOMEM and info.count == 0
    for (off, n, k, o), r in zip(small, ids):
        ok, orr, info = srv.result(r, cid, min(k, n))
        assert info.route == 0
        ek, er = oracle.topk(h[off:off + n], None, k, o, rid_dtype=np.uint64)
        assert_same(ok, orr, ek, er + np.uint64(off), what=f"small off={off} n={n} k={k} o={o}")
    assert srv.stats()["live"] == 0
    srv.close()


def test_served_host_resident_column_and_transfer_gate():
    """A column held only in pinned host memory: the GPU route copies each
    request's rows into the slot's arena.  With the cost gate the routing
    follows the models with the transfer term B = N x key bytes (paper
    sec. II-B); either route equals the oracle."""
    import torch
    from paper_2601_19911_amd.gate import route_gpu
    ncol = 1 << 22
    h = inputgen.generate(inputgen.KIND_U_I64, 31, ncol)
    pinned = torch.from_numpy(h).pin_memory()
    cost = {"cpu_a": 1.0e-9, "cpu_b": 1.3e-8, "cpu_c": 4.4e-5, "gpu_a": 0.0, "gpu_b": 1.5e-8,
            "gpu_c": 5.3e-5}
    h2d = 2.0e10
    rng = np.random.default_rng(41)
    reqs = []
    for _ in range(80):
        n = int(2 ** rng.uniform(10, 21))
        reqs.append((int(rng.integers(0, ncol - n + 1)), n, int(rng.choice([10, 100, 1000])),
                     int(rng.integers(0, 2))))
    for gate in (GATE_GPU, GATE_COST):
        srv = Server(arena_bytes=256 << 20, max_batch=16, slots=2, gate=gate, cost=cost,
                     h2d_bytes_per_s=h2d)
        cid = srv.add_column(None, pinned)  # host-resident: no device copy
        rid = [srv.submit(cid, *r) for r in reqs]
        srv.drain()
        want = route_gpu(cost, [r[1] for r in reqs], [r[2] for r in reqs], 0.0,
                         bytes_per_key=8.0, h2d_bytes_per_s=h2d)
        if gate == GATE_COST:
            say(f"host-resident column: {int(want.sum())} of {len(reqs)} modelled to offload")
            assert 0 < int(want.sum()) < len(reqs)
        for i, ((off, n, k, o), r) in enumerate(zip(reqs, rid)):
            ok, orr, info = srv.result(r, cid, min(k, n))
            assert info.route == (0 if (gate == GATE_GPU or want[i]) else 1)
            ek, er = oracle.topk(h[off:off + n], None, k, o, rid_dtype=np.uint64)
            assert_same(ok, orr, ek, er + np.uint64(off), what=f"host column n={n} k={k} o={o} gate={gate}")
        assert srv.stats()["live"] == 0
        srv.close()
