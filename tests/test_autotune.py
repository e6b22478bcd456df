"""Autotuner: candidate sets and the tuned-parameter cache (CPU), and that a
tuned plan stays exact (GPU)."""
import json

import numpy as np
import pytest

from paper_2601_19911_amd import autotune


def test_candidates_are_valid_plan_params():
    for kb in (4, 8):
        c = autotune.candidates(kb)
        assert len(c) >= 8
        assert len({json.dumps(x, sort_keys=True) for x in c}) == len(c)
        for p in c:
            assert p["tile_keys"] >= 1 << 14 and p["tile_keys"] & (p["tile_keys"] - 1) == 0
            assert p["sample_sigma"] > 0 and 12 <= p["max_sample_log2"] <= 24
        assert autotune.candidates(kb, quick=True)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tuned.json")
    assert autotune.cached_params("dev", "int64", path) is None
    autotune.store("dev", "int64", {"tile_keys": 32768, "sample_sigma": 3.0}, 0.01, path)
    autotune.store("dev", "float32", {"tile_keys": 65536, "sample_sigma": 2.0}, 0.02, path)
    assert autotune.cached_params("dev", "int64", path) == {"tile_keys": 32768, "sample_sigma": 3.0}
    assert autotune.cached_params("dev", "float32", path)["tile_keys"] == 65536
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}


@pytest.mark.gpu
def test_tuned_plan_is_exact(tmp_path):
    import torch

    import inputgen
    import oracle
    from paper_2601_19911_amd.batched import Plan
    from tests.gpu_util import assert_same, say, to_dev, to_np

    off, ks, orders = inputgen.batched_queries(48, seed=21, n_lo_log2=10, n_hi_log2=20, k_max=2048)
    keys = inputgen.generate(inputgen.KIND_U_I64, 21, int(off[-1]))
    kd = to_dev(keys)
    best, secs, table = autotune.tune(off, ks, orders, kd, quick=True, reps=2,
                                      cache_path=str(tmp_path / "t.json"), log=say)
    say(f"best {best} {secs * 1e3:.3f} ms")
    assert len(table) == len(autotune.candidates(8, quick=True))
    s = torch.cuda.Stream()
    plan = Plan(off, ks, orders, key_dtype=torch.int64, rid_dtype=torch.uint32, stream=s, **best)
    ok, orr = plan.alloc_outputs()
    torch.cuda.synchronize()
    plan.launch(kd, ok, orr, stream=s)
    torch.cuda.synchronize()
    okn, orn = to_np(ok), to_np(orr)
    for q in range(len(ks)):
        lo, hi = int(off[q]), int(off[q + 1])
        a, b = int(plan.out_offsets[q]), int(plan.out_offsets[q + 1])
        ek, er = oracle.topk(keys[lo:hi], None, int(ks[q]), int(orders[q]), rid_dtype=np.uint32)
        assert_same(okn[a:b], orn[a:b], ek, er, what=f"tuned q={q}")
