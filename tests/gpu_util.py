"""Helpers for the GPU parity tests: move numpy inputs to the device, run the
library through its C ABI, and compare with the oracle bit for bit."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def torch_mod():
    import torch
    return torch


def to_dev(a: np.ndarray):
    torch = torch_mod()
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda().view(torch.uint32)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda().view(torch.uint64)
    return torch.from_numpy(a).cuda()


def to_np(t) -> np.ndarray:
    torch = torch_mod()
    if t.dtype == torch.uint32:
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    if t.dtype == torch.uint64:
        return t.view(torch.int64).cpu().numpy().view(np.uint64)
    return t.cpu().numpy()


def bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same(got_keys, got_rids, exp_keys, exp_rids, what=""):
    assert got_keys.shape == exp_keys.shape, f"{what}: {got_keys.shape} vs {exp_keys.shape}"
    bad = np.flatnonzero((bits(got_keys) != bits(exp_keys)) |
                         (got_rids.astype(np.uint64) != exp_rids.astype(np.uint64)))
    if bad.size:
        j = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {j}: got ({got_keys[j]!r}, "
                             f"{int(got_rids[j])}) expected ({exp_keys[j]!r}, {int(exp_rids[j])})")


def order_code(order: str) -> int:
    return oracle.DESC if order == "desc" else oracle.ASC
