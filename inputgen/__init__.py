"""Seeded synthetic inputs for key-only Top-K.

This module serves both sides of every parity check: the CPU oracle and the
HIP library.  It holds no Top-K arithmetic, only the input recipes.

Every random value is output ``i`` of a SplitMix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), written
here from its published definition:

    z  = seed + (i + 1) * 0x9E3779B97F4A7C15        (mod 2^64)
    z  = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z  = (z ^ (z >> 27)) * 0x94D049BB133111EB
    h  = z ^ (z >> 31)

The stream is indexable, so any slice can be regenerated without the rest.  A C
and a HIP version of the same recipes live in ``gen.hip`` (library
``libtkgen.so``) for sizes where numpy is too slow; tests check that all three
agree bit for bit.

Recipes (the paper's workloads are a PostgreSQL table of double keys plus text
payload, sec. V-A; these synthetic inputs stand in for it):

* uniform int32 in [0, 2^31):  h >> 33
* uniform int64 over the full range:  h reinterpreted as int64
* uniform float32 in [0, 1):  (h >> 40) * 2^-24   (a 2^-24 grid)
* Zipf(s) over ranks 1..m:  u = (h >> 11) * 2^-53, rank = 1 + #{r : cdf[r] <= u}
  with cdf the float64 running sum of r^-s divided by its last entry
* presorted float32:  floor(i * 2^24 / n) * 2^-24
* presorted int64:    floor(i * 2^24 / n) - 2^23
* float64 payload in [0, 1):  (h >> 11) * 2^-53
* join probe keys (foreign keys into a build side generated as uniform int32 or
  int64 with the same seed):  key_j = build recipe at index (h'_j mod R), with
  h' the stream of seed + 1 and R = n_total.  Index i < n_build is a hit on
  build row i; for int64 an index i >= n_build gives a key that no build row
  holds (SplitMix64 outputs of distinct indices are distinct), so the hit rate
  is n_build / R in expectation.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 260119911

# generator kinds, shared with gen.hip (same numbering)
KIND_U_I32 = 0
KIND_U_I64 = 1
KIND_U_F32 = 2
KIND_ZIPF_I64 = 3
KIND_ZIPF_F32 = 4
KIND_SORTED_F32 = 5
KIND_SORTED_I64 = 6
KIND_IOTA_U32 = 7
KIND_IOTA_U64 = 8
KIND_PAYLOAD_F64 = 9
KIND_ZIPF_I32 = 10
KIND_JOIN_FK_I32 = 11
KIND_JOIN_FK_I64 = 12
KIND_U_F64 = KIND_PAYLOAD_F64  # uniform float64 keys in [0, 1): the same 2^-53 grid

KIND_DTYPE = {
    KIND_U_I32: np.int32,
    KIND_U_I64: np.int64,
    KIND_U_F32: np.float32,
    KIND_ZIPF_I64: np.int64,
    KIND_ZIPF_F32: np.float32,
    KIND_SORTED_F32: np.float32,
    KIND_SORTED_I64: np.int64,
    KIND_IOTA_U32: np.uint32,
    KIND_IOTA_U64: np.uint64,
    KIND_PAYLOAD_F64: np.float64,
    KIND_ZIPF_I32: np.int32,
    KIND_JOIN_FK_I32: np.int32,
    KIND_JOIN_FK_I64: np.int64,
}


def config_seed(config: int, variant: int = 0) -> int:
    """Seed of workload ``config`` (1-based) and variant ``variant``."""
    return BASE_SEED + 100 * config + variant


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream of ``seed``."""
    i = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + (i + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
    return z ^ (z >> np.uint64(31))


def zipf_cdf(s: float, m: int) -> np.ndarray:
    """float64 cumulative table of the Zipf(s) law truncated to ranks 1..m.

    Built once here and handed to the C/HIP generators, so every side uses the
    very same table.  The last entry is exactly 1.0.
    """
    w = np.arange(1, m + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    return c / c[-1]


def _unit53(h: np.ndarray) -> np.ndarray:
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def generate(kind: int, seed: int, n: int, start: int = 0, n_total: int | None = None,
             cdf: np.ndarray | None = None) -> np.ndarray:
    """Elements ``start .. start+n-1`` of input ``kind``.

    ``n_total`` is the full column length (presorted recipes depend on it);
    ``cdf`` is the Zipf table from :func:`zipf_cdf` for the Zipf kinds.
    """
    if n_total is None:
        n_total = start + n
    if kind in (KIND_SORTED_F32, KIND_SORTED_I64, KIND_IOTA_U32, KIND_IOTA_U64):
        i = np.arange(start, start + n, dtype=np.uint64)
        if kind == KIND_IOTA_U32:
            return i.astype(np.uint32)
        if kind == KIND_IOTA_U64:
            return i
        # floor(i * 2^24 / n_total) without overflow: i < 2^40 in every workload
        g = (i << np.uint64(24)) // np.uint64(n_total)
        if kind == KIND_SORTED_F32:
            return (g.astype(np.float32) * np.float32(2.0 ** -24)).astype(np.float32)
        return g.astype(np.int64) - np.int64(1 << 23)
    h = splitmix64(seed, start, n)
    if kind == KIND_U_I32:
        return (h >> np.uint64(33)).astype(np.int32)
    if kind == KIND_U_I64:
        return h.view(np.int64)
    if kind == KIND_U_F32:
        return ((h >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)).astype(np.float32)
    if kind == KIND_PAYLOAD_F64:
        return _unit53(h)
    if kind in (KIND_JOIN_FK_I32, KIND_JOIN_FK_I64):
        idx = splitmix64(seed + 1, start, n) % np.uint64(n_total)
        with np.errstate(over="ignore"):
            z = np.uint64(seed % (1 << 64)) + (idx + np.uint64(1)) * GAMMA
            z = (z ^ (z >> np.uint64(30))) * MIX1
            z = (z ^ (z >> np.uint64(27))) * MIX2
        hb = z ^ (z >> np.uint64(31))
        if kind == KIND_JOIN_FK_I32:
            return (hb >> np.uint64(33)).astype(np.int32)
        return hb.view(np.int64)
    if kind in (KIND_ZIPF_I64, KIND_ZIPF_F32, KIND_ZIPF_I32):
        if cdf is None:
            raise ValueError("Zipf kinds need the cdf table")
        u = _unit53(h)
        r = np.searchsorted(cdf, u, side="right").astype(np.int64) + 1
        if kind == KIND_ZIPF_I64:
            return r
        if kind == KIND_ZIPF_I32:
            return r.astype(np.int32)
        return r.astype(np.float32)
    raise ValueError(f"unknown generator kind {kind}")


# ---- workload shapes ------------------------------------------------------------------------

def batched_queries(q: int = 4096, seed: int | None = None, n_lo_log2: float = 10.0,
                    n_hi_log2: float = 24.0, k_max: int = 4096):
    """Per-query sizes of the batched workload: Q independent Top-K queries.

    N_q = floor(2^(lo + (hi-lo) u)) and K_q = min(N_q, k_max, floor((k_max+1)^v)),
    u and v from stream (seed, 2q) and (seed, 2q+1); half of the queries are
    ascending and half descending, assigned by a seeded shuffle.  Returns
    (offsets uint64[Q+1], ks uint32[Q], orders uint8[Q]).
    """
    if seed is None:
        seed = config_seed(3)
    h = splitmix64(seed, 0, 2 * q)
    u = _unit53(h[0::2])
    v = _unit53(h[1::2])
    n = np.floor(2.0 ** (n_lo_log2 + (n_hi_log2 - n_lo_log2) * u)).astype(np.uint64)
    k = np.minimum(np.floor(float(k_max + 1) ** v), float(k_max)).astype(np.uint64)
    k = np.minimum(np.maximum(k, 1), n).astype(np.uint32)
    orders = np.zeros(q, dtype=np.uint8)
    orders[: q // 2] = 1
    perm_keys = splitmix64(seed + 1, 0, q)
    orders = orders[np.argsort(perm_keys, kind="stable")]
    offsets = np.zeros(q + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(n, dtype=np.uint64)
    return offsets, k, orders


def serving_requests(count: int, seed: int | None = None, col_len: int = 1 << 28):
    """Request mix of the serving workload.

    N: 70 % log-uniform in [2^12, 2^16], 25 % log-uniform in [2^18, 2^22], 5 % at
    2^26; K uniform over {10, 100, 1000, 10000} capped at N; offset uniform in
    [0, col_len - N].  Returns a dict of numpy arrays (n, k, offset, u_col, u_arr)
    where u_col and u_arr are uniforms the caller maps to a column and an arrival.
    """
    if seed is None:
        seed = config_seed(5)
    h = splitmix64(seed, 0, 6 * count).reshape(count, 6)
    u = _unit53(h.reshape(-1)).reshape(count, 6)
    mix = u[:, 0]
    ln = np.where(mix < 0.70, 12.0 + 4.0 * u[:, 1], np.where(mix < 0.95, 18.0 + 4.0 * u[:, 1], 26.0))
    n = np.floor(2.0 ** ln).astype(np.uint64)
    kk = np.array([10, 100, 1000, 10000], dtype=np.uint64)[np.minimum((u[:, 2] * 4).astype(np.int64), 3)]
    k = np.minimum(kk, n)
    off = np.floor(u[:, 3] * (col_len - n + 1).astype(np.float64)).astype(np.uint64)
    off = np.minimum(off, np.uint64(col_len) - n)
    return {"n": n, "k": k, "offset": off, "u_col": u[:, 4], "u_arr": u[:, 5]}
