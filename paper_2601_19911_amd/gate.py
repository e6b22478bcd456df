"""Calibration of the cost gate (paper sec. II-B; the fit and break-even
validation of sec. V-D), host-side arithmetic only.

The gate offloads a request when C_cpu - C_gpu exceeds a margin, with the
two cost models of the served form (K = min(k, N), seconds):

    C_cpu = cpu_a N + cpu_b K log2(K + 1) + cpu_c
    C_gpu = gpu_a N + gpu_b K + gpu_c            (+ B / link rate, host-resident)

``fit_costs`` fits them by least squares to measured times, ``break_even``
solves the models for the smallest N from which offloading saves more than
the margin, ``route_gpu`` is the gate's decision, and ``measured_break_even``
brackets the measured crossover by bisection.  The library's request loop
evaluates the same rule in C++ (tk_server_submit); these functions produce
and check its coefficients.
"""

from __future__ import annotations

import numpy as np

FIELDS = ("cpu_a", "cpu_b", "cpu_c", "gpu_a", "gpu_b", "gpu_c")


def fit_costs(rows, relative=False):
    """Least-squares cost models from rows {n, k, cpu_all_cores_s, gpu_resident_s}.
    relative: residuals taken relative to the measured time, so that the
    small-N points near the break-even weigh as much as the large ones."""
    N = np.array([r["n"] for r in rows], dtype=np.float64)
    K = np.array([min(r["k"], r["n"]) for r in rows], dtype=np.float64)
    cpu = np.array([r["cpu_all_cores_s"] for r in rows])
    gpu = np.array([r["gpu_resident_s"] for r in rows])
    wc = 1.0 / cpu if relative else np.ones_like(cpu)
    wg = 1.0 / gpu if relative else np.ones_like(gpu)
    A = np.stack([N, K * np.log2(K + 1), np.ones_like(N)], 1)
    ca = np.linalg.lstsq(A * wc[:, None], cpu * wc, rcond=None)[0]
    B = np.stack([N, K, np.ones_like(N)], 1)
    ga = np.linalg.lstsq(B * wg[:, None], gpu * wg, rcond=None)[0]
    return {"cpu_a": float(ca[0]), "cpu_b": float(ca[1]), "cpu_c": float(ca[2]),
            "gpu_a": float(ga[0]), "gpu_b": float(ga[1]), "gpu_c": float(ga[2])}


def saving(cost, n, k, bytes_per_key=0.0, h2d_bytes_per_s=5.0e10):
    """C_cpu - C_gpu for requests (n, k), K = min(k, n); bytes_per_key > 0
    adds the host-link transfer of a host-resident column to C_gpu."""
    n = np.asarray(n, dtype=np.float64)
    k = np.minimum(np.asarray(k, dtype=np.float64), n)
    c_cpu = cost["cpu_a"] * n + cost["cpu_b"] * k * np.log2(k + 1.0) + cost["cpu_c"]
    c_gpu = cost["gpu_a"] * n + cost["gpu_b"] * k + cost["gpu_c"] + n * bytes_per_key / h2d_bytes_per_s
    return c_cpu - c_gpu


def route_gpu(cost, n, k, margin_s=0.0, bytes_per_key=0.0, h2d_bytes_per_s=5.0e10):
    """The gate's decision for requests (n, k): True where offloaded."""
    return saving(cost, n, k, bytes_per_key, h2d_bytes_per_s) > margin_s


def break_even(cost, k, margin_s=0.0, bytes_per_key=0.0, h2d_bytes_per_s=5.0e10, n_max=2.0 ** 40):
    """The smallest N from which the modelled saving stays above the margin
    (real-valued; None if it never does up to n_max).

    The models depend on N through K = min(k, N), so the saving is piecewise:
    for N >= k it is linear in N (slope cpu_a - gpu_a - transfer per key),
    for N < k both sides carry the K terms at K = N.  Above k the linear
    solution is exact; when the crossing lies below k it is found by
    bisection on the last interval where the saving is at most the margin."""
    kw = dict(bytes_per_key=bytes_per_key, h2d_bytes_per_s=h2d_bytes_per_s)
    slope = cost["cpu_a"] - cost["gpu_a"] - bytes_per_key / h2d_bytes_per_s
    k = float(k)
    above = float(saving(cost, k, k, **kw)) > margin_s  # at N = k
    if not above:
        if slope <= 0:
            return None
        # linear on [k, inf): saving(N) = saving(k) + slope (N - k)
        n = k + (margin_s - float(saving(cost, k, k, **kw))) / slope
        return n if n <= n_max else None
    if slope < 0:
        return None  # it falls below the margin again somewhere past k
    # the saving exceeds the margin at N = k: look below k for the last point
    # where it does not (on a log grid), then bisect that interval
    grid = np.unique(np.concatenate([np.geomspace(1.0, k, 4096), [k]]))
    s = saving(cost, grid, k, **kw) - margin_s
    bad = np.flatnonzero(s <= 0)
    if bad.size == 0:
        return 1.0
    lo, hi = float(grid[bad[-1]]), float(grid[bad[-1] + 1])
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if float(saving(cost, mid, k, **kw)) > margin_s:
            hi = mid
        else:
            lo = mid
    return hi


def crossover_n(rows, key):
    """Smallest N from which the GPU time (rows[key]) stays below the CPU time."""
    rows = sorted(rows, key=lambda r: r["n"])
    best = None
    for r in reversed(rows):
        if r[key] < r["cpu_all_cores_s"]:
            best = r["n"]
        else:
            break
    return best


def measured_break_even(pt, k, rows, steps, key="gpu_resident_s"):
    """Smallest N from which the GPU route beats the CPU route: the
    bracketing pair of the power-of-two sweep, then `steps` bisections in
    log N (each midpoint measured by pt(n, k) like the sweep)."""
    rows = sorted(rows, key=lambda r: r["n"])
    hi = crossover_n(rows, key)
    if hi is None or hi == rows[0]["n"]:
        return hi, []
    lo = hi // 2
    extra = []
    for _ in range(steps):
        mid = int(round(np.sqrt(float(lo) * float(hi))))
        if mid <= lo or mid >= hi:
            break
        r = pt(mid, k)
        extra.append(r)
        if r[key] < r["cpu_all_cores_s"]:
            hi = mid
        else:
            lo = mid
    return float(np.sqrt(float(lo) * float(hi))), extra
