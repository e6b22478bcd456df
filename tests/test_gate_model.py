"""Host logic of the cost gate's measurement (paper sec. II-B): the least-squares
fit of the two cost models, the break-even N they predict, the routing rule,
and the bisection that measures the break-even; checked on synthetic timings
with a known answer."""
import numpy as np
import pytest

from paper_2601_19911_amd.gate import break_even as predicted_break_even
from paper_2601_19911_amd.gate import crossover_n, fit_costs, measured_break_even
from paper_2601_19911_amd.gate import route_gpu as gate_route_gpu

TRUE = {"cpu_a": 2.0e-10, "cpu_b": 1.0e-8, "cpu_c": 4.0e-5, "gpu_a": 1.0e-12, "gpu_b": 2.0e-8,
        "gpu_c": 6.0e-5}


def _times(n, k, c=TRUE):
    k = min(k, n)
    cpu = c["cpu_a"] * n + c["cpu_b"] * k * np.log2(k + 1.0) + c["cpu_c"]
    gpu = c["gpu_a"] * n + c["gpu_b"] * k + c["gpu_c"]
    return cpu, gpu


def _row(n, k):
    cpu, gpu = _times(n, k)
    return {"n": n, "k": k, "cpu_all_cores_s": cpu, "gpu_resident_s": gpu}


def test_fit_recovers_noise_free_models():
    rows = [_row(1 << lg, k) for k in (10, 100, 1000, 10000) for lg in range(8, 23)]
    got = fit_costs(rows)
    for key, v in TRUE.items():
        assert got[key] == pytest.approx(v, rel=1e-6, abs=1e-15), key


@pytest.mark.parametrize("k", [1, 10, 100, 1000, 10000, 100000])
@pytest.mark.parametrize("margin", [0.0, 2e-5])
def test_break_even_is_where_saving_meets_margin(k, margin):
    """On either side of N = k (the model's K is min(k, N)): the saving equals
    the margin at the predicted N*, and the gate switches there."""
    n_star = predicted_break_even(TRUE, k, margin)
    assert n_star is not None and n_star >= 1.0
    cpu, gpu = _times(n_star, k)
    if n_star > 1.0:
        assert cpu - gpu == pytest.approx(margin, abs=1e-12)
        assert not gate_route_gpu(TRUE, [n_star * 0.99], [k], margin)[0]
    assert gate_route_gpu(TRUE, [n_star * 1.01], [k], margin)[0]
    # offloaded everywhere above N*
    grid = np.geomspace(n_star * 1.01, 1 << 30, 200)
    assert gate_route_gpu(TRUE, grid, np.full(grid.shape, k), margin).all()


def test_break_even_below_k():
    """A model whose crossing lies below k: before the fix the predictor
    clamped it to 1 (it held K = k below N = k)."""
    c = dict(TRUE, cpu_b=4.0e-8, gpu_b=1.0e-8)   # large K strongly favours the GPU
    k = 10000
    n_star = predicted_break_even(c, k)
    assert 1.0 < n_star < k
    n = np.array([n_star * 0.999, n_star * 1.001])
    cpu, gpu = [np.array(x) for x in zip(*[_times(v, k, c) for v in n])]
    assert cpu[0] - gpu[0] < 0 < cpu[1] - gpu[1]


def test_break_even_with_transfer_term():
    """A host-resident column pays B = N x key bytes over the host link: the
    break-even moves up, and vanishes when the link is slower per key than the
    CPU's scan."""
    k = 100
    base = predicted_break_even(TRUE, k)
    with_b = predicted_break_even(TRUE, k, bytes_per_key=4.0, h2d_bytes_per_s=5.0e10)
    assert with_b > base
    assert predicted_break_even(TRUE, k, bytes_per_key=8.0, h2d_bytes_per_s=1.0e10) is None


def test_route_caps_k_at_n():
    # k far above n: the modelled work is n results, not k
    assert gate_route_gpu(TRUE, [4096], [10 ** 6])[0] == gate_route_gpu(TRUE, [4096], [4096])[0]


def test_margin_moves_the_break_even_up():
    a = predicted_break_even(TRUE, 100, 0.0)
    b = predicted_break_even(TRUE, 100, 1e-5)
    assert b > a
    assert b - a == pytest.approx(1e-5 / (TRUE["cpu_a"] - TRUE["gpu_a"]), rel=1e-9)


def test_no_break_even_when_cpu_never_slower_per_key():
    c = dict(TRUE, cpu_a=1e-12, gpu_a=2e-12)
    assert predicted_break_even(c, 100) is None


def test_bisection_brackets_the_true_crossover():
    k = 100
    n_true = predicted_break_even(TRUE, k)
    rows = [_row(1 << lg, k) for lg in range(8, 23)]
    assert crossover_n(rows, "gpu_resident_s") == 1 << int(np.ceil(np.log2(n_true)))
    calls = []

    def pt(n, kk):
        calls.append(n)
        return _row(n, kk)

    meas, extra = measured_break_even(pt, k, rows, steps=6)
    assert len(extra) == len(calls) == 6
    # six halvings of one octave in log N: within 2^(1/128) of the truth
    assert abs(np.log2(meas) - np.log2(n_true)) <= 1.0 / 64


def test_relative_fit_recovers_noise_free_models():
    rows = [_row(1 << lg, k) for k in (10, 100, 1000, 10000) for lg in range(10, 21)]
    got = fit_costs(rows, relative=True)
    for key, v in TRUE.items():
        assert got[key] == pytest.approx(v, rel=1e-6, abs=1e-15), key
