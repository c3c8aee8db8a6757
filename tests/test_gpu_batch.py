"""Many graphs in one call: each result equals the graph's own single-graph
run bitwise (needs an MI355X)."""
import numpy as np
import pytest

from paper_2002_08233_amd import api, inputs as I

pytestmark = pytest.mark.gpu


def _job(kind, n, seed, mode, iters, bs=64, theta=1.0, precision="fp32_kahan", lit=True):
    g = I.erdos_renyi(n, 8.0, seed) if kind == "er" else I.barabasi_albert(n, 4, seed)
    x, y = I.uniform_coords(g.n, seed + 7)
    p = api.params(batch_size=bs, iterations=iters, mode=mode, theta=theta, precision=precision,
                   repulse_adjacent=lit)
    return g, I.to_f32_representable(x), I.to_f32_representable(y), p


def test_mixed_batch_matches_single_runs_bitwise():
    jobs = [
        _job("er", 300, 1, "exact", 12),
        _job("ba", 777, 2, "exact", 9, bs=128),
        _job("er", 1500, 3, "exact", 5, precision="fp64"),
        _job("ba", 640, 4, "exact", 7, lit=False),
        _job("er", 5000, 5, "bh", 6, bs=128, theta=1.0),
        _job("ba", 7000, 6, "bh", 4, bs=256, theta=1.2),
        _job("er", 4500, 7, "bh", 9, bs=100, theta=0.8),
        _job("ba", 9000, 8, "exact", 2, bs=512),      # larger than one workgroup's share
        _job("er", 3000, 9, "exact", 4, bs=128),      # one workgroup in the batch, step kernels alone
    ]
    outs, stats = api.layout_batch([j[0] for j in jobs], [j[1] for j in jobs], [j[2] for j in jobs],
                                   [j[3] for j in jobs])
    for (g, x0, y0, p), (xb, yb), st in zip(jobs, outs, stats):
        xs, ys, es, sts = api.layout(g, x0, y0, p)
        assert np.array_equal(xb, xs) and np.array_equal(yb, ys), (g.n, p.mode)
        assert st["iters_run"] == p.iterations
        assert st["energy_last"] == es[-1]


def test_batch_twice_is_reproducible_and_empty_is_ok():
    jobs = [_job("er", 400 + 50 * q, 20 + q, "exact" if q % 2 else "bh", 3, theta=1.0) for q in range(6)]
    a, _ = api.layout_batch([j[0] for j in jobs], [j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs])
    b, _ = api.layout_batch([j[0] for j in jobs], [j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs])
    for (xa, ya), (xb, yb) in zip(a, b):
        assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert api.layout_batch([], [], [], []) == ([], [])


def test_batch_with_energy_stopping_rule():
    """conv_tol per graph in a batch (one-workgroup exact, step-kernel exact,
    Barnes-Hut engine): each graph stops where it stops alone, with the same
    bits."""
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from _parity import stop_tolerance
    jobs = [_job("er", 600, 41, "exact", 12, bs=64), _job("ba", 9000, 42, "exact", 10, bs=512),
            _job("er", 5000, 43, "bh", 12, bs=128), _job("ba", 700, 44, "exact", 12, bs=32)]
    for g, x0, y0, p in jobs:
        p.step0, p.step_decay = 0.05, 0.97
        _, _, ef, _ = api.layout(g, x0, y0, p)
        p.conv_tol = stop_tolerance(ef)[0]
    outs, stats = api.layout_batch([j[0] for j in jobs], [j[1] for j in jobs], [j[2] for j in jobs],
                                   [j[3] for j in jobs])
    stopped = 0
    for (g, x0, y0, p), (xb, yb), st in zip(jobs, outs, stats):
        xs, ys, es, sts = api.layout(g, x0, y0, p)
        assert np.array_equal(xb, xs) and np.array_equal(yb, ys), (g.n, p.mode)
        assert st["iters_run"] == sts["iters_run"] == len(es)
        stopped += st["iters_run"] < p.iterations
    assert stopped == len(jobs)
