"""Parity at the benchmark workloads' full sizes, in the launch configuration
the benchmark times, on sampled minibatches the oracle can compute one by one
(needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import bh_mask, assert_forces, force_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat17():
    return I.workload_rmat17(mode="bh")


@pytest.fixture(scope="module")
def rgg64k():
    return I.workload_rgg64k()


def _pipeline(w, p, k, stop):
    """Forces of batch `stop` in iteration k (0-based), with the snapshot the
    tree of iteration k was built from and the live coordinates."""
    g = w["graph"]
    with api.Graph(g, p) as h:
        h.set_coords(w["x0"], w["y0"])
        if k > 0:
            h.run(k)
        sx, sy = h.get_coords()
        _, st, fx, fy = h.run(1, start_iter=k, stop_batch=stop)
        xs, ys = h.get_coords()
    return sx, sy, xs, ys, fx, fy, st


@pytest.mark.parametrize("stop", [0, 300, 511])
def test_rmat17_barnes_hut_pipeline(rmat17, stop):
    """131072 vertices, theta 1.2, batch 256: hub rows (batch 0), the middle,
    the last batch; iteration 2 (moved leaves and moved neighbours live)."""
    w, g = rmat17, rmat17["graph"]
    p = api.params(batch_size=256, iterations=2, mode="bh", theta=1.2)
    sx, sy, xs, ys, fx, fy, st = _pipeline(w, p, 1, stop)
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(sx, sy), stop * 256, stop * 256 + 256,
                           theta=1.2)
    r = assert_forces(fx, fy, ref, mask=bh_mask(ref), what="rmat17 bh batch %d" % stop)
    print("rmat17 bh batch", stop, r, "near ties", int(ref.near_tie.sum()))


def test_rmat17_barnes_hut_one_shot(rmat17):
    w, g = rmat17, rmat17["graph"]
    p = api.params(batch_size=256, iterations=1, mode="bh", theta=1.2)
    for b in (1, 257):
        fx, fy = api.forces(g, w["x0"], w["y0"], b, p)
        ref = oracle.forces_bh(g.rowptr, g.colidx, w["x0"], w["y0"], oracle.Tree(w["x0"], w["y0"]),
                               b * 256, b * 256 + 256, theta=1.2)
        assert_forces(fx, fy, ref, mask=bh_mask(ref), what="rmat17 one-shot batch %d" % b)


@pytest.mark.parametrize("stop", [0, 257])
def test_rmat17_exact_pipeline(rmat17, stop):
    """The same graph in exact mode (17.2e9 pairs per iteration): iteration 2."""
    w, g = rmat17, rmat17["graph"]
    p = api.params(batch_size=256, iterations=2, mode="exact")
    _, _, xs, ys, fx, fy, _ = _pipeline(w, p, 1, stop)
    ref = oracle.forces_exact(g.rowptr, g.colidx, xs, ys, stop * 256, stop * 256 + 256)
    r = assert_forces(fx, fy, ref, what="rmat17 exact batch %d" % stop)
    print("rmat17 exact batch", stop, r)


def test_rmat17_exact_persistent_run_equals_step_launches(rmat17, monkeypatch):
    """The benchmark's exact configuration (131072 vertices, batch 256) runs as
    one cooperative launch; the step-by-step launches, which the pipeline test
    above checks against the oracle, give the same bits over 3 iterations."""
    w, g = rmat17, rmat17["graph"]
    p = api.params(batch_size=256, iterations=3, mode="exact")
    xa, ya, ea, sa = api.layout(g, w["x0"], w["y0"], p)
    monkeypatch.setenv("BL_EXACT_STEPWISE", "1")
    xb, yb, eb, sb = api.layout(g, w["x0"], w["y0"], p)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)
    assert sa["iters_run"] == sb["iters_run"] == 3 and sa["nonfinite_events"] == 0


def test_rmat17_barnes_hut_benchmark_run_energies(rmat17):
    """The benchmark's Barnes-Hut configuration as timed (resident job, graph
    replay, 16 chain segments): the first two iterations' energies against the
    oracle's run from the same start (the first within 1e-4; the second within
    1e-2, as a handful of close pairs with |f| ~ 1e6 dominate the sum and FP32
    moves them slightly differently), and a repeat of the run gives the same
    bits."""
    w, g = rmat17, rmat17["graph"]
    p = api.params(batch_size=256, iterations=2, mode="bh", theta=1.2)
    with api.Graph(g, p) as h:
        h.set_coords(w["x0"], w["y0"])
        ea, _ = h.run(2)
        xa, ya = h.get_coords()
        h.set_coords(w["x0"], w["y0"])
        eb, _ = h.run(2)
        xb, yb = h.get_coords()
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)
    _, _, eo, _ = oracle.layout_bh(g.rowptr, g.colidx, w["x0"], w["y0"], 256, 2, theta=1.2)
    assert abs(ea[0] / eo[0] - 1) < 1e-4 and abs(ea[1] / eo[1] - 1) < 1e-2, (ea, eo)


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32", "fp64"])
def test_rgg64k_precision_stress(rgg64k, precision):
    """65536-vertex random geometric graph, batch 512, three precisions: the
    per-step force error against FP64 at iteration 3, batch 64."""
    w, g = rgg64k, rgg64k["graph"]
    p = api.params(batch_size=512, iterations=4, mode="exact", precision=precision)
    _, _, xs, ys, fx, fy, _ = _pipeline(w, p, 3, 64)
    ref = oracle.forces_exact(g.rowptr, g.colidx, xs, ys, 64 * 512, 65 * 512)
    r = force_errors(fx, fy, ref)
    print("rgg64k", precision, r)
    assert r["ok"], r
    if precision == "fp64":
        assert r["normwise"] < 1e-10


@pytest.mark.parametrize("b", [0, 1000, 1171])
def test_sort_above_fused_tile_limit_one_shot(b):
    """300,000 vertices (a 600 x 500 grid, random start) is above 128 sort
    tiles of 2048 keys, where the radix scatter reads scanned histogram
    offsets instead of forming them from the raw counts: one-shot forces of
    the first, a middle and the last (ragged) batch against the oracle's walk
    of its own tree, theta 1.2."""
    g = I.grid(600, 500)
    x0, y0 = I.uniform_coords(g.n, 23)
    x0, y0 = I.to_f32_representable(x0), I.to_f32_representable(y0)
    assert g.n > 128 * 2048
    p = api.params(batch_size=256, iterations=1, mode="bh", theta=1.2)
    fx, fy = api.forces(g, x0, y0, b, p)
    ref = oracle.forces_bh(g.rowptr, g.colidx, x0, y0, oracle.Tree(x0, y0), b * 256, min(b * 256 + 256, g.n),
                           theta=1.2)
    assert_forces(fx, fy, ref, mask=bh_mask(ref), what="grid 600x500 one-shot batch %d" % b)
