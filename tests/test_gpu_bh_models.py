"""(a, r)-energy models of Sec. 2.2 other than (2, -1) in Barnes-Hut mode and
on the batched and served paths: the HIP path against the FP64 oracle (needs
an MI355X).

Barnes-Hut under a general model: an accepted cell adds count times the
repulsion d^(r-1) (c - c_i) at its centroid (reading R13 carried over), the
attraction along edges is d^(a-1) (c_j - c_i) / K.  The oracle's walk is the
same (pinned on the CPU by theta = 0 against exact forces and the two-vertex
closed form for each model)."""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import RUN_TOL, SETTLING, assert_forces, bh_mask, near_grid_init, quality

pytestmark = pytest.mark.gpu

MODELS = [(1, -1), (0, -1), (3, 0), (2, -2)]


@pytest.fixture(scope="module")
def rmat14():
    g = I.rmat(14, 16, seed=41)
    x, y = I.uniform_coords(g.n, 42)
    return g, I.to_f32_representable(x), I.to_f32_representable(y)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("stop", [0, 37, 63])
def test_rmat14_pipeline_forces(rmat14, model, stop):
    """RMAT scale 14 (16384 vertices, hub rows in batch 0), theta 1.2, batch
    256: forces of batch `stop` in iteration 2 (moved leaves and neighbours
    live) against the oracle's walk on the same tree and coordinates."""
    g, x0, y0 = rmat14
    p = api.params(batch_size=256, iterations=2, mode="bh", theta=1.2, model=model)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        h.run(1)
        sx, sy = h.get_coords()
        _, st, fx, fy = h.run(1, start_iter=1, stop_batch=stop)
        xs, ys = h.get_coords()
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(sx, sy), stop * 256, stop * 256 + 256,
                           theta=1.2, model=model)
    assert_forces(fx, fy, ref, mask=bh_mask(ref), what="model %s batch %d" % (model, stop))


@pytest.mark.parametrize("model", MODELS)
def test_theta_zero_equals_exact(model):
    """theta = 0 opens every cell: the Barnes-Hut forces are the exact ones."""
    g = I.erdos_renyi(900, 6.0, 43)
    x, y = I.uniform_coords(g.n, 44)
    x, y = I.to_f32_representable(x), I.to_f32_representable(y)
    p = api.params(batch_size=128, iterations=1, mode="bh", theta=0.0, model=model)
    for b in (0, 7):
        fx, fy = api.forces(g, x, y, b, p)
        ref = oracle.forces_exact(g.rowptr, g.colidx, x, y, 128 * b, min(128 * b + 128, g.n), model=model)
        assert_forces(fx, fy, ref, what="theta 0 model %s batch %d" % (model, b))


@pytest.mark.parametrize("model", [(1, -1), (0, -1), (3, 0)])
def test_one_shot_forces_ragged(model):
    """700 vertices, batch 96 (ragged last batch), theta 0.8, buckets of
    coincident points."""
    g = I.erdos_renyi(700, 8.0, 45)
    x, y = I.uniform_coords(g.n, 46)
    x[600:610] = x[600]
    y[600:610] = y[600]
    x, y = I.to_f32_representable(x), I.to_f32_representable(y)
    p = api.params(batch_size=96, iterations=1, mode="bh", theta=0.8, model=model)
    for b in (0, 6, 7):
        fx, fy = api.forces(g, x, y, b, p)
        ref = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), 96 * b, min(96 * b + 96, g.n),
                               theta=0.8, model=model)
        assert_forces(fx, fy, ref, mask=bh_mask(ref), what="one-shot model %s batch %d" % (model, b))


@pytest.mark.parametrize("model", [(1, -1), (0, -1), (3, 0)])
def test_settling_run(model):
    """32x32 grid from a near-grid start, theta 1.2, 60 iterations on a
    settling schedule: stress and edge energy within 1% of the oracle's run."""
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    xo, yo, eo, _ = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, 128, 60, step0=SETTLING["step0"],
                                     decay=SETTLING["step_decay"], theta=1.2, model=model)
    qo = quality(oracle, g, xo, yo)
    p = api.params(batch_size=128, iterations=60, mode="bh", theta=1.2, model=model, **SETTLING)
    xg, yg, eg, st = api.layout(g, x0, y0, p)
    qg = quality(oracle, g, xg, yg)
    print("model", model, "stress, edge energy gpu", qg, "oracle", qo)
    assert abs(qg[0] / qo[0] - 1) <= RUN_TOL and abs(qg[1] / qo[1] - 1) <= RUN_TOL, (qg, qo)
    assert st["iters_run"] == 60 and st["nonfinite_events"] == 0
    assert np.allclose(eg, eo, rtol=1e-2)


def test_fruchterman_reingold_given_explicitly_is_the_default(rmat14):
    g, x0, y0 = rmat14
    a = api.layout(g, x0, y0, api.params(batch_size=256, iterations=3, mode="bh", theta=1.2))
    b = api.layout(g, x0, y0, api.params(batch_size=256, iterations=3, mode="bh", theta=1.2, model=(2, -1)))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def _mixed_jobs():
    """Graphs of both modes and several models: small exact graphs (the
    one-workgroup kernel runs (2, -1) only, so the others take the
    multi-workgroup path), Barnes-Hut graphs of two models in one job set."""
    jobs = []
    for q, (n, mode, model) in enumerate([(300, "exact", (2, -1)), (500, "exact", (1, -1)),
                                          (5000, "bh", (2, -1)), (6000, "bh", (0, -1)),
                                          (4500, "bh", (3, 0)), (800, "exact", (3, -1))]):
        g = I.erdos_renyi(n, 8.0, 700 + q)
        x, y = I.uniform_coords(g.n, 800 + q)
        jobs.append((g, I.to_f32_representable(x), I.to_f32_representable(y),
                     api.params(batch_size=128, iterations=12, mode=mode, theta=1.0, model=model)))
    return jobs


def test_batched_mixed_models_equal_alone_runs():
    jobs = _mixed_jobs()
    outs, _ = api.layout_batch([j[0] for j in jobs], [j[1] for j in jobs], [j[2] for j in jobs],
                               [j[3] for j in jobs])
    for q, (g, x, y, p) in enumerate(jobs):
        xa, ya, _, _ = api.layout(g, x, y, p)
        assert np.array_equal(outs[q][0], xa) and np.array_equal(outs[q][1], ya), q


def test_served_mixed_models_equal_alone_runs():
    jobs = _mixed_jobs()
    with api.Server(8 << 30, max_slots=16) as s:
        ids = [s.submit(g, x, y, p) for g, x, y, p in jobs]
        for q, (g, x, y, p) in enumerate(jobs):
            s.wait(ids[q], 300.0)
            xs, ys, st = s.fetch(ids[q])
            xa, ya, _, _ = api.layout(g, x, y, p)
            assert np.array_equal(xs, xa) and np.array_equal(ys, ya), q
