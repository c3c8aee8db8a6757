"""(a, r)-energy models of Sec. 2.2 other than (2, -1) in exact mode: the HIP
path against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import RUN_TOL, SETTLING, assert_forces, near_grid_init, quality

pytestmark = pytest.mark.gpu

MODELS = [(1, -1), (0, -1), (3, -1), (2, -2), (1, -2), (3, 0)]


def _f32(a):
    return I.to_f32_representable(a)


def _graph(n, deg, seed):
    r = I.rng(seed)
    iu = np.triu_indices(n, 1)
    keep = r.random(len(iu[0])) < deg / n
    return I.csr_from_edges(n, iu[0][keep], iu[1][keep])


@pytest.fixture(scope="module")
def ragged():
    g = _graph(700, 8.0, 81)
    x, y = I.uniform_coords(g.n, 82)
    return g, _f32(x), _f32(y)


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32", "fp64"])
@pytest.mark.parametrize("model", MODELS)
def test_one_shot_forces(ragged, model, precision):
    """Forces of the first, a middle and the ragged last batch (700 vertices, batch 96)."""
    g, x, y = ragged
    p = api.params(batch_size=96, iterations=1, precision=precision, model=model)
    for b in (0, 3, 7):
        fx, fy = api.forces(g, x, y, b, p)
        ref = oracle.forces_exact(g.rowptr, g.colidx, x, y, 96 * b, min(96 * b + 96, g.n), model=model)
        assert_forces(fx, fy, ref, what="model %s %s batch %d" % (model, precision, b))


@pytest.mark.parametrize("model", [(1, -1), (0, -1)])
def test_literal_mode(ragged, model):
    g, x, y = ragged
    p = api.params(batch_size=96, iterations=1, repulse_adjacent=False, model=model)
    fx, fy = api.forces(g, x, y, 2, p)
    ref = oracle.forces_exact(g.rowptr, g.colidx, x, y, 192, 288, repulse_adjacent=False, model=model)
    assert_forces(fx, fy, ref, what="literal %s" % (model,))


@pytest.mark.parametrize("model", [(1, -1), (3, -1)])
def test_pipeline_forces(model):
    """The state at (iteration 2, batch 5) of a resident run: its forces against the oracle's."""
    g = _graph(1500, 10.0, 83)
    x0, y0 = I.uniform_coords(g.n, 84)
    p = api.params(batch_size=128, iterations=3, model=model)
    with api.Graph(g, p) as h:
        h.set_coords(_f32(x0), _f32(y0))
        h.run(2)
        _, st, fx, fy = h.run(1, start_iter=2, stop_batch=5)
        xs, ys = h.get_coords()
    ref = oracle.forces_exact(g.rowptr, g.colidx, xs, ys, 640, 768, model=model)
    assert_forces(fx, fy, ref, what="pipeline %s" % (model,))


@pytest.mark.parametrize("model", [(1, -1), (0, -1), (3, -1)])
def test_full_run_fp64_and_settling(model):
    """32x32 grid from a near-grid start, 60 iterations on a settling schedule:
    FP64 on the GPU tracks the oracle to 1e-6 and FP32-Kahan is within 1% in
    stress and edge energy."""
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    xo, yo, eo = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 128, 60, step0=SETTLING["step0"],
                                     decay=SETTLING["step_decay"], model=model)
    qo = quality(oracle, g, xo, yo)
    for precision, tol in (("fp64", 1e-6), ("fp32_kahan", RUN_TOL)):
        p = api.params(batch_size=128, iterations=60, precision=precision, model=model, **SETTLING)
        xg, yg, eg, st = api.layout(g, x0, y0, p)
        qg = quality(oracle, g, xg, yg)
        assert abs(qg[0] / qo[0] - 1) <= tol and abs(qg[1] / qo[1] - 1) <= tol, (precision, qg, qo)
        assert st["iters_run"] == 60 and st["nonfinite_events"] == 0
    assert np.allclose(eg, eo, rtol=1e-3)


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp64"])
def test_persistent_run_equals_step_launches(monkeypatch, precision):
    g = _graph(3000, 8.0, 85)
    x0, y0 = I.uniform_coords(g.n, 86)
    p = api.params(batch_size=128, iterations=4, precision=precision, model=(1, -1))
    a = api.layout(g, _f32(x0), _f32(y0), p)
    monkeypatch.setenv("BL_EXACT_STEPWISE", "1")
    b = api.layout(g, _f32(x0), _f32(y0), p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_default_model_is_fruchterman_reingold(ragged):
    g, x, y = ragged
    a = api.layout(g, x, y, api.params(batch_size=96, iterations=3))
    b = api.layout(g, x, y, api.params(batch_size=96, iterations=3, model=(2, -1)))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
