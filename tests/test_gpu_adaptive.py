"""Hu's adaptive step (cited in Sec. 4.3.5) on the GPU against the oracle.  The
step decisions compare consecutive energies; every case here keeps them at
least 0.5% apart in the oracle's run, far above FP32 rounding, so both sides
take the same decisions."""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import RUN_TOL, near_grid_init, quality

pytestmark = pytest.mark.gpu


def _margin(e):
    return float(np.min(np.abs(np.diff(e)) / e[1:]))


def test_fp64_tracks_oracle():
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    p = api.params(batch_size=128, iterations=40, precision="fp64", step_decay=0.9, adaptive_step=True)
    xg, yg, eg, st = api.layout(g, x0, y0, p)
    xo, yo, eo, so = oracle.layout_adaptive(g.rowptr, g.colidx, x0, y0, 128, 40, step0=1.0, t=0.9)
    assert _margin(eo) > 5e-3 and len(set(np.round(so, 12))) > 3
    assert np.allclose(xg, xo, rtol=0, atol=1e-6) and np.allclose(yg, yo, rtol=0, atol=1e-6)
    assert np.allclose(eg, eo, rtol=1e-9)
    assert st["iters_run"] == 40


@pytest.mark.parametrize("mode", ["exact", "bh"])
def test_fp32_within_one_percent(mode):
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    p = api.params(batch_size=100, iterations=60, mode=mode, theta=1.2, step0=0.05, step_decay=0.9,
                   adaptive_step=True)
    xg, yg, eg, st = api.layout(g, x0, y0, p)
    kw = dict(theta=1.2) if mode == "bh" else {}
    xo, yo, eo, _ = oracle.layout_adaptive(g.rowptr, g.colidx, x0, y0, 100, 60, step0=0.05, t=0.9, mode=mode, **kw)
    assert _margin(eo) > 5e-3
    qg, qo = quality(oracle, g, xg, yg), quality(oracle, g, xo, yo)
    assert abs(qg[0] / qo[0] - 1) <= RUN_TOL and abs(qg[1] / qo[1] - 1) <= RUN_TOL, (qg, qo)
    assert np.allclose(eg, eo, rtol=1e-3)


def test_repeat_and_stopping_rule():
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    kw = dict(batch_size=100, step0=0.05, step_decay=0.9, adaptive_step=True)
    xa, ya, ea, _ = api.layout(g, x0, y0, api.params(iterations=30, **kw))
    xb, yb, eb, _ = api.layout(g, x0, y0, api.params(iterations=30, **kw))
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)
    rel = np.abs(np.diff(ea)) / ea[:-1]
    tol = float(np.sort(rel)[len(rel) // 2]) * 1.0000001
    want = int(np.argmax(rel <= tol)) + 2
    xs, ys, es, st = api.layout(g, x0, y0, api.params(iterations=30, conv_tol=tol, **kw))
    assert st["iters_run"] == want and np.array_equal(es, ea[:want])
    xp, yp, _, _ = api.layout(g, x0, y0, api.params(iterations=want, **kw))
    assert np.array_equal(xs, xp) and np.array_equal(ys, yp)
    xo, yo, eo, _ = oracle.layout_adaptive(g.rowptr, g.colidx, x0, y0, 100, 30, step0=0.05, t=0.9, conv_tol=tol)
    assert len(eo) == want


def test_unit_factor_is_the_fixed_step_run():
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    xa, ya, ea, _ = api.layout(g, x0, y0, api.params(batch_size=128, iterations=8, step0=0.2, step_decay=1.0,
                                                     adaptive_step=True))
    xb, yb, eb, _ = api.layout(g, x0, y0, api.params(batch_size=128, iterations=8, step0=0.2, step_decay=1.0))
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)


@pytest.mark.parametrize("precision,model,bs,stepwise", [
    ("fp32_kahan", (2, -1), 96, False), ("fp32", (2, -1), 96, False), ("fp64", (2, -1), 96, False),
    ("fp32_kahan", (1, -1), 96, False), ("fp32_kahan", (2, -1), 96, True), ("fp32_kahan", (2, -1), 2048, False)])
def test_multi_wg_runs_chain_bitwise(monkeypatch, precision, model, bs, stepwise):
    """The multi-workgroup exact path: with t = 1 the adaptive driver's chain
    of one-iteration runs (each leaving the next one's prologue in place)
    gives the bits of one 6-iteration run.  Ragged batches (1600 = 16 x 96 +
    64), FP32 and FP64, a general model, the step-by-step path, one batch."""
    if stepwise:
        monkeypatch.setenv("BL_EXACT_STEPWISE", "1")
    g = I.grid(40, 40)
    x0, y0 = near_grid_init(40, 40)
    kw = dict(batch_size=bs, step0=0.2, step_decay=1.0, multi_wg=True, precision=precision, model=model)
    xa, ya, ea, _ = api.layout(g, x0, y0, api.params(iterations=6, adaptive_step=True, **kw))
    xb, yb, eb, _ = api.layout(g, x0, y0, api.params(iterations=6, **kw))
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)
