"""Barnes-Hut parity: the HIP tree build, far-field walk and minibatch chain
against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import (bh_mask, RUN_TOL, SETTLING, assert_forces, assert_within_oracle_spread, near_grid_init, quality,
                     stop_tolerance)

pytestmark = pytest.mark.gpu


def _f32(a):
    return I.to_f32_representable(a)


@pytest.fixture(scope="module")
def grid32():
    w = I.workload_grid32()
    w["x0"], w["y0"] = _f32(w["x0"]), _f32(w["y0"])
    return w


@pytest.mark.parametrize("theta", [0.0, 0.5, 1.2])
@pytest.mark.parametrize("batch", [0, 5])
def test_one_shot_forces(grid32, theta, batch):
    g, x, y = grid32["graph"], grid32["x0"], grid32["y0"]
    p = api.params(batch_size=128, iterations=1, mode="bh", theta=theta)
    fx, fy = api.forces(g, x, y, batch, p)
    ref = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), batch * 128, batch * 128 + 128,
                           theta=theta)
    assert_forces(fx, fy, ref, mask=bh_mask(ref), what="theta=%g" % theta)
    if theta == 0.0:
        ex = oracle.forces_exact(g.rowptr, g.colidx, x, y, batch * 128, batch * 128 + 128)
        assert_forces(fx, fy, ex, what="theta=0 vs exact")


@pytest.mark.parametrize("iters,stop", [(1, 1), (1, 6), (2, 3)])
@pytest.mark.parametrize("snapshot_leaves", [False, True])
def test_pipeline_step_forces(grid32, iters, stop, snapshot_leaves):
    g = grid32["graph"]
    p = api.params(batch_size=128, iterations=iters, mode="bh", theta=1.2, snapshot_leaves=snapshot_leaves)
    with api.Graph(g, p) as h:
        h.set_coords(grid32["x0"], grid32["y0"])
        if iters > 1:
            h.run(iters - 1)
        sx, sy = h.get_coords()
        _, _, fx, fy = h.run(1, start_iter=iters - 1, stop_batch=stop)
        xs, ys = h.get_coords()
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(sx, sy), stop * 128, stop * 128 + 128,
                           theta=1.2, leaf_live=not snapshot_leaves)
    assert_forces(fx, fy, ref, mask=bh_mask(ref))


def test_rmat_hubs_and_snapshot_argument():
    """Scale-12 RMAT (hub rows of hundreds of entries), mid-iteration state,
    tree from a separate snapshot through the one-shot call."""
    g = I.rmat(12, 16, seed=5)
    x0, y0 = I.uniform_coords(g.n, 6)
    x0, y0 = _f32(x0), _f32(y0)
    p = api.params(batch_size=256, iterations=1, mode="bh", theta=1.2)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        _, st, fx, fy = h.run(1, stop_batch=9)
        xs, ys = h.get_coords()
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(x0, y0), 9 * 256, 10 * 256, theta=1.2)
    assert_forces(fx, fy, ref, mask=bh_mask(ref), what="pipeline")
    fx2, fy2 = api.forces(g, xs, ys, 9, p, snapshot=(x0, y0))
    assert_forces(fx2, fy2, ref, mask=bh_mask(ref), what="one-shot with snapshot")
    for b in (0, 15):    # hub rows sit at low ids
        fx3, fy3 = api.forces(g, xs, ys, b, p, snapshot=(x0, y0))
        ref3 = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(x0, y0), b * 256, b * 256 + 256,
                                theta=1.2)
        assert_forces(fx3, fy3, ref3, mask=bh_mask(ref3), what="batch %d" % b)


def test_late_list_overflow_falls_back_to_full_walk():
    """A dense cluster at small theta lists more than the per-vertex capacity
    of moved leaves; those vertices take a full live walk instead."""
    r = I.rng(77)
    n = 2048
    x0 = np.concatenate([r.normal(0, 1e-3, n // 2), r.uniform(-1, 1, n // 2)])
    y0 = np.concatenate([r.normal(0, 1e-3, n // 2), r.uniform(-1, 1, n // 2)])
    perm = r.permutation(n)
    x0, y0 = _f32(x0[perm]), _f32(y0[perm])
    g = I.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    p = api.params(batch_size=256, iterations=1, mode="bh", theta=0.3)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        _, st, fx, fy = h.run(1, stop_batch=6)
        xs, ys = h.get_coords()
    assert st["late_overflow"] > 0
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(x0, y0), 6 * 256, 7 * 256, theta=0.3)
    assert_forces(fx, fy, ref, mask=bh_mask(ref))


@pytest.mark.parametrize("n,bs", [(1, 4), (2, 1), (3, 2), (600, 100), (777, 1024)])
def test_small_and_ragged(n, bs):
    r = I.rng(n)
    x0, y0 = _f32(r.uniform(-1, 1, n)), _f32(r.uniform(-1, 1, n))
    g = I.csr_from_edges(n, np.arange(max(n - 1, 0)), np.arange(1, n)) if n > 1 else \
        I.csr_from_edges(1, np.array([], np.int64), np.array([], np.int64))
    nb = (n + bs - 1) // bs
    p = api.params(batch_size=bs, iterations=1, mode="bh", theta=1.0)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        _, _, fx, fy = h.run(1, stop_batch=nb - 1)
        xs, ys = h.get_coords()
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(x0, y0), (nb - 1) * bs, n, theta=1.0)
    assert_forces(fx, fy, ref, mask=bh_mask(ref))


def test_coincident_points_bucket():
    """Points sharing a depth-16 cell form a bucket; every member interacts exactly."""
    n = 300
    r = I.rng(3)
    x0 = _f32(np.where(np.arange(n) < 40, 0.25, r.uniform(-1, 1, n)))
    y0 = _f32(np.where(np.arange(n) < 40, -0.5, r.uniform(-1, 1, n)))
    x0[:40] += np.arange(40) * 1e-7        # distinct, but inside one finest cell
    x0 = _f32(x0)
    g = I.csr_from_edges(n, np.array([], np.int64), np.array([], np.int64))
    p = api.params(batch_size=64, iterations=1, mode="bh", theta=1.2)
    fx, fy = api.forces(g, x0, y0, 0, p)
    ref = oracle.forces_bh(g.rowptr, g.colidx, x0, y0, oracle.Tree(x0, y0), 0, 64, theta=1.2)
    assert_forces(fx, fy, ref, mask=bh_mask(ref))


def test_full_run_settling_schedule_within_one_percent():
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    p = api.params(batch_size=128, iterations=100, mode="bh", theta=1.2, **SETTLING)
    xg, yg, eg, st = api.layout(g, x0, y0, p)
    xo, yo, eo, _ = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, 128, 100, theta=1.2,
                                     step0=SETTLING["step0"], decay=SETTLING["step_decay"])
    qg, qo = quality(oracle, g, xg, yg), quality(oracle, g, xo, yo)
    assert abs(qg[0] / qo[0] - 1) <= RUN_TOL and abs(qg[1] / qo[1] - 1) <= RUN_TOL, (qg, qo)
    assert np.allclose(eg, eo, rtol=1e-3)
    assert st["node_visits"] > 0 and st["nonfinite_events"] == 0


def test_full_run_random_start_within_oracle_spread(grid32):
    g = grid32["graph"]
    x0, y0 = grid32["x0"], grid32["y0"]
    p = api.params(batch_size=128, iterations=100, mode="bh", theta=1.2)
    xg, yg, eg, st = api.layout(g, x0, y0, p)
    rep = assert_within_oracle_spread(
        oracle, g, xg, yg,
        lambda a, b: oracle.layout_bh(g.rowptr, g.colidx, a, b, 128, 100, theta=1.2)[:2], x0, y0)
    print("grid32 BH full run:", rep)
    _, _, eo, _ = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, 128, 100, theta=1.2)
    assert abs(eg[0] / eo[0] - 1) < 1e-3


def test_repeat_runs_bitwise(grid32):
    g = grid32["graph"]
    p = api.params(batch_size=128, iterations=5, mode="bh", theta=1.2)
    a = api.layout(g, grid32["x0"], grid32["y0"], p)
    b = api.layout(g, grid32["x0"], grid32["y0"], p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("iters,stop,lag", [(1, 40, 14), (1, 199, 14), (2, 170, 14), (1, 199, None), (2, 170, None)])
def test_segmented_chain_ragged(iters, stop, lag, monkeypatch):
    """A long chain (200 batches of 64 rows, ragged last batch): forces at stop
    batches.  With the lag capped at 14, most moved entries lie more than the
    chain's lag behind (summed by its helper workgroups), the rest in its LDS
    ring; by default the ring holds the whole chain and no helper runs."""
    if lag is not None:
        monkeypatch.setenv("BL_BH_LAG", str(lag))
    g = I.rmat(14, 8, seed=23)
    n = 200 * 64 - 17
    keep = (g.colidx < n)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    sel = keep & (rows < n)
    g = I.csr_from_edges(n, rows[sel], g.colidx[sel])
    x0, y0 = I.uniform_coords(n, 24)
    x0, y0 = _f32(x0), _f32(y0)
    p = api.params(batch_size=64, iterations=iters, mode="bh", theta=1.2)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        if iters > 1:
            h.run(iters - 1)
        sx, sy = h.get_coords()
        _, _, fx, fy = h.run(1, start_iter=iters - 1, stop_batch=stop)
        xs, ys = h.get_coords()
    r1 = min(n, stop * 64 + 64)
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(sx, sy), stop * 64, r1, theta=1.2)
    assert_forces(fx, fy, ref, mask=bh_mask(ref), what="stop %d" % stop)


@pytest.mark.parametrize("stop", [25, 29])
def test_window_forces_segments_at_big_batches(stop):
    """Batch 1024: the chain's LDS ring holds 15 batches (lag 14), so even a
    30-batch chain has old entries for its helpers; forces in the last
    batches, including the ragged last batch."""
    g = I.rmat(15, 8, seed=29)
    n = 29 * 1024 + 300
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    sel = (g.colidx < n) & (rows < n)
    g = I.csr_from_edges(n, rows[sel], g.colidx[sel])
    x0, y0 = I.uniform_coords(n, 30)
    x0, y0 = _f32(x0), _f32(y0)
    p = api.params(batch_size=1024, iterations=1, mode="bh", theta=1.2)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        _, _, fx, fy = h.run(1, stop_batch=stop)
        xs, ys = h.get_coords()
    r1 = min(n, stop * 1024 + 1024)
    ref = oracle.forces_bh(g.rowptr, g.colidx, xs, ys, oracle.Tree(x0, y0), stop * 1024, r1, theta=1.2)
    assert_forces(fx, fy, ref, mask=bh_mask(ref), what="stop %d" % stop)


def test_chain_wait_limit_reports_timeout(monkeypatch):
    """A spin limit of zero makes the first wait of the chain launch that is
    not already met give up (a helper polling for batches the chain has not
    moved yet): every workgroup leaves, the run reports BL_E_TIMEOUT, and a
    new run is unaffected."""
    g = I.rmat(14, 8, seed=23)
    x0, y0 = I.uniform_coords(g.n, 24)
    x0, y0 = _f32(x0), _f32(y0)
    p = api.params(batch_size=64, iterations=2, mode="bh", theta=1.2)
    monkeypatch.setenv("BL_BH_LAG", "14")   # (the ring would hold this chain whole: no helpers, no waits)
    monkeypatch.setenv("BL_BH_SPIN_LIMIT", "0")
    with pytest.raises(api.BLError) as err:
        api.layout(g, x0, y0, p)
    assert err.value.code == -7
    monkeypatch.delenv("BL_BH_SPIN_LIMIT")
    xa, ya, ea, _ = api.layout(g, x0, y0, p)
    xb, yb, eb, _ = api.layout(g, x0, y0, p)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)


@pytest.mark.parametrize("n,bs,lag", [(3000, 128, None), (12783, 64, 14)])
def test_energy_stopping_rule(n, bs, lag, monkeypatch):
    """conv_tol on the Barnes-Hut engine (a chain the ring holds whole, and a
    chain with helpers): the run stops at the same iteration as the oracle and
    equals a plain run of that many iterations bitwise."""
    if lag is not None:
        monkeypatch.setenv("BL_BH_LAG", str(lag))
    g = I.rmat(14, 8, seed=31)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    sel = (g.colidx < n) & (rows < n)
    g = I.csr_from_edges(n, rows[sel], g.colidx[sel])
    x0, y0 = I.uniform_coords(n, 32)
    x0, y0 = _f32(x0), _f32(y0)
    kw = dict(batch_size=bs, mode="bh", theta=1.2, step0=0.05, step_decay=0.97)
    _, _, ef, _ = api.layout(g, x0, y0, api.params(iterations=12, **kw))
    tol, want = stop_tolerance(ef)
    xs, ys, es, st = api.layout(g, x0, y0, api.params(iterations=12, conv_tol=tol, **kw))
    assert st["iters_run"] == want and len(es) == want
    xp, yp, ep, _ = api.layout(g, x0, y0, api.params(iterations=want, **kw))
    assert np.array_equal(xs, xp) and np.array_equal(ys, yp) and np.array_equal(es, ep)
    eo = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, bs, 12, step0=0.05, decay=0.97, theta=1.2, conv_tol=tol)[2]
    assert len(eo) == want
