"""Exact-mode parity: the HIP path against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import (RUN_TOL, SETTLING, assert_forces, assert_within_oracle_spread, force_errors, stop_tolerance,
                     near_grid_init, quality)

pytestmark = pytest.mark.gpu


def _f32(a):
    return I.to_f32_representable(a)


def _rand_graph(n, p, seed):
    r = I.rng(seed)
    iu = np.triu_indices(n, 1)
    keep = r.random(len(iu[0])) < p
    return I.csr_from_edges(n, iu[0][keep], iu[1][keep])


@pytest.fixture(scope="module")
def grid32():
    w = I.workload_grid32()
    w["x0"], w["y0"] = _f32(w["x0"]), _f32(w["y0"])
    return w


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32", "fp64"])
@pytest.mark.parametrize("batch", [0, 3, 7])
def test_one_shot_forces(grid32, precision, batch):
    g, x, y = grid32["graph"], grid32["x0"], grid32["y0"]
    p = api.params(batch_size=128, iterations=1, precision=precision)
    fx, fy = api.forces(g, x, y, batch, p)
    ref = oracle.forces_exact(g.rowptr, g.colidx, x, y, batch * 128, batch * 128 + 128)
    r = assert_forces(fx, fy, ref, what=precision)
    if precision == "fp64":
        assert r["rel_max"] < 1e-12


@pytest.mark.parametrize("iters,stop", [(1, 1), (1, 5), (2, 0), (3, 6)])
def test_pipeline_step_forces(grid32, iters, stop):
    """Forces of batch `stop` after the pipelined panels of earlier steps,
    checked on the exact state they were computed from."""
    g = grid32["graph"]
    p = api.params(batch_size=128, iterations=iters)
    with api.Graph(g, p) as h:
        h.set_coords(grid32["x0"], grid32["y0"])
        _, _, fx, fy = h.run(iters, stop_batch=stop)
        xs, ys = h.get_coords()
    ref = oracle.forces_exact(g.rowptr, g.colidx, xs, ys, stop * 128, stop * 128 + 128)
    assert_forces(fx, fy, ref, what="pipeline k=%d b=%d" % (iters - 1, stop))


@pytest.mark.parametrize("n,bs,lit", [(1000, 96, True), (257, 64, False), (300, 512, True), (40, 1, True),
                                      (130, 7, False)])
def test_ragged_and_literal(n, bs, lit):
    g = _rand_graph(n, 6.0 / n, n + bs)
    x0, y0 = I.uniform_coords(n, 3)
    x0, y0 = _f32(x0), _f32(y0)
    nb = (n + bs - 1) // bs
    stop = nb - 1                       # the ragged last batch
    p = api.params(batch_size=bs, iterations=2, repulse_adjacent=lit)
    with api.Graph(g, p) as h:
        h.set_coords(x0, y0)
        _, _, fx, fy = h.run(2, stop_batch=stop)
        xs, ys = h.get_coords()
    ref = oracle.forces_exact(g.rowptr, g.colidx, xs, ys, stop * bs, n, repulse_adjacent=lit)
    assert len(fx) == n - stop * bs
    assert_forces(fx, fy, ref)


def test_single_vertex_and_no_edges():
    g1 = I.csr_from_edges(1, np.array([], np.int64), np.array([], np.int64))
    x, y, e, st = api.layout(g1, np.array([0.5]), np.array([-0.25]), api.params(batch_size=4, iterations=3))
    assert x[0] == 0.5 and y[0] == -0.25 and np.all(e == 0)
    g0 = I.csr_from_edges(50, np.array([], np.int64), np.array([], np.int64))
    x0, y0 = I.uniform_coords(50, 9)
    x0, y0 = _f32(x0), _f32(y0)
    fx, fy = api.forces(g0, x0, y0, 0, api.params(batch_size=50))
    ref = oracle.forces_exact(g0.rowptr, g0.colidx, x0, y0, 0, 50)
    assert_forces(fx, fy, ref)


def test_full_run_fp64_tracks_oracle():
    """FP64 on the GPU against the FP64 oracle, the paper's schedule, 100 iterations."""
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    xg, yg, eg, st = api.layout(g, x0, y0, api.params(batch_size=128, iterations=100, precision="fp64"))
    xo, yo, eo = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 128, 100)
    qg, qo = quality(oracle, g, xg, yg), quality(oracle, g, xo, yo)
    assert abs(qg[0] / qo[0] - 1) <= 1e-6 and abs(qg[1] / qo[1] - 1) <= 1e-6, (qg, qo)
    assert np.allclose(eg, eo, rtol=1e-8)
    assert st["iters_run"] == 100 and st["nonfinite_events"] == 0


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32"])
def test_full_run_settling_schedule_within_one_percent(precision):
    """FP32 run on a schedule that settles: stress and edge energy within 1%."""
    g = I.grid(32, 32)
    x0, y0 = near_grid_init(32, 32)
    p = api.params(batch_size=128, iterations=100, precision=precision, **SETTLING)
    xg, yg, eg, st = api.layout(g, x0, y0, p)
    xo, yo, eo = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 128, 100, step0=SETTLING["step0"],
                                     decay=SETTLING["step_decay"])
    qg, qo = quality(oracle, g, xg, yg), quality(oracle, g, xo, yo)
    assert abs(qg[0] / qo[0] - 1) <= RUN_TOL and abs(qg[1] / qo[1] - 1) <= RUN_TOL, (qg, qo)
    assert np.allclose(eg, eo, rtol=1e-3)


def test_full_run_random_start_within_oracle_spread(grid32):
    """The 32x32 grid workload (random start, 100 iterations, batch 128)."""
    g = grid32["graph"]
    x0, y0 = grid32["x0"], grid32["y0"]
    xg, yg, eg, st = api.layout(g, x0, y0, api.params(batch_size=128, iterations=100))
    rep = assert_within_oracle_spread(
        oracle, g, xg, yg, lambda a, b: oracle.layout_exact(g.rowptr, g.colidx, a, b, 128, 100)[:2], x0, y0)
    print("grid32 exact full run:", rep)
    _, _, eo = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 128, 100)
    assert abs(eg[0] / eo[0] - 1) < 1e-4


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp64"])
def test_resume_is_bitwise_and_runs_repeat(grid32, precision):
    g = grid32["graph"]
    p = api.params(batch_size=128, iterations=10, precision=precision)
    xa, ya, ea, _ = api.layout(g, grid32["x0"], grid32["y0"], p)
    xb, yb, eb, _ = api.layout(g, grid32["x0"], grid32["y0"], p)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)
    with api.Graph(g, p) as h:
        h.set_coords(grid32["x0"], grid32["y0"])
        e1, _ = h.run(4, start_iter=0)
        e2, _ = h.run(6, start_iter=4)
        xc, yc = h.get_coords()
    assert np.array_equal(xa, xc) and np.array_equal(ya, yc)
    assert np.array_equal(ea, np.concatenate([e1, e2]))


def test_device_pointer_path(grid32):
    import torch
    g = grid32["graph"]
    dev = I.Graph(g.n, torch.as_tensor(g.rowptr, device="cuda"), torch.as_tensor(g.colidx, device="cuda"))
    x0 = torch.as_tensor(grid32["x0"], device="cuda")
    y0 = torch.as_tensor(grid32["y0"], device="cuda")
    p = api.params(batch_size=128, iterations=5)
    xd, yd, ed, _ = api.layout(dev, x0, y0, p)
    xh, yh, eh, _ = api.layout(g, grid32["x0"], grid32["y0"], p)
    assert np.array_equal(xd.cpu().numpy(), xh) and np.array_equal(yd.cpu().numpy(), yh)


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32", "fp64"])
@pytest.mark.parametrize("n,bs,lit", [(1024, 128, True), (700, 96, False), (300, 512, True), (257, 256, True)])
def test_one_workgroup_and_multi_workgroup_paths_agree_bitwise(monkeypatch, precision, n, bs, lit):
    """The one-workgroup kernel (forced with BL_EXACT_ONE_WG=1 above its
    default size) and the step kernels compute the same bits (energies,
    coordinates), resumed or not."""
    monkeypatch.setenv("BL_EXACT_ONE_WG", "1")
    g = I.grid(32, 32) if n == 1024 else _rand_graph(n, 8.0 / n, n + 3)
    x0, y0 = I.uniform_coords(g.n, 12)
    x0, y0 = _f32(x0), _f32(y0)
    kw = dict(batch_size=bs, iterations=7, precision=precision, repulse_adjacent=lit)
    xa, ya, ea, sa = api.layout(g, x0, y0, api.params(**kw))
    xb, yb, eb, sb = api.layout(g, x0, y0, api.params(multi_wg=True, **kw))
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)
    with api.Graph(g, api.params(**kw)) as h:
        h.set_coords(x0, y0)
        e1, _ = h.run(3)
        e2, _ = h.run(4, start_iter=3)
        xc, yc = h.get_coords()
    assert np.array_equal(xa, xc) and np.array_equal(ya, yc) and np.array_equal(ea, np.concatenate([e1, e2]))


def test_multi_workgroup_full_run_within_oracle_spread():
    """A graph above the one-workgroup size (64x64 grid, batch 256): the
    step-kernel path over a whole run, random start, 40 iterations."""
    g = I.grid(64, 64)
    x0, y0 = I.uniform_coords(g.n, 21)
    x0, y0 = _f32(x0), _f32(y0)
    xg, yg, eg, st = api.layout(g, x0, y0, api.params(batch_size=256, iterations=40))
    rep = assert_within_oracle_spread(
        oracle, g, xg, yg, lambda a, b: oracle.layout_exact(g.rowptr, g.colidx, a, b, 256, 40)[:2], x0, y0,
        members=4)
    print("grid64 exact full run:", rep)
    _, _, eo = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 256, 40)
    assert abs(eg[0] / eo[0] - 1) < 1e-4


def test_hub_rows_and_big_batches():
    """Hubs with hundreds of neighbours in one column batch, a batch larger
    than one LDS tile (1500 > 1024 columns), and the single-batch case."""
    r = I.rng(77)
    n = 3000
    src = np.concatenate([np.zeros(900, np.int64), np.full(700, 5), r.integers(0, n, 4000)])
    dst = np.concatenate([r.choice(np.arange(1, n), 900, replace=False), r.choice(np.arange(6, 1500), 700, replace=False),
                          r.integers(0, n, 4000)])
    g = I.csr_from_edges(n, src, dst)
    x0, y0 = I.uniform_coords(n, 5)
    x0, y0 = _f32(x0), _f32(y0)
    for bs, stop in [(1500, 1), (256, 0), (256, 11), (3000, 0)]:
        p = api.params(batch_size=bs, iterations=2)
        with api.Graph(g, p) as h:
            h.set_coords(x0, y0)
            _, _, fx, fy = h.run(2, stop_batch=stop)
            xs, ys = h.get_coords()
        ref = oracle.forces_exact(g.rowptr, g.colidx, xs, ys, stop * bs, min(n, stop * bs + bs))
        assert_forces(fx, fy, ref, what="bs=%d stop=%d" % (bs, stop))


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp64"])
@pytest.mark.parametrize("n,bs", [(3000, 128), (2900, 300), (4100, 512), (1300, 256)])
def test_persistent_run_equals_step_launches_bitwise(monkeypatch, precision, n, bs):
    """A multi-workgroup run is one cooperative launch whose workgroups wait
    on per-batch move counters; launching the steps one by one gives the same
    bits.  Batch sizes below, across and above the 256-row chunks."""
    g = _rand_graph(n, 8.0 / n, n + 11)
    x0, y0 = I.uniform_coords(g.n, 31)
    x0, y0 = _f32(x0), _f32(y0)
    p = api.params(batch_size=bs, iterations=5, precision=precision, multi_wg=True)
    xa, ya, ea, _ = api.layout(g, x0, y0, p)
    monkeypatch.setenv("BL_EXACT_STEPWISE", "1")
    xb, yb, eb, _ = api.layout(g, x0, y0, p)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)


def test_persistent_wait_limit_reports_timeout(monkeypatch):
    """A spin limit of zero makes the first wait that is not already met give
    up: every workgroup leaves, the run reports BL_E_TIMEOUT, and a new run
    on a new job is unaffected."""
    g = _rand_graph(4000, 8.0 / 4000, 4011)
    x0, y0 = I.uniform_coords(g.n, 32)
    x0, y0 = _f32(x0), _f32(y0)
    p = api.params(batch_size=128, iterations=4, multi_wg=True)
    monkeypatch.setenv("BL_EXACT_SPIN_LIMIT", "0")
    with pytest.raises(api.BLError) as err:
        api.layout(g, x0, y0, p)
    assert err.value.code == -7
    monkeypatch.delenv("BL_EXACT_SPIN_LIMIT")
    xa, ya, ea, _ = api.layout(g, x0, y0, p)
    monkeypatch.setenv("BL_EXACT_STEPWISE", "1")
    xb, yb, eb, _ = api.layout(g, x0, y0, p)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp64"])
@pytest.mark.parametrize("lit", [True, False])
def test_hub_rows_one_workgroup_and_multi_workgroup_bitwise(monkeypatch, precision, lit):
    """Rows with far more than 16 neighbours in one column batch take the
    long-segment path (entries 16.. dealt round the wave's 64 lanes, the lane
    sums met in a pairwise tree of cross-lane exchanges); the one-workgroup
    kernel evaluates the same tree one lane per row."""
    monkeypatch.setenv("BL_EXACT_ONE_WG", "1")
    r = I.rng(91)
    n = 2000
    src = np.concatenate([np.zeros(900, np.int64), np.full(600, 7), r.integers(0, n, 3000)])
    dst = np.concatenate([r.choice(np.arange(1, n), 900, replace=False), r.choice(np.arange(8, n), 600, replace=False),
                          r.integers(0, n, 3000)])
    g = I.csr_from_edges(n, src, dst)
    x0, y0 = I.uniform_coords(n, 17)
    x0, y0 = _f32(x0), _f32(y0)
    kw = dict(batch_size=128, iterations=4, precision=precision, repulse_adjacent=lit)
    xa, ya, ea, _ = api.layout(g, x0, y0, api.params(**kw))
    xb, yb, eb, _ = api.layout(g, x0, y0, api.params(multi_wg=True, **kw))
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb) and np.array_equal(ea, eb)


@pytest.mark.parametrize("path", ["one_workgroup", "persistent", "stepwise"])
def test_energy_stopping_rule(monkeypatch, path):
    """conv_tol ends the run where the energy's relative change first falls to
    the tolerance (Sec. 4.5): the same iteration as the oracle, and the same
    bits as a plain run of that many iterations, on every exact path."""
    g = _rand_graph(900, 8.0 / 900, 77)
    x0, y0 = I.uniform_coords(g.n, 78)
    x0, y0 = _f32(x0), _f32(y0)
    multi = path != "one_workgroup"
    if path == "one_workgroup":
        monkeypatch.setenv("BL_EXACT_ONE_WG", "1")
    if path == "stepwise":
        monkeypatch.setenv("BL_EXACT_STEPWISE", "1")
    kw = dict(batch_size=128, step0=0.05, step_decay=0.97, multi_wg=multi)
    _, _, ef, _ = api.layout(g, x0, y0, api.params(iterations=14, **kw))
    tol, want = stop_tolerance(ef)
    xs, ys, es, st = api.layout(g, x0, y0, api.params(iterations=14, conv_tol=tol, **kw))
    assert st["iters_run"] == want and len(es) == want
    xp, yp, ep, _ = api.layout(g, x0, y0, api.params(iterations=want, **kw))
    assert np.array_equal(xs, xp) and np.array_equal(ys, yp) and np.array_equal(es, ep)
    _, _, eo = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 128, 14, step0=0.05, decay=0.97, conv_tol=tol)
    assert len(eo) == want


@pytest.mark.gpu
def test_issue_probe_counts_and_times():
    """The issue-rate probe times each op and counts the instructions it
    issued: blocks x 256 threads x iters x 8 chains (x 7 for the mix)."""
    import ctypes as C
    from paper_2002_08233_amd import _lib
    lib = _lib.load()
    for op, per in ((0, 1), (1, 1), (2, 7)):
        ms, ops = C.c_double(), C.c_double()
        assert lib.bl_probe_issue_rate(op, 64, 128, None, C.byref(ms), C.byref(ops)) == 0
        assert ms.value > 0
        assert ops.value == 64 * 256 * 128 * 8 * per
