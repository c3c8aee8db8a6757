"""Pins for the FP64 oracle: closed forms, invariants, special cases and brute force.

Each test fixes the oracle to something other than itself, so that a dropped
term, a wrong sign, a swapped index or a wrong batch order fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_graph(n, p, seed):
    r = I.rng(seed)
    iu = np.triu_indices(n, 1)
    keep = r.random(len(iu[0])) < p
    return I.csr_from_edges(n, iu[0][keep], iu[1][keep])


def dyadic_coords(n, seed, bits=12):
    """Coordinates on a 2^-bits grid so that shifts, rotations and power-of-two
    scalings are exact in FP64."""
    r = I.rng(seed)
    return (r.integers(-2 ** bits, 2 ** bits, n) / 2.0 ** bits,
            r.integers(-2 ** bits, 2 ** bits, n) / 2.0 ** bits)


# ---------------------------------------------------------------- pair terms

@pytest.mark.parametrize("K,R", [(1.0, 1.0), (0.5, 2.0), (2.0, 0.25)])
def test_two_vertex_force_closed_form(K, R):
    """Sec. 2.2 with a=2, r=-1: |f| = |d^2/K - R K^2/d| along the line, zero at d* = K R^(1/3)."""
    g = I.path(2)
    for d, ang in [(0.3, 0.1), (1.7, 2.0), (K * R ** (1 / 3), -0.7)]:
        x = np.array([0.25, 0.25 + d * math.cos(ang)])
        y = np.array([-0.5, -0.5 + d * math.sin(ang)])
        f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 2, K=K, R=R)
        # force on vertex 0 is along +u (toward vertex 1) with signed magnitude d^2/K - R K^2/d
        u = np.array([math.cos(ang), math.sin(ang)])
        mag = d * d / K - R * K * K / d
        assert f.fx[0] == pytest.approx(mag * u[0], abs=1e-12 * (1 + abs(mag)))
        assert f.fy[0] == pytest.approx(mag * u[1], abs=1e-12 * (1 + abs(mag)))
        assert f.fx[1] == pytest.approx(-mag * u[0], abs=1e-12 * (1 + abs(mag)))
        # attraction and repulsion separately (signs)
        assert f.ax[0] * u[0] + f.ay[0] * u[1] == pytest.approx(d * d / K, rel=1e-13)
        assert f.rx[0] * u[0] + f.ry[0] * u[1] == pytest.approx(-R * K * K / d, rel=1e-13)


@pytest.mark.parametrize("bs", [1, 2])
def test_two_vertex_trajectory_and_equilibrium(bs):
    """Normalised steps make the motion 1-D: with batch 2 both ends move by Step
    (distance changes by 2 Step); with batch 1 the second vertex sees the first
    one's move.  The distance settles within 2*Step_k of d* = K R^(1/3)."""
    g = I.path(2)
    K, R = 1.0, 1.0
    dstar = K * R ** (1 / 3)
    x0 = np.array([0.0, 5.0])
    y0 = np.array([0.0, 0.0])
    iters = 400
    x, y, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, bs, iters, step0=1.0, decay=0.9)
    # independent recurrence on the two abscissae: each end moves by Step toward
    # the other when the gap exceeds d*, away from it when the gap is shorter
    def pull(p, q):
        d = abs(q - p)
        toward = 1.0 if q > p else -1.0
        return toward * (1.0 if d > dstar else (-1.0 if d < dstar else 0.0))

    a, b = 0.0, 5.0
    step = 1.0
    for k in range(iters):
        if bs == 2:
            sa, sb = pull(a, b), pull(b, a)
            a, b = a + step * sa, b + step * sb
        else:
            a = a + step * pull(a, b)
            b = b + step * pull(b, a)
        step *= 0.9
    assert x[0] == pytest.approx(a, abs=1e-12) and x[1] == pytest.approx(b, abs=1e-12)
    assert np.all(y == 0.0)
    assert abs(abs(x[1] - x[0]) - dstar) <= 2 * 0.9 ** (iters - 1) + 1e-12


def test_cycle_equilibrium_radius():
    """Cycle C_k on a circle of radius rho: by symmetry forces are radial,
    F(rho) = (k-1) R K^2 / (2 rho) - 8 rho^2 sin^3(pi/k) / K, so the
    equilibrium radius is rho*^3 = (k-1) R K^3 / (16 sin^3(pi/k))."""
    for k, K, R in [(5, 1.0, 1.0), (12, 0.7, 1.5), (31, 1.3, 0.4)]:
        g = I.cycle(k)
        rho_star = (((k - 1) * R * K ** 3) / (16 * math.sin(math.pi / k) ** 3)) ** (1 / 3)
        for rho in [0.5 * rho_star, rho_star, 2.0 * rho_star]:
            phi = 2 * math.pi * np.arange(k) / k
            x, y = rho * np.cos(phi), rho * np.sin(phi)
            f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, k, K=K, R=R)
            radial = f.fx * np.cos(phi) + f.fy * np.sin(phi)
            tangential = -f.fx * np.sin(phi) + f.fy * np.cos(phi)
            expect = (k - 1) * R * K * K / (2 * rho) - 8 * rho ** 2 * math.sin(math.pi / k) ** 3 / K
            scale = f.scale.max()
            assert np.allclose(radial, expect, atol=1e-12 * scale)
            assert np.abs(tangential).max() <= 1e-12 * scale


# ------------------------------------------------------------ force invariants

def test_newton_third_law():
    """With all vertices in one batch, repulsions and attractions each sum to zero."""
    g = random_graph(60, 0.1, 11)
    x, y = I.uniform_coords(60, 12)
    f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 60)
    s = f.scale.sum()
    assert abs(f.rx.sum()) < 1e-12 * s and abs(f.ry.sum()) < 1e-12 * s
    assert abs(f.ax.sum()) < 1e-12 * s and abs(f.ay.sum()) < 1e-12 * s


def test_literal_mode_skips_adjacent_repulsion():
    """Algorithms 1/2 skip repulsion between adjacent vertices: the literal force
    equals the all-pairs force minus the repulsion of each neighbour."""
    g = random_graph(40, 0.15, 3)
    x, y = I.uniform_coords(40, 4)
    fa = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 40, repulse_adjacent=True)
    fl = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 40, repulse_adjacent=False)
    for i in range(40):
        nb = g.colidx[g.rowptr[i]:g.rowptr[i + 1]]
        dx, dy = x[nb] - x[i], y[nb] - y[i]
        d2 = dx * dx + dy * dy
        cx, cy = (-dx / d2).sum(), (-dy / d2).sum()
        assert fl.fx[i] == pytest.approx(fa.fx[i] - cx, abs=1e-11 * fa.scale[i])
        assert fl.fy[i] == pytest.approx(fa.fy[i] - cy, abs=1e-11 * fa.scale[i])


def test_translation_invariance_bitwise():
    g = random_graph(50, 0.1, 5)
    x, y = dyadic_coords(50, 6)
    f0 = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 50)
    f1 = oracle.forces_exact(g.rowptr, g.colidx, x + 3.25, y - 0.5, 0, 50)
    assert np.array_equal(f0.fx, f1.fx) and np.array_equal(f0.fy, f1.fy)


def test_rotation_and_reflection_covariance_bitwise():
    """(x,y) -> (-y,x) and x -> -x are exact in floating point, so the forces
    transform exactly."""
    g = random_graph(50, 0.1, 7)
    x, y = dyadic_coords(50, 8)
    f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 50)
    fr = oracle.forces_exact(g.rowptr, g.colidx, -y, x, 0, 50)
    assert np.array_equal(fr.fx, -f.fy) and np.array_equal(fr.fy, f.fx)
    fm = oracle.forces_exact(g.rowptr, g.colidx, -x, y, 0, 50)
    assert np.array_equal(fm.fx, -f.fx) and np.array_equal(fm.fy, f.fy)


def test_scaling_law():
    """c -> s c: attraction scales by s^2, repulsion by 1/s (exact for s = 2^k)."""
    g = random_graph(40, 0.1, 9)
    x, y = dyadic_coords(40, 10)
    f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 40)
    f4 = oracle.forces_exact(g.rowptr, g.colidx, 4 * x, 4 * y, 0, 40)
    assert np.allclose(f4.ax, 16 * f.ax, rtol=0, atol=1e-14 * np.abs(16 * f.ax).max())
    assert np.array_equal(f4.rx, f.rx / 4) and np.array_equal(f4.ry, f.ry / 4)


def test_coincident_vertices_contribute_nothing():
    g = I.csr_from_edges(4, np.array([0]), np.array([1]))
    x = np.array([0.0, 0.0, 1.0, 0.0])
    y = np.array([0.0, 0.0, 0.0, 2.0])
    f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 4)
    assert np.all(np.isfinite(f.fx)) and np.all(np.isfinite(f.fy))
    # vertex 0 feels only vertices 2 and 3
    assert f.rx[0] == pytest.approx(-1.0) and f.ry[0] == pytest.approx(-0.5)
    assert f.ax[0] == 0.0 and f.ay[0] == 0.0


# --------------------------------------------------------- minibatch semantics

def _py_force(rp, ci, x, y, i, K=1.0, R=1.0, literal=False):
    """Sec. 2.2 written with the paper's f_a, f_r and unit vectors."""
    nb = set(ci[rp[i]:rp[i + 1]].tolist())
    fx = fy = 0.0
    for j in range(len(x)):
        if j == i:
            continue
        dx, dy = x[j] - x[i], y[j] - y[i]
        d = math.hypot(dx, dy)
        if d == 0:
            continue
        if j in nb:
            fa = d ** 2 / K
            fx += fa * dx / d
            fy += fa * dy / d
            if literal:
                continue
        fr = -R * K * K / d
        fx += fr * dx / d
        fy += fr * dy / d
    return fx, fy


def _py_layout(rp, ci, x, y, bs, iters, literal=False, step=1.0, decay=0.999):
    x, y = list(x), list(y)
    n = len(x)
    energies = []
    for _ in range(iters):
        e = 0.0
        for b0 in range(0, n, bs):
            batch = range(b0, min(b0 + bs, n))
            forces = [_py_force(rp, ci, x, y, i, literal=literal) for i in batch]
            for i, (fx, fy) in zip(batch, forces):
                norm = math.hypot(fx, fy)
                if norm > 0:
                    x[i] += step * fx / norm
                    y[i] += step * fy / norm
                e += fx * fx + fy * fy
        energies.append(e)
        step *= decay
    return np.array(x), np.array(y), np.array(energies)


def test_batch_one_is_algorithm1():
    """Batch size 1 is the sequential Algorithm 1 (literal neighbour exclusion)."""
    g = random_graph(24, 0.2, 21)
    x0, y0 = I.uniform_coords(24, 22)
    xr, yr, er = _py_layout(g.rowptr, g.colidx, x0, y0, 1, 5, literal=True)
    x, y, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 1, 5, repulse_adjacent=False)
    assert np.allclose(x, xr, atol=1e-10) and np.allclose(y, yr, atol=1e-10)
    assert np.allclose(e, er, rtol=1e-10)


@pytest.mark.parametrize("bs", [24, 5, 7])
def test_batch_n_is_jacobi_and_ragged_batches(bs):
    """Batch n is a fully synchronous update; other sizes give consecutive-id
    batches with a ragged last batch."""
    g = random_graph(24, 0.2, 23)
    x0, y0 = I.uniform_coords(24, 24)
    xr, yr, er = _py_layout(g.rowptr, g.colidx, x0, y0, bs, 4)
    x, y, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, bs, 4)
    assert np.allclose(x, xr, atol=1e-10) and np.allclose(y, yr, atol=1e-10)
    assert np.allclose(e, er, rtol=1e-10)


def test_fig2_schedule_golden():
    """Fig. 2: batch b's forces use the already-moved coordinates of batch b-1."""
    gold = json.load(open(os.path.join(GOLDEN, "fig2_minibatch_schedule.json")))
    n, bs = gold["n"], gold["batch_size"]
    g = I.cycle(n)
    x0, y0 = I.uniform_coords(n, 31)
    x, y = x0.copy(), y0.copy()
    for batch in gold["batches"]:
        i0, i1 = batch[0], batch[-1] + 1
        f = oracle.forces_exact(g.rowptr, g.colidx, x, y, i0, i1)
        norm = np.hypot(f.fx, f.fy)
        x[i0:i1] += f.fx / norm
        y[i0:i1] += f.fy / norm
        xs, ys, _ = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, bs, 1, stop_batch=i1 // bs)
        assert np.allclose(xs, x, atol=1e-13) and np.allclose(ys, y, atol=1e-13)
    assert len(gold["batches"]) == gold["steps"] == (n + bs - 1) // bs


def test_energy_is_sum_of_squared_forces():
    """The energy of an iteration is the sum of |f_i|^2 at the moment of each move."""
    g = random_graph(30, 0.15, 41)
    x0, y0 = I.uniform_coords(30, 42)
    f = oracle.forces_exact(g.rowptr, g.colidx, x0, y0, 0, 30)
    _, _, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 30, 1)
    assert e[0] == pytest.approx(float(np.sum(f.fx ** 2 + f.fy ** 2)), rel=1e-14)


def test_step_schedule():
    """Step_k = Step_0 * 0.999^k (Sec. 4.3.5); resuming at iteration k continues it."""
    assert oracle.step_at(1.0, 0.999, 0) == 1.0
    for k in [1, 10, 599]:
        assert oracle.step_at(1.0, 0.999, k) == pytest.approx(0.999 ** k, rel=1e-13)
    g = random_graph(20, 0.2, 51)
    x0, y0 = I.uniform_coords(20, 52)
    xa, ya, ea = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 8, 6)
    xb, yb, eb = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 8, 3)
    xc, yc, ec = oracle.layout_exact(g.rowptr, g.colidx, xb, yb, 8, 3, start_iter=3)
    assert np.array_equal(xa, xc) and np.array_equal(ya, yc)
    assert np.array_equal(ea, np.concatenate([eb, ec]))


def test_single_vertex_and_empty_graph():
    g1 = I.csr_from_edges(1, np.array([], np.int64), np.array([], np.int64))
    x, y, e = oracle.layout_exact(g1.rowptr, g1.colidx, [0.5], [0.25], 4, 3)
    assert x[0] == 0.5 and y[0] == 0.25 and np.all(e == 0)
    g0 = I.csr_from_edges(3, np.array([], np.int64), np.array([], np.int64))
    x0 = np.array([0.0, 1.0, 0.0]); y0 = np.array([0.0, 0.0, 1.0])
    f = oracle.forces_exact(g0.rowptr, g0.colidx, x0, y0, 0, 3)
    assert np.all(f.ax == 0) and f.rx[0] == pytest.approx(-1.0) and f.ry[0] == pytest.approx(-1.0)


def test_mpmath_bruteforce():
    """Forces, one iteration and its energy against 50-digit arithmetic."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    n, bs = 12, 5
    g = random_graph(n, 0.3, 61)
    x0, y0 = I.uniform_coords(n, 62)
    K, R = 0.8, 1.3
    X = [mp.mpf(v) for v in x0]
    Y = [mp.mpf(v) for v in y0]
    nbs = [set(g.colidx[g.rowptr[i]:g.rowptr[i + 1]].tolist()) for i in range(n)]

    def force(i):
        fx = fy = mp.mpf(0)
        for j in range(n):
            if j == i:
                continue
            dx, dy = X[j] - X[i], Y[j] - Y[i]
            d = mp.sqrt(dx * dx + dy * dy)
            if j in nbs[i]:
                fx += d * d / K * dx / d
                fy += d * d / K * dy / d
            fx += -R * K * K / d * dx / d
            fy += -R * K * K / d * dy / d
        return fx, fy

    f = oracle.forces_exact(g.rowptr, g.colidx, x0, y0, 0, n, K=K, R=R)
    for i in range(n):
        fx, fy = force(i)
        assert abs(f.fx[i] - float(fx)) <= 1e-13 * f.scale[i]
        assert abs(f.fy[i] - float(fy)) <= 1e-13 * f.scale[i]
    energy = mp.mpf(0)
    for b0 in range(0, n, bs):
        batch = list(range(b0, min(b0 + bs, n)))
        fs = [force(i) for i in batch]
        for i, (fx, fy) in zip(batch, fs):
            nrm = mp.sqrt(fx * fx + fy * fy)
            X[i] += fx / nrm
            Y[i] += fy / nrm
            energy += fx * fx + fy * fy
    x, y, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, bs, 1, K=K, R=R)
    assert np.allclose(x, [float(v) for v in X], atol=1e-12)
    assert np.allclose(y, [float(v) for v in Y], atol=1e-12)
    assert e[0] == pytest.approx(float(energy), rel=1e-13)


# ---------------------------------------------------------------- Barnes-Hut

def test_bh_theta_zero_is_exact():
    """theta = 0 never accepts a cell, so the walk reaches every vertex (any batch size)."""
    w = I.workload_grid32()
    g = w["graph"]
    x, y = w["x0"], w["y0"]
    t = oracle.Tree(x, y)
    fe = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, g.n)
    fb = oracle.forces_bh(g.rowptr, g.colidx, x, y, t, 0, g.n, theta=0.0)
    assert np.abs(fe.fx - fb.fx).max() <= 1e-12 * fe.scale.max()
    assert np.abs(fe.fy - fb.fy).max() <= 1e-12 * fe.scale.max()
    # full runs, several batch sizes: theta = 0 equals exact up to rounding order
    gs = random_graph(40, 0.1, 71)
    x0, y0 = I.uniform_coords(40, 72)
    for bs in [1, 7, 40]:
        xe, ye, ee = oracle.layout_exact(gs.rowptr, gs.colidx, x0, y0, bs, 2)
        xb, yb, eb, _ = oracle.layout_bh(gs.rowptr, gs.colidx, x0, y0, bs, 2, theta=0.0)
        assert np.allclose(xe, xb, atol=1e-9) and np.allclose(ee, eb, rtol=1e-11)


def test_bh_tree_invariants():
    r = I.rng(81)
    n = 500
    x = np.concatenate([r.normal(0, 1, n - 20), np.full(20, 0.75)])   # 20 coincident points
    y = np.concatenate([r.normal(0, 2, n - 20), np.full(20, -0.25)])
    t = oracle.Tree(x, y)
    nodes = t.nodes()
    order, keys = t.order()
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    assert sorted(order.tolist()) == list(range(n))
    assert nodes[0]["lo"] == 0 and nodes[0]["hi"] == n and nodes[0]["level"] == 0
    W = t.width
    assert W == pytest.approx(max(x.max() - x.min(), y.max() - y.min()), rel=1e-6)
    nb = 0
    for nd in nodes:
        members = order[nd["lo"]:nd["hi"]]
        assert nd["cx"] == pytest.approx(x[members].mean(), abs=1e-14 * (1 + abs(x).max()))
        assert nd["cy"] == pytest.approx(y[members].mean(), abs=1e-14 * (1 + abs(y).max()))
        assert nd["level"] <= 16
        if nd["children"]:
            kids = [nodes[c] for c in nd["children"]]
            assert kids[0]["lo"] == nd["lo"] and kids[-1]["hi"] == nd["hi"]
            for a, b in zip(kids, kids[1:]):
                assert a["hi"] == b["lo"]
            assert all(k["level"] == nd["level"] + 1 for k in kids)
        if nd["bucket"]:
            nb += 1
            assert nd["level"] == 16 and nd["hi"] - nd["lo"] >= 2
    assert nb == 1


def test_bh_coincident_far_cell_is_k_times_single():
    """k vertices at one far point act as one accepted cell with k times the force."""
    k = 7
    x = np.array([0.0] + [10.0] * k)
    y = np.array([0.0] + [5.0] * k)
    g = I.csr_from_edges(len(x), np.array([], np.int64), np.array([], np.int64))
    f = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), 0, 1, theta=1.2)
    assert f.visits[0] < 4          # root opened, far cell accepted without descending
    x1, y1 = x[:2], y[:2]
    g1 = I.csr_from_edges(2, np.array([], np.int64), np.array([], np.int64))
    single = oracle.forces_bh(g1.rowptr, g1.colidx, x1, y1, oracle.Tree(x1, y1), 0, 1, theta=1.2)
    assert f.rx[0] == pytest.approx(k * single.rx[0], rel=1e-14)
    assert f.ry[0] == pytest.approx(k * single.ry[0], rel=1e-14)
    assert single.rx[0] == pytest.approx(-10.0 / 125.0, rel=1e-14)


def _py_bh_force(x, y, i, theta, K=1.0, R=1.0, r=-1):
    """Independent Barnes-Hut walk: cells found by recursive geometric
    subdivision of the bounding square (no Morton keys); repulsion magnitude
    R K^2 d^r, an accepted cell counting once per member."""
    xs = x.astype(np.float32).astype(np.float64)
    ys = y.astype(np.float32).astype(np.float64)
    x0, y0 = xs.min(), ys.min()
    W = max(xs.max() - x0, ys.max() - y0)
    fx = fy = 0.0

    def rep(px, py, mult):
        dx, dy = px - x[i], py - y[i]
        d = math.hypot(dx, dy)
        if d == 0:
            return 0.0, 0.0
        m = mult * R * K * K * d ** r
        return (-m * dx / d, -m * dy / d)

    def walk(members, cx0, cy0, side, level):
        nonlocal fx, fy
        if len(members) == 1 or level == 16:
            for j in members:
                if j != i:
                    a, b = rep(x[j], y[j], 1)
                    fx += a; fy += b
            return
        if i not in members:
            cx, cy = x[members].mean(), y[members].mean()
            if side < theta * math.hypot(cx - x[i], cy - y[i]):
                a, b = rep(cx, cy, len(members))
                fx += a; fy += b
                return
        h = side / 2
        for qy in (0, 1):
            for qx in (0, 1):
                sub = [j for j in members
                       if (xs[j] >= cx0 + qx * h or qx == 0) and (xs[j] < cx0 + h or qx == 1)
                       and (ys[j] >= cy0 + qy * h or qy == 0) and (ys[j] < cy0 + h or qy == 1)]
                if sub:
                    walk(sub, cx0 + qx * h, cy0 + qy * h, h, level + 1)

    walk(list(range(len(x))), x0, y0, W, 0)
    return fx, fy


@pytest.mark.parametrize("theta", [0.5, 1.2, 2.5])
@pytest.mark.parametrize("clustered", [False, True])
def test_bh_matches_independent_geometric_walk(theta, clustered):
    """Also with groups of distinct points inside one finest cell: the cells
    above such a group hold the same members and may be accepted."""
    r = I.rng(91)
    n = 60
    x = r.uniform(-1, 1, n)
    y = r.uniform(-1, 1, n)
    if clustered:
        x[:8] = 0.3 + np.arange(8) * 2e-7
        y[:8] = -0.4
        x[8:12] = -0.7
        y[8:12] = 0.1 + np.arange(4) * 3e-7
    x = x.astype(np.float32).astype(np.float64)
    y = y.astype(np.float32).astype(np.float64)
    g = I.csr_from_edges(n, np.array([], np.int64), np.array([], np.int64))
    t = oracle.Tree(x, y)
    f = oracle.forces_bh(g.rowptr, g.colidx, x, y, t, 0, n, theta=theta)
    for i in range(n):
        fx, fy = _py_bh_force(x, y, i, theta)
        assert f.rx[i] == pytest.approx(fx, abs=1e-11 * f.scale[i])
        assert f.ry[i] == pytest.approx(fy, abs=1e-11 * f.scale[i])


def test_bh_error_shrinks_with_theta():
    w = I.workload_grid32()
    g = w["graph"]
    x, y = w["x0"], w["y0"]
    t = oracle.Tree(x, y)
    fe = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, g.n)
    errs = []
    for theta in [2.0, 1.2, 0.8, 0.4, 0.2]:
        fb = oracle.forces_bh(g.rowptr, g.colidx, x, y, t, 0, g.n, theta=theta)
        errs.append(np.hypot(fb.rx - fe.rx, fb.ry - fe.ry).sum() / np.hypot(fe.rx, fe.ry).sum())
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3


def test_bh_live_leaves_vs_snapshot():
    """Leaves use live coordinates: after one batch has moved, a later vertex's
    force changes only through the moved vertices it reaches as leaves."""
    g = random_graph(64, 0.05, 95)
    x0, y0 = I.uniform_coords(64, 96)
    x, y, _, _, sx, sy = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, 16, 1, theta=0.0,
                                          stop_batch=2, want_snapshot=True)
    t = oracle.Tree(sx, sy)
    live = oracle.forces_bh(g.rowptr, g.colidx, x, y, t, 32, 48, theta=0.0, leaf_live=True)
    exact = oracle.forces_exact(g.rowptr, g.colidx, x, y, 32, 48)
    assert np.allclose(live.fx, exact.fx, atol=1e-12 * exact.scale.max())
    snap = oracle.forces_bh(g.rowptr, g.colidx, x, y, t, 32, 48, theta=0.0, leaf_live=False)
    assert not np.allclose(snap.fx, exact.fx, atol=1e-6 * exact.scale.max())


# ------------------------------------------------------------ quality measures

def test_stress_zero_for_metric_layout_and_optimal_scale():
    g = I.path(10)
    x = np.arange(10, dtype=float) * 3.0
    y = np.zeros(10)
    st, s = oracle.stress(g.rowptr, g.colidx, x, y)
    assert st == pytest.approx(0.0, abs=1e-9) and s == pytest.approx(1 / 3.0)
    from scipy.optimize import minimize_scalar
    g2 = random_graph(30, 0.15, 101)
    x2, y2 = I.uniform_coords(30, 102)
    st2, s2 = oracle.stress(g2.rowptr, g2.colidx, x2, y2)
    # brute-force stress as a function of the scale, independent of the closed form
    D = np.full((30, 30), -1)
    for p in range(30):
        D[p, p] = 0
        frontier = [p]
        while frontier:
            nxt = []
            for u in frontier:
                for v in g2.colidx[g2.rowptr[u]:g2.rowptr[u + 1]]:
                    if D[p, v] < 0:
                        D[p, v] = D[p, u] + 1
                        nxt.append(v)
            frontier = nxt
    iu = np.triu_indices(30, 1)
    dd = D[iu].astype(float)
    gg = np.hypot(x2[iu[0]] - x2[iu[1]], y2[iu[0]] - y2[iu[1]])
    ok = dd > 0
    fun = lambda sc: float(np.sum((sc * gg[ok] - dd[ok]) ** 2 / dd[ok] ** 2))
    res = minimize_scalar(fun, bounds=(1e-3, 1e3), method="bounded", options=dict(xatol=1e-12))
    assert s2 == pytest.approx(res.x, rel=1e-6)
    assert st2 == pytest.approx(res.fun, rel=1e-9)


def test_edge_energy_and_uniformity_closed_forms():
    g = I.cycle(8)
    phi = 2 * math.pi * np.arange(8) / 8
    x, y = 2 * np.cos(phi), 2 * np.sin(phi)
    assert oracle.edge_uniformity(g.rowptr, g.colidx, x, y) == pytest.approx(0.0, abs=1e-12)
    side = 2 * 2 * math.sin(math.pi / 8)
    assert oracle.edge_energy(g.rowptr, g.colidx, x, y, K=1.5) == pytest.approx(8 * side ** 3 / 4.5)
    gp = I.path(3)
    assert oracle.edge_uniformity(gp.rowptr, gp.colidx, np.array([0.0, 1.0, 4.0]), np.zeros(3)) == \
        pytest.approx(math.sqrt(((1 - 2) ** 2 + (3 - 2) ** 2) / (2 * 4)))


def test_paper_defaults_golden():
    gold = json.load(open(os.path.join(GOLDEN, "paper_defaults.json")))
    assert gold["step_decay"]["value"] == 0.999 and gold["theta"]["value"] == 1.2
    assert gold["batch_size"]["value"] == 256 and gold["step0"]["value"] == 1.0


def _first_stop(e, tol):
    """Iterations run under the energy stopping rule, straight from its
    definition: the first k >= 1 with |E_k - E_{k-1}| <= tol * E_{k-1}."""
    for k in range(1, len(e)):
        if abs(e[k] - e[k - 1]) <= tol * e[k - 1]:
            return k + 1
    return len(e)


@pytest.mark.parametrize("mode", ["exact", "bh"])
def test_energy_stopping_rule(mode):
    """Sec. 4.5's energy stopping rule read as a relative change (R11): the run
    stops at the first iteration (not the run's first) whose relative energy
    change is at or below the tolerance, and its layout is the plain run's
    layout after that many iterations.  Tolerances taken from the plain run's
    own changes, one that always holds, and 0 (off)."""
    g = I.grid(6, 7)
    x0, y0 = I.uniform_coords(g.n, 41)
    if mode == "exact":
        run = lambda it, tol=0.0: oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 8, it, conv_tol=tol)[:3]
    else:
        run = lambda it, tol=0.0: oracle.layout_bh(g.rowptr, g.colidx, x0, y0, 8, it, theta=0.7,
                                                   conv_tol=tol)[:3]
    xf, yf, ef = run(16)
    rel = np.abs(np.diff(ef)) / ef[:-1]
    assert np.all(np.isfinite(rel)) and rel.size == 15
    tols = [10.0, 0.0] + sorted(set(float(r) * 1.0001 for r in rel[1:8]))
    for tol in tols:
        want = _first_stop(ef, tol) if tol > 0 else 16
        xs, ys, es = run(16, tol)
        assert len(es) == want, (tol, len(es), want)
        xp, yp, ep = run(want)
        assert np.array_equal(xs, xp) and np.array_equal(ys, yp) and np.array_equal(es, ep)
    assert len(run(16, 10.0)[2]) == 2


# --------------------------------------------------- greedy initialisation

def _angle(dx, dy):
    return math.atan2(dy, dx) % (2 * math.pi)


def test_greedy_path_from_an_end_is_the_unit_line():
    """Alg. 3 from an end of a path: every vertex is one unit further along +x (angle 0 each time)."""
    g = I.path(9)
    x, y, par = oracle.greedy_init(g.rowptr, g.colidx, 0)
    assert np.array_equal(x, np.arange(9.0)) and np.array_equal(y, np.zeros(9))
    assert list(par) == [-1] + list(range(8))


def test_greedy_uses_the_papers_pi_and_a_stack():
    """Path 0-1-2-3-4 from 2: vertex 1 at angle 0, vertex 3 at 180 degrees of the paper's PI = 3.1416,
    so 3 lies sin(3.1416) = -(3.1416 - pi) + O(eps^3) below the axis; 3 is popped first (last pushed)
    and places 4 at angle 0 from itself; then 1 places 0."""
    g = I.path(5)
    x, y, par = oracle.greedy_init(g.rowptr, g.colidx, 2)
    assert (x[2], y[2]) == (0.0, 0.0)
    assert (x[1], y[1]) == (1.0, 0.0) and (x[0], y[0]) == (2.0, 0.0)
    eps = 3.1416 - math.pi
    assert y[3] == pytest.approx(-eps, rel=1e-9)
    assert x[3] == pytest.approx(-1.0 + eps * eps / 2, abs=1e-15)
    assert x[4] == x[3] + 1.0 and y[4] == y[3]
    assert list(par) == [1, 2, -1, 2, 3]


def test_greedy_depth_first_not_breadth_first():
    """Square 0-1-3-2-0 from 0: 1 and 2 are pushed in that order, 2 is popped first and places 3
    at angle 0 from itself, next to the origin (a queue would let 1 place it, at (2, 0))."""
    g = I.csr_from_edges(4, np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3]))
    x, y, par = oracle.greedy_init(g.rowptr, g.colidx, 0)
    assert par[3] == 2
    assert x[3] == x[2] + 1.0 and y[3] == y[2]
    assert abs(x[3]) < 1e-9 and abs(y[3]) < 1e-5


@pytest.mark.parametrize("m", [3, 7, 12])
def test_greedy_star_angles_count_every_neighbour(m):
    """Star with centre 0.  From the centre the leaves sit on the unit circle 2*3.1416/m radians apart
    in row order.  From leaf 1 the centre lands at (1, 0) and places the other m - 1 leaves at the
    same spacing: the degree counts the visited neighbour too."""
    g = I.csr_from_edges(m + 1, np.zeros(m, np.int64), np.arange(1, m + 1))
    step = 2 * 3.1416 / m
    x, y, _ = oracle.greedy_init(g.rowptr, g.colidx, 0)
    assert (x[1], y[1]) == (1.0, 0.0)
    for k in range(1, m + 1):
        assert math.hypot(x[k], y[k]) == pytest.approx(1.0, abs=1e-15)
        assert _angle(x[k], y[k]) == pytest.approx((k - 1) * step % (2 * math.pi), abs=1e-12)
    x, y, _ = oracle.greedy_init(g.rowptr, g.colidx, 1)
    assert (x[0], y[0]) == (1.0, 0.0) and (x[2], y[2]) == (2.0, 0.0)
    for k in range(2, m + 1):
        assert _angle(x[k] - x[0], y[k] - y[0]) == pytest.approx((k - 2) * step % (2 * math.pi), abs=1e-12)


def test_greedy_tree_invariants_and_components():
    """Random graph with several components and isolated vertices: every vertex is placed once;
    a non-root lies at distance 1 from the neighbour that placed it; the children of a vertex
    sit at angles 0, s, 2s, ... with s = 2*3.1416/deg in row order; the start is at the origin and
    each other component's root is its lowest id, at its given position."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    g = random_graph(300, 0.006, 41)
    n = g.n
    xr, yr = I.uniform_coords(n, 42)
    start = 17
    x, y, par = oracle.greedy_init(g.rowptr, g.colidx, start, xr, yr)
    A = csr_matrix((np.ones(g.nnz), g.colidx, g.rowptr), shape=(n, n))
    ncomp, lab = connected_components(A, directed=False)
    assert ncomp > 5
    roots = np.flatnonzero(par < 0)
    assert len(roots) == ncomp and len(set(lab[roots])) == ncomp
    assert (x[start], y[start]) == (0.0, 0.0)
    for r in roots:
        if r != start:
            assert r == np.flatnonzero(lab == lab[r]).min()
            assert (x[r], y[r]) == (xr[r], yr[r])
    kids = {}
    for v in range(n):
        u = par[v]
        if u < 0:
            continue
        assert v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]]
        assert math.hypot(x[v] - x[u], y[v] - y[u]) == pytest.approx(1.0, abs=1e-12)
        kids.setdefault(u, []).append(v)
    for u, vs in kids.items():
        s = 2 * 3.1416 / (g.rowptr[u + 1] - g.rowptr[u])
        for k, v in enumerate(sorted(vs)):
            assert _angle(x[v] - x[u], y[v] - y[u]) == pytest.approx(k * s % (2 * math.pi), abs=1e-9)
    # the tree is acyclic: following parents always reaches a root
    for v in range(n):
        seen, u = 0, v
        while par[u] >= 0:
            u = par[u]
            seen += 1
            assert seen <= n


# ------------------------------------------------------ (a, r) energy models

AR_MODELS = [(1, -1), (0, -1), (3, -1), (2, -2), (1, -2), (3, 0)]


@pytest.mark.parametrize("a,r", AR_MODELS)
def test_ar_two_vertex_closed_form(a, r):
    """Sec. 2.2 with general (a, r): on two vertices the force on vertex 0 is
    (d^a/K - R K^2 d^r) along the unit vector toward vertex 1, zero at
    d* = (R K^3)^(1/(a - r))."""
    g = I.path(2)
    K, R = 0.7, 1.6
    dstar = (R * K ** 3) ** (1.0 / (a - r))
    for d, ang in [(0.37, 0.3), (2.2, -1.1), (dstar, 2.5)]:
        x = np.array([-0.25, -0.25 + d * math.cos(ang)])
        y = np.array([0.5, 0.5 + d * math.sin(ang)])
        f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 2, K=K, R=R, model=(a, r))
        u = np.array([math.cos(ang), math.sin(ang)])
        mag = d ** a / K - R * K * K * d ** r
        tol = 1e-12 * (d ** a / K + R * K * K * d ** r)
        assert f.fx[0] == pytest.approx(mag * u[0], abs=tol) and f.fy[0] == pytest.approx(mag * u[1], abs=tol)
        assert f.fx[1] == pytest.approx(-mag * u[0], abs=tol) and f.fy[1] == pytest.approx(-mag * u[1], abs=tol)
        assert np.hypot(f.ax[0], f.ay[0]) == pytest.approx(d ** a / K, rel=1e-12)
        assert np.hypot(f.rx[0], f.ry[0]) == pytest.approx(R * K * K * d ** r, rel=1e-12)
    # the attraction points toward the neighbour, the repulsion away from it
    assert f.ax[0] * u[0] + f.ay[0] * u[1] > 0 and f.rx[0] * u[0] + f.ry[0] * u[1] < 0


@pytest.mark.parametrize("a,r", AR_MODELS)
def test_ar_newton_third_law(a, r):
    """At BS = n every pair term appears with both signs: the attraction and
    the repulsion each sum to zero over all vertices."""
    g = random_graph(60, 0.1, 71)
    x, y = I.uniform_coords(60, 72)
    f = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 60, model=(a, r))
    s = f.scale.sum()
    assert abs(f.ax.sum()) < 1e-12 * s and abs(f.ay.sum()) < 1e-12 * s
    assert abs(f.rx.sum()) < 1e-12 * s and abs(f.ry.sum()) < 1e-12 * s


@pytest.mark.parametrize("a,r", AR_MODELS)
def test_ar_scaling_law_and_literal_identity(a, r):
    """c -> 2c scales the attraction by 2^a and the repulsion by 2^r; literal
    mode is the default force minus the neighbours' repulsion terms."""
    g = random_graph(40, 0.15, 73)
    x, y = dyadic_coords(40, 74)
    f1 = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 40, model=(a, r))
    f2 = oracle.forces_exact(g.rowptr, g.colidx, 2 * x, 2 * y, 0, 40, model=(a, r))
    np.testing.assert_allclose(f2.ax, 2.0 ** a * f1.ax, rtol=1e-13, atol=1e-13 * 2.0 ** a * f1.scale.max())
    np.testing.assert_allclose(f2.rx, 2.0 ** r * f1.rx, rtol=1e-13, atol=1e-13 * 2.0 ** r * f1.scale.max())
    lit = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 40, repulse_adjacent=False, model=(a, r))
    for i in range(40):
        cx = cy = 0.0
        for j in g.colidx[g.rowptr[i]:g.rowptr[i + 1]]:
            dx, dy = x[j] - x[i], y[j] - y[i]
            d = math.hypot(dx, dy)
            cx += -(d ** r) * dx / d
            cy += -(d ** r) * dy / d
        assert lit.rx[i] == pytest.approx(f1.rx[i] - cx, abs=1e-12 * f1.scale[i])
        assert lit.ry[i] == pytest.approx(f1.ry[i] - cy, abs=1e-12 * f1.scale[i])


@pytest.mark.parametrize("a,r", [(1, -1), (0, -2), (3, 0)])
def test_ar_mpmath_bruteforce(a, r):
    """Forces and one iteration under (a, r) against 50-digit arithmetic."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    n, bs = 11, 4
    g = random_graph(n, 0.35, 75)
    x0, y0 = I.uniform_coords(n, 76)
    K, R = 1.3, 0.6
    nbs = [set(g.colidx[g.rowptr[i]:g.rowptr[i + 1]].tolist()) for i in range(n)]

    def forces(X, Y, i):
        fx = fy = mp.mpf(0)
        for j in range(n):
            if j == i:
                continue
            dx, dy = X[j] - X[i], Y[j] - Y[i]
            d = mp.sqrt(dx * dx + dy * dy)
            m = -R * K * K * d ** r + (d ** a / K if j in nbs[i] else 0)
            fx += m * dx / d
            fy += m * dy / d
        return fx, fy

    X = [mp.mpf(v) for v in x0]
    Y = [mp.mpf(v) for v in y0]
    f = oracle.forces_exact(g.rowptr, g.colidx, x0, y0, 0, n, K=K, R=R, model=(a, r))
    for i in range(n):
        fx, fy = forces(X, Y, i)
        assert abs(f.fx[i] - float(fx)) <= 1e-13 * f.scale[i]
        assert abs(f.fy[i] - float(fy)) <= 1e-13 * f.scale[i]
    # one iteration of the minibatch schedule, step 1
    for b0 in range(0, n, bs):
        batch = list(range(b0, min(b0 + bs, n)))
        fs = [forces(X, Y, i) for i in batch]
        for i, (fx, fy) in zip(batch, fs):
            nrm = mp.sqrt(fx * fx + fy * fy)
            X[i] += fx / nrm
            Y[i] += fy / nrm
    x1, y1, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, bs, 1, K=K, R=R, model=(a, r))
    for i in range(n):
        assert x1[i] == pytest.approx(float(X[i]), abs=1e-12) and y1[i] == pytest.approx(float(Y[i]), abs=1e-12)


# ------------------------------------------- (a, r) models in Barnes-Hut mode

@pytest.mark.parametrize("a,r", AR_MODELS)
def test_ar_bh_theta_zero_is_exact(a, r):
    """theta = 0 opens every cell, so the Barnes-Hut force under (a, r) is the
    exact one (up to summation order), per step and over whole runs."""
    g = random_graph(70, 0.08, 301)
    x, y = I.uniform_coords(70, 302)
    fe = oracle.forces_exact(g.rowptr, g.colidx, x, y, 0, 70, model=(a, r))
    fb = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), 0, 70, theta=0.0, model=(a, r))
    assert np.all(np.abs(fe.fx - fb.fx) <= 1e-12 * fe.scale) and np.all(np.abs(fe.fy - fb.fy) <= 1e-12 * fe.scale)
    assert np.allclose(fe.scale, fb.scale, rtol=1e-12)
    for bs in (1, 9, 70):
        xe, ye, ee = oracle.layout_exact(g.rowptr, g.colidx, x, y, bs, 2, step0=0.05, model=(a, r))
        xb, yb, eb, _ = oracle.layout_bh(g.rowptr, g.colidx, x, y, bs, 2, step0=0.05, theta=0.0, model=(a, r))
        assert np.allclose(xe, xb, atol=1e-10) and np.allclose(ye, yb, atol=1e-10) and np.allclose(ee, eb, rtol=1e-10)


@pytest.mark.parametrize("a,r", AR_MODELS)
def test_ar_bh_two_vertex_closed_form(a, r):
    """Two vertices: the other vertex is a leaf at any theta, so the force is
    (d^a/K - R K^2 d^r) along the unit vector, as in exact mode."""
    g = I.path(2)
    K, R = 0.8, 1.3
    d, ang = 1.7, 0.4
    x = np.array([0.1, 0.1 + d * math.cos(ang)])
    y = np.array([-0.2, -0.2 + d * math.sin(ang)])
    f = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), 0, 2, K=K, R=R, theta=5.0, model=(a, r))
    mag = d ** a / K - R * K * K * d ** r
    tol = 1e-12 * (d ** a / K + R * K * K * d ** r)
    assert f.fx[0] == pytest.approx(mag * math.cos(ang), abs=tol)
    assert f.fy[0] == pytest.approx(mag * math.sin(ang), abs=tol)
    assert f.fx[1] == pytest.approx(-mag * math.cos(ang), abs=tol)


@pytest.mark.parametrize("a,r", AR_MODELS)
def test_ar_bh_far_cell_is_count_times_single(a, r):
    """k coincident vertices far away form one accepted cell whose repulsion
    is k times a single vertex's, R K^2 d^r away from it."""
    k = 5
    x = np.array([0.0] + [12.0] * k)
    y = np.array([0.0] + [-9.0] * k)
    g = I.csr_from_edges(len(x), np.array([], np.int64), np.array([], np.int64))
    f = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), 0, 1, theta=1.2, model=(a, r))
    assert f.visits[0] < 4
    d = 15.0
    assert f.rx[0] == pytest.approx(-k * d ** r * 12.0 / d, rel=1e-13)
    assert f.ry[0] == pytest.approx(k * d ** r * 9.0 / d, rel=1e-13)


@pytest.mark.parametrize("a,r", [(1, -1), (0, -2), (3, 0)])
@pytest.mark.parametrize("theta", [0.7, 1.2])
def test_ar_bh_matches_independent_geometric_walk(a, r, theta):
    """The repulsion under (a, r) against the independent recursive walk."""
    rr = I.rng(303)
    n = 50
    x = rr.uniform(-1, 1, n).astype(np.float32).astype(np.float64)
    y = rr.uniform(-1, 1, n).astype(np.float32).astype(np.float64)
    g = I.csr_from_edges(n, np.array([], np.int64), np.array([], np.int64))
    f = oracle.forces_bh(g.rowptr, g.colidx, x, y, oracle.Tree(x, y), 0, n, theta=theta, model=(a, r))
    for i in range(n):
        fx, fy = _py_bh_force(x, y, i, theta, r=r)
        assert f.rx[i] == pytest.approx(fx, abs=1e-11 * f.scale[i])
        assert f.ry[i] == pytest.approx(fy, abs=1e-11 * f.scale[i])


# ------------------------------------------------- neighbourhood preservation

def test_np_metric_layouts_preserve_every_neighbourhood():
    """A path at unit spacing on a line, a cycle on a regular polygon and a
    grid at unit spacing: each vertex's deg nearest vertices are exactly its
    neighbours, so the measure is 1 over all vertices."""
    n = 12
    g = I.path(n)
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, np.arange(n, dtype=float), np.zeros(n))
    assert v == 1.0 and c == n
    g = I.cycle(9)
    t = 2 * np.pi * np.arange(9) / 9
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, np.cos(t), np.sin(t))
    assert v == 1.0 and c == 9
    g = I.grid(4, 5)
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, (np.arange(20) % 5).astype(float),
                                            (np.arange(20) // 5).astype(float))
    assert v == 1.0 and c == 20


def test_np_crossed_matching_is_zero():
    """Edges (0,2), (1,3), (4,6), (5,7) with vertex v at x = v: every vertex's
    nearest other vertex (ties to the lower id) is not its partner."""
    src = np.array([0, 1, 4, 5])
    dst = np.array([2, 3, 6, 7])
    g = I.csr_from_edges(8, src, dst)
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, np.arange(8, dtype=float), np.zeros(8))
    assert v == 0.0 and c == 8


def test_np_worked_example_with_ties_and_isolated_vertex():
    """Star 0-{1,2,3} and an isolated vertex 4, worked by hand:
    vertex 0 at the origin, degree 3: nearest 4 (d^2 .25), then 1 and 2 (d^2 1):
    2 of 3 neighbours, Jaccard 2/4; vertex 1 at (1,0): nearest 4, a miss;
    vertex 2 at (0,1): nearest 0, a hit; vertex 3 at (5,5): 1 and 2 tie at
    d^2 41, the lower id 1 is taken, a miss; vertex 4 is isolated and skipped.
    Mean (0.5 + 0 + 1 + 0) / 4."""
    g = I.csr_from_edges(5, np.array([0, 0, 0]), np.array([1, 2, 3]))
    x = np.array([0.0, 1.0, 0.0, 5.0, 0.5])
    y = np.array([0.0, 0.0, 1.0, 5.0, 0.0])
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, x, y)
    assert v == 0.375 and c == 4
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, x, y, sample=[0, 0, 2, 4])
    assert v == pytest.approx(2.0 / 3.0, rel=1e-15) and c == 3
    v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, x, y, sample=[4])
    assert v == 0.0 and c == 0


def test_np_invariant_under_similarity_transforms():
    """Translation by a dyadic offset, scaling by 2 and a 90 degree rotation
    keep every distance order, so the measure is unchanged."""
    g = random_graph(80, 0.06, 321)
    x, y = dyadic_coords(80, 322)
    v0, c0 = oracle.neighborhood_preservation(g.rowptr, g.colidx, x, y)
    assert 0.0 < v0 < 1.0
    for xs, ys in [(x + 0.5, y - 0.25), (2 * x, 2 * y), (-y, x)]:
        v, c = oracle.neighborhood_preservation(g.rowptr, g.colidx, xs, ys)
        assert v == v0 and c == c0
