"""Pins of the batch-randomisation oracle (Sec. 4.3.3) and of Hu's adaptive step
(cited in Sec. 4.3.5).  Batch order: the generator against
published outputs, the shuffle's uniformity, and the shuffled run against a
brute-force statement of randomised minibatches on the original labels."""
import collections
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import inputs as I
from test_oracle_pins import _py_force, random_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_stream():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.json")) as f:
        gold = json.load(f)
    got = [oracle.splitmix64(gold["seed"] + t * oracle._SM_GAMMA) for t in (1, 2, 3)]
    assert got == [int(h, 16) for h in gold["outputs_hex"]]


@pytest.mark.parametrize("n", [1, 2, 17, 300])
def test_batch_permutation_is_a_permutation(n):
    for k in range(3):
        p = oracle.batch_permutation(n, 12345, k)
        assert sorted(p.tolist()) == list(range(n))
    if n > 2:
        assert not np.array_equal(oracle.batch_permutation(n, 12345, 0), oracle.batch_permutation(n, 12345, 1))
        assert not np.array_equal(oracle.batch_permutation(n, 1, 0), oracle.batch_permutation(n, 2, 0))


@pytest.mark.parametrize("n", [3, 4])
def test_batch_permutation_is_uniform(n):
    """Every order equally likely (a swap partner drawn from all n positions
    instead of the first i+1 would skew these counts far beyond the bound)."""
    draws = 600 * math.factorial(n)
    counts = collections.Counter(tuple(oracle.batch_permutation(n, 77, k).tolist()) for k in range(draws))
    assert len(counts) == math.factorial(n)
    expect = draws / math.factorial(n)
    chi2 = sum((c - expect) ** 2 / expect for c in counts.values())
    # chi-square with 5 or 23 degrees of freedom: these bounds hold with p > 0.999
    assert chi2 < {3: 20.5, 4: 49.7}[n], (chi2, counts)


def _py_layout_shuffled(rp, ci, x, y, bs, iters, seed, step=1.0, decay=0.999):
    """Randomised minibatches on the original labels: iteration k takes the
    runs of bs entries of the permutation, each run's forces from the
    positions before it, then moves the run (Jacobi within, Gauss-Seidel
    across)."""
    x, y = list(x), list(y)
    n = len(x)
    energies = []
    for k in range(iters):
        order = oracle.batch_permutation(n, seed, k).tolist()
        e = 0.0
        for b0 in range(0, n, bs):
            batch = order[b0:b0 + bs]
            forces = [_py_force(rp, ci, x, y, i) for i in batch]
            for i, (fx, fy) in zip(batch, forces):
                norm = math.hypot(fx, fy)
                if norm > 0:
                    x[i] += step * fx / norm
                    y[i] += step * fy / norm
                e += fx * fx + fy * fy
        energies.append(e)
        step *= decay
    return np.array(x), np.array(y), np.array(energies)


@pytest.mark.parametrize("bs", [1, 5, 8])
def test_shuffled_run_is_randomised_minibatches(bs):
    g = random_graph(24, 0.2, 41)
    x0, y0 = I.uniform_coords(24, 42)
    xr, yr, er = _py_layout_shuffled(g.rowptr, g.colidx, x0, y0, bs, 4, seed=99)
    x, y, e = oracle.layout_shuffled(g.rowptr, g.colidx, x0, y0, bs, 4, seed=99)
    assert np.allclose(x, xr, atol=1e-10) and np.allclose(y, yr, atol=1e-10)
    assert np.allclose(e, er, rtol=1e-10)
    xu, yu, _ = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, bs, 4)
    assert not np.allclose(x, xu, atol=1e-6)      # the order matters at these batch sizes


def test_one_batch_is_the_unshuffled_run():
    """With a single batch of all n vertices the order is irrelevant."""
    g = random_graph(30, 0.15, 43)
    x0, y0 = I.uniform_coords(30, 44)
    x, y, e = oracle.layout_shuffled(g.rowptr, g.colidx, x0, y0, 30, 5, seed=3)
    xu, yu, eu = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 30, 5)
    assert np.allclose(x, xu, atol=1e-12) and np.allclose(y, yu, atol=1e-12) and np.allclose(e, eu, rtol=1e-12)


def test_shuffled_resume_and_bh_one_batch():
    g = random_graph(30, 0.15, 45)
    x0, y0 = I.uniform_coords(30, 46)
    xa, ya, ea = oracle.layout_shuffled(g.rowptr, g.colidx, x0, y0, 4, 6, seed=5)
    xb, yb, eb = oracle.layout_shuffled(g.rowptr, g.colidx, x0, y0, 4, 2, seed=5)
    xc, yc, ec = oracle.layout_shuffled(g.rowptr, g.colidx, xb, yb, 4, 4, seed=5, start_iter=2)
    assert np.array_equal(xa, xc) and np.array_equal(ya, yc) and np.array_equal(ea, np.concatenate([eb, ec]))
    x, y, e = oracle.layout_shuffled(g.rowptr, g.colidx, x0, y0, 30, 3, seed=3, mode="bh", theta=1.2)
    xu, yu, eu, _ = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, 30, 3, theta=1.2)
    assert np.allclose(x, xu, atol=1e-10) and np.allclose(y, yu, atol=1e-10) and np.allclose(e, eu, rtol=1e-10)


@pytest.mark.parametrize("bs", [1, 7])
def test_shuffled_bh_run_is_randomised_minibatches(bs):
    """Barnes-Hut: the tree of the iteration's start snapshot, live leaves,
    the permutation's runs as minibatches, on the original labels."""
    g = random_graph(40, 0.1, 47)
    x, y = (a.copy() for a in I.uniform_coords(40, 48))
    x0, y0 = x.copy(), y.copy()
    step, er = 1.0, []
    for k in range(3):
        tree = oracle.Tree(x.copy(), y.copy())
        order = oracle.batch_permutation(40, 11, k)
        e = 0.0
        for b0 in range(0, 40, bs):
            batch = order[b0:b0 + bs]
            f = [oracle.forces_bh(g.rowptr, g.colidx, x, y, tree, int(i), int(i) + 1, theta=1.2) for i in batch]
            for i, fi in zip(batch, f):
                fx, fy = fi.fx[0], fi.fy[0]
                norm = math.hypot(fx, fy)
                if norm > 0:
                    x[i] += step * fx / norm
                    y[i] += step * fy / norm
                e += fx * fx + fy * fy
        er.append(e)
        step *= 0.999
    xs, ys, es = oracle.layout_shuffled(g.rowptr, g.colidx, x0, y0, bs, 3, seed=11, mode="bh", theta=1.2)
    assert np.allclose(xs, x, atol=1e-10) and np.allclose(ys, y, atol=1e-10) and np.allclose(es, er, rtol=1e-10)


def _relabel(rowptr, colidx, perm):
    """The graph with vertex perm[q] renamed q (rows sorted again)."""
    rp = np.asarray(rowptr, dtype=np.int64)
    ci = np.asarray(colidx, dtype=np.int64)
    n = len(rp) - 1
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    rows = [np.sort(inv[ci[rp[v]:rp[v + 1]]]) for v in perm]
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum([len(r) for r in rows])
    ci2 = np.concatenate(rows) if len(ci) else np.zeros(0, dtype=np.int64)
    return rp2.astype(np.int32), ci2.astype(np.int32)


@pytest.mark.parametrize("mode,bs", [("exact", 6), ("exact", 13), ("bh", 6)])
def test_shuffled_run_is_invariant_under_relabelling(mode, bs):
    """Renaming vertex pi_k[q] to q turns the permutation's runs into id
    ranges; one ordinary iteration on the renamed graph, mapped back, is the
    shuffled iteration (same arithmetic up to summation order)."""
    g = random_graph(45, 0.12, 311)
    x, y = I.uniform_coords(45, 312)
    kw = dict(theta=1.2) if mode == "bh" else {}
    xs, ys, es = oracle.layout_shuffled(g.rowptr, g.colidx, x, y, bs, 3, seed=21, mode=mode, **kw)
    xr, yr, er = x.copy(), y.copy(), []
    for k in range(3):
        perm = oracle.batch_permutation(45, 21, k)
        rp2, ci2 = _relabel(g.rowptr, g.colidx, perm)
        if mode == "exact":
            xk, yk, ek = oracle.layout_exact(rp2, ci2, xr[perm], yr[perm], bs, 1, k)
        else:
            xk, yk, ek, _ = oracle.layout_bh(rp2, ci2, xr[perm], yr[perm], bs, 1, k, **kw)
        xr[perm], yr[perm] = xk, yk
        er.append(ek[0])
    assert np.allclose(xs, xr, atol=1e-10) and np.allclose(ys, yr, atol=1e-10) and np.allclose(es, er, rtol=1e-10)


# ------------------------------------------------------- Hu's adaptive step

def test_hu_update_worked_sequence():
    """Hu's rule worked by hand for t = 0.5 on a scripted energy sequence:
    five drops grow the step once; a rise shrinks it and restarts the count."""
    energies = [10, 9, 8, 7, 6, 5, 4, 6, 5, 4, 3, 2, 1, 0.5]
    # step used by each iteration, from 1.0
    want = [1, 1, 1, 1, 1, 2, 2, 2, 1, 1, 1, 1, 1, 2]
    step, prog, prev, got = 1.0, 0, float("inf"), []
    for e in energies:
        got.append(step)
        step, prog = oracle.hu_step_update(step, prog, e, prev, 0.5)
        prev = e
    assert got == want


def test_adaptive_with_unit_factor_is_the_fixed_step_run():
    g = random_graph(30, 0.15, 51)
    x0, y0 = I.uniform_coords(30, 52)
    x, y, e, steps = oracle.layout_adaptive(g.rowptr, g.colidx, x0, y0, 7, 6, step0=0.3, t=1.0)
    xf, yf, ef = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, 7, 6, step0=0.3, decay=1.0)
    assert np.array_equal(x, xf) and np.array_equal(y, yf) and np.array_equal(e, ef)
    assert np.all(steps == 0.3)


def test_adaptive_steps_follow_the_energies():
    """The recorded steps obey the rule against the run's own energies, and
    the run equals the fixed-step iterations replayed with those steps."""
    g = random_graph(30, 0.15, 53)
    x0, y0 = I.uniform_coords(30, 54)
    x, y, e, steps = oracle.layout_adaptive(g.rowptr, g.colidx, x0, y0, 8, 25, step0=0.5, t=0.9)
    assert len(set(np.round(steps, 12))) > 2             # the step moved both ways or more than once
    prev, prog, s = float("inf"), 0, 0.5
    xr, yr = x0, y0
    for k in range(25):
        assert steps[k] == s
        xr, yr, ek = oracle.layout_exact(g.rowptr, g.colidx, xr, yr, 8, 1, step0=steps[k], decay=1.0)
        assert ek[0] == e[k]
        s, prog = (s / 0.9, 0) if (e[k] < prev and prog + 1 >= 5) else \
                  ((s, prog + 1) if e[k] < prev else (s * 0.9, 0))
        prev = e[k]
    assert np.array_equal(x, xr) and np.array_equal(y, yr)
