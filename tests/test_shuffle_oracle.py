"""Pins of the batch-randomisation oracle (Sec. 4.2): the generator against
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
