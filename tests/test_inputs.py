"""Seeded synthetic inputs: shapes, sizes and structure of the workloads."""
import math

import numpy as np
import pytest

from paper_2002_08233_amd import inputs as I


def test_grid32_shape():
    w = I.workload_grid32()
    g = w["graph"]
    I.validate_csr(g)
    assert g.n == 1024 and g.nnz == 2 * 1984
    assert w["batch_size"] == 128 and w["iterations"] == 100
    assert np.all(np.abs(w["x0"]) <= 1) and np.all(np.abs(w["y0"]) <= 1)


def test_rmat_small_is_canonical_and_seeded():
    g1 = I.rmat(10, 16, seed=3)
    g2 = I.rmat(10, 16, seed=3)
    I.validate_csr(g1)
    assert np.array_equal(g1.colidx, g2.colidx)
    d = g1.degrees()
    # skewed: vertex 0 gets quadrant a at every level, so it is the hub
    assert d.argmax() < 16 and d.max() > 10 * d.mean()


def test_rmat_non_power_of_two_keeps_prefix():
    g = I.rmat_n(3000, 8, seed=9)
    I.validate_csr(g)
    assert g.n == 3000


def test_rgg_mean_degree():
    n = 4096
    r = math.sqrt(10.0 / (math.pi * (n - 1)))
    g, pts = I.rgg(n, r, 3)
    I.validate_csr(g)
    assert 8.0 < g.nnz / n < 10.5     # boundary effects lower the mean a little


def test_er_and_ba():
    g = I.erdos_renyi(2000, 8.0, 5)
    I.validate_csr(g)
    assert 7.0 < g.nnz / g.n < 9.0
    b = I.barabasi_albert(2000, 4, 6)
    I.validate_csr(b)
    assert b.degrees().min() >= 4 and abs(b.nnz / b.n - 8.0) < 0.1


def test_validate_rejects_bad_csr():
    g = I.path(4)
    bad = I.Graph(4, g.rowptr.copy(), g.colidx.copy())
    bad.colidx[0] = 0            # self loop at row 0
    with pytest.raises(ValueError):
        I.validate_csr(bad)


def test_served_stream_recipe():
    s = I.served_stream(rate=20, duration=10, seed=6)
    assert 100 < len(s) < 300
    ns = np.array([n for _, n, _ in s])
    assert ns.min() >= 2 ** 10 and ns.max() <= 2 ** 20
    assert np.all(np.diff([t for t, _, _ in s]) > 0)
