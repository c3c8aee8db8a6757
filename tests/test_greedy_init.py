"""Greedy initial layout (Sec. 3.6, Algorithm 3): the library's host routine
against the oracle.

The traversal is the same integer decision sequence on both sides (which
vertex places which, at which angle slot), so a wrong pop order, angle slot or
component root moves a vertex by O(1).  Positions agree to rounding: the
routines call the host's cos and sin, which are not correctly rounded and may
differ by an ulp between a sin/cos pair and a fused sincos; the error adds up
along the traversal's tree paths, so the bound scales with the largest
coordinate.  No device work: these run in the CPU suite.
"""
import ctypes as C
import os

import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from paper_2002_08233_amd import _lib


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def _check(g, start, xr=None, yr=None):
    x, y = api.greedy_init(g, start, xr, yr)
    xo, yo, par = oracle.greedy_init(g.rowptr, g.colidx, start, xr, yr)
    tol = 1e-12 * max(1.0, np.abs(xo).max(), np.abs(yo).max())
    np.testing.assert_allclose(x, xo, rtol=0, atol=tol)
    np.testing.assert_allclose(y, yo, rtol=0, atol=tol)
    # vertices placed from the start and component roots: exact
    assert (x[start], y[start]) == (0.0, 0.0)
    for r in np.flatnonzero(par < 0):
        if r != start:
            assert (x[r], y[r]) == (xr[r], yr[r])
    return x, y, par


def test_small_cases():
    _check(I.path(9), 0)
    _check(I.path(9), 4)
    _check(I.cycle(11), 3)
    _check(I.grid(7, 9), 31)
    star = I.csr_from_edges(13, np.zeros(12, np.int64), np.arange(1, 13))
    _check(star, 0)
    _check(star, 5)
    sq = I.csr_from_edges(4, np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3]))
    _check(sq, 0)


def test_single_vertex_and_edgeless():
    g = I.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    x, y = api.greedy_init(g, 0)
    assert (x[0], y[0]) == (0.0, 0.0)
    g = I.csr_from_edges(5, np.zeros(0, np.int64), np.zeros(0, np.int64))
    xr, yr = I.uniform_coords(5, 3)
    x, y = api.greedy_init(g, 2, xr, yr)
    assert (x[2], y[2]) == (0.0, 0.0)
    keep = [0, 1, 3, 4]
    assert np.array_equal(x[keep], xr[keep]) and np.array_equal(y[keep], yr[keep])


@pytest.mark.parametrize("kind,seed", [("er", 1), ("er", 2), ("ba", 3), ("rmat", 4), ("rgg", 5)])
def test_random_graphs_with_components(kind, seed):
    if kind == "er":
        g = I.erdos_renyi(3000, 1.5, seed)          # many components, isolated vertices
    elif kind == "ba":
        g = I.barabasi_albert(4000, 4, seed)
    elif kind == "rmat":
        g = I.rmat(12, 8, seed=seed)
    else:
        g, _ = I.rgg(4000, 0.015, seed)
    xr, yr = I.uniform_coords(g.n, 100 + seed)
    r = I.rng(200 + seed)
    for start in r.integers(0, g.n, 3):
        _check(g, int(start), xr, yr)


def test_rmat17_full_size():
    """The default workload's graph (131072 vertices, ~3.7M entries, ~41k isolated vertices)."""
    w = I.workload_rmat17()
    x, y, par = _check(w["graph"], 0, w["x0"], w["y0"])
    assert (par < 0).sum() > 40000


def test_bad_arguments():
    lib = _lib.load()
    g = I.path(4)
    with pytest.raises(_lib.BLError):
        api.greedy_init(g, 4)
    with pytest.raises(_lib.BLError):
        api.greedy_init(g, -1)
    keep = api._Keep()
    csr = api._csr(g, keep)
    x = np.zeros(4)
    assert lib.bl_greedy_init(C.byref(csr), 0, None, x.ctypes.data) == _lib.BL_E_INVAL
    assert lib.bl_greedy_init(None, 0, x.ctypes.data, x.ctypes.data) == _lib.BL_E_INVAL
    bad = I.path(4)
    ci = bad.colidx.copy()
    ci[0] = 7
    csr.colidx = keep.ptr(ci, np.int32)
    assert lib.bl_greedy_init(C.byref(csr), 0, x.ctypes.data, x.ctypes.data) == _lib.BL_E_INVAL
