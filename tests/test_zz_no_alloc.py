"""The allocation-free quality entry point against bl_quality_eval.

bl_quality_eval_noalloc runs the same kernels as bl_quality_eval with its
work buffers in the library's static device array.  Two calls in a row (the
second on a smaller graph, so stale contents of the array from the first
call would show) must give bl_quality_eval's results bit for bit, and the
limits and argument checks must return BL_E_INVAL without device work
beyond the CSR check.
"""
import numpy as np
import pytest

from paper_2002_08233_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dev_graph(g):
    import torch
    return I.Graph(g.n, torch.as_tensor(g.rowptr, device="cuda"), torch.as_tensor(g.colidx, device="cuda"), g.name)


def _both(g, x, y, pivots):
    import torch
    from paper_2002_08233_amd import api
    ref = api.quality(g, x, y, pivots)
    got = api.quality_noalloc(_dev_graph(g), torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda"),
                              pivots)
    return ref, got


def test_noalloc_equals_allocating_call_twice_in_a_row():
    big = I.rmat(14, 16, seed=23)             # hub rows above 256 entries take the heavy BFS kernel
    assert np.max(np.diff(big.rowptr)) > 256
    xb, yb = I.uniform_coords(big.n, 31)
    piv = I.stress_pivots(big.n, 200, seed=7)
    small = I.grid(20, 23)                    # all pairs, 460 vertices
    xs, ys = I.uniform_coords(small.n, 32)
    for g, x, y, p in ((big, xb, yb, piv), (small, xs, ys, None)):
        print("noalloc case", g.name, g.n, "pivots", None if p is None else len(p), flush=True)
        ref, got = _both(g, x, y, p)
        assert ref["pairs"] > 0 and ref["edges"] == g.nnz // 2
        for k in ref:
            assert got[k] == ref[k], (g.name, k, got[k], ref[k])


def test_noalloc_single_vertex_and_edgeless():
    for g in (I.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64), "one"),
              I.csr_from_edges(70, np.zeros(0, np.int64), np.zeros(0, np.int64), "edgeless")):
        x, y = I.uniform_coords(g.n, 5)
        ref, got = _both(g, x, y, None)
        for k in ref:
            assert got[k] == ref[k], (g.name, k)


def test_noalloc_limits_and_checks():
    import torch
    from paper_2002_08233_amd import _lib as L
    from paper_2002_08233_amd import api
    g = I.grid(8, 8)
    x, y = I.uniform_coords(g.n, 3)
    dg = _dev_graph(g)
    dx, dy = torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda")
    with pytest.raises(ValueError):
        api.quality_noalloc(g, x, y)                         # host arrays
    with pytest.raises(L.BLError) as e:
        api.quality_noalloc(dg, dx, dy, np.zeros(65537, np.int32))
    assert e.value.code == L.BL_E_INVAL
    # n above the limit: rejected before any device access
    big = I.Graph(262145, torch.zeros(262146, dtype=torch.int32, device="cuda"),
                  torch.zeros(0, dtype=torch.int32, device="cuda"), "big")
    zx = torch.zeros(262145, dtype=torch.float64, device="cuda")
    with pytest.raises(L.BLError) as e:
        api.quality_noalloc(big, zx, zx)
    assert e.value.code == L.BL_E_INVAL
    # a column id out of range is caught by the device-side CSR check
    bad_ci = g.colidx.copy()
    bad_ci[5] = g.n
    bad = I.Graph(g.n, torch.as_tensor(g.rowptr, device="cuda"), torch.as_tensor(bad_ci, device="cuda"), "bad")
    with pytest.raises(L.BLError) as e:
        api.quality_noalloc(bad, dx, dy)
    assert e.value.code == L.BL_E_INVAL
    # and the next good call is still right
    ref, got = _both(g, x, y, None)
    for k in ref:
        assert got[k] == ref[k], k
