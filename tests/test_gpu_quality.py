"""Quality measures of Sec. 3.7 on the GPU (bl_quality_eval) against the
oracle's FP64 evaluators (needs an MI355X).

Pair and edge counts are integers and must match exactly; they pin the BFS
(hop distances, unreachable pairs, the i < j rule, pivot repeats).  The sums
are FP64 in another order than the oracle's, so they agree to a relative
1e-9 (stress, whose closed form N - A^2/B cancels) and 1e-11 (the rest).
"""
import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I

pytestmark = pytest.mark.gpu


def _ref(g, x, y, pivots=None, K=1.0):
    s, scale = oracle.stress(g.rowptr, g.colidx, x, y, pivots)
    return dict(stress=s, scale=scale, edge_energy=oracle.edge_energy(g.rowptr, g.colidx, x, y, K),
                edge_uniformity=oracle.edge_uniformity(g.rowptr, g.colidx, x, y))


def _pairs(g, pivots=None):
    """Reachable pairs counted by a scipy BFS (independent of both sides)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    A = csr_matrix((np.ones(g.nnz), g.colidx, g.rowptr), shape=(g.n, g.n))
    if pivots is None:
        d = shortest_path(A, unweighted=True, directed=False)
        iu = np.triu_indices(g.n, 1)
        return int(np.isfinite(d[iu]).sum())
    d = shortest_path(A, unweighted=True, directed=False, indices=np.asarray(pivots))
    return int(np.isfinite(d).sum() - len(pivots))


def _check(g, x, y, pivots=None, K=1.0):
    q = api.quality(g, x, y, pivots, K)
    r = _ref(g, x, y, pivots, K)
    assert q["pairs"] == _pairs(g, pivots)
    assert q["edges"] == g.nnz // 2
    assert q["stress"] == pytest.approx(r["stress"], rel=1e-9, abs=1e-9)
    assert q["scale"] == pytest.approx(r["scale"], rel=1e-11)
    assert q["edge_energy"] == pytest.approx(r["edge_energy"], rel=1e-11)
    assert q["edge_uniformity"] == pytest.approx(r["edge_uniformity"], rel=1e-10, abs=1e-14)
    return q


def test_grid_all_pairs():
    g = I.grid(32, 32)
    for seed in (1, 2):
        x, y = I.uniform_coords(g.n, seed)
        _check(g, x, y)
    gx = (np.arange(g.n) % 32).astype(float)
    gy = (np.arange(g.n) // 32).astype(float)
    q = _check(g, gx + 0.1 * np.sin(gy), gy)
    assert q["pairs"] == g.n * (g.n - 1) // 2


def test_path_on_a_line_has_zero_stress():
    """A layout equal to the graph metric: stress 0 at scale 1."""
    g = I.path(300)
    q = api.quality(g, np.arange(300.0), np.zeros(300))
    assert abs(q["stress"]) <= 1e-9 * q["pairs"] and q["scale"] == pytest.approx(1.0, rel=1e-14)
    assert q["edge_uniformity"] == 0.0


@pytest.mark.parametrize("n,deg,seed", [(1000, 1.2, 3), (2000, 3.0, 4)])
def test_components_and_ragged_passes_all_pairs(n, deg, seed):
    """Several components (unreachable pairs skipped); n not a multiple of 64."""
    g = I.erdos_renyi(n, deg, seed)
    x, y = I.uniform_coords(n, seed + 10)
    _check(g, x, y, K=0.7)


def test_pivots_with_repeats_and_isolated_vertices():
    g = I.rmat(12, 8, seed=5)
    x, y = I.uniform_coords(g.n, 6)
    iso = int(np.flatnonzero(np.diff(g.rowptr) == 0)[0])
    r = I.rng(7)
    piv = np.concatenate([r.integers(0, g.n, 100), [iso, 3, 3]]).astype(np.int32)
    _check(g, x, y, piv)


def test_rgg_long_diameter():
    g, pts = I.rgg(3000, 0.04, 8)
    _check(g, pts[:, 0], pts[:, 1])


def test_single_vertex_and_edgeless():
    g = I.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    q = api.quality(g, np.zeros(1), np.zeros(1))
    assert q["pairs"] == 0 and q["edges"] == 0 and q["stress"] == 0.0
    g = I.csr_from_edges(70, np.zeros(0, np.int64), np.zeros(0, np.int64))
    x, y = I.uniform_coords(70, 1)
    q = api.quality(g, x, y)
    assert q["pairs"] == 0 and q["edges"] == 0 and q["edge_energy"] == 0.0


def test_rmat17_pivots_full_size():
    """The default workload's graph and start, 64 sampled pivots."""
    w = I.workload_rmat17()
    g = w["graph"]
    piv = I.rng(9).integers(0, g.n, 64).astype(np.int32)
    _check(g, w["x0"], w["y0"], piv)


def test_device_pointers_and_repeat_bitwise():
    import torch
    g = I.rmat(11, 16, seed=3)
    x, y = I.uniform_coords(g.n, 4)
    piv = np.arange(0, g.n, 7, dtype=np.int32)
    a = api.quality(g, x, y, piv)
    b = api.quality(g, x, y, piv)
    dev = I.Graph(g.n, torch.as_tensor(g.rowptr, device="cuda"), torch.as_tensor(g.colidx, device="cuda"))
    c = api.quality(dev, torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda"), piv)
    assert a == b == c
