"""Seeded synthetic inputs: graphs in CSR form and initial coordinates.

This module holds no arithmetic of the layout method.  It only draws graphs
and starting points, so that the HIP path and the CPU oracle can be fed the
same inputs.  Every generator takes its own ``numpy.random.Generator(PCG64)``
seed; nothing depends on global random state.

Workload recipes (shapes and distributions of the paper's benchmark graphs,
which are not shipped here; synthetic graphs stand in for them):

* ``grid``: 2D lattice graph.
* ``rmat``: recursive-matrix graph (Chakrabarti, Zhan & Faloutsos 2004),
  edge factor x n edges drawn by choosing one of four quadrants per level
  with probabilities (a, b, c, d); symmetrised, self-loops and duplicates
  dropped.  A vertex count that is not a power of two is drawn at the next
  power of two and vertices >= n are dropped.
* ``rgg``: random geometric graph in the unit square.
* ``erdos_renyi``: G(n, M) with M drawn from Binomial(n(n-1)/2, p).
* ``barabasi_albert``: preferential attachment from a (m+1)-clique, m distinct
  degree-proportional targets per new vertex.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Graph:
    """Symmetric CSR graph: sorted rows, no self-loops, no duplicates."""
    n: int
    rowptr: np.ndarray   # int32 [n+1]
    colidx: np.ndarray   # int32 [nnz]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, name: str = "") -> Graph:
    """Symmetrise an edge list, drop self-loops and duplicates, sort rows."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = (src != dst) & (src >= 0) & (dst >= 0) & (src < n) & (dst < n)
    src, dst = src[keep], dst[keep]
    u = np.concatenate([src, dst])
    v = np.concatenate([dst, src])
    code = np.unique(u * n + v)
    u = (code // n).astype(np.int64)
    v = (code % n).astype(np.int32)
    counts = np.bincount(u, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, rowptr.astype(np.int32), v.astype(np.int32), name)


def validate_csr(g: Graph) -> None:
    """Raise ValueError unless g is a symmetric CSR with sorted rows, no self-loops or duplicates."""
    rp, ci, n = g.rowptr, g.colidx, g.n
    if len(rp) != n + 1 or rp[0] != 0 or np.any(np.diff(rp) < 0) or rp[-1] != len(ci):
        raise ValueError("bad rowptr")
    if len(ci) and (ci.min() < 0 or ci.max() >= n):
        raise ValueError("colidx out of range")
    rows = np.repeat(np.arange(n), np.diff(rp))
    if np.any(rows == ci):
        raise ValueError("self-loop")
    code = rows.astype(np.int64) * n + ci
    if np.any(np.diff(code) <= 0):
        raise ValueError("rows not strictly sorted")
    tcode = np.sort(ci.astype(np.int64) * n + rows)
    if not np.array_equal(code, tcode):
        raise ValueError("not symmetric")


def grid(rows: int, cols: int) -> Graph:
    idx = np.arange(rows * cols).reshape(rows, cols)
    src = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    dst = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return csr_from_edges(rows * cols, src, dst, "grid%dx%d" % (rows, cols))


def path(n: int) -> Graph:
    a = np.arange(n - 1)
    return csr_from_edges(n, a, a + 1, "path%d" % n)


def cycle(n: int) -> Graph:
    a = np.arange(n)
    return csr_from_edges(n, a, (a + 1) % n, "cycle%d" % n)


def rmat(scale: int, edge_factor: int, a=0.57, b=0.19, c=0.19, d=0.05, seed=17,
         n: int | None = None) -> Graph:
    n_full = 1 << scale
    n = n_full if n is None else n
    m = edge_factor * n
    r = rng(seed)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    cut_a, cut_b, cut_c = a, a + b, a + b + c
    for level in range(scale):
        u = r.random(m)
        bit = 1 << (scale - 1 - level)
        src_bit = u >= cut_b                       # quadrants c, d: lower half of rows
        dst_bit = ((u >= cut_a) & (u < cut_b)) | (u >= cut_c)   # quadrants b, d
        src |= src_bit.astype(np.int64) * bit
        dst |= dst_bit.astype(np.int64) * bit
    g = csr_from_edges(n, src, dst, "rmat%d_ef%d" % (scale, edge_factor))
    g.meta.update(scale=scale, edge_factor=edge_factor, abcd=(a, b, c, d), seed=seed)
    return g


def rmat_n(n: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19, d=0.05) -> Graph:
    """RMAT with an arbitrary vertex count (drawn at the next power of two)."""
    scale = max(1, int(math.ceil(math.log2(max(n, 2)))))
    return rmat(scale, edge_factor, a, b, c, d, seed=seed, n=n)


def rgg(n: int, radius: float, seed: int):
    """Random geometric graph in the unit square; returns (graph, points)."""
    from scipy.spatial import cKDTree
    pts = rng(seed).random((n, 2))
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    g = csr_from_edges(n, pairs[:, 0], pairs[:, 1], "rgg%d" % n)
    g.meta.update(radius=radius, seed=seed)
    return g, pts


def erdos_renyi(n: int, mean_degree: float, seed: int) -> Graph:
    r = rng(seed)
    p = min(1.0, mean_degree / max(n - 1, 1))
    pairs = n * (n - 1) // 2
    m = int(r.binomial(pairs, p))
    chosen = set()
    codes = []
    while len(codes) < m:
        k = m - len(codes)
        u = r.integers(0, n, size=2 * k + 16)
        v = r.integers(0, n, size=2 * k + 16)
        for a_, b_ in zip(u.tolist(), v.tolist()):
            if a_ == b_:
                continue
            lo, hi = (a_, b_) if a_ < b_ else (b_, a_)
            c_ = lo * n + hi
            if c_ in chosen:
                continue
            chosen.add(c_)
            codes.append(c_)
            if len(codes) == m:
                break
    codes = np.asarray(codes, dtype=np.int64)
    g = csr_from_edges(n, codes // n, codes % n, "er%d" % n)
    g.meta.update(kind="er", mean_degree=mean_degree, seed=seed)
    return g


def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    r = rng(seed)
    m0 = m + 1
    src, dst = [], []
    targets_pool = []
    for i in range(m0):
        for j in range(i + 1, m0):
            src.append(i); dst.append(j)
            targets_pool += [i, j]
    for v in range(m0, n):
        chosen = set()
        while len(chosen) < m:
            chosen.add(targets_pool[int(r.integers(0, len(targets_pool)))])
        for t in sorted(chosen):
            src.append(v); dst.append(t)
            targets_pool += [v, t]
    g = csr_from_edges(n, np.array(src), np.array(dst), "ba%d" % n)
    g.meta.update(kind="ba", m=m, seed=seed)
    return g


def uniform_coords(n: int, seed: int, lo: float = -1.0, hi: float = 1.0):
    """Initial coordinates uniform in [lo, hi]^2 (FP64)."""
    r = rng(seed)
    xy = r.uniform(lo, hi, size=(2, n))
    return xy[0].copy(), xy[1].copy()


def to_f32_representable(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest float32 and back (a shared FP32 state)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def stress_pivots(n: int, count: int = 1024, seed: int = 10):
    """BFS sources of a sampled stress (reading R23): `count` ids drawn
    uniformly with repetition from one seeded generator, or None (all pairs)
    when n <= 65536 and no count is forced."""
    return rng(seed).integers(0, n, count).astype(np.int32)


def ulp_perturbed(x: np.ndarray, seed: int):
    """A copy of x with one entry, chosen by the seed, moved up by one
    float32 ulp (a start that differs from x in one coordinate by one ulp)."""
    xp = np.array(x, dtype=np.float64, copy=True)
    i = int(rng(seed).integers(0, len(xp)))
    xp[i] = float(np.nextafter(np.float32(xp[i]), np.float32(np.inf)))
    return xp, i


# --------------------------------------------------------------------------
# Workload recipes.  Each returns a dict with graph, x0, y0 and run knobs.

def workload_grid32(seed: int = 1):
    """32x32 grid (1024 vertices, 1984 edges); init uniform in [-1,1]^2 FP64;
    batch 128; 100 iterations, exact repulsion."""
    g = grid(32, 32)
    x, y = uniform_coords(g.n, seed)
    return dict(name="grid32x32-exact", graph=g, x0=x, y0=y, batch_size=128, iterations=100,
                mode="exact", theta=0.0)


def workload_rmat17(graph_seed: int = 17, init_seed: int = 2, mode: str = "bh"):
    """RMAT scale 17 (131072 vertices), edge factor 16, (.57,.19,.19,.05),
    symmetrised; init uniform in [-1,1]^2; batch 256; theta 1.2; 600 iterations."""
    g = rmat(17, 16, seed=graph_seed)
    x, y = uniform_coords(g.n, init_seed)
    x, y = to_f32_representable(x), to_f32_representable(y)
    return dict(name="rmat17-ef16-%s" % mode, graph=g, x0=x, y0=y, batch_size=256,
                iterations=600, mode=mode, theta=1.2)


def workload_rgg64k(point_seed: int = 3, noise_seed: int = 4, n: int = 65536):
    """Random geometric graph, 65536 vertices, radius for mean degree 10;
    init = points + N(0, 0.01^2); batch 512; 300 iterations; exact."""
    radius = math.sqrt(10.0 / (math.pi * (n - 1)))
    g, pts = rgg(n, radius, point_seed)
    noise = rng(noise_seed).normal(0.0, 0.01, size=(n, 2))
    x = to_f32_representable(pts[:, 0] + noise[:, 0])
    y = to_f32_representable(pts[:, 1] + noise[:, 1])
    return dict(name="rgg64k-exact", graph=g, x0=x, y0=y, batch_size=512, iterations=300,
                mode="exact", theta=0.0)


def batched_sizes(count: int = 512, seed: int = 5, lo: int = 200, hi: int = 20000):
    r = rng(seed)
    return np.exp(r.uniform(math.log(lo), math.log(hi), size=count)).astype(np.int64)


def workload_batched(count: int = 512, seed: int = 5, scale_down: float = 1.0):
    """Many independent graphs: n log-uniform in [200, 20000], half Erdos-Renyi
    (mean degree 8), half Barabasi-Albert (m=4) by seed; init uniform in
    [-1,1]^2; batch 128; exact below 4096 vertices, Barnes-Hut theta 1.0 above;
    200 iterations."""
    sizes = batched_sizes(count, seed)
    if scale_down != 1.0:
        sizes = np.maximum(8, (sizes * scale_down).astype(np.int64))
    jobs = []
    for gi, n in enumerate(sizes.tolist()):
        s = 5000 + gi
        if rng(s).random() < 0.5:
            g = erdos_renyi(int(n), 8.0, s)
        else:
            g = barabasi_albert(int(n), 4, s)
        x, y = uniform_coords(g.n, s + 100000)
        x, y = to_f32_representable(x), to_f32_representable(y)
        mode = "exact" if g.n < 4096 else "bh"
        jobs.append(dict(graph=g, x0=x, y0=y, batch_size=128, iterations=200, mode=mode,
                         theta=1.0 if mode == "bh" else 0.0))
    return jobs


def served_stream(rate: float = 20.0, duration: float = 120.0, seed: int = 6,
                  lo_log2: float = 10, hi_log2: float = 20):
    """Poisson arrivals; each request an RMAT graph (edge factor 8) with n
    log-uniform in [2^lo, 2^hi]; returns a list of (arrival_time, n, seed)."""
    r = rng(seed)
    t = 0.0
    out = []
    k = 0
    while True:
        t += r.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(round(2.0 ** r.uniform(lo_log2, hi_log2)))
        out.append((t, n, 6000 + k))
        k += 1
    return out


def served_request(n: int, seed: int):
    g = rmat_n(n, 8, seed)
    x, y = uniform_coords(g.n, seed + 100000)
    return dict(graph=g, x0=to_f32_representable(x), y0=to_f32_representable(y),
                batch_size=256, iterations=300, mode="bh", theta=1.2)
