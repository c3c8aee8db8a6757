"""FP64 CPU oracle for the BatchLayout force step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports, links or executes anything here.

The arithmetic lives in ``bl_oracle.c`` (plain C, FP64, compiled with
``-O2 -fno-fast-math -ffp-contract=off``); this module marshals numpy arrays
through ctypes and applies the energy stopping rule between iterations (one
comparison of two energies).  Every function cites the passage of the paper
it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bl_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = C.CDLL(_LIB_PATH)
    lib.orc_forces_exact.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int,
                                     C.c_double, C.c_double, C.c_int,
                                     _f64p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_forces_exact_ar.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int,
                                        C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                        _f64p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_layout_exact_ar.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int, C.c_int,
                                        C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                        C.c_int, C.c_int, C.c_int, _f64p]
    lib.orc_layout_exact_ord.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int, C.c_int,
                                         C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                         C.c_int, C.c_int, C.c_int, C.c_void_p, _f64p]
    lib.orc_step_at.argtypes = [C.c_double, C.c_double, C.c_int]
    lib.orc_step_at.restype = C.c_double
    lib.orc_layout_exact.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int, C.c_int,
                                     C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                     C.c_int, _f64p]
    lib.orc_tree_build.argtypes = [C.c_int, _f64p, _f64p]
    lib.orc_tree_build.restype = C.c_void_p
    lib.orc_tree_free.argtypes = [C.c_void_p]
    lib.orc_tree_nnodes.argtypes = [C.c_void_p]
    lib.orc_tree_width.argtypes = [C.c_void_p]
    lib.orc_tree_width.restype = C.c_double
    lib.orc_tree_node.argtypes = [C.c_void_p, C.c_int] + [C.POINTER(C.c_int)] * 4 + \
        [C.POINTER(C.c_int * 4), C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.orc_tree_order.argtypes = [C.c_void_p, _i32p, _u32p]
    lib.orc_forces_bh.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_void_p, C.c_int, C.c_int,
                                  C.c_double, C.c_double, C.c_double, C.c_int,
                                  _f64p, _f64p, _f64p, _f64p, _f64p, _i64p, _i32p]
    lib.orc_forces_bh_ar.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_void_p, C.c_int, C.c_int,
                                     C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                     _f64p, _f64p, _f64p, _f64p, _f64p, _i64p, _i32p]
    lib.orc_layout_bh_ord.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int, C.c_int,
                                      C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, _f64p,
                                      C.c_void_p, C.c_void_p, C.POINTER(C.c_long)]
    lib.orc_layout_bh.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_int, C.c_int,
                                  C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_int, C.c_int, _f64p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_long)]
    lib.orc_edge_energy.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_double]
    lib.orc_edge_energy.restype = C.c_double
    lib.orc_edge_uniformity.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p]
    lib.orc_edge_uniformity.restype = C.c_double
    lib.orc_stress.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_void_p,
                               C.POINTER(C.c_double)]
    lib.orc_stress.restype = C.c_double
    lib.orc_neighborhood_preservation.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, C.c_void_p,
                                                  C.POINTER(C.c_long)]
    lib.orc_neighborhood_preservation.restype = C.c_double
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_get_threads.restype = C.c_int
    lib.orc_greedy_init.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _f64p, _f64p, _f64p, _f64p, _i32p]
    _lib = lib
    return lib


def set_threads(t: int) -> int:
    """Threads for the oracle's parallel loops (t <= 0: one per host core).
    Results do not depend on it.  Returns the count now in effect."""
    lib = _load()
    lib.orc_set_threads(int(t))
    return lib.orc_get_threads()


def threads() -> int:
    return _load().orc_get_threads()


def _csr(rowptr, colidx):
    return (np.ascontiguousarray(rowptr, dtype=np.int32),
            np.ascontiguousarray(colidx if len(colidx) else np.zeros(1, np.int32), dtype=np.int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Forces:
    """Per-vertex attraction (ax, ay), repulsion (rx, ry), scale S_i = sum |term|."""

    def __init__(self, ax, ay, rx, ry, scale, visits=None, near_tie=None):
        self.ax, self.ay, self.rx, self.ry, self.scale = ax, ay, rx, ry, scale
        self.visits, self.near_tie = visits, near_tie

    @property
    def fx(self):
        return self.ax + self.rx

    @property
    def fy(self):
        return self.ay + self.ry


def step_at(step0: float, decay: float, k: int) -> float:
    """Step length at iteration k (step0 times decay, once per finished iteration)."""
    return _load().orc_step_at(step0, decay, k)


def forces_exact(rowptr, colidx, x, y, i0, i1, K=1.0, R=1.0, repulse_adjacent=True, model=(2, -1)) -> Forces:
    """Exact net forces on vertices [i0, i1) from coordinates (x, y) (Sec. 2.2; Alg. 2).

    model = (a, r): attraction magnitude d^a / K, repulsion magnitude R K^2 d^r
    (integers; (2, -1) is Fruchterman-Reingold)."""
    lib = _load()
    rp, ci = _csr(rowptr, colidx)
    n = len(rp) - 1
    m = i1 - i0
    out = [np.zeros(max(m, 1)) for _ in range(5)]
    rc = lib.orc_forces_exact_ar(n, rp, ci, _f64(x), _f64(y), i0, i1, K, R, int(repulse_adjacent),
                                 int(model[0]), int(model[1]), *out)
    if rc != 0:
        raise ValueError("orc_forces_exact: bad arguments")
    return Forces(*[o[:m] for o in out])


def _converged(e, conv_tol):
    """The energy stopping rule (Sec. 4.5), read as a relative change: after
    an iteration that is not the run's first, stop when |E_k - E_{k-1}| <=
    conv_tol * E_{k-1}."""
    return conv_tol > 0 and len(e) >= 2 and abs(e[-1] - e[-2]) <= conv_tol * e[-2]


def _order_arg(order, n):
    if order is None:
        return None, None
    o = np.ascontiguousarray(order, dtype=np.int32)
    if len(o) != n or not np.array_equal(np.sort(o), np.arange(n)):
        raise ValueError("order must be a permutation of 0..n-1")
    return o, o.ctypes.data_as(C.c_void_p)


def layout_exact(rowptr, colidx, x0, y0, bs, iters, start_iter=0, step0=1.0, decay=0.999,
                 K=1.0, R=1.0, repulse_adjacent=True, stop_batch=-1, conv_tol=0.0, model=(2, -1),
                 order=None):
    """Exact BatchLayout (Alg. 2 semantics) with the (a, r) model of Sec. 2.2.
    order: a permutation whose runs of bs entries are the batches (default:
    consecutive ids).  Returns (x, y, energy per iteration); with conv_tol > 0
    the run ends where the energy stopping rule holds."""
    if conv_tol > 0:
        assert stop_batch < 0
        x, y, es = x0, y0, []
        for t in range(iters):
            x, y, e = layout_exact(rowptr, colidx, x, y, bs, 1, start_iter + t, step0, decay, K, R,
                                   repulse_adjacent, model=model, order=order)
            es.append(e[0])
            if _converged(es, conv_tol):
                break
        return _f64(x), _f64(y), np.array(es)
    lib = _load()
    rp, ci = _csr(rowptr, colidx)
    n = len(rp) - 1
    x = _f64(x0).copy()
    y = _f64(y0).copy()
    e = np.zeros(max(iters, 1))
    keep, optr = _order_arg(order, n)
    rc = lib.orc_layout_exact_ord(n, rp, ci, x, y, bs, iters, start_iter, step0, decay, K, R,
                                  int(repulse_adjacent), int(model[0]), int(model[1]), stop_batch, optr, e)
    if rc != 0:
        raise ValueError("orc_layout_exact failed (%d)" % rc)
    return x, y, e[:iters]


class Tree:
    """Quadtree of a snapshot (Alg. S1) built by the oracle."""

    def __init__(self, sx, sy):
        self._lib = _load()
        self.n = len(sx)
        self.h = self._lib.orc_tree_build(self.n, _f64(sx), _f64(sy))
        if not self.h:
            raise ValueError("orc_tree_build failed")

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.orc_tree_free(self.h)
            self.h = None

    @property
    def width(self):
        return self._lib.orc_tree_width(self.h)

    def nodes(self):
        out = []
        lv, lo, hi, nc, bk = (C.c_int() for _ in range(5))
        ch = (C.c_int * 4)()
        cx, cy = C.c_double(), C.c_double()
        for i in range(self._lib.orc_tree_nnodes(self.h)):
            self._lib.orc_tree_node(self.h, i, C.byref(lv), C.byref(lo), C.byref(hi), C.byref(nc),
                                    C.byref(ch), C.byref(bk), C.byref(cx), C.byref(cy))
            out.append(dict(level=lv.value, lo=lo.value, hi=hi.value, children=list(ch)[:nc.value],
                            bucket=bool(bk.value), cx=cx.value, cy=cy.value))
        return out

    def order(self):
        order = np.zeros(self.n, np.int32)
        keys = np.zeros(self.n, np.uint32)
        self._lib.orc_tree_order(self.h, order, keys)
        return order, keys


def forces_bh(rowptr, colidx, x, y, tree: Tree, i0, i1, K=1.0, R=1.0, theta=1.2,
              leaf_live=True, model=(2, -1)) -> Forces:
    """Barnes-Hut forces on [i0, i1): CSR attraction + tree repulsion (Alg. S2,
    S3) under the (a, r) model of Sec. 2.2 (an accepted cell adds count times
    the repulsion from its centroid)."""
    lib = _load()
    rp, ci = _csr(rowptr, colidx)
    n = len(rp) - 1
    m = i1 - i0
    out = [np.zeros(max(m, 1)) for _ in range(5)]
    vis = np.zeros(max(m, 1), np.int64)
    tie = np.zeros(max(m, 1), np.int32)
    rc = lib.orc_forces_bh_ar(n, rp, ci, _f64(x), _f64(y), tree.h, i0, i1, K, R, theta,
                              int(leaf_live), int(model[0]), int(model[1]), *out, vis, tie)
    if rc != 0:
        raise ValueError("orc_forces_bh: bad arguments")
    return Forces(*[o[:m] for o in out], visits=vis[:m], near_tie=tie[:m].astype(bool))


def layout_bh(rowptr, colidx, x0, y0, bs, iters, start_iter=0, step0=1.0, decay=0.999,
              K=1.0, R=1.0, theta=1.2, leaf_live=True, stop_batch=-1, want_snapshot=False, conv_tol=0.0,
              model=(2, -1), order=None):
    """BatchLayoutBH (Alg. S3 with the step decay of Alg. 2) under the (a, r)
    model; order as in layout_exact.

    Returns (x, y, energy, visits) or, with want_snapshot, also the snapshot
    (sx, sy) taken at the start of the last iteration.  With conv_tol > 0 the
    run ends where the energy stopping rule holds."""
    if conv_tol > 0:
        assert stop_batch < 0 and not want_snapshot
        x, y, es, vt = x0, y0, [], 0
        for t in range(iters):
            x, y, e, v = layout_bh(rowptr, colidx, x, y, bs, 1, start_iter + t, step0, decay, K, R, theta,
                                   leaf_live, model=model, order=order)
            es.append(e[0])
            vt += v
            if _converged(es, conv_tol):
                break
        return _f64(x), _f64(y), np.array(es), vt
    lib = _load()
    rp, ci = _csr(rowptr, colidx)
    n = len(rp) - 1
    x = _f64(x0).copy()
    y = _f64(y0).copy()
    e = np.zeros(max(iters, 1))
    sx = np.zeros(n)
    sy = np.zeros(n)
    vt = C.c_long(0)
    keep, optr = _order_arg(order, n)
    rc = lib.orc_layout_bh_ord(n, rp, ci, x, y, bs, iters, start_iter, step0, decay, K, R, theta,
                               int(leaf_live), int(model[0]), int(model[1]), stop_batch, optr, e,
                               sx.ctypes.data_as(C.c_void_p) if want_snapshot else None,
                               sy.ctypes.data_as(C.c_void_p) if want_snapshot else None,
                               C.byref(vt))
    if rc != 0:
        raise ValueError("orc_layout_bh failed (%d)" % rc)
    if want_snapshot:
        return x, y, e[:iters], vt.value, sx, sy
    return x, y, e[:iters], vt.value


def hu_step_update(step, progress, e, e_prev, t):
    """One update of Hu's adaptive step (Hu 2005, the scheme Sec. 4.3.5 cites):
    an energy drop advances a progress count, and the fifth in a row resets
    it and grows the step by 1/t; any other outcome resets the count and
    shrinks the step by t.  Returns (step, progress)."""
    if e < e_prev:
        progress += 1
        if progress >= 5:
            return step / t, 0
        return step, progress
    return step * t, 0


def layout_adaptive(rowptr, colidx, x0, y0, bs, iters, step0=1.0, t=0.9, mode="exact", conv_tol=0.0, **kw):
    """BatchLayout with Hu's adaptive step instead of the fixed decay:
    iteration k runs at step s_k (s_0 = step0, E_{-1} = +inf), then
    hu_step_update gives s_{k+1}.  Returns (x, y, energy, steps)."""
    x, y = _f64(x0).copy(), _f64(y0).copy()
    step, progress, e_prev = step0, 0, float("inf")
    es, steps = [], []
    for k in range(iters):
        steps.append(step)
        if mode == "exact":
            x, y, e = layout_exact(rowptr, colidx, x, y, bs, 1, 0, step0=step, decay=1.0, **kw)
        else:
            x, y, e, _ = layout_bh(rowptr, colidx, x, y, bs, 1, 0, step0=step, decay=1.0, **kw)
        es.append(e[0])
        if _converged(es, conv_tol):
            break
        step, progress = hu_step_update(step, progress, e[0], e_prev, t)
        e_prev = e[0]
    return x, y, np.array(es), np.array(steps)


_M64 = (1 << 64) - 1
_SM_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) of
    one state word: xor-shift 30, multiply, xor-shift 27, multiply,
    xor-shift 31.  The t-th output (t >= 1) of a stream seeded with s is
    splitmix64(s + t * gamma)."""
    z = state & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def batch_permutation(n: int, seed: int, k: int) -> np.ndarray:
    """The vertex order of iteration k under batch randomisation (Sec. 4.3.3;
    the paper fixes no generator, so this is the library's documented one):
    Durstenfeld's Fisher-Yates shuffle of 0..n-1, for i = n-1 down to 1
    swapping positions i and u mod (i+1), u = the (c+1)-th SplitMix64 output
    of seed for the counter c = k * 2^32 + i.  Pure Python (small n)."""
    perm = list(range(n))
    for i in range(n - 1, 0, -1):
        c = (k << 32) + i
        u = splitmix64(seed + (c + 1) * _SM_GAMMA)
        j = u % (i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return np.array(perm, dtype=np.int64)


def layout_shuffled(rowptr, colidx, x0, y0, bs, iters, seed, start_iter=0, mode="exact", conv_tol=0.0,
                    **kw):
    """BatchLayout with randomised minibatches (Sec. 4.3.3): iteration k takes
    its batches as the consecutive runs of bs entries of
    batch_permutation(n, seed, k), on the original labels, with the usual
    Jacobi-within and Gauss-Seidel-across semantics and the iteration's own
    step length.  Returns (x, y, energy per iteration)."""
    x = _f64(x0).copy()
    y = _f64(y0).copy()
    n = len(x)
    es = []
    for t in range(iters):
        k = start_iter + t
        perm = batch_permutation(n, seed, k)
        if mode == "exact":
            x, y, e = layout_exact(rowptr, colidx, x, y, bs, 1, k, order=perm, **kw)
        else:
            x, y, e, _ = layout_bh(rowptr, colidx, x, y, bs, 1, k, order=perm, **kw)
        es.append(e[0])
        if _converged(es, conv_tol):
            break
    return x, y, np.array(es)


def edge_energy(rowptr, colidx, x, y, K=1.0) -> float:
    """Sum over undirected edges of d^3/(3K), the attractive potential."""
    rp, ci = _csr(rowptr, colidx)
    return _load().orc_edge_energy(len(rp) - 1, rp, ci, _f64(x), _f64(y), K)


def edge_uniformity(rowptr, colidx, x, y) -> float:
    """Normalised standard deviation of edge lengths (Sec. 3.7)."""
    rp, ci = _csr(rowptr, colidx)
    return _load().orc_edge_uniformity(len(rp) - 1, rp, ci, _f64(x), _f64(y))


def stress(rowptr, colidx, x, y, pivots=None):
    """Stress after optimal uniform scaling (Sec. 3.7).  Returns (stress, scale)."""
    rp, ci = _csr(rowptr, colidx)
    s = C.c_double()
    if pivots is None:
        v = _load().orc_stress(len(rp) - 1, rp, ci, _f64(x), _f64(y), 0, None, C.byref(s))
    else:
        pv = np.ascontiguousarray(pivots, dtype=np.int32)
        v = _load().orc_stress(len(rp) - 1, rp, ci, _f64(x), _f64(y), len(pv),
                               pv.ctypes.data_as(C.c_void_p), C.byref(s))
    return v, s.value


def neighborhood_preservation(rowptr, colidx, x, y, sample=None):
    """Neighbourhood preservation (Sec. 3.7): the mean over vertices with
    k = deg > 0 of the Jaccard index of their graph neighbours and their k
    nearest vertices in the layout (FP64 squared distances, ties by id).
    sample: vertices to average over (repeats count again), default all.
    Returns (np, vertices counted)."""
    rp, ci = _csr(rowptr, colidx)
    cnt = C.c_long(0)
    if sample is None:
        v = _load().orc_neighborhood_preservation(len(rp) - 1, rp, ci, _f64(x), _f64(y), 0, None, C.byref(cnt))
    else:
        sv = np.ascontiguousarray(sample, dtype=np.int32)
        v = _load().orc_neighborhood_preservation(len(rp) - 1, rp, ci, _f64(x), _f64(y), len(sv),
                                                  sv.ctypes.data_as(C.c_void_p), C.byref(cnt))
    if v < 0:
        raise MemoryError("orc_neighborhood_preservation")
    return v, cnt.value


def greedy_init(rowptr, colidx, start, xr=None, yr=None):
    """Greedy initial layout (Sec. 3.6, Algorithm 3) from `start` at (0, 0).

    Components the start cannot reach begin, lowest unvisited id first, at
    their positions in (xr, yr) (zeros when not given).  Returns (x, y, parent).
    """
    rp, ci = _csr(rowptr, colidx)
    n = len(rp) - 1
    xr = np.zeros(n) if xr is None else _f64(xr)
    yr = np.zeros(n) if yr is None else _f64(yr)
    x, y, par = np.empty(n), np.empty(n), np.empty(n, np.int32)
    rc = _load().orc_greedy_init(n, rp, ci, int(start), xr, yr, x, y, par)
    if rc != 0:
        raise ValueError("greedy_init: bad arguments (%d)" % rc)
    return x, y, par
