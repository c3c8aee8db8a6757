"""Python front end of the BatchLayout HIP library (marshalling only).

Arrays may be numpy (host) or torch device tensors; device tensors are passed
as device pointers (BL_DEVICE_PTRS), host arrays are copied by the library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import (BL_ADAPTIVE_STEP, BL_BH, BL_BH_SNAPSHOT_LEAVES, BL_DEVICE_PTRS, BL_EXACT, BL_EXACT_MULTI_WG, BL_FP32_KAHAN,
                   BL_FP32_PLAIN, BL_FP64, BL_VALIDATE, BLError, Params, Stats, check, load)

PRECISIONS = {"fp32_kahan": BL_FP32_KAHAN, "fp32": BL_FP32_PLAIN, "fp32_plain": BL_FP32_PLAIN,
              "fp64": BL_FP64}
MODES = {"exact": BL_EXACT, "bh": BL_BH}


def params(batch_size=256, iterations=600, start_iter=0, mode="exact", precision="fp32_kahan",
           repulse_adjacent=True, step0=1.0, step_decay=0.999, K=1.0, R=1.0, theta=1.2,
           validate=False, snapshot_leaves=False, multi_wg=False, conv_tol=0.0, model=(2, -1),
           adaptive_step=False) -> Params:
    p = Params()
    check(load().bl_params_init(C.byref(p)))
    p.batch_size = int(batch_size)
    p.iterations = int(iterations)
    p.start_iter = int(start_iter)
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.repulse_adjacent = 1 if repulse_adjacent else 0
    p.step0, p.step_decay, p.K, p.R, p.theta = step0, step_decay, K, R, theta
    p.conv_tol = conv_tol
    p.model_a, p.model_r = int(model[0]), int(model[1])
    p.flags = ((BL_VALIDATE if validate else 0) | (BL_BH_SNAPSHOT_LEAVES if snapshot_leaves else 0) |
               (BL_EXACT_MULTI_WG if multi_wg else 0) | (BL_ADAPTIVE_STEP if adaptive_step else 0))
    return p


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Keep:
    """Holds converted arrays alive while their pointers are in use."""

    def __init__(self):
        self.items = []

    def host(self, a, dtype):
        arr = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(arr)
        return arr.ctypes.data

    def ptr(self, a, dtype):
        if a is None:
            return None
        if _is_torch(a):
            import torch
            t = a.contiguous()
            want = {np.float64: torch.float64, np.int32: torch.int32}[dtype]
            if t.dtype != want:
                t = t.to(want)
            self.items.append(t)
            return t.data_ptr()
        return self.host(a, dtype)


def _device(*arrays):
    dev = [_is_torch(a) and a.is_cuda for a in arrays if a is not None]
    if any(dev) and not all(dev):
        raise ValueError("mix of device tensors and host arrays")
    return bool(dev) and all(dev)


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    return getattr(stream, "cuda_stream", stream)


def _csr(graph, keep: _Keep) -> L.CSR:
    rowptr = graph.rowptr
    colidx = graph.colidx
    n = (len(rowptr) - 1) if not _is_torch(rowptr) else rowptr.numel() - 1
    nnz = (len(colidx)) if not _is_torch(colidx) else colidx.numel()
    c = L.CSR()
    c.n = n
    c.nnz = nnz
    c.rowptr = keep.ptr(rowptr, np.int32)
    c.colidx = keep.ptr(colidx, np.int32) if nnz else None
    return c


def layout(graph, x0, y0, p: Params, stream=None, energy=True):
    """Run p.iterations of the layout.  Returns (x, y, energy, stats)."""
    lib = load()
    keep = _Keep()
    dev = _device(graph.rowptr, x0, y0)
    csr = _csr(graph, keep)
    pp = Params.from_buffer_copy(p)
    if dev:
        pp.flags |= BL_DEVICE_PTRS
        import torch
        xo = torch.empty_like(x0, dtype=torch.float64)
        yo = torch.empty_like(y0, dtype=torch.float64)
        xptr, yptr = xo.data_ptr(), yo.data_ptr()
    else:
        xo = np.empty(csr.n)
        yo = np.empty(csr.n)
        xptr, yptr = xo.ctypes.data, yo.ctypes.data
    en = np.zeros(max(p.iterations, 1))
    st = Stats()
    check(lib.bl_layout(C.byref(csr), keep.ptr(x0, np.float64), keep.ptr(y0, np.float64), C.byref(pp),
                        _stream(stream), xptr, yptr, en.ctypes.data if energy else None, C.byref(st)))
    return xo, yo, en[:st.iters_run], st.as_dict()


def layout_shuffled(graph, x0, y0, p: Params, seed: int, stream=None):
    """Run p.iterations with randomised minibatches (Sec. 4.3.3): in iteration k
    the batches are consecutive runs of a permutation drawn from (seed, k).
    Host arrays only.  Returns (x, y, energy, stats)."""
    lib = load()
    keep = _Keep()
    if _device(graph.rowptr, x0, y0):
        raise ValueError("layout_shuffled takes host arrays")
    csr = _csr(graph, keep)
    xo = np.empty(csr.n)
    yo = np.empty(csr.n)
    en = np.zeros(max(p.iterations, 1))
    st = Stats()
    check(lib.bl_layout_shuffled(C.byref(csr), keep.ptr(x0, np.float64), keep.ptr(y0, np.float64), C.byref(p),
                                 int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream), xo.ctypes.data, yo.ctypes.data,
                                 en.ctypes.data, C.byref(st)))
    return xo, yo, en[:st.iters_run], st.as_dict()


def greedy_init(graph, start, x=None, y=None):
    """Greedy initial layout (Sec. 3.6, Algorithm 3) from vertex `start` at (0, 0).

    (x, y): host positions whose entries for the lowest id of each component
    that `start` does not reach are kept as that component's origin (zeros
    when not given).  Returns new host arrays (x, y).
    """
    lib = load()
    keep = _Keep()
    if _device(graph.rowptr, x, y):
        raise ValueError("greedy_init takes host arrays")
    csr = _csr(graph, keep)
    xo = np.zeros(csr.n) if x is None else np.array(x, dtype=np.float64)
    yo = np.zeros(csr.n) if y is None else np.array(y, dtype=np.float64)
    if xo.shape != (csr.n,) or yo.shape != (csr.n,):
        raise ValueError("x and y need n entries")
    check(lib.bl_greedy_init(C.byref(csr), int(start), xo.ctypes.data, yo.ctypes.data))
    return xo, yo


def quality(graph, x, y, pivots=None, K=1.0, stream=None):
    """Stress (optimal scale, BFS hop distances), edge energy and edge
    uniformity of the layout (x, y) (Sec. 3.7), computed on the GPU.

    pivots=None: all unordered pairs; else pairs (p, j) for each pivot p.
    Returns a dict (stress, scale, pairs, edge_energy, edge_uniformity, edges,
    bfs_levels).
    """
    lib = load()
    keep = _Keep()
    dev = _device(graph.rowptr, x, y)
    csr = _csr(graph, keep)
    piv = None if pivots is None else np.ascontiguousarray(pivots, dtype=np.int32)
    q = L.Quality()
    check(lib.bl_quality_eval(C.byref(csr), keep.ptr(x, np.float64), keep.ptr(y, np.float64),
                              0 if piv is None else len(piv), None if piv is None else piv.ctypes.data,
                              float(K), BL_DEVICE_PTRS if dev else 0, _stream(stream), C.byref(q)))
    return q.as_dict()


def neighborhood_preservation(graph, x, y, sample=None, stream=None):
    """Neighbourhood preservation (Sec. 3.7) of the layout (x, y) on the GPU:
    mean Jaccard index of each vertex's graph neighbours and its deg nearest
    layout vertices.  sample=None: all vertices.  Returns (np, counted)."""
    lib = load()
    keep = _Keep()
    dev = _device(graph.rowptr, x, y)
    csr = _csr(graph, keep)
    smp = None if sample is None else np.ascontiguousarray(sample, dtype=np.int32)
    v = C.c_double(0.0)
    cnt = C.c_int64(0)
    check(lib.bl_neighborhood_preservation(C.byref(csr), keep.ptr(x, np.float64), keep.ptr(y, np.float64),
                                           0 if smp is None else len(smp), None if smp is None else smp.ctypes.data,
                                           BL_DEVICE_PTRS if dev else 0, _stream(stream), C.byref(v),
                                           C.byref(cnt)))
    return v.value, cnt.value


def quality_noalloc(graph, x, y, pivots=None, K=1.0, stream=None):
    """quality() through bl_quality_eval_noalloc: the graph (a Graph whose
    rowptr/colidx are device tensors) and x, y must be device tensors; the
    library uses its static device work array instead of allocating."""
    lib = load()
    keep = _Keep()
    if not _device(graph.rowptr, x, y):
        raise ValueError("quality_noalloc takes device tensors only")
    csr = _csr(graph, keep)
    piv = None if pivots is None else np.ascontiguousarray(pivots, dtype=np.int32)
    q = L.Quality()
    check(lib.bl_quality_eval_noalloc(C.byref(csr), keep.ptr(x, np.float64), keep.ptr(y, np.float64),
                                      0 if piv is None else len(piv), None if piv is None else piv.ctypes.data,
                                      float(K), BL_DEVICE_PTRS, _stream(stream), C.byref(q)))
    return q.as_dict()


def forces(graph, x, y, batch_index, p: Params, snapshot=None, stream=None):
    """Net forces on one batch from (x, y); BH tree from `snapshot` (sx, sy) if given."""
    lib = load()
    keep = _Keep()
    csr = _csr(graph, keep)
    pp = Params.from_buffer_copy(p)
    sx, sy = snapshot if snapshot is not None else (None, None)
    if _device(graph.rowptr, x, y, sx, sy):
        pp.flags |= BL_DEVICE_PTRS
    R = min(p.batch_size, csr.n - batch_index * p.batch_size)
    fx = np.zeros(max(R, 1))
    fy = np.zeros(max(R, 1))
    check(lib.bl_forces(C.byref(csr), keep.ptr(x, np.float64), keep.ptr(y, np.float64),
                        keep.ptr(sx, np.float64), keep.ptr(sy, np.float64), int(batch_index), C.byref(pp),
                        _stream(stream), fx.ctypes.data, fy.ctypes.data))
    return fx[:R], fy[:R]


def layout_batch(graphs, x0s, y0s, plist, stream=None):
    """Lay out many graphs at once (host arrays).  Returns ([(x, y)], [stats])."""
    lib = load()
    G = len(graphs)
    keep = _Keep()
    csrs = [_csr(g, keep) for g in graphs]
    pp = [Params.from_buffer_copy(p) for p in plist]
    CP = C.POINTER(L.CSR)
    PP = C.POINTER(Params)
    csr_arr = (CP * G)(*[C.pointer(c) for c in csrs])
    par_arr = (PP * G)(*[C.pointer(p) for p in pp])
    xin = (C.c_void_p * G)(*[keep.host(x, np.float64) for x in x0s])
    yin = (C.c_void_p * G)(*[keep.host(y, np.float64) for y in y0s])
    outs = [(np.empty(c.n), np.empty(c.n)) for c in csrs]
    xo = (C.c_void_p * G)(*[o[0].ctypes.data for o in outs])
    yo = (C.c_void_p * G)(*[o[1].ctypes.data for o in outs])
    st = (Stats * G)()
    check(lib.bl_layout_batch(G, csr_arr, xin, yin, par_arr, _stream(stream), xo, yo, st))
    return outs, [st[q].as_dict() for q in range(G)]


def footprint_bytes(n, nnz, p: Params) -> int:
    return int(load().bl_footprint_bytes(int(n), int(nnz), C.byref(p)))


class Graph:
    """A resident layout job (CSR, coordinates and buffers kept on the device)."""

    def __init__(self, graph, p: Params, stream=None):
        self._lib = load()
        keep = _Keep()
        self.p = Params.from_buffer_copy(p)
        if _device(graph.rowptr):
            self.p.flags |= BL_DEVICE_PTRS
        csr = _csr(graph, keep)
        self.n = csr.n
        self.h = C.c_void_p()
        check(self._lib.bl_graph_create(C.byref(csr), C.byref(self.p), _stream(stream), C.byref(self.h)))

    def set_coords(self, x, y):
        keep = _Keep()
        flags = BL_DEVICE_PTRS if _device(x, y) else 0
        check(self._lib.bl_graph_set_coords(self.h, keep.ptr(x, np.float64), keep.ptr(y, np.float64), flags))

    def get_coords(self, out=None):
        if out is not None:
            x, y = out
            check(self._lib.bl_graph_get_coords(self.h, x.data_ptr(), y.data_ptr(), BL_DEVICE_PTRS))
            return x, y
        x = np.empty(self.n)
        y = np.empty(self.n)
        check(self._lib.bl_graph_get_coords(self.h, x.ctypes.data, y.ctypes.data, 0))
        return x, y

    def run(self, iterations, start_iter=0, stop_batch=-1, energy=True):
        """Returns (energy, stats) or, with stop_batch >= 0, (energy, stats, fx, fy)."""
        en = np.zeros(max(iterations, 1))
        st = Stats()
        fx = fy = None
        fptr = (None, None)
        if stop_batch >= 0:
            R = min(self.p.batch_size, self.n - stop_batch * self.p.batch_size)
            fx = np.zeros(max(R, 1))
            fy = np.zeros(max(R, 1))
            fptr = (fx.ctypes.data, fy.ctypes.data)
        check(self._lib.bl_graph_run(self.h, int(iterations), int(start_iter), int(stop_batch),
                                     en.ctypes.data if energy else None, fptr[0], fptr[1], C.byref(st)))
        full = iterations - 1 if stop_batch >= 0 else st.iters_run
        if stop_batch >= 0:
            return en[:full], st.as_dict(), fx[:R], fy[:R]
        return en[:full], st.as_dict()

    def profile(self, enable=True):
        check(self._lib.bl_graph_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel):
        """(total_ms, launches) of one kernel since profiling was enabled."""
        ms = C.c_double()
        cnt = C.c_int64()
        check(self._lib.bl_graph_profile_read(self.h, kernel.encode(), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self._lib.bl_graph_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Server:
    """Continuous-batching layout server (host arrays in and out)."""

    def __init__(self, hbm_budget_bytes, max_slots=256, stream=None):
        self._lib = load()
        self.h = C.c_void_p()
        check(self._lib.bl_server_create(C.c_size_t(int(hbm_budget_bytes)), int(max_slots), None,
                                         C.byref(self.h)))
        self.n = {}

    def submit(self, graph, x0, y0, p: Params) -> int:
        keep = _Keep()
        csr = _csr(graph, keep)
        job = C.c_int64()
        check(self._lib.bl_server_submit(self.h, C.byref(csr), keep.host(x0, np.float64),
                                         keep.host(y0, np.float64), C.byref(p), C.byref(job)))
        self.n[job.value] = csr.n
        return job.value

    def poll(self, job) -> bool:
        d = C.c_int32()
        check(self._lib.bl_server_poll(self.h, C.c_int64(job), C.byref(d)))
        return bool(d.value)

    def wait(self, job, timeout=600.0):
        check(self._lib.bl_server_wait(self.h, C.c_int64(job), C.c_double(timeout)))

    def fetch(self, job):
        n = self.n[job]
        x = np.empty(n)
        y = np.empty(n)
        st = Stats()
        check(self._lib.bl_server_fetch(self.h, C.c_int64(job), x.ctypes.data, y.ctypes.data, C.byref(st)))
        return x, y, st.as_dict()

    def release(self, job):
        check(self._lib.bl_server_release(self.h, C.c_int64(job)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self._lib.bl_server_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
