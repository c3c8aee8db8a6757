"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host (no device work is started by these calls)."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "batchlayout.h")).read()
    return sorted(set(re.findall(r"\b(bl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_08233_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2002_08233_amd import _lib
    names = _declared()
    assert len(names) >= 21
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTED)


def test_params_defaults_are_the_papers(lib):
    from paper_2002_08233_amd import api
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_defaults.json")))
    p = api.Params()
    assert lib.bl_params_init(C.byref(p)) == 0
    assert p.batch_size == gold["batch_size"]["value"]
    assert p.iterations == gold["iterations"]["value"]
    assert p.step0 == gold["step0"]["value"] and p.step_decay == gold["step_decay"]["value"]
    assert p.theta == gold["theta"]["value"]
    assert p.mode == api.BL_EXACT and p.repulse_adjacent == 1 and p.K == 1.0 and p.R == 1.0


def _call_layout(lib, g, p):
    from paper_2002_08233_amd import _lib as L
    csr = L.CSR()
    csr.n = g.n
    csr.nnz = g.nnz
    rp = np.ascontiguousarray(g.rowptr, np.int32)
    ci = np.ascontiguousarray(g.colidx, np.int32)
    csr.rowptr = rp.ctypes.data
    csr.colidx = ci.ctypes.data if g.nnz else None
    x = np.zeros(g.n)
    return lib.bl_layout(C.byref(csr), x.ctypes.data, x.ctypes.data, C.byref(p), None,
                         x.ctypes.data, x.ctypes.data, None, None)


@pytest.mark.parametrize("field,value", [("batch_size", 0), ("iterations", -1), ("K", 0.0), ("R", -1.0),
                                         ("theta", -0.5), ("step_decay", 1.5), ("mode", 7),
                                         ("precision", 9), ("step0", 0.0), ("conv_tol", -1.0),
                                         ("reserved0", 3)])
def test_bad_params_rejected(lib, field, value):
    from paper_2002_08233_amd import api, inputs
    p = api.params(iterations=1)
    setattr(p, field, value)
    assert _call_layout(lib, inputs.path(5), p) == api.BL_BH * 0 - 1
    assert lib.bl_last_error()


def test_bad_csr_rejected(lib):
    from paper_2002_08233_amd import api, inputs
    g = inputs.path(6)
    bad = inputs.Graph(6, g.rowptr.copy(), g.colidx.copy())
    bad.colidx[3] = 99                       # out of range: always checked
    assert _call_layout(lib, bad, api.params(iterations=1)) == -1
    bad2 = inputs.Graph(6, g.rowptr.copy(), g.colidx.copy())
    bad2.rowptr[3] = bad2.rowptr[2] - 1      # decreasing row pointer
    assert _call_layout(lib, bad2, api.params(iterations=1)) == -1
    bad3 = inputs.Graph(6, g.rowptr.copy(), g.colidx.copy())
    bad3.colidx[0] = 0                       # self loop: caught with BL_VALIDATE
    assert _call_layout(lib, bad3, api.params(iterations=1, validate=True)) == -1
    one = inputs.Graph(0, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert _call_layout(lib, one, api.params(iterations=1)) == -1


def test_bh_rejects_fp64_and_literal(lib):
    from paper_2002_08233_amd import api, inputs
    assert _call_layout(lib, inputs.path(5), api.params(iterations=1, mode="bh", precision="fp64")) == -1
    assert _call_layout(lib, inputs.path(5), api.params(iterations=1, mode="bh", repulse_adjacent=False)) == -1


def test_footprint_grows_with_size(lib):
    from paper_2002_08233_amd import api
    p = api.params(mode="bh")
    a = api.footprint_bytes(1000, 8000, p)
    b = api.footprint_bytes(100000, 800000, p)
    assert 0 < a < b
    assert api.footprint_bytes(0, 0, p) == 0
    e = api.footprint_bytes(100000, 800000, api.params(mode="exact"))
    assert 0 < e < b


def test_server_argument_checks(lib):
    import ctypes as C
    from paper_2002_08233_amd import api
    h = C.c_void_p()
    assert lib.bl_server_create(C.c_size_t(0), 4, None, C.byref(h)) == api.BL_BH * 0 - 1
    assert lib.bl_server_create(C.c_size_t(1 << 30), 0, None, C.byref(h)) == -1
    assert lib.bl_server_create(C.c_size_t(1 << 30), 5000, None, C.byref(h)) == -1
    assert lib.bl_server_destroy(None) == 0


def test_batch_argument_checks(lib):
    import ctypes as C
    assert lib.bl_layout_batch(0, None, None, None, None, None, None, None, None) == 0
    assert lib.bl_layout_batch(-1, None, None, None, None, None, None, None, None) == -1
    assert lib.bl_layout_batch(2, None, None, None, None, None, None, None, None) == -1


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets that a C
    compiler gives the header's structs."""
    import ctypes as C
    import subprocess
    from paper_2002_08233_amd import _lib
    src = tmp_path / "layout.c"
    fields = [f for f, _ in _lib.Params._fields_]
    sfields = [f for f, _ in _lib.Stats._fields_]
    qfields = [f for f, _ in _lib.Quality._fields_]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "batchlayout.h"', 'int main(void) {',
             '  printf("%zu\\n", sizeof(bl_params));']
    lines += ['  printf("%%zu\\n", offsetof(bl_params, %s));' % f for f in fields]
    lines += ['  printf("%zu\\n", sizeof(bl_stats));']
    lines += ['  printf("%%zu\\n", offsetof(bl_stats, %s));' % f for f in sfields]
    lines += ['  printf("%zu\\n", sizeof(bl_quality));']
    lines += ['  printf("%%zu\\n", offsetof(bl_quality, %s));' % f for f in qfields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(_lib.Params)] + [getattr(_lib.Params, f).offset for f in fields]
    want += [C.sizeof(_lib.Stats)] + [getattr(_lib.Stats, f).offset for f in sfields]
    want += [C.sizeof(_lib.Quality)] + [getattr(_lib.Quality, f).offset for f in qfields]
    assert got == want


def test_quality_rejects_bad_arguments(lib):
    """Argument checks of bl_quality_eval run on the host before any device work."""
    import ctypes as C
    from paper_2002_08233_amd import _lib, api, inputs
    g = inputs.path(5)
    keep = api._Keep()
    csr = api._csr(g, keep)
    x = np.zeros(5)
    q = _lib.Quality()
    piv = np.array([0, 7], np.int32)
    assert lib.bl_quality_eval(C.byref(csr), x.ctypes.data, x.ctypes.data, 0, None, 1.0, 0, None, None) == -1
    assert lib.bl_quality_eval(C.byref(csr), None, x.ctypes.data, 0, None, 1.0, 0, None, C.byref(q)) == -1
    assert lib.bl_quality_eval(C.byref(csr), x.ctypes.data, x.ctypes.data, 0, None, 0.0, 0, None, C.byref(q)) == -1
    assert lib.bl_quality_eval(C.byref(csr), x.ctypes.data, x.ctypes.data, 2, piv.ctypes.data, 1.0, 0, None,
                               C.byref(q)) == -1
    assert lib.bl_quality_eval(C.byref(csr), x.ctypes.data, x.ctypes.data, 2, None, 1.0, 0, None, C.byref(q)) == -1
    assert lib.bl_quality_eval(C.byref(csr), x.ctypes.data, x.ctypes.data, 0, None, 1.0, 64, None, C.byref(q)) == -1
    bad = inputs.Graph(5, g.rowptr.copy(), g.colidx.copy())
    bad.colidx[2] = 9
    csr2 = api._csr(bad, keep)
    assert lib.bl_quality_eval(C.byref(csr2), x.ctypes.data, x.ctypes.data, 0, None, 1.0, 0, None, C.byref(q)) == -1
    assert lib.bl_last_error()


@pytest.mark.parametrize("a,r", [(1, 1), (-1, 2), (9, -1), (2, -9), (0, 0)])
def test_model_out_of_range_rejected(lib, a, r):
    from paper_2002_08233_amd import api, inputs
    p = api.params(iterations=1, model=(a, r))
    assert _call_layout(lib, inputs.path(5), p) == -1
    assert b"model" in lib.bl_last_error()


def test_default_model_is_fruchterman_reingold(lib):
    """bl_params_init gives the (2, -1) model; a model outside -8 <= r < a <= 8
    is rejected on the host in Barnes-Hut mode as in exact mode."""
    from paper_2002_08233_amd import api, inputs
    p = api.params()
    assert (p.model_a, p.model_r) == (2, -1)
    assert _call_layout(lib, inputs.path(5), api.params(iterations=1, mode="bh", model=(1, 2))) == -1
    assert b"model" in lib.bl_last_error()


def test_shuffled_layout_host_checks(lib):
    """bl_layout_shuffled: bad arguments are rejected before any device work;
    zero iterations return the start layout."""
    from paper_2002_08233_amd import api, inputs, _lib
    g = inputs.path(6)
    keep = api._Keep()
    csr = api._csr(g, keep)
    x = np.linspace(0.0, 1.0, 6)
    y = np.zeros(6)
    xo, yo = np.empty(6), np.empty(6)

    def call(p, xa=x, ya=y, graph=C.byref(csr)):
        return lib.bl_layout_shuffled(graph, xa.ctypes.data, ya.ctypes.data, C.byref(p), 7, None,
                                      xo.ctypes.data, yo.ctypes.data, None, None)
    dev = api.params(iterations=1)
    dev.flags |= _lib.BL_DEVICE_PTRS
    assert call(dev) == -1
    assert call(api.params(batch_size=0)) == -1
    assert call(api.params(iterations=1), graph=None) == -1
    bad = x.copy()
    bad[2] = np.nan
    assert call(api.params(iterations=1), xa=bad) == -1
    assert lib.bl_last_error()
    st = _lib.Stats()
    assert lib.bl_layout_shuffled(C.byref(csr), x.ctypes.data, y.ctypes.data, C.byref(api.params(iterations=0)),
                                  7, None, xo.ctypes.data, yo.ctypes.data, None, C.byref(st)) == 0
    assert np.array_equal(xo, x) and np.array_equal(yo, y) and st.iters_run == 0


@pytest.mark.parametrize("rows", [[[1], []], [[1, 2], [0], [0, 1]], [[2], [2], [0]]])
def test_shuffled_layout_rejects_asymmetric_csr(lib, rows):
    """An asymmetric CSR whose ids are in range (so the always-on checks pass)
    is rejected by bl_layout_shuffled before any device work, with or without
    BL_VALIDATE: its relabelling reads the graph through the transpose and
    would otherwise write past the relabelled rows."""
    from paper_2002_08233_amd import api, inputs, _lib
    n = len(rows)
    g = inputs.Graph(n, np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32),
                     np.array(sum(rows, []), np.int32))
    keep = api._Keep()
    csr = api._csr(g, keep)
    x = np.linspace(0.0, 1.0, n)
    xo, yo = np.empty(n), np.empty(n)
    for flags in (0, _lib.BL_VALIDATE):
        p = api.params(iterations=1, batch_size=1)
        p.flags |= flags
        assert lib.bl_layout_shuffled(C.byref(csr), x.ctypes.data, x.ctypes.data, C.byref(p), 3, None,
                                      xo.ctypes.data, yo.ctypes.data, None, None) == -1
        assert "symmetric" in lib.bl_last_error().decode()


def test_adaptive_step_is_a_layout_option(lib):
    """BL_ADAPTIVE_STEP: start_iter must be 0; the graph API, the batched call
    and the shuffled layout reject it (all before any device work)."""
    from paper_2002_08233_amd import api, inputs
    g = inputs.path(5)
    assert _call_layout(lib, g, api.params(iterations=1, start_iter=1, adaptive_step=True)) == -1
    keep = api._Keep()
    csr = api._csr(g, keep)
    h = C.c_void_p()
    assert lib.bl_graph_create(C.byref(csr), C.byref(api.params(adaptive_step=True)), None, C.byref(h)) == -1
    x = np.zeros(5)
    assert lib.bl_layout_shuffled(C.byref(csr), x.ctypes.data, x.ctypes.data,
                                  C.byref(api.params(iterations=1, adaptive_step=True)), 1, None,
                                  x.ctypes.data, x.ctypes.data, None, None) == -1
    gp = (C.c_void_p * 1)(C.addressof(csr))
    xp = (C.c_void_p * 1)(x.ctypes.data)
    pp = api.params(iterations=1, adaptive_step=True)
    ppp = (C.c_void_p * 1)(C.addressof(pp))
    assert lib.bl_layout_batch(1, gp, xp, xp, ppp, None, xp, xp, None) == -1
    assert "ADAPTIVE" in lib.bl_last_error().decode()


@pytest.mark.parametrize("op,blocks,iters,null_ms", [(3, 1, 1, False), (-1, 1, 1, False), (0, 0, 1, False),
                                                     (1, 1, 0, False), (2, 1, 1, True)])
def test_issue_probe_rejects_bad_arguments(lib, op, blocks, iters, null_ms):
    """The issue-rate probe checks its arguments before touching the device."""
    ms, ops = C.c_double(), C.c_double()
    rc = lib.bl_probe_issue_rate(op, blocks, iters, None, None if null_ms else C.byref(ms), C.byref(ops))
    assert rc == -1
    assert b"bl_probe_issue_rate" in lib.bl_last_error()
