"""Full runs at the benchmark workloads, to the end, against the oracle's
full runs (needs an MI355X).

tests/golden/fullrun_<workload>.json holds, from the FP64 oracle alone
(tests/golden/make_fullrun_golden.py), the final layout's stress (Sec. 3.7,
1024 seeded BFS pivots), edge energy and last iteration energy of the run
from the workload's seeded start, and of runs whose starts differ from it by
one float32 ulp in one coordinate.  The spread of those runs is the
problem's own sensitivity to rounding-sized changes.

The bar: the GPU run's stress and edge energy, evaluated by the oracle's own
evaluators on the GPU's final layout, lie within 1% of the oracle runs'
range: [min * 0.99, max * 1.01].  The deviation from the unperturbed oracle
run and the ensemble spread are printed beside it.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2002_08233_amd import api, inputs as I
from _parity import RUN_TOL

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, "fullrun_%s.json" % name)) as f:
        return json.load(f)


def _check(gold, g, x, y, what):
    piv = I.stress_pivots(g.n)
    got = dict(stress=oracle.stress(g.rowptr, g.colidx, x, y, piv)[0],
               edge_energy=oracle.edge_energy(g.rowptr, g.colidx, x, y))
    rep = {}
    for k, v in got.items():
        vals = np.array([r[k] for r in gold["runs"]])
        lo, hi = vals.min() * (1 - RUN_TOL), vals.max() * (1 + RUN_TOL)
        rep[k] = dict(gpu=v, dev_from_oracle_run=v / vals[0] - 1, oracle_spread=gold["spread"][k],
                      oracle_min=float(vals.min()), oracle_max=float(vals.max()))
        assert lo <= v <= hi, "%s %s: gpu %r outside [%r, %r]" % (what, k, v, lo, hi)
    print(what, json.dumps(rep), flush=True)
    return rep


def test_rmat17_barnes_hut_full_run():
    """131072-vertex RMAT, theta 1.2, batch 256, all 600 iterations as the
    benchmark runs them (resident job, replayed iteration graph)."""
    gold = _golden("rmat17_bh")
    w = I.workload_rmat17(mode="bh")
    g = w["graph"]
    assert gold["n"] == g.n and gold["nnz"] == g.nnz and gold["iterations"] == w["iterations"] == 600
    p = api.params(batch_size=256, iterations=600, mode="bh", theta=1.2)
    print("rmat17 bh full run: 600 iterations", flush=True)
    with api.Graph(g, p) as h:
        h.set_coords(w["x0"], w["y0"])
        e, st = h.run(600)
        x, y = h.get_coords()
    assert st["iters_run"] == 600 and st["nonfinite_events"] == 0
    assert abs(e[0] / gold["runs"][0]["energy_first"] - 1) < 1e-4
    _check(gold, g, x, y, "rmat17 bh")


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32", "fp64"])
def test_rgg64k_exact_full_run(precision):
    """65536-vertex random geometric graph, exact repulsion, batch 512, all 300
    iterations in each precision (the persistent run the benchmark times)."""
    gold = _golden("rgg64k")
    w = I.workload_rgg64k()
    g = w["graph"]
    assert gold["n"] == g.n and gold["nnz"] == g.nnz and gold["iterations"] == w["iterations"] == 300
    p = api.params(batch_size=512, iterations=300, mode="exact", precision=precision)
    print("rgg64k exact full run:", precision, flush=True)
    with api.Graph(g, p) as h:
        h.set_coords(w["x0"], w["y0"])
        e, st = h.run(300)
        x, y = h.get_coords()
    assert st["iters_run"] == 300 and st["nonfinite_events"] == 0
    rep = _check(gold, g, x, y, "rgg64k " + precision)
    rep["energy_last_dev"] = float(e[-1] / gold["runs"][0]["energy_last"] - 1)
    print("rgg64k", precision, "last energy deviation", rep["energy_last_dev"], flush=True)
