"""Write the oracle's full-run quality figures for the benchmark workloads.

For each workload this runs the FP64 oracle for the workload's whole
iteration count from its seeded start, and again from MEMBERS - 1 starts that
differ from it in one coordinate by one float32 ulp (the run's intrinsic
spread: how far rounding-sized changes move the end result).  It records,
per run, the layout's stress (Sec. 3.7, optimal uniform scale, BFS hop
distances; all pairs for the grid, 1024 seeded pivots otherwise), its edge
energy (sum over edges of d^3 / 3K) and the last iteration's energy
sum |f_i|^2, and writes tests/golden/fullrun_<workload>.json.

It calls only the oracle and the seeded input generators.  The GPU tests
compare the library's full runs with these values.

    python tests/golden/make_fullrun_golden.py grid32 rmat17_bh rgg64k
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_08233_amd import inputs as I  # noqa: E402

MEMBERS = 5


def _workload(name):
    if name == "grid32":
        return I.workload_grid32(), None
    if name == "rmat17_bh":
        w = I.workload_rmat17(mode="bh")
        return w, I.stress_pivots(w["graph"].n)
    if name == "rgg64k":
        w = I.workload_rgg64k()
        return w, I.stress_pivots(w["graph"].n)
    raise SystemExit("unknown workload " + name)


def _run(w, x0, y0):
    g = w["graph"]
    if w["mode"] == "bh":
        x, y, e, _ = oracle.layout_bh(g.rowptr, g.colidx, x0, y0, w["batch_size"], w["iterations"],
                                      theta=w["theta"])
    else:
        x, y, e = oracle.layout_exact(g.rowptr, g.colidx, x0, y0, w["batch_size"], w["iterations"])
    return x, y, e


def make(name):
    w, piv = _workload(name)
    g = w["graph"]
    runs = []
    for m in range(MEMBERS):
        if m == 0:
            x0, y0, moved = w["x0"], w["y0"], None
        else:
            x0, moved = I.ulp_perturbed(w["x0"], 900 + m)
            y0 = w["y0"]
        t0 = time.perf_counter()
        x, y, e = _run(w, x0, y0)
        sec = time.perf_counter() - t0
        s, scale = oracle.stress(g.rowptr, g.colidx, x, y, piv)
        ee = oracle.edge_energy(g.rowptr, g.colidx, x, y)
        runs.append(dict(perturbed_vertex=moved, stress=s, scale=scale, edge_energy=ee,
                         energy_last=float(e[-1]), energy_first=float(e[0]), seconds=sec))
        print(name, m, runs[-1], flush=True)
    keys = ("stress", "edge_energy", "energy_last")
    base = runs[0]
    spread = {k: (max(r[k] for r in runs) - min(r[k] for r in runs)) / abs(base[k]) for k in keys}
    out = dict(workload=w["name"], n=g.n, nnz=int(g.nnz), batch_size=w["batch_size"],
               iterations=w["iterations"], mode=w["mode"], theta=w["theta"],
               step0=1.0, step_decay=0.999, K=1.0, R=1.0,
               stress_sources="all pairs" if piv is None else "1024 pivots, inputs.stress_pivots(n)",
               perturbation="one x coordinate moved up by one float32 ulp, inputs.ulp_perturbed(x0, 900+m)",
               oracle_threads=oracle.threads(), runs=runs, spread=spread,
               made_by="tests/golden/make_fullrun_golden.py (oracle FP64, fixed summation order)")
    path = os.path.join(HERE, "fullrun_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "spread", spread, flush=True)


if __name__ == "__main__":
    oracle.set_threads(0)
    for nm in sys.argv[1:] or ["grid32", "rmat17_bh", "rgg64k"]:
        make(nm)
