"""Benchmark of the BatchLayout force step on one MI355X.

A step is one layout iteration of the whole hot path over the graph: for
Barnes-Hut the quadtree build, the far-field walks and the chain of all
minibatches (attraction, moved leaves, update); for exact mode all minibatch
steps of one iteration.  The default workload is the RMAT scale-17 graph
(131072 vertices, edge factor 16, a,b,c,d = .57,.19,.19,.05), Barnes-Hut with
theta 1.2, batch 256, 600 iterations from a seeded uniform start.

Prints one JSON line: force-updates/s = n * timed iterations / seconds, with
inputs resident in device memory before the timed region, plus the roofline of
the dominant kernel (live hipEvent timing inside the library) and the oracle's
throughput on the host cores for a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "force-updates/s (exact & BH) vs plain on 1 GPU; served p50/p99 layout latency"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 78.6     # 256 CU x 64 lanes x 2 FLOP (FMA) x 2.4 GHz, non-packed FP32
FP64_VALU_PEAK_TFLOPS = 78.6     # MI355X vector FP64
# Algorithmic work per unit (see the design notes):
BYTES_PER_VISIT = 24.0           # float4 (centroid, side^2, count) + int2 (skip, vertex) per node visit
BYTES_PER_WALK_VERTEX = 32.0     # order id 4 + own x,y 8 + far-field sum 16 + late count 4
BYTES_PER_ENTRY = 12.0           # CSR or moved-leaf entry: 4 B id + 8 B live x,y
BYTES_PER_CHAIN_VERTEX = 52.0    # rowptr 8 + late count 4 + far sum 16 + x,y read 8 + write 8 + force 8
FLOP_PER_PAIR = 10.0             # 2 sub, d^2 (2 mul + 1 add), 1 reciprocal, 2 FMA


def workload(name):
    from paper_2002_08233_amd import inputs as I
    if name == "c2-bh":
        return I.workload_rmat17(mode="bh")
    if name == "c2-exact":
        w = I.workload_rmat17(mode="exact")
        w["theta"] = 0.0
        return w
    if name == "c1":
        w = I.workload_grid32()
        w["x0"], w["y0"] = I.to_f32_representable(w["x0"]), I.to_f32_representable(w["y0"])
        return w
    if name == "c3":
        return I.workload_rgg64k()
    raise SystemExit("unknown config %s" % name)


def describe(w, iters):
    g = w["graph"]
    mode = "Barnes-Hut theta=%g" % w["theta"] if w["mode"] == "bh" else "exact all-pairs"
    return {"workload": "%s, %d vertices, %d CSR entries, %s, batch %d, %d iterations" % (
        w["name"], g.n, g.nnz, mode, w["batch_size"], iters),
        "n": g.n, "nnz": g.nnz, "mode": w["mode"], "theta": w["theta"], "batch_size": w["batch_size"],
        "iterations": iters, "init": "seeded uniform [-1,1]^2 (float32-representable)"}


def cpu_baseline(w, budget_s):
    """The FP64 oracle, single-threaded, on the host: as many whole iterations of
    the same workload as fit in the budget (at least one)."""
    import oracle
    g = w["graph"]
    x, y = w["x0"].copy(), w["y0"].copy()
    done = 0
    t0 = time.perf_counter()
    while True:
        if w["mode"] == "bh":
            x, y, _, _ = oracle.layout_bh(g.rowptr, g.colidx, x, y, w["batch_size"], 1, start_iter=done,
                                          theta=w["theta"])
        else:
            x, y, _ = oracle.layout_exact(g.rowptr, g.colidx, x, y, w["batch_size"], 1, start_iter=done)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / done * (done + 1) > 2.5 * budget_s:
            break
    return {"value": g.n * done / el, "unit": "force-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d of %d iterations of the same workload from the same start, FP64 C oracle, "
                      "1 thread, %.1f s" % (done, w["iterations"], el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed iterations (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2-bh", choices=["c2-bh", "c2-exact", "c1", "c3"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel hipEvent timing")
    ap.add_argument("--precision", default="fp32_kahan")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs the layout of a graph on a single "
              "MI355X; --gpus %d is not supported." % args.gpus, file=sys.stderr)
        return 2

    import torch
    from paper_2002_08233_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = workload(args.config)
    g = w["graph"]
    steps = args.steps if args.steps is not None else w["iterations"]
    p = api.params(batch_size=w["batch_size"], iterations=steps, mode=w["mode"],
                   theta=w["theta"] if w["mode"] == "bh" else 1.2, precision=args.precision)

    # inputs resident on the device before the timed region
    dev = api.Graph(g, p)
    x0 = torch.as_tensor(w["x0"], device="cuda")
    y0 = torch.as_tensor(w["y0"], device="cuda")
    dev.set_coords(x0, y0)
    if args.warmup > 0:
        dev.run(args.warmup)
    dev.set_coords(x0, y0)
    if not args.no_profile:
        dev.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energy, st = dev.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    value = g.n * steps / wall
    out = {"metric": METRIC, "value": value, "unit": "force-updates/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * wall / max(steps, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
           "config": describe(w, steps)}

    if not args.no_profile:
        kern = {}
        for name in ("tree_build", "far_kernel", "chain_kernel", "rows_kernel", "step_kernel",
                     "finalize_kernel", "exact_graph_kernel"):
            ms, cnt = dev.profile_read(name)
            if cnt:
                kern[name] = {"total_ms": ms, "launches": cnt, "avg_us": 1e3 * ms / cnt}
        late = dev.profile_read("late_entries")[1]
        if w["mode"] == "bh":
            visits = st["node_visits"]
            far = kern["far_kernel"]
            chain = kern["chain_kernel"]
            far_bytes = (BYTES_PER_VISIT * visits + BYTES_PER_WALK_VERTEX * g.n * far["launches"]) / far["launches"]
            chain_bytes = (BYTES_PER_ENTRY * (g.nnz * chain["launches"] + late) +
                           BYTES_PER_CHAIN_VERTEX * g.n * chain["launches"]) / chain["launches"]
            far["achieved_GBs"] = far_bytes / (far["avg_us"] * 1e-6) / 1e9
            chain["achieved_GBs"] = chain_bytes / (chain["avg_us"] * 1e-6) / 1e9
            far["bytes_per_launch"], chain["bytes_per_launch"] = far_bytes, chain_bytes
            dom_name = max(("far_kernel", "chain_kernel", "tree_build"), key=lambda k: kern[k]["total_ms"])
            dom = kern[dom_name] if dom_name != "tree_build" else far
            if dom_name == "tree_build":
                dom_name = "far_kernel"
            out["roofline"] = {"bound": "hbm", "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": dom["achieved_GBs"] / HBM_PEAK_GBS, "traffic": None,
                               "kernel": dom_name}
            out["bh"] = {"node_visits_per_vertex": visits / (g.n * steps), "late_entries_per_vertex":
                         late / (g.n * steps), "late_overflow": st["late_overflow"]}
        else:
            nb = (g.n + w["batch_size"] - 1) // w["batch_size"]
            pairs = float(g.n) * g.n * steps
            if "step_kernel" in kern:
                dom_name = "step_kernel"
                dom = kern[dom_name]
                flop_per_launch = FLOP_PER_PAIR * float(g.n) * w["batch_size"]
            else:   # small graph: the whole run is one launch of the one-workgroup kernel
                dom_name = "exact_graph_kernel"
                dom = kern[dom_name]
                flop_per_launch = FLOP_PER_PAIR * pairs / dom["launches"]
            dom["achieved_TFLOPs"] = flop_per_launch / (dom["avg_us"] * 1e-6) / 1e12
            dom["flop_per_launch"] = flop_per_launch
            peak = FP32_VALU_PEAK_TFLOPS if args.precision != "fp64" else FP64_VALU_PEAK_TFLOPS
            out["roofline"] = {"bound": "alu", "achieved": dom["achieved_TFLOPs"], "peak": peak,
                               "unit": "TFLOP/s", "frac": dom["achieved_TFLOPs"] / peak,
                               "traffic": None, "kernel": dom_name,
                               "frac_of_packed_fp32_peak": (dom["achieved_TFLOPs"] / 157.3
                                                            if args.precision != "fp64" else None)}
            out["exact"] = {"pairs_per_s": pairs / wall, "batches_per_iteration": nb}
        out["kernels"] = kern
    out["energy_last"] = float(energy[-1]) if len(energy) else None

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    dev.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
