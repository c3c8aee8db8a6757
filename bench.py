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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "force-updates/s (exact & BH) vs plain on 1 GPU; served p50/p99 layout latency"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 78.6     # 256 CU x 64 lanes x 2 FLOP (FMA) x 2.4 GHz, non-packed FP32
FP64_VALU_PEAK_TFLOPS = 78.6     # MI355X vector FP64
# Algorithmic work per unit (bytes a kernel must move, or FLOP it must do, per unit of work):
BYTES_PER_VISIT = 24.0           # a tree-node visit: centroid and side (16) + skip link and count or vertex (8)
BYTES_PER_WALK_VERTEX = 32.0     # order id 4 + own x,y 8 + far-field sum 16 + late count 4
BYTES_PER_ENTRY = 12.0           # a CSR or moved-leaf entry: its id 4 + the x,y it gathers 8
BYTES_PER_UPDATE = 16.0          # a vertex update: x,y read 8 + x,y written 8
BYTES_PER_TREE_VERTEX = 200.0    # quadtree build per vertex and iteration: keys 8, four radix passes x 16,
                                 # about two 24-byte nodes, their reads
FLOP_PER_PAIR = 10.0             # 2 sub, d^2 (2 mul + 1 add), 1 reciprocal, 2 FMA


def flop_per_pair(model):
    """Repulsion FLOP per pair under the (a, r) model: 2 sub, d^2 (3), the
    power d^(r-1) from d^2, 2 FMA (4).  r = -1 (any a) takes one reciprocal;
    other r |h| multiplications by d^2 (h = floor((r-1)/2)), a reciprocal
    when h < 0, and a square root and a multiplication when r - 1 is odd."""
    if model[1] == -1:
        return FLOP_PER_PAIR
    k = model[1] - 1
    h = k >> 1
    return 9.0 + abs(h) + (1.0 if h < 0 else 0.0) + (2.0 if k & 1 else 0.0)
# HBM bytes per launch of a workload's dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (FETCH_SIZE scaled by 2.0, the factor a plain copy of known size shows; WRITE_SIZE by 1.0).
# Valid only while the kernel's source file is the one the counters were taken on.
MEASURED_TRAFFIC = {
    ("c2-bh", "chain_kernel"): (33942475.6, "bl_bh.hip", "24a68aa275f9dc75"),
}


def measured_traffic(config, kernel):
    import hashlib
    m = MEASURED_TRAFFIC.get((config, kernel))
    if not m:
        return None
    path = os.path.join(ROOT, "paper_2002_08233_amd", "csrc", m[1])
    try:
        digest = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return m[0] if digest == m[2] else None


def persistent_pairs(n, bs, iters):
    """Pairs of one exact run's steps after the first finish: step e adds
    batch (e-1) % nb to every row, except in the last iteration, where only
    the rows of later batches take it."""
    nb = (n + bs - 1) // bs
    pairs = 0.0
    for c in range(nb):
        cols = min(bs, n - c * bs)
        pairs += cols * float(n) * (iters - 1)                 # iterations before the last
        if c < nb - 1:
            pairs += cols * float(n - (c + 1) * bs)           # last iteration: later rows only
    return pairs


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


def _oracle_iterations(w, budget_s):
    """Whole iterations of the workload's oracle run from its start until the
    budget is spent (at least one); returns (iterations, seconds)."""
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
            return done, el


def cpu_baseline(w, budget_s, quality_layout=None):
    """The FP64 oracle on the host: as many whole iterations of the same
    workload as fit in the budget (at least one), on the oracle's OpenMP
    threads (OMP_NUM_THREADS, else one per host core; results do not depend
    on the count), and again on one thread.  Also times, under "other", the
    oracle's greedy initialisation of the graph and its stress evaluator per
    BFS source (16 sources) on `quality_layout` when given."""
    import oracle
    g0 = w["graph"]
    other = {}
    nthreads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
    t0 = time.perf_counter()
    oracle.greedy_init(g0.rowptr, g0.colidx, 0, w["x0"], w["y0"])
    other["greedy_init_seconds"] = time.perf_counter() - t0
    if quality_layout is not None:
        from paper_2002_08233_amd import inputs as I
        sp = I.rng(11).integers(0, g0.n, 16).astype(np.int32)
        t0 = time.perf_counter()
        oracle.stress(g0.rowptr, g0.colidx, quality_layout[0], quality_layout[1], sp)
        other["stress_seconds_per_source"] = (time.perf_counter() - t0) / len(sp)
    g = w["graph"]
    done, el = _oracle_iterations(w, budget_s)
    oracle.set_threads(1)
    done1, el1 = _oracle_iterations(w, budget_s)
    oracle.set_threads(nthreads)
    return {"value": g.n * done / el, "unit": "force-updates/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d of %d iterations of the same workload from the same start, FP64 C oracle, "
                      "%d OpenMP threads, %.1f s" % (done, w["iterations"], nthreads, el),
            "one_thread": {"value": g.n * done1 / el1, "unit": "force-updates/s", "cores": 1,
                           "sample": "%d iterations, 1 thread, %.1f s" % (done1, el1)},
            "other": other}


QUALITY_PIVOTS = 1024             # BFS pivots of the stress sample at 131072 vertices


def quality_report(api, g, x, y):
    """Stress (1024 seeded pivots, or all pairs below 65536 vertices), edge
    energy and edge uniformity of the timed run's layout (Sec. 3.7), on the
    GPU."""
    from paper_2002_08233_amd import inputs as I
    piv = None if g.n <= 65536 else I.rng(10).integers(0, g.n, QUALITY_PIVOTS).astype(np.int32)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q = api.quality(g, x, y, piv)
    sec = time.perf_counter() - t0
    nsrc = g.n if piv is None else len(piv)
    rep = dict(q, seconds=sec, sources=nsrc, pairs_per_s=q["pairs"] / sec,
               note="bl_quality_eval from host arrays: upload, edge passes, 64-source BFS passes")
    return rep


def greedy_report(api, w, p, steps, energy_random):
    """The greedy initial layout (Sec. 3.6) of the workload's graph from vertex
    0, the library's host routine timed (median of 5), and the same run as the
    timed one started from it instead of the random start (its last energy
    beside the random start's)."""
    g = w["graph"]
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        xg, yg = api.greedy_init(g, 0, w["x0"], w["y0"])
        ts.append(time.perf_counter() - t0)
    sec = float(np.median(ts))
    rep = {"seconds": sec, "entries_per_s": (g.n + g.nnz) / sec, "start": 0,
           "note": "host routine; unreached components start from the random layout"}
    _, _, en, _ = api.layout(g, xg, yg, p)
    rep["energy_last"] = float(en[-1]) if len(en) else None
    rep["energy_last_random_start"] = energy_random
    return rep


def shuffle_report(api, w, p, steps, seed=2020):
    """Randomised minibatches (Sec. 4.3.3) for `steps` iterations from the
    workload's start through bl_layout_shuffled, which relabels and uploads
    the graph every iteration, beside bl_layout from the same host arrays for
    the same iterations (both end to end, host arrays in and out)."""
    g = w["graph"]
    q = api.Params.from_buffer_copy(p)
    q.iterations = steps
    t0 = time.perf_counter()
    _, _, es, st = api.layout_shuffled(g, w["x0"], w["y0"], q, seed=seed)
    ts = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _, eu, _ = api.layout(g, w["x0"], w["y0"], q)
    tu = time.perf_counter() - t0
    return {"steps": steps, "seed": seed, "force_updates_per_s": g.n * steps / ts, "seconds": ts,
            "device_seconds": st["seconds"], "device_force_updates_per_s": g.n * steps / max(st["seconds"], 1e-12),
            "sequential_end_to_end_force_updates_per_s": g.n * steps / tu,
            "energy_last": float(es[-1]) if len(es) else None,
            "energy_last_sequential": float(eu[-1]) if len(eu) else None}


def adaptive_report(api, w, p, steps, t=0.9):
    """Hu's adaptive step for `steps` iterations from the workload's start
    (one device run per iteration on the resident graph), beside the fixed
    decay, both through bl_layout from host arrays."""
    g = w["graph"]
    q = api.Params.from_buffer_copy(p)
    q.iterations = steps
    a = api.Params.from_buffer_copy(q)
    a.step_decay = t
    a.flags |= api.BL_ADAPTIVE_STEP
    t0 = time.perf_counter()
    _, _, ea, st = api.layout(g, w["x0"], w["y0"], a)
    ta = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _, ef, sf = api.layout(g, w["x0"], w["y0"], q)
    tf = time.perf_counter() - t0
    return {"steps": steps, "t": t, "force_updates_per_s": g.n * steps / ta, "seconds": ta,
            "device_seconds": st["seconds"], "device_force_updates_per_s": g.n * steps / max(st["seconds"], 1e-12),
            "fixed_decay_end_to_end_force_updates_per_s": g.n * steps / tf,
            "fixed_decay_device_seconds": sf["seconds"],
            "energy_last": float(ea[-1]) if len(ea) else None,
            "energy_last_fixed_decay": float(ef[-1]) if len(ef) else None}


def bench_single(args, api, config, steps=None, warmup=None, precision=None, extras=True):
    """One workload's timed run on resident device buffers (the benchmark
    step = one iteration of the whole path), with its per-kernel timing and,
    when `extras`, the reports beside it.  Returns the JSON-ready dict."""
    import torch
    w = workload(config)
    if steps is None:
        steps = args.steps if args.steps is not None else w["iterations"]
    if warmup is None:
        warmup = args.warmup
    if precision is None:
        precision = args.precision
    g = w["graph"]
    model = tuple(int(v) for v in args.model.split(","))
    p = api.params(batch_size=w["batch_size"], iterations=steps, mode=w["mode"],
                   theta=w["theta"] if w["mode"] == "bh" else 1.2, precision=precision, model=model)

    # inputs resident on the device before the timed region
    dev = api.Graph(g, p)
    x0 = torch.as_tensor(w["x0"], device="cuda")
    y0 = torch.as_tensor(w["y0"], device="cuda")
    dev.set_coords(x0, y0)
    if warmup > 0:
        dev.run(warmup)
    dev.set_coords(x0, y0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energy, st = dev.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    xf, yf = dev.get_coords()   # the timed run's layout (quality report)

    value = g.n * steps / wall
    out = {"metric": METRIC, "value": value, "unit": "force-updates/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": 1e3 * wall / max(steps, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if precision == "fp64" else "f32", "data": "synthetic",
           "config": dict(describe(w, steps), model=list(model))}

    if not args.no_profile:
        # per-kernel hipEvent timing in a separate run from the same start (its
        # event records between launches would slow the timed run)
        psteps = min(steps, args.profile_steps)
        dev.set_coords(x0, y0)
        dev.profile(True)
        _, st = dev.run(psteps)
        out["profiled_steps"] = psteps
        kern = {}
        for name in ("tree_build", "far_kernel", "chain_kernel", "rows_kernel", "step_kernel",
                     "steps_kernel", "finalize_kernel", "exact_graph_kernel"):
            ms, cnt = dev.profile_read(name)
            if cnt:
                kern[name] = {"total_ms": ms, "launches": cnt, "avg_us": 1e3 * ms / cnt}
        late = dev.profile_read("late_entries")[1]
        if w["mode"] == "bh":
            visits = st["node_visits"]
            old_e, recent_e = dev.profile_read("old_entries")[1], dev.profile_read("recent_entries")[1]
            tests = dev.profile_read("cell_tests")[1]
            rows = float(g.n) * psteps   # every row once per iteration in each kernel below
            work = {"far_kernel": BYTES_PER_VISIT * visits + BYTES_PER_WALK_VERTEX * rows,
                    "chain_kernel": BYTES_PER_UPDATE * rows + BYTES_PER_ENTRY * (recent_e + old_e)}
            for k, total in work.items():
                if k in kern:
                    kern[k]["bytes_per_launch"] = total / kern[k]["launches"]
                    kern[k]["achieved_GBs"] = kern[k]["bytes_per_launch"] / (kern[k]["avg_us"] * 1e-6) / 1e9
            dom_name = max((k for k in work if k in kern), key=lambda k: kern[k]["total_ms"])
            dom = kern[dom_name]
            out["roofline"] = {"bound": "hbm", "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": dom["achieved_GBs"] / HBM_PEAK_GBS,
                               "traffic": measured_traffic(config, dom_name), "kernel": dom_name,
                               "algorithmic_bytes_per_launch": dom["bytes_per_launch"]}
            nb = (g.n + w["batch_size"] - 1) // w["batch_size"]
            out["bh"] = {"node_visits_per_vertex": visits / rows, "cell_tests_per_vertex": tests / rows,
                         "node_visits_per_s": visits / rows * g.n * steps / wall,
                         "late_entries_per_vertex": late / rows,
                         "old_entries_per_vertex": old_e / rows, "recent_entries_per_vertex": recent_e / rows,
                         "late_overflow": st["late_overflow"],
                         "chain_us_per_batch": 1e3 * kern["chain_kernel"]["total_ms"] / (nb * psteps)}
            # the whole Barnes-Hut iteration on the same units: walks, every CSR
            # entry's attraction, moved leaves, updates and the tree build
            path_bytes = (BYTES_PER_VISIT * visits / psteps + BYTES_PER_ENTRY * (g.nnz + late / psteps)
                          + (BYTES_PER_UPDATE + BYTES_PER_TREE_VERTEX) * g.n)
            path_gbs = path_bytes / (1e-3 * out["ms_per_step"]) / 1e9
            out["bh"]["path"] = {"algorithmic_bytes_per_iteration": path_bytes, "achieved_GBs": path_gbs,
                                 "frac_of_hbm_peak": path_gbs / HBM_PEAK_GBS,
                                 "note": "24 B per node visit, 12 B per CSR or moved-leaf entry, 16 B per "
                                         "update and 200 B per vertex of tree build, over the timed "
                                         "iteration time"}
        else:
            nb = (g.n + w["batch_size"] - 1) // w["batch_size"]
            pairs = float(g.n) * g.n * steps
            if "steps_kernel" in kern:   # the run's steps as one persistent launch
                dom_name = "steps_kernel"
                dom = kern[dom_name]
                flop_per_launch = flop_per_pair(model) * persistent_pairs(g.n, w["batch_size"], psteps) / dom["launches"]
            elif "step_kernel" in kern:
                dom_name = "step_kernel"
                dom = kern[dom_name]
                flop_per_launch = flop_per_pair(model) * float(g.n) * w["batch_size"]
            else:   # small graph: the whole run is one launch of the one-workgroup kernel
                dom_name = "exact_graph_kernel"
                dom = kern[dom_name]
                flop_per_launch = flop_per_pair(model) * float(g.n) * g.n * psteps / dom["launches"]
            dom["achieved_TFLOPs"] = flop_per_launch / (dom["avg_us"] * 1e-6) / 1e12
            dom["flop_per_launch"] = flop_per_launch
            peak = FP32_VALU_PEAK_TFLOPS if precision != "fp64" else FP64_VALU_PEAK_TFLOPS
            out["roofline"] = {"bound": "alu", "achieved": dom["achieved_TFLOPs"], "peak": peak,
                               "unit": "TFLOP/s", "frac": dom["achieved_TFLOPs"] / peak,
                               "traffic": measured_traffic(config, dom_name.split("<")[0]), "kernel": dom_name,
                               "frac_of_packed_fp32_peak": (dom["achieved_TFLOPs"] / 157.3
                                                            if precision != "fp64" else None)}
            out["exact"] = {"pairs_per_s": pairs / wall, "batches_per_iteration": nb}
        out["kernels"] = kern
        dev.profile(False)   # (this also clears the totals just read)
    out["energy_last"] = float(energy[-1]) if len(energy) else None

    if extras and not args.no_end_to_end:
        # the same run through the host-array boundary: graph and coordinates
        # uploaded, the run, coordinates copied back (never the headline value)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.layout(g, w["x0"], w["y0"], p)
        e2e = time.perf_counter() - t0
        out["end_to_end"] = {"force_updates_per_s": g.n * steps / e2e, "seconds": e2e,
                             "note": "bl_layout from host arrays: CSR and coordinates uploaded, "
                                     "device state built, the run, coordinates back"}
    if extras and args.shuffle_steps > 0:
        out["shuffled"] = shuffle_report(api, w, p, args.shuffle_steps)
    if extras and args.adaptive_steps > 0:
        out["adaptive"] = adaptive_report(api, w, p, args.adaptive_steps)
    if extras and not args.no_quality:
        out["quality"] = quality_report(api, g, xf, yf)
    if extras and not args.no_greedy:
        out["greedy_init"] = greedy_report(api, w, p, steps, float(energy[-1]) if len(energy) else None)
    if extras and config == "c3" and precision == "fp32_kahan" and not args.no_precision:
        out["precision"] = precision_report(api, w, x0, y0, w["iterations"])
    if extras and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, None if args.no_quality else (xf, yf))
    dev.close()
    return out


def other_configs(args, api, reqs):
    """Compact measurements of the other workloads, for the default line:
    rgg64k exact (all 300 iterations, with the three-precision comparison
    against the oracle's full runs), rmat17 exact, grid32 exact, the 512
    uneven graphs batched against the same graphs alone, and a short served
    stream against its requests alone."""
    keep = ("value", "unit", "steps", "ms_per_step", "dtype", "config", "roofline", "exact", "precision",
            "energy_last")
    res = {}
    for name in ("c3", "c2-exact", "c1"):
        t0 = time.perf_counter()
        # rgg64k and grid32 run all their iterations (under two seconds); rmat17
        # exact the timed iterations of the line (6 ms each)
        steps = workload(name)["iterations"] if name != "c2-exact" else (args.steps if args.steps is not None else 20)
        r = bench_single(args, api, name, steps=steps, warmup=1, precision="fp32_kahan", extras=False)
        if name == "c3" and not args.no_precision:
            import torch
            w = workload(name)
            x0 = torch.as_tensor(w["x0"], device="cuda")
            y0 = torch.as_tensor(w["y0"], device="cuda")
            r["precision"] = precision_report(api, w, x0, y0, w["iterations"])
        r = {k: v for k, v in r.items() if k in keep}
        r["wall_seconds"] = time.perf_counter() - t0
        res[name] = r
    t0 = time.perf_counter()
    res["c4"] = {k: v for k, v in bench_batched(args, api).items() if k != "metric"}
    res["c4"]["wall_seconds"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    res["c5"] = {k: v for k, v in bench_served(args, api, reqs, window=args.compact_serve_seconds).items()
                 if k != "metric"}
    res["c5"]["wall_seconds"] = time.perf_counter() - t0
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed iterations (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2-bh", choices=["c2-bh", "c2-exact", "c1", "c3", "c4", "c5"])
    ap.add_argument("--batch-count", type=int, default=512, help="c4: graphs in the batch")
    ap.add_argument("--plain-every", type=int, default=8, help="c4: run every k-th graph alone for the plain rate")
    ap.add_argument("--serve-seconds", type=float, default=6.0, help="c5: length of the arrival window")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="c5: arrivals per second")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel hipEvent timing")
    ap.add_argument("--profile-steps", type=int, default=100, help="iterations of the per-kernel timing run")
    ap.add_argument("--no-end-to-end", action="store_true", help="skip the run through host arrays")
    ap.add_argument("--no-greedy", action="store_true", help="skip the greedy-initialisation report")
    ap.add_argument("--no-quality", action="store_true", help="skip the layout-quality report")
    ap.add_argument("--precision", default="fp32_kahan")
    ap.add_argument("--adaptive-steps", type=int, default=0,
                    help="also run this many iterations with Hu's adaptive step (0: off)")
    ap.add_argument("--shuffle-steps", type=int, default=0,
                    help="also run this many iterations with randomised minibatches (0: off)")
    ap.add_argument("--model", default="2,-1", help="exact mode: the (a, r) energy model, e.g. 1,-1")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="default run: skip the compact measurements of the other workloads")
    ap.add_argument("--compact-serve-seconds", type=float, default=6.0,
                    help="default run: arrival window of the compact served measurement")
    ap.add_argument("--no-precision", action="store_true", help="c3: skip the three-precision comparison")
    ap.add_argument("--no-bs-study", action="store_true", help="c4: skip the minibatch-size study")
    ap.add_argument("--rcp-probe", action="store_true",
                    help="measure the FMA and reciprocal issue rates and the exact kernel's pair ceiling")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs the layout of a graph on a single "
              "MI355X; --gpus %d is not supported." % args.gpus, file=sys.stderr)
        return 2

    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.rcp_probe:
        return rcp_probe()
    reqs = None
    if args.config == "c5" or (args.config == "c2-bh" and not args.no_other_configs):
        # request graphs are generated before anything touches the GPU
        import multiprocessing as mp
        from paper_2002_08233_amd import inputs as I
        secs = args.serve_seconds if args.config == "c5" else args.compact_serve_seconds
        stream = I.served_stream(rate=args.serve_rate, duration=secs)
        with mp.get_context("fork").Pool(min(16, os.cpu_count() or 4)) as pool:
            reqs = []
            for r in pool.imap(_served_request, stream, chunksize=4):
                reqs.append(r)
                if len(reqs) % 200 == 0:
                    print("served stream: %d of %d request graphs generated" % (len(reqs), len(stream)),
                          file=sys.stderr, flush=True)

    import torch
    from paper_2002_08233_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.config == "c4":
        print(json.dumps(bench_batched(args, api)))
        return 0
    if args.config == "c5":
        print(json.dumps(bench_served(args, api, reqs)))
        return 0
    if args.config == "c2-bh" and not args.no_other_configs:
        out = bench_single(args, api, "c2-bh")
        out["other_configs"] = other_configs(args, api, reqs)
    else:
        out = bench_single(args, api, args.config)
    print(json.dumps(out))
    return 0


def rcp_probe():
    """Issue rates of v_fma_f32, v_rcp_f32 and their repulsion-term mix (one
    reciprocal to six multiply-adds) through the library's probe, and the
    instruction-bound ceiling of the exact kernel's repulsion pairs that
    follows: a pair takes six FMA-class instructions and one reciprocal."""
    import ctypes as C
    from paper_2002_08233_amd import _lib
    lib = _lib.load()
    blocks, iters = 256 * 16, 4096
    res = {}
    for op, name in ((0, "fma"), (1, "rcp"), (2, "rep_mix")):
        ms, ops = C.c_double(), C.c_double()
        rc = lib.bl_probe_issue_rate(op, blocks, iters, None, C.byref(ms), C.byref(ops))
        if rc != 0:
            raise RuntimeError("bl_probe_issue_rate(%d) failed: %d" % (op, rc))
        res[name] = {"ms": ms.value, "lane_ops_per_s": ops.value / (ms.value * 1e-3)}
    lanes_clk = 256 * 64 * 2.4e9   # lanes of the chip's SIMDs per second at 2.4 GHz
    fma = res["fma"]["lane_ops_per_s"]
    out = {"rcp_probe": res,
           "fma_fraction_of_2p4GHz_issue": fma / lanes_clk,
           "rcp_rate_vs_fma": res["rcp"]["lane_ops_per_s"] / fma,
           "pair_ceiling_per_s": res["rep_mix"]["lane_ops_per_s"] / 7.0,
           "flop_ceiling_tflops": 10.0 * res["rep_mix"]["lane_ops_per_s"] / 7.0 / 1e12}
    print(json.dumps(out))
    return 0


def copy_probe(mib):
    """A plain copy of known size: reads and writes mib MiB once per launch,
    three launches.  Its FETCH_SIZE / WRITE_SIZE calibrate the counters."""
    import torch
    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": mib << 20, "launches": 3}))
    return 0


def edge_energy(g, x, y):
    """Sum over undirected edges of d^3 / 3 (K = 1): the attractive potential."""
    import numpy as np
    row = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    keep = row < g.colidx
    d = np.hypot(x[g.colidx[keep]] - x[row[keep]], y[g.colidx[keep]] - y[row[keep]])
    return float(np.sum(d ** 3) / 3.0)


def precision_report(api, w, x0, y0, iters):
    """The same iterations in FP32 with compensated sums, plain FP32 and FP64
    on the GPU: throughput of each; the final layout's stress (Sec. 3.7, 1024
    seeded pivots) and edge energy, from the GPU evaluator, against the FP64
    oracle's full run of the workload and the spread of its one-ulp-perturbed
    runs (tests/golden/fullrun_<workload>.json, written by the oracle alone)
    when the run is the full one; and the FP32 runs' deviation from the FP64
    run on the GPU (per-iteration energy, coordinates)."""
    import numpy as np
    import torch
    from paper_2002_08233_amd import inputs as I
    g = w["graph"]
    res = {}
    for prec in ("fp32_kahan", "fp32", "fp64"):
        p = api.params(batch_size=w["batch_size"], iterations=iters, mode="exact", precision=prec)
        with api.Graph(g, p) as h:
            h.set_coords(x0, y0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            en, _ = h.run(iters)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            x, y = h.get_coords()
        res[prec] = dict(x=x, y=y, en=en, fu_s=g.n * iters / dt)
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "fullrun_%s.json" % w["name"].split("-")[0])
    if iters == w["iterations"] and os.path.exists(gpath):
        with open(gpath) as f:
            gold = json.load(f)
    piv = I.stress_pivots(g.n) if g.n > 65536 or gold is not None else None
    ref = res["fp64"]
    ext = max(np.ptp(ref["x"]), np.ptp(ref["y"]))
    out = {"iterations": iters, "reference": "fp64 on the GPU; oracle full run when the run is the full one",
           "stress_sources": "all pairs" if piv is None else "%d pivots" % len(piv)}
    if gold is not None:
        out["oracle"] = {k: {"run": gold["runs"][0][k], "min": min(r[k] for r in gold["runs"]),
                             "max": max(r[k] for r in gold["runs"]), "spread": gold["spread"][k]}
                         for k in ("stress", "edge_energy")}
    for prec in ("fp32_kahan", "fp32", "fp64"):
        r = res[prec]
        q = api.quality(g, r["x"], r["y"], piv)
        o = {"force_updates_per_s": r["fu_s"], "stress": q["stress"], "edge_energy": q["edge_energy"]}
        if gold is not None:
            for k in ("stress", "edge_energy"):
                o[k + "_dev_from_oracle"] = o[k] / gold["runs"][0][k] - 1
                lo = min(x[k] for x in gold["runs"]) * 0.99
                hi = max(x[k] for x in gold["runs"]) * 1.01
                o[k + "_within_1pct_of_oracle_range"] = bool(lo <= o[k] <= hi)
        if prec != "fp64":
            o.update({
                "energy_rel_dev_from_fp64_max": float(np.max(np.abs(r["en"] / ref["en"] - 1))),
                "coord_rms_dev_from_fp64_over_extent": float(np.sqrt(np.mean((r["x"] - ref["x"]) ** 2 +
                                                                             (r["y"] - ref["y"]) ** 2)) / ext)})
        out[prec] = o
    return out


def bench_batched(args, api):
    """Batched uneven graphs: all of them in one bl_layout_batch call, against
    the same graphs run alone one after the other (a sample of them), on the
    same GPU.  Layouts are identical bit for bit either way (so at equal
    stress).  Device time from the library (inputs already uploaded)."""
    import numpy as np
    from paper_2002_08233_amd import inputs as I
    jobs = I.workload_batched(count=args.batch_count)
    graphs = [j["graph"] for j in jobs]
    plist = [api.params(batch_size=j["batch_size"], iterations=j["iterations"], mode=j["mode"],
                        theta=j["theta"] if j["mode"] == "bh" else 1.2) for j in jobs]
    fu = float(sum(g.n * j["iterations"] for g, j in zip(graphs, jobs)))
    api.layout_batch(graphs[:4], [j["x0"] for j in jobs[:4]], [j["y0"] for j in jobs[:4]], plist[:4])  # warm-up
    t0 = time.perf_counter()
    outs, stats = api.layout_batch(graphs, [j["x0"] for j in jobs], [j["y0"] for j in jobs], plist)
    wall = time.perf_counter() - t0
    dev_s = stats[0]["seconds"]
    sample = list(range(0, len(jobs), max(1, args.plain_every)))
    plain_s = 0.0
    plain_fu = 0.0
    same = True
    for q in sample:
        x, y, _, st = api.layout(graphs[q], jobs[q]["x0"], jobs[q]["y0"], plist[q], energy=False)
        plain_s += st["seconds"]
        plain_fu += graphs[q].n * jobs[q]["iterations"]
        same &= bool(np.array_equal(x, outs[q][0]) and np.array_equal(y, outs[q][1]))
    value = fu / dev_s
    plain = plain_fu / plain_s
    nex = sum(1 for j in jobs if j["mode"] == "exact")
    out = {"metric": METRIC, "value": value, "unit": "force-updates/s", "n_gpus": 1, "steps": 200,
           "warmup": 1, "ms_per_step": 1e3 * dev_s / 200, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batched: %d graphs (n log-uniform in [200, 20000], ER mean degree 8 / BA m=4), "
                                  "%d vertices, batch 128, 200 iterations, exact below 4096 vertices (%d graphs), "
                                  "Barnes-Hut theta 1.0 above" % (len(jobs), sum(g.n for g in graphs), nex),
                      "graphs": len(jobs), "vertices": int(sum(g.n for g in graphs))},
           "batched": {"device_seconds": dev_s, "wall_seconds_with_transfers": wall,
                       "force_updates_per_s_with_transfers": fu / wall},
           "plain": {"force_updates_per_s": plain, "sample_graphs": len(sample),
                     "note": "each sampled graph alone through bl_layout, device time summed"},
           "speedup_vs_plain": value / plain, "equal_stress": "bitwise-identical layouts" if same else "MISMATCH",
           "roofline": None}
    if not args.no_bs_study:
        out["minibatch_study"] = minibatch_study(api, jobs)
    return out


MINIBATCH_CANDIDATES = (64, 128, 256, 512)


def minibatch_study(api, jobs, count=24, ref_bs=128, tol=0.01):
    """The minibatch size at equal stress (Sec. 4.3.2): a size-stratified
    sample of the batched graphs is laid out in one bl_layout_batch call per
    candidate batch size; each layout's stress (all pairs, on the GPU) is
    compared with the same graph's at the configured size.  The pick is the
    fastest candidate whose mean stress ratio lies within `tol` of 1.  Batch
    size changes the layout, so the parity path keeps the configured 128; the
    pick is reported, not applied."""
    import numpy as np
    order = np.argsort([j["graph"].n for j in jobs])
    sample = [jobs[q] for q in order[np.linspace(0, len(order) - 1, min(count, len(order))).astype(int)]]
    graphs = [j["graph"] for j in sample]
    fu = float(sum(g.n * j["iterations"] for g, j in zip(graphs, sample)))
    res = {}
    for bs in MINIBATCH_CANDIDATES:
        plist = [api.params(batch_size=bs, iterations=j["iterations"], mode=j["mode"],
                            theta=j["theta"] if j["mode"] == "bh" else 1.2) for j in sample]
        outs, stats = api.layout_batch(graphs, [j["x0"] for j in sample], [j["y0"] for j in sample], plist)
        stress = [api.quality(g, o[0], o[1])["stress"] for g, o in zip(graphs, outs)]
        res[bs] = dict(force_updates_per_s=fu / stats[0]["seconds"], stress=stress)
    ref = np.array(res[ref_bs]["stress"])
    rows = {}
    for bs, r in res.items():
        ratio = np.array(r["stress"]) / ref
        rows[str(bs)] = {"force_updates_per_s": r["force_updates_per_s"],
                         "stress_ratio_mean": float(ratio.mean()), "stress_ratio_min": float(ratio.min()),
                         "stress_ratio_max": float(ratio.max())}
    ok = [bs for bs in res if abs(rows[str(bs)]["stress_ratio_mean"] - 1) <= tol]
    pick = max(ok, key=lambda bs: res[bs]["force_updates_per_s"])
    return {"graphs": len(sample), "reference_batch_size": ref_bs, "tolerance": tol, "candidates": rows,
            "pick_at_equal_stress": pick,
            "note": "batched throughput per candidate batch size on a size-stratified sample; equal stress = "
                    "mean stress ratio to the reference size within the tolerance (all pairs, GPU evaluator)"}


def _served_request(args):
    from paper_2002_08233_amd import inputs as I
    t, n, seed = args
    r = I.served_request(n, seed)
    return t, r["graph"], r["x0"], r["y0"]


def bench_served(args, api, reqs, window=None):
    """Served stream: Poisson arrivals, each an RMAT graph (edge factor 8, n
    log-uniform in [2^10, 2^20]), Barnes-Hut theta 1.2, batch 256, 300
    iterations, submitted to the continuous-batching server at its arrival
    time.  Reports p50/p99 latency (submit to done) and the aggregate rate,
    and the plain rate (a sample of the same requests run alone)."""
    import threading
    import numpy as np
    p = api.params(batch_size=256, iterations=300, mode="bh", theta=1.2)
    srv = api.Server(200 << 30, max_slots=512)
    ids = [None] * len(reqs)
    t_start = time.perf_counter()

    def submitter():
        for q, (t, g, x0, y0) in enumerate(reqs):
            delay = t - (time.perf_counter() - t_start)
            if delay > 0:
                time.sleep(delay)
            ids[q] = srv.submit(g, x0, y0, p)
            if (q + 1) % 100 == 0:
                print("served stream: %d requests submitted at %.1f s" % (q + 1, time.perf_counter() - t_start),
                      file=sys.stderr, flush=True)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    lat = []
    for q in range(len(reqs)):
        srv.wait(ids[q], 3600.0)
        _, _, st = srv.fetch(ids[q])
        lat.append(st["seconds"])
        if (q + 1) % 100 == 0:
            print("served stream: %d requests done at %.1f s" % (q + 1, time.perf_counter() - t_start),
                  file=sys.stderr, flush=True)
    t_end = time.perf_counter()
    srv.close()
    fu = float(sum(g.n * 300 for _, g, _, _ in reqs))
    span = t_end - t_start
    # plain: a size-stratified sample of the same requests, each alone
    order = np.argsort([g.n for _, g, _, _ in reqs])
    sample = order[np.linspace(0, len(order) - 1, min(12, len(order))).astype(int)]
    ps, pf = 0.0, 0.0
    for q in sample:
        _, g, x0, y0 = reqs[q]
        _, _, _, st = api.layout(g, x0, y0, p, energy=False)
        ps += st["seconds"]
        pf += g.n * 300
    lat = np.array(lat)
    out = {"metric": METRIC, "value": fu / span, "unit": "force-updates/s", "n_gpus": 1, "steps": 300,
           "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "served: Poisson %.0f requests/s for %.0f s (%d requests), RMAT edge factor 8, "
                                  "n log-uniform in [2^10, 2^20], Barnes-Hut theta 1.2, batch 256, 300 iterations"
                                  % (args.serve_rate, window or args.serve_seconds, len(reqs)),
                      "requests": len(reqs), "vertices": int(sum(g.n for _, g, _, _ in reqs))},
           "served": {"latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
                      "latency_max_s": float(lat.max()), "span_s": span},
           "plain": {"force_updates_per_s": pf / ps, "sample_requests": int(len(sample)),
                     "note": "sampled requests alone through bl_layout, device time summed"},
           "speedup_vs_plain": (fu / span) / (pf / ps), "roofline": None}
    return out


if __name__ == "__main__":
    sys.exit(main())
