"""Shared parity measures: GPU results against the FP64 oracle."""
import numpy as np

# Per-step force bar: |f_gpu - f_64| <= TOL * max(|f_64|, FLOOR * S_i), where
# S_i = sum of |term| over all terms of vertex i (its condition scale).
FORCE_TOL = 1e-5
FLOOR = 1e-2
# Full runs: stress and edge energy within 1% of the oracle's run.
RUN_TOL = 0.01


def force_errors(fx, fy, ref, mask=None):
    """Per-vertex errors of (fx, fy) against an oracle Forces object."""
    dx = fx - ref.fx
    dy = fy - ref.fy
    err = np.hypot(dx, dy)
    mag = np.hypot(ref.fx, ref.fy)
    bound = FORCE_TOL * np.maximum(mag, FLOOR * ref.scale)
    if mask is not None:
        err, mag, bound = err[mask], mag[mask], bound[mask]
    rel = err / np.maximum(mag, 1e-300)
    return dict(ok=bool(np.all(err <= bound)), worst=float(np.max(err / bound)) if len(err) else 0.0,
                rel_max=float(rel.max()) if len(rel) else 0.0,
                rel_p99=float(np.percentile(rel, 99)) if len(rel) else 0.0,
                rel_median=float(np.median(rel)) if len(rel) else 0.0,
                normwise=float(np.linalg.norm(np.hypot(dx, dy)) / max(np.linalg.norm(mag), 1e-300)))


def assert_forces(fx, fy, ref, mask=None, what=""):
    r = force_errors(fx, fy, ref, mask)
    assert r["ok"], "%s force parity failed: %s" % (what, r)
    return r


def perturbed_inits(x0, y0, count, seed=123):
    """(x0, y0) and count-1 copies in which every coordinate moved by one
    float32 ulp up or down (random signs): rounding-sized changes of the whole
    state, like those an FP32 run makes at every update."""
    r = np.random.default_rng(seed)
    out = [(x0, y0)]

    def nudge(a):
        up = r.random(len(a)) < 0.5
        f = a.astype(np.float32)
        return np.where(up, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))).astype(
            np.float64)

    for _ in range(count - 1):
        out.append((nudge(x0), nudge(y0)))
    return out


def quality(oracle, g, x, y):
    return (oracle.stress(g.rowptr, g.colidx, x, y)[0], oracle.edge_energy(g.rowptr, g.colidx, x, y))


def assert_within_oracle_spread(oracle, g, xg, yg, run_oracle, x0, y0, members=16, what=""):
    """Chaotic runs: from a random start, rounding-sized changes of the input
    move the oracle's own final stress by up to several percent.
    The GPU run's stress and edge energy must lie within RUN_TOL of the range
    of an ensemble of such oracle runs, [min * (1 - RUN_TOL), max * (1 +
    RUN_TOL)]; the ensemble's own spread is reported beside the result, not
    added to the bound."""
    qs = np.array([quality(oracle, g, *run_oracle(xp, yp)) for xp, yp in perturbed_inits(x0, y0, members)])
    qg = np.array(quality(oracle, g, xg, yg))
    lo = qs.min(axis=0) * (1 - RUN_TOL)
    hi = qs.max(axis=0) * (1 + RUN_TOL)
    spread = (qs.max(axis=0) - qs.min(axis=0)) / qs[0]
    rep = dict(gpu=qg.tolist(), oracle_min=qs.min(axis=0).tolist(), oracle_max=qs.max(axis=0).tolist(),
               spread=spread.tolist(), dev_from_oracle_run=(qg / qs[0] - 1).tolist())
    print(what, "stress, edge energy:", rep)
    assert np.all((qg >= lo) & (qg <= hi)), "%s: gpu %s outside %s..%s (oracle spread %s)" % (
        what, qg, lo, hi, spread)
    return rep


# Barnes-Hut: the oracle flags a vertex whose walk met a cell with
# |side - theta * d| <= 1e-5 theta d, where an FP32 distance may take the
# other branch of the acceptance test.  Such vertices are left out of the
# force bar, and there must be few of them.
NEAR_TIE_MAX_FRAC = 0.02


def bh_mask(ref, what=""):
    """Rows checked against the force bar: all but the oracle's near-tie
    vertices, whose number is bounded by NEAR_TIE_MAX_FRAC of the rows (at
    least one allowed)."""
    ties = int(np.sum(ref.near_tie))
    rows = len(ref.near_tie)
    assert ties <= max(1, NEAR_TIE_MAX_FRAC * rows), "%s: %d of %d rows are near ties" % (what, ties, rows)
    return ~ref.near_tie


# A schedule whose runs settle: total travel step0 / (1 - decay) ~ 1.7 edge
# lengths.  With the paper's schedule Step is still ~0.9 after 100 iterations,
# and FP32 rounding of the state alone moves the final stress by ~1%.
SETTLING = dict(step0=0.05, step_decay=0.97)


def near_grid_init(rows, cols, seed=11, noise=0.15):
    """Grid coordinates at unit spacing plus Gaussian noise."""
    r = np.random.default_rng(seed)
    n = rows * cols
    gx = (np.arange(n) % cols).astype(float)
    gy = (np.arange(n) // cols).astype(float)
    x = np.float32(gx + r.normal(0, noise, n)).astype(np.float64)
    y = np.float32(gy + r.normal(0, noise, n)).astype(np.float64)
    return x, y


def stop_tolerance(energies, kmax=10):
    """A tolerance for the energy stopping rule that first holds at an
    iteration k* with a margin on both sides (so that runs whose energies
    differ by rounding stop at the same k*): the k* in 2..kmax whose relative
    change is furthest below all earlier ones, else k* = 1.  Returns
    (tolerance, iterations the stopped run completes = k* + 1)."""
    e = np.asarray(energies, float)
    rel = np.abs(np.diff(e)) / e[:-1]          # rel[k - 1]: change at iteration k
    best, kbest = 1.0, 1
    for k in range(2, min(kmax, len(rel)) + 1):
        ratio = float(np.min(rel[:k - 1])) / max(float(rel[k - 1]), 1e-300)
        if ratio > best:
            best, kbest = ratio, k
    if kbest == 1 or best < 1.3:
        return 2.0 * float(rel[0]) + 1e-12, 2
    return float(np.sqrt(rel[kbest - 1] * np.min(rel[:kbest - 1]))), kbest + 1
