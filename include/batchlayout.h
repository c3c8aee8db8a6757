/*
 * batchlayout.h -- C ABI of the MI355X (gfx950) BatchLayout force-step library.
 *
 * The library lays out an undirected graph in 2D with the minibatch
 * force-directed method of Rahman, Sujon & Azad ("BatchLayout: A
 * Batch-Parallel Force-Directed Graph Layout Algorithm in Shared Memory"):
 * per minibatch of consecutive vertex ids it computes attraction along CSR
 * edges and repulsion (exact over all pairs, or through a Barnes-Hut
 * quadtree), then moves every vertex of the batch by Step along its
 * normalised net force; Step decays geometrically per iteration.
 *
 * Conventions shared by every call:
 *  - Every function returns an int status: BL_OK (0) or a negative BL_E_*
 *    code.  No call aborts or throws.  bl_last_error() returns a message for
 *    the last non-OK status of the calling thread.
 *  - Graphs are CSR (Sec. 2.1 of the paper): rowptr[n+1], colidx[nnz], int32,
 *    symmetric, rows sorted ascending, no self-loops, no duplicates.
 *  - Coordinates cross the ABI as FP64 structure-of-arrays x[n], y[n].  The
 *    FP32 paths round them to nearest float32 on entry; results are returned
 *    as FP64 copies of the device values.
 *  - Pointers are host memory unless the call's flags contain BL_DEVICE_PTRS;
 *    then they are device pointers (for instance torch tensors' data_ptr()),
 *    stay owned by the caller and must stay valid until the call returns.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Calls are
 *    synchronous with respect to the host: they return after their device
 *    work on that stream has finished.
 *  - Host arrays are owned by the caller; the library copies what it needs
 *    before returning (the server copies on submit).  Device state created by
 *    a handle is owned by the library until the matching destroy/release.
 */
#ifndef BATCHLAYOUT_H
#define BATCHLAYOUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define BL_OK            0
#define BL_E_INVAL      -1   /* bad argument (see each call)                     */
#define BL_E_NOMEM      -2   /* device or host allocation failed                 */
#define BL_E_HIP        -3   /* a HIP runtime call failed                        */
#define BL_E_NOTREADY   -4   /* server job still running                         */
#define BL_E_REJECTED   -5   /* server job can never fit the HBM budget          */
#define BL_E_NONFINITE  -6   /* a NaN or Inf force or coordinate appeared        */
#define BL_E_TIMEOUT    -7   /* a bounded device wait ran out                    */

/* ------------------------------------------------------------------ knobs */
#define BL_EXACT 0           /* exact all-pairs repulsion (Alg. 2)               */
#define BL_BH    1           /* Barnes-Hut repulsion (Sec. 3.5, Alg. S1-S3)      */

#define BL_FP32_KAHAN 0      /* FP32 pair math, compensated per-vertex sums      */
#define BL_FP32_PLAIN 1      /* FP32 pair math, plain FP32 sums                  */
#define BL_FP64       2      /* FP64 pair math and sums (exact mode only)        */

#define BL_DEVICE_PTRS        1u  /* array arguments are device pointers         */
#define BL_VALIDATE           2u  /* full CSR check on the host (sorted rows,
                                     range, no self-loops/duplicates, symmetry) */
#define BL_BH_SNAPSHOT_LEAVES 4u  /* BH leaves use the per-iteration snapshot
                                     instead of live coordinates                */
#define BL_EXACT_MULTI_WG     8u  /* exact mode: always use the multi-workgroup
                                     step kernels (graphs of at most 24,576
                                     pairs per step, n * batch_size, otherwise
                                     run in one workgroup); the result is the
                                     same bits                                   */
#define BL_ADAPTIVE_STEP     16u  /* bl_layout only: the adaptive step of Hu
                                     (2005), cited in Sec. 4.3.5, replaces the
                                     fixed decay (see bl_layout)                */

typedef struct {
    int32_t n;               /* vertices, >= 1                                   */
    int64_t nnz;             /* CSR entries (2 x undirected edges), >= 0         */
    const int32_t *rowptr;   /* [n+1], rowptr[0] = 0, non-decreasing             */
    const int32_t *colidx;   /* [nnz]                                            */
} bl_csr;

/* Run parameters.  bl_params_init() fills the paper's defaults: batch 256
 * (Sec. 4.3.2), 600 iterations (supplement run example), Step_0 = 1 and decay
 * 0.999 (Alg. 2, Sec. 4.3.5), K = R = 1 (Sec. 2.2 leaves them open),
 * theta = 1.2 (Sec. 4.1), exact mode, FP32 with compensated sums,
 * repulsion over all pairs. */
typedef struct {
    int32_t batch_size;      /* >= 1; the minibatch, consecutive vertex ids      */
    int32_t iterations;      /* >= 0                                             */
    int32_t start_iter;      /* >= 0; Step at iteration k = step0 * decay^k      */
    int32_t mode;            /* BL_EXACT | BL_BH                                 */
    int32_t precision;       /* BL_FP32_KAHAN | BL_FP32_PLAIN | BL_FP64          */
    int32_t repulse_adjacent;/* 1: repulsion over every j != i (default);
                                0: skip neighbours as Alg. 1/2 do (exact only)  */
    double step0;            /* > 0                                              */
    double step_decay;       /* in (0, 1]                                        */
    double K;                /* > 0, optimal spring length                       */
    double R;                /* > 0, relative strength of repulsion              */
    double theta;            /* >= 0, BH acceptance: side < theta * distance     */
    uint32_t flags;          /* BL_VALIDATE | BL_BH_SNAPSHOT_LEAVES | BL_EXACT_MULTI_WG
                                | BL_ADAPTIVE_STEP                               */
    int32_t reserved0;       /* must be zero                                     */
    double conv_tol;         /* >= 0; 0 = off.  The energy stopping rule of
                                Sec. 4.5 read as a relative change: after an
                                iteration k that is not the run's first, stop
                                when |E_k - E_{k-1}| <= conv_tol * E_{k-1}; the
                                layout is the one after iteration k and
                                stats.iters_run counts the iterations done.
                                Not with a stop batch, nor in the server.       */
    int32_t model_a;         /* the (a, r)-energy model of Sec. 2.2: attraction   */
    int32_t model_r;         /* magnitude d^a / K, repulsion magnitude R K^2 d^r
                                (r read as the power of d in the force, so the
                                default (2, -1) is Fruchterman-Reingold).
                                Integers, -8 <= r < a <= 8, in exact and
                                Barnes-Hut mode, on every path (an accepted
                                Barnes-Hut cell adds count times the repulsion
                                at its centroid).                                */
    int32_t reserved[2];     /* must be zero                                     */
} bl_params;

typedef struct {
    int32_t iters_run;       /* iterations completed                             */
    int32_t late_overflow;   /* BH: vertices whose late-leaf list overflowed     */
    double  energy_last;     /* energy sum |f_i|^2 of the last full iteration    */
    double  seconds;         /* device time of the run (hipEvent)                */
    int64_t node_visits;     /* BH: tree nodes visited by the far-field walk     */
    int64_t nonfinite_events;/* NaN/Inf net forces seen (those vertices stay)    */
} bl_stats;

/* Fill *p with the paper's defaults (see bl_params).  Returns BL_E_INVAL for NULL. */
int bl_params_init(bl_params *p);

/* Message for the last non-OK status returned to this thread ("" if none). */
const char *bl_last_error(void);

/* Library version string. */
const char *bl_version(void);

/* Bytes of device memory a resident layout job of this size needs (CSR,
 * coordinates, accumulators, tree and sort buffers).  0 on invalid input. */
size_t bl_footprint_bytes(int32_t n, int64_t nnz, const bl_params *p);

/* ------------------------------------------------------- one-shot layout
 * Lay out g from (x0, y0) for p->iterations iterations (Alg. 2 in exact mode,
 * Alg. S3 in BH mode, both with the minibatch semantics of Sec. 3.3) and write
 * the final coordinates to (x_out, y_out), which may alias (x0, y0).
 * energy_out (may be NULL) receives p->iterations values, the energy
 * sum_i |f_i|^2 of each iteration (Sec. 2.2), reduced in FP64 on the GPU.
 * stats may be NULL.  Errors: BL_E_INVAL for bad sizes/params/NULL arrays,
 * BL_E_NONFINITE if a net force was NaN/Inf (coordinates are still written).
 * With BL_ADAPTIVE_STEP in p->flags the step length follows Hu's adaptive
 * rule instead of step0 * step_decay^k, with t = p->step_decay (Hu uses 0.9):
 * iteration 0 takes p->step0; after each iteration k, if E_k < E_{k-1}
 * (E_{-1} = +inf) a progress count goes up by one and on reaching 5 is reset
 * while the step is divided by t; otherwise the count is reset and the step
 * multiplied by t.  p->start_iter must be 0; each iteration is then its own
 * device run on the resident graph.  The graph API, bl_layout_shuffled,
 * bl_layout_batch and the server reject the flag. */
int bl_layout(const bl_csr *g, const double *x0, const double *y0, const bl_params *p,
              void *hip_stream, double *x_out, double *y_out, double *energy_out,
              bl_stats *stats);

/* ------------------------------------------- randomised minibatches
 * bl_layout with the batch randomisation of Sec. 4.3.3: in iteration k the
 * minibatches are the consecutive runs of p->batch_size entries of a
 * permutation pi_k of the vertex ids (the last run may be shorter), processed
 * in that order, each with the usual Jacobi-within / Gauss-Seidel-across
 * semantics; the step length is p->step0 * p->step_decay^k as in bl_layout.
 * pi_k is Durstenfeld's Fisher-Yates shuffle of the identity, for i = n-1
 * down to 1 swapping positions i and (u mod (i+1)), where u is SplitMix64's
 * output function (Steele, Lea and Flood 2014) applied to the state
 * seed + (c+1) * 0x9E3779B97F4A7C15 with c = k * 2^32 + i; so pi_k depends on
 * (seed, k) only.  The paper gives no generator; this one is the library's.
 * Host arrays only (BL_DEVICE_PTRS in p->flags is BL_E_INVAL); exact and
 * Barnes-Hut modes; conv_tol applies between iterations as in bl_layout.
 * Each iteration relabels the graph on the host and uploads it, the
 * reshuffling cost the paper notes.  stats->seconds sums the device time of
 * the iterations (host relabelling excluded).  Errors as bl_layout. */
int bl_layout_shuffled(const bl_csr *g, const double *x0, const double *y0, const bl_params *p,
                       uint64_t seed, void *hip_stream, double *x_out, double *y_out,
                       double *energy_out, bl_stats *stats);

/* ------------------------------------------------ greedy initial layout
 * The greedy initialisation of Sec. 3.6 (Algorithm 3): `start` is placed at
 * (0, 0) and pushed on a stack; each popped vertex U places every neighbour
 * that is not yet placed, in row order, on the unit circle around U, at
 * angles 0, d, 2d, ... degrees with d = 360 / deg(U) (deg counts all of U's
 * neighbours) and pi taken as the paper's 3.1416, and pushes it.  The paper
 * draws `start` at random; the caller passes it.
 * x, y (host FP64, length n) are in/out.  On entry only the entries of
 * vertices that `start` cannot reach are read: the lowest-id vertex of each
 * such component keeps its position and the component is placed from it the
 * same way, components in increasing order of that id.  On return they hold
 * the initial layout for bl_layout.  g must be host memory (no
 * BL_DEVICE_PTRS); rows in the order the traversal should see them.
 * Runs on the host (a sequential O(n + m) traversal), no device work.
 * Errors: BL_E_INVAL for NULL arrays, start out of range or a malformed CSR
 * (rowptr not monotone, colidx out of range), BL_E_NOMEM. */
int bl_greedy_init(const bl_csr *g, int32_t start, double *x, double *y);

/* ------------------------------------------------------ layout quality
 * The quality measures of Sec. 3.7 for the layout (x, y) of g, in FP64 on
 * the GPU:
 *  - stress after the best uniform scaling s: sum over pairs of
 *    d_ij^-2 (s |c_i - c_j| - d_ij)^2, minimised over s in closed form
 *    (N - A^2/B with A = sum |.|/d, B = sum |.|^2/d^2, N the pair count),
 *    d_ij the BFS hop distance, pairs that cannot reach each other skipped;
 *  - edge energy: sum over undirected edges of d^3 / (3K), the attractive
 *    potential whose gradient is the attraction term of Sec. 2.2;
 *  - edge uniformity: the standard deviation of edge lengths over their
 *    mean (normalised as in Sec. 3.7).
 * npivots = 0: stress over all unordered pairs i < j; otherwise over pairs
 * (p, j), j != p, for each pivot p of the host array pivots[npivots]
 * (repeats count again).  Hop distances come from a bit-parallel BFS with 64
 * sources per pass.  With BL_DEVICE_PTRS in flags, g, x and y are device
 * pointers (pivots stay host memory).  The work runs on hip_stream and the
 * call returns when it is done; temporary device memory is allocated and
 * freed inside.  Sums run in a fixed order: the same inputs give the same bits.
 * Errors: BL_E_INVAL (NULL arrays, bad CSR, K <= 0, a pivot out of range),
 * BL_E_NOMEM, BL_E_HIP. */
typedef struct {
    double  stress;          /* at the optimal scale                          */
    double  scale;           /* the optimal s = A / B (0 when B = 0)          */
    int64_t pairs;           /* pairs in the stress sum                       */
    double  edge_energy;     /* sum over edges of d^3 / (3K)                  */
    double  edge_uniformity; /* std(edge length) / mean(edge length)          */
    int64_t edges;           /* undirected edges                              */
    int64_t bfs_levels;      /* BFS levels launched, all passes               */
    double  reserved[2];
} bl_quality;

int bl_quality_eval(const bl_csr *g, const double *x, const double *y, int32_t npivots,
                    const int32_t *pivots, double K, uint32_t flags, void *hip_stream,
                    bl_quality *out);

/* Neighbourhood preservation (Sec. 3.7, the measure of tsNET and Maxent):
 * the mean, over vertices i with k = deg(i) > 0, of the Jaccard index
 * |N(i) & L(i)| / |N(i) | L(i)| of i's graph neighbours N(i) and the k
 * vertices L(i) nearest to i in the layout.  The paper names the measure but
 * not its neighbourhood size; k = deg(i) is the reading used here.  Distances
 * are squared Euclidean in FP64 without fused multiply-add, equal distances
 * ordered by vertex id, so every membership decision is exact.
 * nsample = 0: over all vertices; otherwise over the vertices of the host
 * array sample[nsample] (repeats count again).  Isolated vertices are
 * skipped; *counted (may be NULL) receives how many vertices were averaged
 * and *np_out the mean (0 when none).  With BL_DEVICE_PTRS in flags, g, x and
 * y are device pointers (sample stays host memory).  Coordinates must be
 * finite.  One workgroup per sampled vertex runs a radix selection over all
 * n vertices.  Temporary device memory is allocated and freed inside; the
 * same inputs give the same bits.
 * Errors: BL_E_INVAL (NULL arrays, bad CSR, a sample vertex out of range),
 * BL_E_NOMEM, BL_E_HIP. */
int bl_neighborhood_preservation(const bl_csr *g, const double *x, const double *y, int32_t nsample,
                                 const int32_t *sample, uint32_t flags, void *hip_stream,
                                 double *np_out, int64_t *counted);

/* bl_quality_eval for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same results, bit for bit, with every work buffer in
 * one static device array of the library (about 11.9 MiB per GPU, reserved
 * from the first use on that GPU until the process ends) instead of device
 * memory allocated per call.  No hipMalloc, hipFree or other allocation.
 *  - flags must be exactly BL_DEVICE_PTRS: g's arrays, x and y are device
 *    memory the caller owns; pivots (npivots of them, or NULL for all pairs)
 *    stay host memory and are copied into the array.
 *  - Limits: 1 <= n <= 262144 vertices, npivots <= 65536 (BL_E_INVAL above).
 *  - The CSR is checked on the device (rowptr from 0 to nnz, non-decreasing,
 *    colidx in [0, n)); BL_VALIDATE's full checks are not available here.
 *  - Calls on one GPU share its array: calls that overlap in time on one GPU
 *    (from several host threads or streams) race and give wrong results; the
 *    caller serialises them.  Each call starts from cleared state, so a call
 *    never depends on the previous one.
 * Errors: as bl_quality_eval, plus BL_E_INVAL for the limits above. */
int bl_quality_eval_noalloc(const bl_csr *g, const double *x, const double *y, int32_t npivots,
                            const int32_t *pivots, double K, uint32_t flags, void *hip_stream,
                            bl_quality *out);

/* --------------------------------------------------------- one minibatch
 * Net forces (attraction + repulsion, no update) on the vertices of batch
 * `batch_index` (ids [b*BS, min((b+1)*BS, n))) from coordinates (x, y)
 * (Sec. 2.2, the combined force f(i,c)).  In BH mode the quadtree is built
 * from the snapshot (sx, sy) -- the coordinates at the start of the
 * iteration -- or from (x, y) when sx/sy are NULL; leaves use (x, y).
 * fx, fy receive BS (or the ragged remainder) values as FP64.
 * Errors: BL_E_INVAL if batch_index is out of range or arguments are bad. */
int bl_forces(const bl_csr *g, const double *x, const double *y,
              const double *sx, const double *sy, int32_t batch_index,
              const bl_params *p, void *hip_stream, double *fx, double *fy);

/* ------------------------------------------------------ resident handle
 * A layout job whose CSR, coordinates and work buffers live on the device
 * between calls (used by the benchmark, the batched path and the server). */
typedef struct bl_graph bl_graph;

/* Upload g (host, or device with BL_DEVICE_PTRS in p->flags) and allocate the
 * work buffers for parameters p.  Coordinates start at zero. */
int bl_graph_create(const bl_csr *g, const bl_params *p, void *hip_stream, bl_graph **out);

/* Replace the coordinates (FP64 arrays of length n; flags may hold BL_DEVICE_PTRS). */
int bl_graph_set_coords(bl_graph *h, const double *x, const double *y, uint32_t flags);

/* Copy the current coordinates out as FP64 (flags may hold BL_DEVICE_PTRS). */
int bl_graph_get_coords(bl_graph *h, double *x, double *y, uint32_t flags);

/* Run iterations [start_iter, start_iter + iterations) on the resident state.
 * stop_batch < 0: run them all.  stop_batch = b >= 0: the last iteration
 * stops after computing the forces of batch b, which are written to (fx, fy)
 * (host FP64, BS values or the ragged remainder) without moving the batch;
 * the coordinates then hold the state those forces were computed from.
 * energy_out (host, may be NULL) receives one value per full iteration.
 * Resuming is exact: run(k1) followed by run(k2, start_iter = k1) gives the
 * same coordinates as run(k1 + k2). */
int bl_graph_run(bl_graph *h, int32_t iterations, int32_t start_iter, int32_t stop_batch,
                 double *energy_out, double *fx, double *fy, bl_stats *stats);

/* Release the device state of h.  NULL is accepted. */
int bl_graph_destroy(bl_graph *h);

/* Per-kernel device time of this job's launches, measured with hipEvents on
 * the job's stream.  enable != 0 switches recording on (and resets the
 * totals); 0 switches it off.  Adds two event records per profiled launch. */
int bl_graph_profile(bl_graph *h, int32_t enable);

/* Totals since the last bl_graph_profile(h, 1) for one kernel: "rows_kernel",
 * "step_kernel", "finalize_kernel", "exact_graph_kernel", "steps_kernel" (exact mode),
 * "tree_build" (the whole quadtree build sequence, one entry per iteration),
 * "far_kernel", "chain_kernel" (Barnes-Hut, one entry per launch; the chain
 * launch holds the chain and its helper workgroups).  Counts instead of times,
 * returned in *launches: "late_entries" (moved-leaf entries the far-field
 * walks listed), "old_entries" and "recent_entries" (moved-neighbour and
 * moved-leaf entries summed by the chain's helpers and by the chain itself),
 * "cell_tests" (cells the far-field walks tested with the acceptance
 * criterion). */
int bl_graph_profile_read(bl_graph *h, const char *kernel, double *total_ms, int64_t *launches);

/* -------------------------------------------------- diagnostics
 * Instruction issue rate of the device, for stating the exact kernel's
 * instruction-bound ceiling (no part of the layout path).  Runs `blocks`
 * workgroups of 256 threads, each thread `iters` rounds over 8 independent
 * chains of: op 0, one FP32 fused multiply-add (v_fma_f32); op 1, one
 * hardware reciprocal (v_rcp_f32); op 2, one reciprocal and six multiply-adds
 * of other chains (the repulsion term's mix).  One untimed launch, then one
 * timed with hipEvents on hip_stream (NULL: the default stream).  *ms gets
 * the timed launch's duration; *lane_ops (may be NULL) the instructions it
 * issued, counted per lane.  The probe allocates and frees its own 1 KiB per
 * workgroup of device memory.  Errors: BL_E_INVAL (op not 0..2, blocks or
 * iters not positive, ms NULL), BL_E_NOMEM, BL_E_HIP. */
int bl_probe_issue_rate(int32_t op, int32_t blocks, int32_t iters, void *hip_stream, double *ms,
                        double *lane_ops);

/* -------------------------------------------------- many graphs at once
 * Lay out G independent graphs; graph i uses params[i] (iterations, batch
 * size, mode, theta may differ).  Graphs small enough for one workgroup run
 * in one persistent launch, one workgroup per graph; larger graphs run
 * through the single-graph path on the same stream.  Each result equals the
 * graph's own bl_layout result bitwise.  x_out[i] may alias x0[i].
 * stats (may be NULL) has G entries. */
int bl_layout_batch(int32_t G, const bl_csr *const *graphs, const double *const *x0,
                    const double *const *y0, const bl_params *const *params,
                    void *hip_stream, double *const *x_out, double *const *y_out,
                    bl_stats *stats);

/* ------------------------------------------------------------- server
 * Continuous batching of layout jobs: a host scheduler thread admits queued
 * jobs while their bl_footprint_bytes fits the remaining HBM budget and a
 * slot is free, keeps admitted jobs' state on the device, and interleaves
 * their iterations on the device.  A job's result equals its alone result
 * bitwise. */
typedef struct bl_server bl_server;

/* hbm_budget_bytes > 0; 1 <= max_slots <= 4096.  The server runs on the
 * current device on its own stream (hip_stream is reserved, may be NULL). */
int bl_server_create(size_t hbm_budget_bytes, int32_t max_slots, void *hip_stream,
                     bl_server **out);
/* Copies the graph and coordinates (host pointers only) and queues the job.
 * BL_E_REJECTED if the job alone exceeds the whole budget. */
int bl_server_submit(bl_server *s, const bl_csr *g, const double *x0, const double *y0,
                     const bl_params *p, int64_t *job);
/* *done = 1 when the job has finished (successfully or not). Non-blocking. */
int bl_server_poll(bl_server *s, int64_t job, int32_t *done);
/* Block until the job is done or timeout_s seconds passed (BL_E_TIMEOUT). */
int bl_server_wait(bl_server *s, int64_t job, double timeout_s);
/* Copy the result out; BL_E_NOTREADY while running.  stats may be NULL; its
 * `seconds` is the job's latency from submit to completion. */
int bl_server_fetch(bl_server *s, int64_t job, double *x, double *y, bl_stats *stats);
/* Forget a finished job (or cancel a queued one). */
int bl_server_release(bl_server *s, int64_t job);
/* Stop the scheduler, cancel pending work, free everything.  NULL accepted. */
int bl_server_destroy(bl_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BATCHLAYOUT_H */
