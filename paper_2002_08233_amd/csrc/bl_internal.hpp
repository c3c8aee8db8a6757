// Host-side internals of the BatchLayout library: the resident job state and
// the launchers each kernel file provides.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/batchlayout.h"

namespace bl {

void set_error(const char *fmt, ...);

#define BL_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::bl::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                            __FILE__, __LINE__);                                      \
            return BL_E_HIP;                                                          \
        }                                                                             \
    } while (0)

#define BL_TRY(expr)               \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != BL_OK) return rc_; \
    } while (0)

// Late-leaf list capacity per vertex (Barnes-Hut near field, see bl_bh.hip).
constexpr int kLateCap = 96;

// Device counters shared by the kernels of one job.
struct Counters {
    unsigned long long nonfinite;
    unsigned long long visits;
    unsigned long long late_overflow;
    unsigned long long late_total;
    unsigned long long old_total;      // late entries summed by the segment kernel
    unsigned long long recent_total;   // late entries summed by the chain
    unsigned long long wait_abort;     // a bounded device wait ran out (the launch left early)
    unsigned long long halted;         // the energy stopping rule held after this many iterations
    unsigned long long cell_tests;     // far-field walks: cells tested by the acceptance criterion
};

// Per-kernel device time, measured with hipEvents around launches when a
// job's profiling is on.
enum ProfKernel { PK_ROWS = 0, PK_PANEL, PK_FINALIZE, PK_TREE, PK_FAR, PK_CHAIN, PK_GRAPH, PK_STEPS, PK_COUNT };
constexpr int kProfPool = 8192;
struct Prof {
    bool on = false;
    int used = 0;
    hipEvent_t ev[2 * kProfPool] = {};
    int kid[kProfPool] = {};
    double ms[PK_COUNT] = {};
    long long launches[PK_COUNT] = {};
    long long late_total = 0;
    long long old_total = 0, recent_total = 0, cell_tests = 0;
};

struct BHEngine;
struct BHJob;

// Barnes-Hut buffers of one job (device memory unless noted).
struct BHBuffers {
    float *bbox;            // [6]: xmin, ymin, W, scale, pad, pad
    float *bbox_part;       // [2 * 4 * kBBoxBlocks] block partial min/max
    unsigned *key[2];       // Morton keys, double-buffered for the radix sort
    int *val[2];            // vertex ids
    int *hist;              // radix histogram [256 * tiles]
    int tiles;
    unsigned *mask;         // [n] per sorted position: bit l set if a kept cell of level l starts here
    int *cellcnt;           // [n + 1] exclusive scan of popcount(mask)
    int *scan_part;         // scan block partials
    double *pdd;            // [4 * (n + 1)]: double-double prefix sums of sorted x, y
    double *pdd_part;       // [4 * blocks]
    float4 *nodeA;          // [2n]: centroid hi x, y, side^2 (inf for buckets), centroid lo x, y as two bf16
    int2 *nodeB;            // [2n]: skip, vertex (leaves) or -count (cells)
    int *leafpos;           // [n]: pre-order index of each vertex's leaf
    int *nnodes;            // [1]
    float4 *far;            // [n]: Kahan (sx, sy, cx, cy) of the far-field sum
    int *late_cnt;          // [n]
    int *late_ids;          // [n * kLateCap]
    float *snap;            // [2n] snapshot given to the one-shot force call
    void *fbuf;             // [BS] float2 net forces of the current batch
    int *late_att;          // [n] length of the moved-neighbour prefix of each CSR row
    int *old_att;           // [n] its part in earlier chain segments
    int *roff_old;          // [n] offset of each row's old entries within its batch list
    int *bold;              // [nb + 1] length of each batch list's old part
    float4 *rec;            // [n] chain row records: x, y, force apart from recent entries
    int2 *rmeta;            // [n] offset in the batch's recent list, late-leaf count
    float2 *oldf;           // [n] old-entry sums, from the helpers to the chain
    int *sync;              // [nb + 2] progress words of the chain launch
    int *hbase;             // [nb + 1] helper parts per batch, then (scanned) the first part's item
    int2 *hitem;            // helper items: (batch, part)
    int *heavy;             // [n] rows with many early neighbours (first *nheavy used)
    int *nheavy;            // [1]
    float2 *atte;           // [n] early attraction (neighbours not yet moved)
    int *roff;              // [n] offset of each row's late entries within its batch list
    int *bbase;             // [nb + 1] start of each batch's late entry list
    unsigned long long *ent;// late entries (row in batch << 32 | vertex, bit 31: leaf)
    int *pstart;            // [n] first slot of each row's run within its batch's slot plan
    int *pbase;             // [nb + 1] slot counts, then first slots of the batches' plans
    unsigned long long *slots;  // the batches' slot plans (one word per lane of the chain)
    int *pflag;             // [nb] batch flags of the chain's slot plan
    int4 *bmeta;            // [nb] per batch: first slot, slot count, recent-list start, flags
    int *kiter;             // [2] current iteration, first iteration of the run
    int host_kiter[2];      // host staging for kiter
    bool prefix_ready;      // late_att/heavy computed for this job
    BHEngine *engine;       // one-job launch tables (host object)
};

// What one run of a Barnes-Hut job computes.
struct BHRunSpec {
    int all_live = 0;             // one-shot forces: all leaves and neighbours live
    int first_batch = 0, last_batch = 0, stop_batch = -1;
    const float2 *src = nullptr;  // tree source (NULL: the live coordinates)
};

// Exact-mode buffers (all device memory).
struct ExactBuffers {
    void *accS[2];          // [n] T2 (float2 / double2): per-row force sums, by iteration parity
    float2 *accC[2];        // [n] Kahan compensation (FP32 Kahan only)
    int2 *segs;             // CSR segments: (column batch, first entry) of each run of a row's
                            // neighbours that fall in one batch, rows in order
    size_t segs_cap;        // segments segs holds room for (kept across CSR reloads)
    int *segoff;            // [n + 1] first segment of each row
    int *cursor;            // [n] next segment of each row in the column-batch cycle
    double *epart;          // energy partials of the row chunks of one batch
    unsigned *ticket;       // last-workgroup counter of the batch finalize
    double *echunk;         // persistent run: [2][nb][BS / kRows + 2] chunk energies by iteration parity
    double *ebatch;         // persistent run: [2][nb] batch energies by iteration parity
    unsigned *eticket;      // persistent run: [2][nb + 1] chunks combined per batch, then batches combined
    void *d_job;            // one-job table of the one-workgroup kernel
    unsigned *moved;        // [nb] chunk moves of each batch in the current persistent run
};

}  // namespace bl

// The resident layout job.
struct bl_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    bl_params p{};
    hipStream_t stream = nullptr;
    bool fp64 = false;
    bool aos = false;           // coordinates stored as interleaved float2 (Barnes-Hut)
    int nb = 0;                 // number of batches
    int *rowptr = nullptr;      // device CSR
    int *colidx = nullptr;
    void *x = nullptr;          // device coordinates: float/double x[n] (exact), or float2 xy[n] (BH)
    void *y = nullptr;          // y[n] (exact mode only)
    double *erow = nullptr;     // [n] per-vertex |f|^2 of the current iteration
    // Exact mode, multi-workgroup path: a run that ends with keep_next set
    // also adds the last iteration's panels toward the next iteration, and
    // cont_iter records that iteration, so a run starting there skips its
    // prologue (the same sums, already in place).  Anything else that runs
    // or writes coordinates resets cont_iter to -1.
    int cont_iter = -1;
    bool keep_next = false;
    double *energy = nullptr;   // [energy_cap] per-iteration energies
    int energy_cap = 0;
    double *fout = nullptr;     // [2 * BS] forces of a stopped batch (FP64)
    double *stage = nullptr;    // [2 * n] FP64 staging for coordinate transfers
    bl::Counters *counters = nullptr;
    bl::ExactBuffers ex{};
    bl::BHBuffers bh{};
    void *owned[64] = {};       // every device allocation of this job
    int nowned = 0;
    bl::Prof *prof = nullptr;   // profiling state (NULL when never enabled)
    bool async_mem = false;     // device memory is stream-ordered (hipMallocAsync / hipFreeAsync on stream)
    bool coop = true;           // may run an exact layout as one cooperative (persistent) launch; off when
                                // the job shares the device with other work of this library
};

namespace bl {

int graph_alloc(bl_graph *g, void **ptr, size_t bytes);
// bl_graph_create with stream-ordered device memory when async_mem (nothing
// in create or destroy then waits for other streams).
int graph_create_ex(const bl_csr *csr, const bl_params *p, hipStream_t s, bool async_mem, bl_graph **out);
// Replace g's CSR by another of the same n and nnz (host arrays, already
// checked) and rebuild what the layout derives from it; the next run starts
// with its prologue.
int graph_reload_csr(bl_graph *g, const int32_t *rowptr, const int32_t *colidx);
int fail_code(int code, const char *msg);
// Host CSR checks: sizes, monotone rowptr, colidx in range; with `full` also
// sorted rows, no self-loops or duplicates, symmetry.
int check_csr_host(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, bool full);
// The same checks on a graph given in host or (BL_DEVICE_PTRS) device memory.
int check_csr(const bl_csr *g, uint32_t flags, hipStream_t s);
int params_check(const bl_params *p);
// The (a, r) model is not Fruchterman-Reingold's (2, -1).
inline bool model_general(const bl_params &p) { return p.model_a != 2 || p.model_r != -1; }
int stats_fill(bl_graph *g, bl_stats *st, int iters_run, double seconds);

// exact mode (bl_exact.hip)
int exact_alloc(bl_graph *g);
int exact_prepare(bl_graph *g);   // after the CSR upload
int exact_run(bl_graph *g, int iters, int start_iter, int stop_batch);
int exact_forces(bl_graph *g, int batch);
// The same under (a, r) models other than (2, -1) (bl_exact_models.hip).
int exact_run_model(bl_graph *g, int iters, int start_iter, int stop_batch);
int exact_forces_model(bl_graph *g, int batch);
int exact_graph_launch(bl_graph *const *gs, int G, int threads, hipStream_t s, void *d_jobs, int iters_override,
                       int start_override = -1);
size_t exact_job_size();
size_t exact_footprint(int n, int64_t nnz, int BS, bool fp64);

// Barnes-Hut mode (bl_bh.hip)
int bh_alloc(bl_graph *g);
int bh_run(bl_graph *g, int iters, int start_iter, int stop_batch);
int bh_forces(bl_graph *g, int batch, const double *snap_x, const double *snap_y);
size_t bh_footprint(int n, int64_t nnz, int batch_size);
int bh_set_iteration(bl_graph *g, int k);

// Multi-job launches: one launch per kernel serves every job of the set.
int bh_engine_create(hipStream_t s, BHEngine **out);
void bh_engine_destroy(BHEngine *e);
int bh_fill_job(bl_graph *g, BHJob *J, const BHRunSpec &spec);
int bh_engine_set(BHEngine *e, const BHJob *jobs, int G);
int bh_engine_setup(BHEngine *e);
int bh_engine_iteration(BHEngine *e, bl_graph *prof);
int bh_engine_run(BHEngine *e, int iters, bool use_graph);
size_t bh_job_size();

// shared kernels (bl_common.hip)
int energy_sum(bl_graph *g, int k);
int convert_coords_in(bl_graph *g, const double *x, const double *y);   // device FP64 -> state
int convert_coords_out(bl_graph *g, double *x, double *y);              // state -> device FP64
int convert_to_float2(bl_graph *g, const double *x, const double *y, float2 *o);

double step_at(const bl_params &p, int k);

// Profiling around launches (no-ops unless enabled on the job).
int prof_begin(bl_graph *g, int kid, int *slot);
int prof_end(bl_graph *g, int slot);
int prof_collect(bl_graph *g);

}  // namespace bl
