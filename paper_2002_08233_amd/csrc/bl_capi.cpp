// C ABI of the BatchLayout library: argument checks, the resident job handle,
// and the one-shot calls built on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "bl_internal.hpp"

namespace bl {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

static int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int graph_alloc(bl_graph *g, void **ptr, size_t bytes) {
    if (g->nowned >= (int)(sizeof(g->owned) / sizeof(g->owned[0])))
        return fail(BL_E_NOMEM, "too many allocations in one job");
    if (bytes == 0) bytes = 16;
    void *p = nullptr;
    hipError_t e = g->async_mem ? hipMallocAsync(&p, bytes, g->stream) : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BL_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    g->owned[g->nowned++] = p;
    *ptr = p;
    return BL_OK;
}

int check_params(const bl_params *p);
int fail_code(int code, const char *msg) { return fail(code, "%s", msg); }
int params_check(const bl_params *p) { return check_params(p); }

int check_params(const bl_params *p) {
    if (!p) return fail(BL_E_INVAL, "params is NULL");
    if (p->batch_size < 1) return fail(BL_E_INVAL, "batch_size must be >= 1");
    if (p->iterations < 0) return fail(BL_E_INVAL, "iterations must be >= 0");
    if (p->start_iter < 0) return fail(BL_E_INVAL, "start_iter must be >= 0");
    if (p->mode != BL_EXACT && p->mode != BL_BH) return fail(BL_E_INVAL, "unknown mode %d", p->mode);
    if (p->precision < BL_FP32_KAHAN || p->precision > BL_FP64)
        return fail(BL_E_INVAL, "unknown precision %d", p->precision);
    if (p->mode == BL_BH && p->precision == BL_FP64)
        return fail(BL_E_INVAL, "FP64 precision is provided for exact mode only");
    if (p->mode == BL_BH && p->batch_size > 1024)
        return fail(BL_E_INVAL, "Barnes-Hut mode supports batch sizes up to 1024");
    if (p->mode == BL_BH && !p->repulse_adjacent)
        return fail(BL_E_INVAL, "Barnes-Hut mode repels all pairs (repulse_adjacent must be 1)");
    if (!(p->step0 > 0) || !std::isfinite(p->step0)) return fail(BL_E_INVAL, "step0 must be > 0");
    if (!(p->step_decay > 0 && p->step_decay <= 1)) return fail(BL_E_INVAL, "step_decay must be in (0,1]");
    if (!(p->K > 0) || !std::isfinite(p->K)) return fail(BL_E_INVAL, "K must be > 0");
    if (!(p->R > 0) || !std::isfinite(p->R)) return fail(BL_E_INVAL, "R must be > 0");
    if (!(p->theta >= 0) || !std::isfinite(p->theta)) return fail(BL_E_INVAL, "theta must be >= 0");
    if (p->flags & ~(BL_DEVICE_PTRS | BL_VALIDATE | BL_BH_SNAPSHOT_LEAVES | BL_EXACT_MULTI_WG | BL_ADAPTIVE_STEP))
        return fail(BL_E_INVAL, "unknown flags 0x%x", p->flags);
    if (!(p->conv_tol >= 0) || !std::isfinite(p->conv_tol)) return fail(BL_E_INVAL, "conv_tol must be >= 0");
    if (p->reserved0) return fail(BL_E_INVAL, "reserved fields must be zero");
    for (int q = 0; q < 2; ++q)
        if (p->reserved[q]) return fail(BL_E_INVAL, "reserved fields must be zero");
    if (!(p->model_r < p->model_a) || p->model_r < -8 || p->model_a > 8)
        return fail(BL_E_INVAL, "the (a, r) model needs integers -8 <= r < a <= 8");
    return BL_OK;
}

// Host-side CSR checks.  Always: sizes, rowptr monotone, colidx in range (an
// out-of-range id would make a kernel read outside its buffers).  With
// BL_VALIDATE also: sorted rows, no self-loops or duplicates, symmetry.
int check_csr_host(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, bool full) {
    if (rp[0] != 0) return fail(BL_E_INVAL, "rowptr[0] must be 0");
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(BL_E_INVAL, "rowptr decreases at row %d", i);
    if ((int64_t)rp[n] != nnz) return fail(BL_E_INVAL, "rowptr[n] != nnz");
    for (int64_t e = 0; e < nnz; ++e)
        if (ci[e] < 0 || ci[e] >= n) return fail(BL_E_INVAL, "colidx[%lld] out of range", (long long)e);
    if (!full) return BL_OK;
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] == i) return fail(BL_E_INVAL, "self-loop at row %d", i);
            if (e > rp[i] && ci[e] <= ci[e - 1]) return fail(BL_E_INVAL, "row %d unsorted or duplicate", i);
        }
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            if (!std::binary_search(ci + rp[j], ci + rp[j + 1], i))
                return fail(BL_E_INVAL, "not symmetric: (%d,%d) without (%d,%d)", i, j, j, i);
        }
    return BL_OK;
}

int check_csr(const bl_csr *g, uint32_t flags, hipStream_t s) {
    if (!g) return fail(BL_E_INVAL, "graph is NULL");
    if (g->n < 1) return fail(BL_E_INVAL, "n must be >= 1");
    if (g->nnz < 0 || g->nnz > 0x7fffffffLL) return fail(BL_E_INVAL, "nnz out of range");
    if (!g->rowptr || (g->nnz > 0 && !g->colidx)) return fail(BL_E_INVAL, "CSR arrays are NULL");
    const bool full = (flags & BL_VALIDATE) != 0;
    if (!(flags & BL_DEVICE_PTRS)) return check_csr_host(g->n, g->nnz, g->rowptr, g->colidx, full);
    std::vector<int32_t> rp(g->n + 1), ci(std::max<int64_t>(g->nnz, 1));
    BL_HIP(hipMemcpyAsync(rp.data(), g->rowptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost, s));
    if (g->nnz)
        BL_HIP(hipMemcpyAsync(ci.data(), g->colidx, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    return check_csr_host(g->n, g->nnz, rp.data(), ci.data(), full);
}

static void free_graph(bl_graph *g) {
    if (!g) return;
    if (g->p.mode == BL_BH && g->bh.engine) bh_engine_destroy(g->bh.engine);
    for (int q = 0; q < g->nowned; ++q) {
        if (g->async_mem) (void)hipFreeAsync(g->owned[q], g->stream);
        else (void)hipFree(g->owned[q]);
    }
    if (g->prof) {
        for (int q = 0; q < 2 * kProfPool; ++q)
            if (g->prof->ev[q]) (void)hipEventDestroy(g->prof->ev[q]);
        delete g->prof;
    }
    delete g;
}

static int ensure_energy(bl_graph *g, int iters) {
    if (iters <= g->energy_cap) return BL_OK;
    int cap = std::max(iters, 64);
    BL_TRY(graph_alloc(g, (void **)&g->energy, sizeof(double) * cap));
    g->energy_cap = cap;
    return BL_OK;
}

// Stats of a finished run of g (device counters and per-iteration energies).
int stats_fill(bl_graph *g, bl_stats *st, int iters_run, double seconds) {
    Counters c{};
    BL_HIP(hipMemcpy(&c, g->counters, sizeof c, hipMemcpyDeviceToHost));
    if (c.halted) iters_run = std::min(iters_run, (int)c.halted);
    double e_last = 0.0;
    if (iters_run > 0) BL_HIP(hipMemcpy(&e_last, g->energy + iters_run - 1, 8, hipMemcpyDeviceToHost));
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->iters_run = iters_run;
        st->energy_last = e_last;
        st->seconds = seconds;
        st->node_visits = (int64_t)c.visits;
        st->nonfinite_events = (int64_t)c.nonfinite;
        st->late_overflow = (int32_t)c.late_overflow;
    }
    if (c.wait_abort) return fail(BL_E_TIMEOUT, "a bounded device wait ran out (the launch left early)");
    return c.nonfinite ? BL_E_NONFINITE : BL_OK;
}

}  // namespace bl

using namespace bl;

extern "C" {

int bl_params_init(bl_params *p) {
    if (!p) return fail(BL_E_INVAL, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->batch_size = 256;
    p->iterations = 600;
    p->start_iter = 0;
    p->mode = BL_EXACT;
    p->precision = BL_FP32_KAHAN;
    p->repulse_adjacent = 1;
    p->step0 = 1.0;
    p->step_decay = 0.999;
    p->K = 1.0;
    p->R = 1.0;
    p->theta = 1.2;
    p->model_a = 2;
    p->model_r = -1;
    p->flags = 0;
    return BL_OK;
}

const char *bl_last_error(void) { return g_err; }

const char *bl_version(void) { return "batchlayout-gfx950 0.1"; }

size_t bl_footprint_bytes(int32_t n, int64_t nnz, const bl_params *p) {
    if (n < 1 || nnz < 0 || !p || check_params(p) != BL_OK) return 0;
    const size_t N = (size_t)n, T = (p->precision == BL_FP64) ? 8 : 4;
    size_t b = 4 * (N + 1) + 4 * (size_t)nnz;      // CSR
    b += 2 * T * N;                                 // coordinates
    b += 16 * N + 2 * 8 * N;                        // staging, per-row energy
    b += 2 * 8 * (size_t)p->batch_size + 4096;      // forces out, counters
    b += 8 * (size_t)std::max(p->iterations, 64);   // energy per iteration
    if (p->mode == BL_EXACT)
        b += exact_footprint(n, nnz, p->batch_size, p->precision == BL_FP64);
    else
        b += bh_footprint(n, nnz, p->batch_size);
    return b;
}

int bl_graph_create(const bl_csr *csr, const bl_params *p, void *hip_stream, bl_graph **out) {
    return graph_create_ex(csr, p, (hipStream_t)hip_stream, false, out);
}

}  // extern "C"

int bl::graph_reload_csr(bl_graph *g, const int32_t *rowptr, const int32_t *colidx) {
    const size_t N = (size_t)g->n;
    BL_HIP(hipMemcpyAsync(g->rowptr, rowptr, 4 * (N + 1), hipMemcpyHostToDevice, g->stream));
    if (g->nnz) BL_HIP(hipMemcpyAsync(g->colidx, colidx, 4 * (size_t)g->nnz, hipMemcpyHostToDevice, g->stream));
    g->cont_iter = -1;
    g->keep_next = false;
    if (g->p.mode == BL_EXACT) BL_TRY(exact_prepare(g));   // CSR segments by column batch
    else g->bh.prefix_ready = false;                       // moved-neighbour prefixes, heavy rows
    BL_HIP(hipStreamSynchronize(g->stream));
    return BL_OK;
}

int bl::graph_create_ex(const bl_csr *csr, const bl_params *p, hipStream_t s, bool async_mem, bl_graph **out) {
    if (!out) return fail(BL_E_INVAL, "out is NULL");
    *out = nullptr;
    BL_TRY(check_params(p));
    if (p->flags & BL_ADAPTIVE_STEP) return fail(BL_E_INVAL, "BL_ADAPTIVE_STEP is a bl_layout option");
    BL_TRY(check_csr(csr, p->flags, s));
    bl_graph *g = new bl_graph();
    g->async_mem = async_mem;
    g->n = csr->n;
    g->nnz = csr->nnz;
    g->p = *p;
    g->stream = s;
    g->fp64 = (p->precision == BL_FP64);
    g->aos = (p->mode == BL_BH);
    g->nb = (g->n + p->batch_size - 1) / p->batch_size;
    const size_t N = (size_t)g->n, T = g->fp64 ? 8 : 4;
    int rc = BL_OK;
    auto A = [&](void **ptr, size_t bytes) {
        if (rc == BL_OK) rc = graph_alloc(g, ptr, bytes);
    };
    A((void **)&g->rowptr, 4 * (N + 1));
    A((void **)&g->colidx, 4 * (size_t)std::max<int64_t>(g->nnz, 1));
    A(&g->x, 2 * T * N);
    A(&g->y, T * N);
    A((void **)&g->stage, 16 * N);
    A((void **)&g->erow, 8 * N);
    A((void **)&g->fout, 16 * (size_t)p->batch_size);
    A((void **)&g->counters, sizeof(Counters));
    if (rc == BL_OK) rc = ensure_energy(g, std::max(p->iterations, 1));
    if (rc == BL_OK) rc = (p->mode == BL_EXACT) ? exact_alloc(g) : bh_alloc(g);
    if (rc != BL_OK) {
        free_graph(g);
        return rc;
    }
    const hipMemcpyKind kind = (p->flags & BL_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpyAsync(g->rowptr, csr->rowptr, 4 * (N + 1), kind, s);
    if (e == hipSuccess && g->nnz)
        e = hipMemcpyAsync(g->colidx, csr->colidx, 4 * (size_t)g->nnz, kind, s);
    if (e == hipSuccess) e = hipMemsetAsync(g->x, 0, 2 * T * N, s);
    if (e == hipSuccess) e = hipMemsetAsync(g->y, 0, T * N, s);
    if (e == hipSuccess) e = hipMemsetAsync(g->counters, 0, sizeof(Counters), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("graph upload failed: %s", hipGetErrorString(e));
        free_graph(g);
        return BL_E_HIP;
    }
    if (p->mode == BL_EXACT) {
        rc = exact_prepare(g);
        if (rc != BL_OK) {
            free_graph(g);
            return rc;
        }
    }
    *out = g;
    return BL_OK;
}

extern "C" {

int bl_graph_destroy(bl_graph *g) {
    if (!g) return BL_OK;
    (void)hipStreamSynchronize(g->stream);
    free_graph(g);
    return BL_OK;
}

int bl_graph_set_coords(bl_graph *g, const double *x, const double *y, uint32_t flags) {
    if (!g || !x || !y) return fail(BL_E_INVAL, "NULL argument");
    const size_t N = (size_t)g->n;
    if (flags & BL_DEVICE_PTRS) {
        BL_TRY(convert_coords_in(g, x, y));
    } else {
        for (size_t i = 0; i < N; ++i)
            if (!std::isfinite(x[i]) || !std::isfinite(y[i]))
                return fail(BL_E_INVAL, "coordinate %zu is not finite", i);
        BL_HIP(hipMemcpyAsync(g->stage, x, 8 * N, hipMemcpyHostToDevice, g->stream));
        BL_HIP(hipMemcpyAsync(g->stage + N, y, 8 * N, hipMemcpyHostToDevice, g->stream));
        BL_TRY(convert_coords_in(g, g->stage, g->stage + N));
    }
    BL_HIP(hipStreamSynchronize(g->stream));
    return BL_OK;
}

int bl_graph_get_coords(bl_graph *g, double *x, double *y, uint32_t flags) {
    if (!g || !x || !y) return fail(BL_E_INVAL, "NULL argument");
    const size_t N = (size_t)g->n;
    if (flags & BL_DEVICE_PTRS) {
        BL_TRY(convert_coords_out(g, x, y));
    } else {
        BL_TRY(convert_coords_out(g, g->stage, g->stage + N));
        BL_HIP(hipMemcpyAsync(x, g->stage, 8 * N, hipMemcpyDeviceToHost, g->stream));
        BL_HIP(hipMemcpyAsync(y, g->stage + N, 8 * N, hipMemcpyDeviceToHost, g->stream));
    }
    BL_HIP(hipStreamSynchronize(g->stream));
    return BL_OK;
}

static int run_impl(bl_graph *g, int32_t iterations, int32_t start_iter, int32_t stop_batch,
                    double *energy_out, double *fx, double *fy, bl_stats *st) {
    if (!g) return fail(BL_E_INVAL, "graph is NULL");
    if (iterations < 0 || start_iter < 0) return fail(BL_E_INVAL, "iterations/start_iter must be >= 0");
    if (stop_batch >= g->nb) return fail(BL_E_INVAL, "stop_batch %d out of range (%d batches)", stop_batch, g->nb);
    if (stop_batch >= 0 && iterations < 1) return fail(BL_E_INVAL, "stop_batch needs iterations >= 1");
    if (stop_batch >= 0 && (!fx || !fy)) return fail(BL_E_INVAL, "stop_batch needs fx, fy");
    if (stop_batch >= 0 && g->p.conv_tol > 0) return fail(BL_E_INVAL, "stop_batch cannot be combined with conv_tol");
    BL_TRY(ensure_energy(g, std::max(iterations, 1)));
    BL_HIP(hipMemsetAsync(g->counters, 0, sizeof(Counters), g->stream));
    hipEvent_t e0, e1;
    BL_HIP(hipEventCreate(&e0));
    BL_HIP(hipEventCreate(&e1));
    BL_HIP(hipEventRecord(e0, g->stream));
    int rc = (g->p.mode == BL_EXACT) ? exact_run(g, iterations, start_iter, stop_batch)
                                     : bh_run(g, iterations, start_iter, stop_batch);
    hipError_t he = hipEventRecord(e1, g->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(g->stream);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != BL_OK) return rc;
    if (he != hipSuccess) return fail(BL_E_HIP, "layout run failed: %s", hipGetErrorString(he));
    Counters c{};
    BL_HIP(hipMemcpy(&c, g->counters, sizeof c, hipMemcpyDeviceToHost));
    int full = (stop_batch >= 0) ? iterations - 1 : iterations;
    if (c.halted) full = std::min(full, (int)c.halted);   // the energy stopping rule ended the run
    std::vector<double> en(std::max(full, 1));
    if (full > 0) BL_HIP(hipMemcpy(en.data(), g->energy, 8 * (size_t)full, hipMemcpyDeviceToHost));
    if (energy_out && full > 0) std::memcpy(energy_out, en.data(), 8 * (size_t)full);
    if (stop_batch >= 0) {
        const int BS = g->p.batch_size;
        const int R = std::min(BS, g->n - stop_batch * BS);
        std::vector<double> f(2 * (size_t)R);
        BL_HIP(hipMemcpy(f.data(), g->fout, 16 * (size_t)R, hipMemcpyDeviceToHost));
        for (int q = 0; q < R; ++q) {
            fx[q] = f[2 * q];
            fy[q] = f[2 * q + 1];
        }
    }
    if (g->prof) {
        BL_TRY(prof_collect(g));
        g->prof->late_total += (long long)c.late_total;
        g->prof->old_total += (long long)c.old_total;
        g->prof->recent_total += (long long)c.recent_total;
        g->prof->cell_tests += (long long)c.cell_tests;
    }
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->iters_run = full;
        st->energy_last = full > 0 ? en[full - 1] : 0.0;
        st->seconds = ms * 1e-3;
        st->node_visits = (int64_t)c.visits;
        st->nonfinite_events = (int64_t)c.nonfinite;
        st->late_overflow = (int32_t)c.late_overflow;
    }
    if (c.wait_abort) return fail(BL_E_TIMEOUT, "a bounded device wait ran out (the launch left early)");
    if (c.nonfinite) return fail(BL_E_NONFINITE, "%llu non-finite net forces", c.nonfinite);
    return BL_OK;
}

int bl_graph_run(bl_graph *g, int32_t iterations, int32_t start_iter, int32_t stop_batch,
                 double *energy_out, double *fx, double *fy, bl_stats *st) {
    return run_impl(g, iterations, start_iter, stop_batch, energy_out, fx, fy, st);
}

static const char *kProfNames[PK_COUNT] = {"rows_kernel", "step_kernel",        "finalize_kernel",
                                           "tree_build",  "far_kernel",         "chain_kernel",
                                           "exact_graph_kernel", "steps_kernel"};

int bl_graph_profile(bl_graph *g, int32_t enable) {
    if (!g) return fail(BL_E_INVAL, "graph is NULL");
    if (!g->prof) {
        g->prof = new Prof();
        for (int q = 0; q < 2 * kProfPool; ++q) BL_HIP(hipEventCreate(&g->prof->ev[q]));
    }
    BL_TRY(prof_collect(g));
    Prof &P = *g->prof;
    for (int q = 0; q < PK_COUNT; ++q) {
        P.ms[q] = 0.0;
        P.launches[q] = 0;
    }
    P.late_total = 0;
    P.old_total = 0;
    P.recent_total = 0;
    P.cell_tests = 0;
    P.on = enable != 0;
    return BL_OK;
}

int bl_graph_profile_read(bl_graph *g, const char *kernel, double *total_ms, int64_t *launches) {
    if (!g || !kernel || !total_ms || !launches) return fail(BL_E_INVAL, "NULL argument");
    *total_ms = 0.0;
    *launches = 0;
    if (!g->prof) return BL_OK;
    BL_TRY(prof_collect(g));
    if (!std::strcmp(kernel, "late_entries")) {
        *launches = g->prof->late_total;
        return BL_OK;
    }
    if (!std::strcmp(kernel, "old_entries")) {
        *launches = g->prof->old_total;
        return BL_OK;
    }
    if (!std::strcmp(kernel, "recent_entries")) {
        *launches = g->prof->recent_total;
        return BL_OK;
    }
    if (!std::strcmp(kernel, "cell_tests")) {
        *launches = g->prof->cell_tests;
        return BL_OK;
    }
    for (int q = 0; q < PK_COUNT; ++q)
        if (!std::strcmp(kernel, kProfNames[q])) {
            *total_ms = g->prof->ms[q];
            *launches = g->prof->launches[q];
            return BL_OK;
        }
    return fail(BL_E_INVAL, "unknown kernel name '%s'", kernel);
}

// Hu's adaptive step (Hu 2005, the scheme Sec. 4.3.5 cites): one device run
// per iteration on the resident graph, the step of the next iteration set
// from the energies of the last two.
static int run_adaptive(bl_graph *g, const bl_params *p, double *energy_out, bl_stats *st) {
    const double t = p->step_decay;
    double step = p->step0, e_prev = HUGE_VAL;
    int progress = 0;
    bl_stats acc{};
    int rc = BL_OK;
    g->keep_next = true;   // exact mode: each run leaves the next one's prologue done
    for (int k = 0; k < p->iterations; ++k) {
        g->p.step0 = step;                 // step_decay is 1 on this graph: iteration k runs at `step`
        bl_stats s1{};
        double e = 0.0;
        rc = run_impl(g, 1, k, -1, &e, nullptr, nullptr, &s1);
        if (rc != BL_OK && rc != BL_E_NONFINITE) {
            g->keep_next = false;
            return rc;
        }
        acc.iters_run += s1.iters_run;
        acc.late_overflow = std::max(acc.late_overflow, s1.late_overflow);
        acc.seconds += s1.seconds;
        acc.node_visits += s1.node_visits;
        acc.nonfinite_events += s1.nonfinite_events;
        acc.energy_last = e;
        if (energy_out) energy_out[k] = e;
        if (st) *st = acc;
        if (rc == BL_E_NONFINITE) {
            g->keep_next = false;
            return rc;
        }
        if (p->conv_tol > 0 && k >= 1 && std::fabs(e - e_prev) <= p->conv_tol * e_prev) break;
        if (e < e_prev) {
            if (++progress >= 5) {
                progress = 0;
                step /= t;
            }
        } else {
            progress = 0;
            step *= t;
        }
        e_prev = e;
    }
    g->keep_next = false;
    if (st) *st = acc;
    return BL_OK;
}

int bl_layout(const bl_csr *csr, const double *x0, const double *y0, const bl_params *p,
              void *hip_stream, double *x_out, double *y_out, double *energy_out, bl_stats *st) {
    if (!x0 || !y0 || !x_out || !y_out) return fail(BL_E_INVAL, "coordinate arrays are NULL");
    if (!p) return fail(BL_E_INVAL, "params is NULL");
    const bool adaptive = (p->flags & BL_ADAPTIVE_STEP) != 0;
    if (adaptive && p->start_iter != 0) return fail(BL_E_INVAL, "BL_ADAPTIVE_STEP needs start_iter 0");
    bl_params q = *p;
    if (adaptive) {
        q.flags &= ~(uint32_t)BL_ADAPTIVE_STEP;
        q.step_decay = 1.0;
        q.conv_tol = 0.0;
    }
    bl_graph *g = nullptr;
    BL_TRY(bl_graph_create(csr, &q, hip_stream, &g));
    const uint32_t cf = p->flags & BL_DEVICE_PTRS;
    int rc = bl_graph_set_coords(g, x0, y0, cf);
    int rc_run = BL_OK;
    if (rc == BL_OK)
        rc_run = adaptive ? run_adaptive(g, p, energy_out, st)
                          : bl_graph_run(g, p->iterations, p->start_iter, -1, energy_out, nullptr, nullptr, st);
    if (rc == BL_OK && (rc_run == BL_OK || rc_run == BL_E_NONFINITE)) rc = bl_graph_get_coords(g, x_out, y_out, cf);
    char saved[512];
    std::strncpy(saved, g_err, sizeof saved);
    bl_graph_destroy(g);
    std::strncpy(g_err, saved, sizeof g_err);
    return rc != BL_OK ? rc : rc_run;
}

int bl_forces(const bl_csr *csr, const double *x, const double *y, const double *sx, const double *sy,
              int32_t batch_index, const bl_params *p, void *hip_stream, double *fx, double *fy) {
    if (!x || !y || !fx || !fy) return fail(BL_E_INVAL, "NULL argument");
    if (!p) return fail(BL_E_INVAL, "params is NULL");
    if (!csr || csr->n < 1 || p->batch_size < 1) return fail(BL_E_INVAL, "bad graph or batch size");
    const int nb = (csr->n + p->batch_size - 1) / p->batch_size;
    if (batch_index < 0 || batch_index >= nb) return fail(BL_E_INVAL, "batch_index out of range");
    if ((sx == nullptr) != (sy == nullptr)) return fail(BL_E_INVAL, "give both sx and sy or neither");
    bl_graph *g = nullptr;
    BL_TRY(bl_graph_create(csr, p, hip_stream, &g));
    const uint32_t cf = p->flags & BL_DEVICE_PTRS;
    const size_t N = (size_t)csr->n;
    int rc = bl_graph_set_coords(g, x, y, cf);
    if (rc == BL_OK) {
        if (p->mode == BL_EXACT) {
            rc = exact_forces(g, batch_index);
        } else {
            // Barnes-Hut: tree from the snapshot, leaves and attraction from (x, y).
            const double *dsx = sx, *dsy = sy;
            if (sx && !cf) {
                for (size_t i = 0; i < N; ++i)
                    if (!std::isfinite(sx[i]) || !std::isfinite(sy[i]))
                        rc = fail(BL_E_INVAL, "snapshot coordinate %zu is not finite", i);
                hipError_t e = hipMemcpyAsync(g->stage, sx, 8 * N, hipMemcpyHostToDevice, g->stream);
                if (e == hipSuccess) e = hipMemcpyAsync(g->stage + N, sy, 8 * N, hipMemcpyHostToDevice, g->stream);
                if (e != hipSuccess) rc = fail(BL_E_HIP, "copy failed: %s", hipGetErrorString(e));
                dsx = g->stage;
                dsy = g->stage + N;
            }
            if (rc == BL_OK) rc = bh_forces(g, batch_index, dsx, dsy);
        }
    }
    if (rc == BL_OK) {
        hipError_t e = hipStreamSynchronize(g->stream);
        const int BS = p->batch_size, R = std::min(BS, csr->n - batch_index * BS);
        std::vector<double> f(2 * (size_t)R);
        if (e == hipSuccess) e = hipMemcpy(f.data(), g->fout, 16 * (size_t)R, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(BL_E_HIP, "forces failed: %s", hipGetErrorString(e));
        for (int q = 0; rc == BL_OK && q < R; ++q) {
            fx[q] = f[2 * q];
            fy[q] = f[2 * q + 1];
        }
    }
    char saved[512];
    std::strncpy(saved, g_err, sizeof saved);
    bl_graph_destroy(g);
    std::strncpy(g_err, saved, sizeof g_err);
    return rc;
}

}  // extern "C"
