// Many independent layouts in few launches.
//
//  - Exact-mode graphs up to kWGMaxN vertices: one workgroup per graph, one
//    launch per precision for the whole group (exact_graph_kernel), on a
//    side stream so that it overlaps the Barnes-Hut work.  The workgroup
//    size is picked by a small autotuner (timed on one iteration of the
//    group); the result does not depend on the pick.
//  - Barnes-Hut graphs: one job set in the multi-job engine; one iteration
//    of all jobs is captured into a hipGraph and replayed.  Jobs that need
//    fewer iterations leave the set when they are done.
//  - Larger exact-mode graphs: the multi-workgroup step kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "bl_internal.hpp"

namespace bl {
namespace {

constexpr int kWGMaxN = 8192;

struct TuneKey {
    int prec, bucket;
    bool operator<(const TuneKey &o) const { return prec < o.prec || (prec == o.prec && bucket < o.bucket); }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;   // chosen workgroup size per (precision, size class)

int size_bucket(const std::vector<bl_graph *> &gs) {
    int mx = 1;
    for (auto *g : gs) mx = std::max(mx, g->n);
    int b = 0;
    while ((1 << b) < mx) ++b;
    return b;
}

// Time one iteration of the group per candidate size, restoring coordinates
// in between, and keep the fastest.
int autotune_threads(const std::vector<bl_graph *> &gs, hipStream_t s, void *d_jobs,
                     const std::vector<std::vector<double>> &xy0, int *out) {
    const TuneKey key{gs[0]->p.precision, size_bucket(gs)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *out = it->second;
            return BL_OK;
        }
    }
    const int cand[3] = {256, 512, 1024};
    float best = 1e30f;
    int pick = 1024;
    hipEvent_t e0, e1;
    BL_HIP(hipEventCreate(&e0));
    BL_HIP(hipEventCreate(&e1));
    for (int c : cand) {
        BL_HIP(hipEventRecord(e0, s));
        BL_TRY(exact_graph_launch(gs.data(), (int)gs.size(), c, s, d_jobs, 1));
        BL_HIP(hipEventRecord(e1, s));
        BL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        BL_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // undo the trial iterations
    for (size_t q = 0; q < gs.size(); ++q) {
        const size_t N = (size_t)gs[q]->n;
        BL_HIP(hipMemcpy(gs[q]->stage, xy0[q].data(), 16 * N, hipMemcpyHostToDevice));
        BL_TRY(convert_coords_in(gs[q], gs[q]->stage, gs[q]->stage + N));
        BL_HIP(hipMemsetAsync(gs[q]->counters, 0, sizeof(Counters), gs[q]->stream));
        BL_HIP(hipStreamSynchronize(gs[q]->stream));
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = pick;
    *out = pick;
    return BL_OK;
}

struct BatchState {
    std::vector<bl_graph *> gs;
    hipStream_t s_ex = nullptr, s_bh = nullptr;
    BHEngine *eng = nullptr;
    void *d_jobs = nullptr;
    ~BatchState() {
        if (s_ex) (void)hipStreamSynchronize(s_ex);
        if (s_bh) (void)hipStreamSynchronize(s_bh);
        if (eng) bh_engine_destroy(eng);
        for (auto *g : gs) bl_graph_destroy(g);
        if (d_jobs) (void)hipFree(d_jobs);
        if (s_ex) (void)hipStreamDestroy(s_ex);
        if (s_bh) (void)hipStreamDestroy(s_bh);
    }
};

}  // namespace
}  // namespace bl

using namespace bl;

extern "C" int bl_layout_batch(int32_t G, const bl_csr *const *graphs, const double *const *x0,
                               const double *const *y0, const bl_params *const *params, void *hip_stream,
                               double *const *x_out, double *const *y_out, bl_stats *stats) {
    if (G < 0) return fail_code(BL_E_INVAL, "G must be >= 0");
    if (G == 0) return BL_OK;
    if (!graphs || !x0 || !y0 || !params || !x_out || !y_out) return fail_code(BL_E_INVAL, "NULL array argument");
    for (int q = 0; q < G; ++q) {
        if (!graphs[q] || !x0[q] || !y0[q] || !params[q] || !x_out[q] || !y_out[q])
            return fail_code(BL_E_INVAL, "NULL entry in an array argument");
        if (params[q]->flags & BL_DEVICE_PTRS)
            return fail_code(BL_E_INVAL, "bl_layout_batch takes host arrays only");
        BL_TRY(params_check(params[q]));
        if (params[q]->flags & BL_ADAPTIVE_STEP)
            return fail_code(BL_E_INVAL, "BL_ADAPTIVE_STEP is a bl_layout option");
    }
    BatchState B;
    // non-blocking: the legacy stream of other threads does not wait for them
    // (nor for the graph captured on s_bh)
    BL_HIP(hipStreamCreateWithFlags(&B.s_ex, hipStreamNonBlocking));
    BL_HIP(hipStreamCreateWithFlags(&B.s_bh, hipStreamNonBlocking));
    hipStream_t user = (hipStream_t)hip_stream;
    BL_HIP(hipStreamSynchronize(user));
    B.gs.assign(G, nullptr);
    std::vector<std::vector<double>> xy0(G);
    for (int q = 0; q < G; ++q) {
        const bool bh = params[q]->mode == BL_BH;
        BL_TRY(bl_graph_create(graphs[q], params[q], bh ? B.s_bh : B.s_ex, &B.gs[q]));
        B.gs[q]->coop = false;   // runs beside the other graphs' launches
        BL_TRY(bl_graph_set_coords(B.gs[q], x0[q], y0[q], 0));
        const size_t N = (size_t)graphs[q]->n;
        xy0[q].resize(2 * N);
        std::memcpy(xy0[q].data(), x0[q], 8 * N);
        std::memcpy(xy0[q].data() + N, y0[q], 8 * N);
    }
    const auto t0 = std::chrono::steady_clock::now();
    // groups
    std::vector<bl_graph *> wg[3], big, bhs;
    std::vector<int> wg_idx[3];
    for (int q = 0; q < G; ++q) {
        bl_graph *g = B.gs[q];
        if (g->p.mode == BL_BH) bhs.push_back(g);
        else if (g->n <= kWGMaxN && !model_general(g->p)) {   // the one-workgroup kernel runs (2, -1)
            wg[g->p.precision].push_back(g);
            wg_idx[g->p.precision].push_back(q);
        } else big.push_back(g);
    }
    // largest graphs first: their workgroups start at once and bound the
    // launch, the small ones fill in behind them
    for (int c = 0; c < 3; ++c) {
        std::vector<size_t> ord(wg[c].size());
        for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
            return (int64_t)wg[c][a]->n * wg[c][a]->nb > (int64_t)wg[c][b]->n * wg[c][b]->nb;
        });
        std::vector<bl_graph *> g2;
        std::vector<int> i2;
        for (size_t q : ord) {
            g2.push_back(wg[c][q]);
            i2.push_back(wg_idx[c][q]);
        }
        wg[c].swap(g2);
        wg_idx[c].swap(i2);
    }
    size_t maxwg = 0;
    for (int c = 0; c < 3; ++c) maxwg = std::max(maxwg, wg[c].size());
    if (maxwg) BL_HIP(hipMalloc(&B.d_jobs, exact_job_size() * maxwg));
    // exact groups, one workgroup per graph
    for (int c = 0; c < 3; ++c) {
        if (wg[c].empty()) continue;
        std::vector<std::vector<double>> sub;
        for (int q : wg_idx[c]) sub.push_back(xy0[q]);
        int threads = 1024;
        BL_TRY(autotune_threads(wg[c], B.s_ex, B.d_jobs, sub, &threads));
        BL_TRY(exact_graph_launch(wg[c].data(), (int)wg[c].size(), threads, B.s_ex, B.d_jobs, -1));
    }
    // Barnes-Hut job set
    if (!bhs.empty()) {
        BL_TRY(bh_engine_create(B.s_bh, &B.eng));
        std::vector<int> left(bhs.size());
        for (size_t q = 0; q < bhs.size(); ++q) {
            left[q] = bhs[q]->p.iterations;
            BL_TRY(bh_set_iteration(bhs[q], bhs[q]->p.start_iter));
        }
        bool setup = true;
        for (;;) {
            std::vector<BHJob *> dummy;
            std::vector<char> desc;
            int m = 0x7fffffff, cnt = 0;
            for (size_t q = 0; q < bhs.size(); ++q)
                if (left[q] > 0) {
                    m = std::min(m, left[q]);
                    ++cnt;
                }
            if (cnt == 0) break;
            desc.resize(bh_job_size() * cnt);
            int j = 0;
            for (size_t q = 0; q < bhs.size(); ++q)
                if (left[q] > 0) {
                    BHRunSpec spec;
                    spec.last_batch = bhs[q]->nb - 1;
                    BL_TRY(bh_fill_job(bhs[q], (BHJob *)(desc.data() + bh_job_size() * j), spec));
                    ++j;
                }
            BL_TRY(bh_engine_set(B.eng, (const BHJob *)desc.data(), cnt));
            if (setup) {
                BL_TRY(bh_engine_setup(B.eng));
                setup = false;
            }
            BL_TRY(bh_engine_run(B.eng, m, true));
            for (size_t q = 0; q < bhs.size(); ++q)
                if (left[q] > 0) left[q] -= m;
        }
    }
    // larger exact graphs, one after the other
    for (bl_graph *g : big) {
        BL_TRY(exact_run(g, g->p.iterations, g->p.start_iter, -1));
    }
    BL_HIP(hipStreamSynchronize(B.s_ex));
    BL_HIP(hipStreamSynchronize(B.s_bh));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = BL_OK;
    for (int q = 0; q < G; ++q) {
        bl_graph *g = B.gs[q];
        int r1 = stats_fill(g, stats ? &stats[q] : nullptr, g->p.iterations, secs);
        BL_TRY(bl_graph_get_coords(g, x_out[q], y_out[q], 0));
        if (r1 != BL_OK && rc == BL_OK) rc = r1;
    }
    if (rc != BL_OK) return fail_code(rc, "non-finite net forces in the batch");
    return BL_OK;
}
