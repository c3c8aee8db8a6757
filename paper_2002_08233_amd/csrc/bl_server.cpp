// Continuous batching of layout jobs.
//
// A scheduler thread owns the device work.  Submitted jobs wait in a FIFO;
// the scheduler admits queued jobs first-fit while a slot is free and their
// bl_footprint_bytes fits the remaining HBM budget, and keeps admitted jobs'
// graphs, coordinates and trees resident until they finish.  Resident jobs
// are grouped into lanes by the length of their minibatch chain (batches per
// iteration), each lane with its own stream: a lane advances all its jobs a
// few iterations at a time (Barnes-Hut jobs of a lane share every kernel
// launch of one replayed iteration graph; exact jobs run resumable quanta),
// and lanes run concurrently, so short jobs are not paced by long ones and
// the device overlaps their work.  A lane's jobs are retired and new jobs
// joined between its quanta.  Graph memory is stream-ordered, so admission
// and retirement never wait for other lanes.  A job's result equals its
// alone result bitwise: the kernels it runs and their arithmetic do not
// depend on the other jobs, and runs resume exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bl_internal.hpp"

namespace bl {
namespace {

using Clock = std::chrono::steady_clock;

enum JobState { JS_QUEUED = 0, JS_RUNNING, JS_DONE, JS_FAILED, JS_CANCELLED };

constexpr int kQuantum = 8;   // iterations a lane runs between scheduling decisions
constexpr int kLanes = 4;     // lanes by batches per iteration: <= 16, <= 128, <= 1024, more

int lane_of(int nb) {
    if (nb <= 16) return 0;
    if (nb <= 128) return 1;
    if (nb <= 1024) return 2;
    return 3;
}

struct Job {
    int64_t id = 0;
    JobState state = JS_QUEUED;
    bl_params p{};
    int n = 0;
    int64_t nnz = 0;
    std::vector<int32_t> rowptr, colidx;
    std::vector<double> x0, y0, x, y;
    size_t footprint = 0;
    bl_graph *g = nullptr;
    int left = 0, done_iters = 0;
    int last_q = 0;   // iterations of the job's last quantum
    bool in_flight = false;   // part of its lane's quantum in flight
    bool cancel = false;
    Clock::time_point t_submit, t_done;
    bl_stats stats{};
    int rc = BL_OK;
    std::string err;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    BHEngine *eng = nullptr;
    bool busy = false;       // a quantum is in flight
    int q = 0;               // its iterations
    bool set_dirty = true;   // the Barnes-Hut job set changed
    std::vector<std::shared_ptr<Job>> jobs;
};

}  // namespace
}  // namespace bl

struct bl_server {
    size_t budget = 0, used = 0;
    int max_slots = 0, nresident = 0;
    int device = 0;
    hipStream_t setup = nullptr;     // admission uploads
    bl::Lane lanes[bl::kLanes];
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;        // wakes the scheduler
    std::condition_variable done_cv;   // wakes waiters
    bool stop = false;
    int64_t next_id = 1;
    std::map<int64_t, std::shared_ptr<bl::Job>> jobs;
    std::deque<int64_t> queue;
};

namespace bl {
namespace {

void finish(const std::shared_ptr<Job> &j, int rc, const char *msg) {
    j->t_done = Clock::now();
    j->rc = rc;
    if (msg) j->err = msg;
    j->state = (rc == BL_OK || rc == BL_E_NONFINITE) ? JS_DONE : JS_FAILED;
    if (j->cancel) j->state = JS_CANCELLED;
    j->stats.seconds = std::chrono::duration<double>(j->t_done - j->t_submit).count();
}

// Admit queued jobs first-fit (caller holds the lock).  Graphs are built on
// the setup stream with stream-ordered memory, then handed to their lane.
void admit(bl_server *s) {
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (s->nresident >= s->max_slots) break;
        auto jit = s->jobs.find(*it);
        if (jit == s->jobs.end()) {
            it = s->queue.erase(it);
            continue;
        }
        std::shared_ptr<Job> j = jit->second;
        if (j->cancel) {
            finish(j, BL_OK, nullptr);
            it = s->queue.erase(it);
            s->done_cv.notify_all();
            continue;
        }
        if (s->used + j->footprint > s->budget) {
            ++it;
            continue;
        }
        bl_csr csr{j->n, j->nnz, j->rowptr.data(), j->colidx.data()};
        int rc = graph_create_ex(&csr, &j->p, s->setup, true, &j->g);
        if (rc == BL_OK) j->g->coop = false;   // shares the device with the other lanes
        if (rc == BL_OK) rc = bl_graph_set_coords(j->g, j->x0.data(), j->y0.data(), 0);
        if (rc == BL_OK && j->p.mode == BL_BH) rc = bh_set_iteration(j->g, j->p.start_iter);
        if (rc == BL_OK && hipStreamSynchronize(s->setup) != hipSuccess)
            rc = fail_code(BL_E_HIP, "admission upload failed");
        if (rc != BL_OK) {
            std::string m = bl_last_error();
            if (j->g) bl_graph_destroy(j->g);
            j->g = nullptr;
            finish(j, rc, m.c_str());
            it = s->queue.erase(it);
            s->done_cv.notify_all();
            continue;
        }
        Lane &L = s->lanes[lane_of(j->g->nb)];
        j->g->stream = L.stream;
        j->state = JS_RUNNING;
        j->left = j->p.iterations;
        s->used += j->footprint;
        ++s->nresident;
        L.jobs.push_back(j);
        if (j->p.mode == BL_BH) L.set_dirty = true;
        it = s->queue.erase(it);
    }
}

// Enqueue one quantum of a lane's jobs (no waiting on the device).
int launch(Lane &L) {
    std::vector<std::shared_ptr<Job>> bh, ex;
    int q = kQuantum;
    for (auto &j : L.jobs) {
        if (j->left <= 0 || j->cancel) continue;
        q = std::min(q, j->left);
        (j->p.mode == BL_BH ? bh : ex).push_back(j);
    }
    if (bh.empty() && ex.empty()) return BL_OK;
    for (auto &j : bh) j->in_flight = true;
    for (auto &j : ex) j->in_flight = true;
    if (!bh.empty()) {
        if (L.set_dirty) {
            std::vector<char> desc(bh_job_size() * bh.size());
            for (size_t k = 0; k < bh.size(); ++k) {
                BHRunSpec spec;
                spec.last_batch = bh[k]->g->nb - 1;
                BL_TRY(bh_fill_job(bh[k]->g, (BHJob *)(desc.data() + bh_job_size() * k), spec));
            }
            BL_TRY(bh_engine_set(L.eng, (const BHJob *)desc.data(), (int)bh.size()));
            BL_TRY(bh_engine_setup(L.eng));
            L.set_dirty = false;
        }
        // (launched directly, not replayed from a captured graph: a capture in
        // progress on this thread would make legacy-stream calls of other
        // threads of the process fail)
        BL_TRY(bh_engine_run(L.eng, q, false));
    }
    for (auto &j : ex) BL_TRY(exact_run(j->g, q, j->p.start_iter + j->done_iters, -1));
    BL_HIP(hipEventRecord(L.done, L.stream));
    L.busy = true;
    L.q = q;
    return BL_OK;
}

// After a lane's quantum: progress, then retire finished or cancelled jobs
// (caller holds the lock).
void complete(bl_server *s, Lane &L) {
    L.busy = false;
    // only the jobs that took part in the quantum advance (jobs that joined
    // the lane while it ran start with the next one)
    for (auto &j : L.jobs)
        if (j->in_flight) {
            j->in_flight = false;
            j->left -= L.q;
            j->done_iters += L.q;
            j->last_q = L.q;
        }
    for (auto it = L.jobs.begin(); it != L.jobs.end();) {
        std::shared_ptr<Job> j = *it;
        if (j->left > 0 && !j->cancel) {
            ++it;
            continue;
        }
        int rc = BL_OK;
        std::string m;
        if (!j->cancel) {
            j->x.resize(j->n);
            j->y.resize(j->n);
            rc = bl_graph_get_coords(j->g, j->x.data(), j->y.data(), 0);
            // Barnes-Hut runs index energies from the job's first iteration,
            // resumed exact runs from the quantum's first iteration
            if (rc == BL_OK)
                rc = stats_fill(j->g, &j->stats, j->p.mode == BL_BH ? j->done_iters : j->last_q, 0.0);
            j->stats.iters_run = j->done_iters;
            if (rc != BL_OK && rc != BL_E_NONFINITE) m = bl_last_error();
        }
        if (j->p.mode == BL_BH) L.set_dirty = true;
        bl_graph_destroy(j->g);
        j->g = nullptr;
        s->used -= j->footprint;
        --s->nresident;
        finish(j, rc, m.empty() ? nullptr : m.c_str());
        it = L.jobs.erase(it);
    }
    s->done_cv.notify_all();
}

void fail_lane(bl_server *s, Lane &L, int rc) {
    std::string m = bl_last_error();
    (void)hipStreamSynchronize(L.stream);
    L.busy = false;
    for (auto &j : L.jobs) {
        if (j->g) bl_graph_destroy(j->g);
        j->g = nullptr;
        s->used -= j->footprint;
        --s->nresident;
        finish(j, rc, m.c_str());
    }
    L.jobs.clear();
    L.set_dirty = true;
    s->done_cv.notify_all();
}

void scheduler(bl_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        admit(s);
        bool any_busy = false;
        for (auto &L : s->lanes) {
            if (L.busy) {
                const hipError_t q = hipEventQuery(L.done);
                if (q == hipErrorNotReady) {
                    any_busy = true;
                    continue;
                }
                if (q != hipSuccess) {
                    set_error("lane quantum failed: %s", hipGetErrorString(q));
                    fail_lane(s, L, BL_E_HIP);
                    continue;
                }
                complete(s, L);
            }
            if (!L.jobs.empty()) {
                const int rc = launch(L);
                if (rc != BL_OK) {
                    fail_lane(s, L, rc);
                    continue;
                }
                any_busy |= L.busy;
            }
        }
        if (!any_busy) {
            s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
            continue;
        }
        // poll the lanes' events; new submissions wake us at once
        s->cv.wait_for(lk, std::chrono::microseconds(100));
    }
    for (auto &L : s->lanes) {
        (void)hipStreamSynchronize(L.stream);
        L.busy = false;
        for (auto &j : L.jobs) {
            if (j->g) bl_graph_destroy(j->g);
            j->g = nullptr;
            s->used -= j->footprint;
            --s->nresident;
            j->cancel = true;
            finish(j, BL_OK, nullptr);
        }
        L.jobs.clear();
    }
    s->done_cv.notify_all();
}

void server_free(bl_server *s) {
    for (auto &L : s->lanes) {
        if (L.eng) bh_engine_destroy(L.eng);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) {
            (void)hipStreamSynchronize(L.stream);
            (void)hipStreamDestroy(L.stream);
        }
    }
    if (s->setup) (void)hipStreamDestroy(s->setup);
    delete s;
}

}  // namespace
}  // namespace bl

using namespace bl;

extern "C" {

int bl_server_create(size_t hbm_budget_bytes, int32_t max_slots, void *hip_stream, bl_server **out) {
    (void)hip_stream;
    if (!out) return fail_code(BL_E_INVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return fail_code(BL_E_INVAL, "hbm_budget_bytes must be > 0");
    if (max_slots < 1 || max_slots > 4096) return fail_code(BL_E_INVAL, "max_slots must be in [1, 4096]");
    bl_server *s = new bl_server();
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking);
    for (auto &L : s->lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        server_free(s);
        set_error("server streams: %s", hipGetErrorString(e));
        return BL_E_HIP;
    }
    for (auto &L : s->lanes) {
        const int rc = bh_engine_create(L.stream, &L.eng);
        if (rc != BL_OK) {
            server_free(s);
            return rc;
        }
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return BL_OK;
}

int bl_server_submit(bl_server *s, const bl_csr *g, const double *x0, const double *y0, const bl_params *p,
                     int64_t *job) {
    if (!s || !g || !x0 || !y0 || !p || !job) return fail_code(BL_E_INVAL, "NULL argument");
    BL_TRY(params_check(p));
    if (p->flags & BL_DEVICE_PTRS) return fail_code(BL_E_INVAL, "bl_server_submit takes host arrays only");
    if (p->conv_tol > 0) return fail_code(BL_E_INVAL, "the server runs a fixed number of iterations (conv_tol must be 0)");
    if (p->flags & BL_ADAPTIVE_STEP) return fail_code(BL_E_INVAL, "BL_ADAPTIVE_STEP is a bl_layout option");
    if (g->n < 1 || g->nnz < 0 || !g->rowptr || (g->nnz > 0 && !g->colidx))
        return fail_code(BL_E_INVAL, "bad graph");
    const size_t fp = bl_footprint_bytes(g->n, g->nnz, p);
    if (fp == 0) return fail_code(BL_E_INVAL, "bad graph or parameters");
    if (fp > s->budget) return fail_code(BL_E_REJECTED, "job needs more device memory than the whole budget");
    auto j = std::make_shared<Job>();
    j->p = *p;
    j->n = g->n;
    j->nnz = g->nnz;
    j->rowptr.assign(g->rowptr, g->rowptr + g->n + 1);
    if (g->nnz) j->colidx.assign(g->colidx, g->colidx + g->nnz);
    j->x0.assign(x0, x0 + g->n);
    j->y0.assign(y0, y0 + g->n);
    j->footprint = fp;
    j->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    j->id = s->next_id++;
    s->jobs[j->id] = j;
    s->queue.push_back(j->id);
    *job = j->id;
    s->cv.notify_all();
    return BL_OK;
}

int bl_server_poll(bl_server *s, int64_t job, int32_t *done) {
    if (!s || !done) return fail_code(BL_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail_code(BL_E_INVAL, "unknown job");
    *done = it->second->state >= JS_DONE;
    return BL_OK;
}

int bl_server_wait(bl_server *s, int64_t job, double timeout_s) {
    if (!s) return fail_code(BL_E_INVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail_code(BL_E_INVAL, "unknown job");
    std::shared_ptr<Job> j = it->second;
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double>(std::max(timeout_s, 0.0)));
    if (!s->done_cv.wait_until(lk, until, [&] { return j->state >= JS_DONE; }))
        return fail_code(BL_E_TIMEOUT, "job still running");
    return BL_OK;
}

int bl_server_fetch(bl_server *s, int64_t job, double *x, double *y, bl_stats *st) {
    if (!s || !x || !y) return fail_code(BL_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail_code(BL_E_INVAL, "unknown job");
    std::shared_ptr<Job> j = it->second;
    if (j->state < JS_DONE) return fail_code(BL_E_NOTREADY, "job still running");
    if (j->state == JS_CANCELLED) return fail_code(BL_E_INVAL, "job was cancelled");
    if (j->state == JS_FAILED) return fail_code(j->rc, j->err.c_str());
    std::memcpy(x, j->x.data(), 8 * (size_t)j->n);
    std::memcpy(y, j->y.data(), 8 * (size_t)j->n);
    if (st) *st = j->stats;
    return j->rc;
}

int bl_server_release(bl_server *s, int64_t job) {
    if (!s) return fail_code(BL_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail_code(BL_E_INVAL, "unknown job");
    std::shared_ptr<Job> j = it->second;
    if (j->state >= JS_DONE) {
        s->jobs.erase(it);
        return BL_OK;
    }
    j->cancel = true;   // queued: dropped at admission; running: after its lane's quantum
    s->cv.notify_all();
    return BL_OK;
}

int bl_server_destroy(bl_server *s) {
    if (!s) return BL_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    server_free(s);
    return BL_OK;
}

}  // extern "C"
