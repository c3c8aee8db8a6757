// Continuous batching of layout jobs.
//
// A scheduler thread owns the device work.  Submitted jobs wait in a FIFO;
// at every quantum boundary the scheduler admits queued jobs first-fit while
// a slot is free and their bl_footprint_bytes fits the remaining HBM budget,
// keeps admitted jobs' graphs, coordinates and trees resident, and advances
// all resident Barnes-Hut jobs together through the multi-job engine (one
// launch per kernel serves every job, so their work overlaps on the device);
// exact-mode jobs advance by resumable runs on the same stream.  Finished
// jobs are copied out and their memory is returned to the budget.  A job's
// result equals its alone result bitwise: the kernels it runs and their
// arithmetic do not depend on the other jobs, and runs resume exactly.
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

constexpr int kQuantum = 8;   // iterations between scheduling decisions

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
    bool cancel = false;
    Clock::time_point t_submit, t_done;
    bl_stats stats{};
    int rc = BL_OK;
    std::string err;
};

}  // namespace
}  // namespace bl

struct bl_server {
    size_t budget = 0, used = 0;
    int max_slots = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;        // wakes the scheduler
    std::condition_variable done_cv;   // wakes waiters
    bool stop = false;
    int64_t next_id = 1;
    std::map<int64_t, std::shared_ptr<bl::Job>> jobs;
    std::deque<int64_t> queue;
    std::vector<std::shared_ptr<bl::Job>> resident;
    bl::BHEngine *eng = nullptr;
    bool set_dirty = true;
};

namespace bl {
namespace {

void finish(bl_server *s, const std::shared_ptr<Job> &j, int rc, const char *msg) {
    j->t_done = Clock::now();
    j->rc = rc;
    if (msg) j->err = msg;
    j->state = (rc == BL_OK || rc == BL_E_NONFINITE) ? JS_DONE : JS_FAILED;
    if (j->cancel) j->state = JS_CANCELLED;
    j->stats.seconds = std::chrono::duration<double>(j->t_done - j->t_submit).count();
}

// Admit queued jobs first-fit (caller holds the lock; device work without it
// would race with nothing else, the scheduler is the only device user).
void admit(bl_server *s) {
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if ((int)s->resident.size() >= s->max_slots) break;
        auto jit = s->jobs.find(*it);
        if (jit == s->jobs.end()) {
            it = s->queue.erase(it);
            continue;
        }
        std::shared_ptr<Job> j = jit->second;
        if (j->cancel) {
            finish(s, j, BL_OK, nullptr);
            it = s->queue.erase(it);
            continue;
        }
        if (s->used + j->footprint > s->budget) {
            ++it;
            continue;
        }
        bl_csr csr{j->n, j->nnz, j->rowptr.data(), j->colidx.data()};
        int rc = bl_graph_create(&csr, &j->p, s->stream, &j->g);
        if (rc == BL_OK) rc = bl_graph_set_coords(j->g, j->x0.data(), j->y0.data(), 0);
        if (rc == BL_OK && j->p.mode == BL_BH) rc = bh_set_iteration(j->g, j->p.start_iter);
        if (rc != BL_OK) {
            std::string m = bl_last_error();
            if (j->g) bl_graph_destroy(j->g);
            j->g = nullptr;
            finish(s, j, rc, m.c_str());
            it = s->queue.erase(it);
            s->done_cv.notify_all();
            continue;
        }
        j->state = JS_RUNNING;
        j->left = j->p.iterations;
        s->used += j->footprint;
        s->resident.push_back(j);
        s->set_dirty = true;
        it = s->queue.erase(it);
    }
}

// One quantum of device work for all resident jobs.
int advance(bl_server *s) {
    std::vector<std::shared_ptr<Job>> bh, ex;
    int q = kQuantum;
    for (auto &j : s->resident) {
        if (j->left <= 0) continue;
        q = std::min(q, j->left);
        (j->p.mode == BL_BH ? bh : ex).push_back(j);
    }
    if (!bh.empty()) {
        if (s->set_dirty) {
            std::vector<char> desc(bh_job_size() * bh.size());
            for (size_t k = 0; k < bh.size(); ++k) {
                BHRunSpec spec;
                spec.last_batch = bh[k]->g->nb - 1;
                BL_TRY(bh_fill_job(bh[k]->g, (BHJob *)(desc.data() + bh_job_size() * k), spec));
            }
            BL_TRY(bh_engine_set(s->eng, (const BHJob *)desc.data(), (int)bh.size()));
            BL_TRY(bh_engine_setup(s->eng));
            s->set_dirty = false;
        }
        BL_TRY(bh_engine_run(s->eng, q, q > 1));
    }
    for (auto &j : ex) BL_TRY(exact_run(j->g, q, j->p.start_iter + j->done_iters, -1));
    BL_HIP(hipStreamSynchronize(s->stream));
    for (auto &j : s->resident)
        if (j->left > 0) {
            j->left -= q;
            j->done_iters += q;
            j->last_q = q;
        }
    return BL_OK;
}

void retire(bl_server *s) {
    for (auto it = s->resident.begin(); it != s->resident.end();) {
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
            if (rc != BL_OK) m = bl_last_error();
        }
        bl_graph_destroy(j->g);
        j->g = nullptr;
        s->used -= j->footprint;
        finish(s, j, rc, m.empty() ? nullptr : m.c_str());
        it = s->resident.erase(it);
        s->set_dirty = true;
    }
    s->done_cv.notify_all();
}

void scheduler(bl_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        admit(s);
        if (s->resident.empty()) {
            s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
            continue;
        }
        // device work without the lock: only this thread touches the
        // resident set and the engine; submitters and pollers proceed
        lk.unlock();
        const int rc = advance(s);
        lk.lock();
        if (rc != BL_OK) {
            std::string m = bl_last_error();
            for (auto &j : s->resident) {
                if (j->g) bl_graph_destroy(j->g);
                j->g = nullptr;
                s->used -= j->footprint;
                finish(s, j, rc, m.c_str());
            }
            s->resident.clear();
            s->set_dirty = true;
            s->done_cv.notify_all();
            continue;
        }
        retire(s);
    }
    for (auto &j : s->resident) {
        if (j->g) bl_graph_destroy(j->g);
        j->g = nullptr;
        j->cancel = true;
        finish(s, j, BL_OK, nullptr);
    }
    s->resident.clear();
    s->done_cv.notify_all();
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
    if (e == hipSuccess) e = hipStreamCreate(&s->stream);
    if (e != hipSuccess) {
        delete s;
        set_error("server stream: %s", hipGetErrorString(e));
        return BL_E_HIP;
    }
    int rc = bh_engine_create(s->stream, &s->eng);
    if (rc != BL_OK) {
        (void)hipStreamDestroy(s->stream);
        delete s;
        return rc;
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
    j->cancel = true;   // queued: dropped at admission; running: at the next quantum
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
    if (s->eng) bh_engine_destroy(s->eng);
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return BL_OK;
}

}  // extern "C"
