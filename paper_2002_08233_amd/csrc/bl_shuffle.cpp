// Randomised minibatches (Sec. 4.3.3, batch randomisation), a host driver of the
// library around the ordinary single-graph path.
//
// In iteration k the minibatches are consecutive runs of BS vertices of a
// permutation pi_k of the vertex ids instead of consecutive id ranges.  The
// force kernels need no change for this: giving vertex pi_k[q] the label q
// makes the permuted batches the ordinary ones, so each iteration relabels the
// graph and the coordinates on the host, runs one iteration of the resident
// path (start_iter = k, so the step length is the run's own), and scatters the
// coordinates back.  The relabelling is the reshuffling cost the paper notes;
// it is O(n + m) host work and one CSR upload per iteration into one resident
// device graph (what the layout derives from the CSR is rebuilt each time).
//
// pi_k is drawn with Durstenfeld's form of the Fisher-Yates shuffle, for
// i = n-1 down to 1 swapping positions i and u mod (i+1), where u is the
// SplitMix64 output (Steele, Lea and Flood, OOPSLA 2014) for the counter
// c = k * 2^32 + i: the mix of the state seed + (c + 1) * 0x9E3779B97F4A7C15,
// which is the (c+1)-th output of a SplitMix64 stream seeded with `seed`.
// Every u depends only on (seed, k, i), so a run restarted at start_iter
// draws the same batches.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "bl_internal.hpp"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t splitmix_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// perm[q] = the vertex that gets label q in iteration k.
void draw_perm(uint64_t seed, int64_t k, int n, std::vector<int32_t> &perm) {
    perm.resize(n);
    for (int q = 0; q < n; ++q) perm[q] = q;
    for (int i = n - 1; i >= 1; --i) {
        const uint64_t c = ((uint64_t)k << 32) + (uint64_t)i;
        const uint64_t u = splitmix_out(seed + (c + 1) * kGamma);
        const int j = (int)(u % (uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
    }
}

// f(lo, hi) over [0, n) in contiguous parts on up to 16 host threads (one
// when the work is small).
template <typename F>
void parallel_range(int64_t n, int64_t work, F f) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = work < (1 << 18) ? 1 : (int)std::min<unsigned>(16u, hw);
    if (T == 1 || n < 2 * T) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) th.emplace_back(f, n * t / T, n * (t + 1) / T);
    for (auto &x : th) x.join();
}

}  // namespace

using namespace bl;

int bl_layout_shuffled(const bl_csr *csr, const double *x0, const double *y0, const bl_params *p, uint64_t seed,
                       void *hip_stream, double *x_out, double *y_out, double *energy_out, bl_stats *st) {
    if (!x0 || !y0 || !x_out || !y_out) return fail_code(BL_E_INVAL, "coordinate arrays are NULL");
    if (!p) return fail_code(BL_E_INVAL, "params is NULL");
    BL_TRY(params_check(p));
    if (p->flags & BL_DEVICE_PTRS) return fail_code(BL_E_INVAL, "bl_layout_shuffled takes host arrays");
    if (p->flags & BL_ADAPTIVE_STEP) return fail_code(BL_E_INVAL, "BL_ADAPTIVE_STEP is a bl_layout option");
    if (!csr) return fail_code(BL_E_INVAL, "graph is NULL");
    BL_TRY(check_csr(csr, p->flags, (hipStream_t)hip_stream));
    const int n = csr->n;
    const int32_t *rp = csr->rowptr, *ci = csr->colidx;
    // The method lays out undirected graphs, stored as symmetric CSRs
    // (BL_VALIDATE checks that in full).  Whatever the flags, a CSR whose
    // in-degrees differ from its row lengths is rejected here, as the batch
    // randomisation has always done.
    {
        std::vector<int64_t> indeg(n, 0);
        for (int64_t e = 0; e < csr->nnz; ++e) ++indeg[ci[e]];
        for (int i = 0; i < n; ++i)
            if (indeg[i] != rp[i + 1] - rp[i])
                return fail_code(BL_E_INVAL, "bl_layout_shuffled needs a symmetric CSR "
                                             "(a vertex's in-degree differs from its row length)");
    }
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x0[i]) || !std::isfinite(y0[i]))
            return fail_code(BL_E_INVAL, "a start coordinate is not finite");

    std::vector<double> x(x0, x0 + n), y(y0, y0 + n), xs(n), ys(n);
    std::vector<int32_t> perm, inv(n), rp2(n + 1), ci2;
    // the relabelled column ids, uploaded every iteration: pinned host memory
    // when it can be had (the copy then goes straight to DMA), else pageable
    const size_t ci_bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(csr->nnz, 1);
    int32_t *ci_pin = nullptr;
    if (hipHostMalloc((void **)&ci_pin, ci_bytes, hipHostMallocDefault) != hipSuccess) {
        ci_pin = nullptr;
        (void)hipGetLastError();
        ci2.resize((size_t)std::max<int64_t>(csr->nnz, 1));
    }
    int32_t *const ci_out = ci_pin ? ci_pin : ci2.data();
    bl_params q = *p;
    q.iterations = 1;
    q.conv_tol = 0.0;
    bl_stats acc{};
    std::vector<double> es;
    int rc = BL_OK;
    bl_graph *g = nullptr;   // the relabelled graph, resident across iterations
    auto done = [&](int code) {
        if (g) {
            char saved[512];
            std::strncpy(saved, bl_last_error(), sizeof saved - 1);
            saved[sizeof saved - 1] = 0;
            bl_graph_destroy(g);
            if (code != BL_OK) set_error("%s", saved);
        }
        if (ci_pin) (void)hipHostFree(ci_pin);   // every copy from it has completed
        return code;
    };
    for (int t = 0; t < p->iterations; ++t) {
        const int k = p->start_iter + t;
        draw_perm(seed, k, n, perm);
        for (int l = 0; l < n; ++l) inv[perm[l]] = l;
        // Row l of the relabelled graph is old row perm[l] with every
        // neighbour u renamed inv[u], in increasing new label: each row is
        // gathered and sorted on its own, rows in parallel.
        rp2[0] = 0;
        for (int l = 0; l < n; ++l) rp2[l + 1] = rp2[l] + (rp[perm[l] + 1] - rp[perm[l]]);
        parallel_range(n, csr->nnz, [&](int64_t l0, int64_t l1) {
            for (int64_t l = l0; l < l1; ++l) {
                const int v = perm[l];
                int32_t *row = ci_out + rp2[l];
                for (int e = rp[v]; e < rp[v + 1]; ++e) row[e - rp[v]] = inv[ci[e]];
                std::sort(row, row + (rp[v + 1] - rp[v]));
                xs[l] = x[v];
                ys[l] = y[v];
            }
        });
        q.start_iter = k;
        q.flags = p->flags & ~(uint32_t)BL_VALIDATE;   // the relabelled graph is valid if the input is
        if (!g) {
            const bl_csr g2{n, csr->nnz, rp2.data(), ci_out};
            rc = bl_graph_create(&g2, &q, hip_stream, &g);
            if (rc != BL_OK) return done(rc);
        } else {
            rc = graph_reload_csr(g, rp2.data(), ci_out);
            if (rc != BL_OK) return done(rc);
        }
        bl_stats s1{};
        rc = bl_graph_set_coords(g, xs.data(), ys.data(), 0);
        if (rc != BL_OK) return done(rc);
        rc = bl_graph_run(g, 1, k, -1, nullptr, nullptr, nullptr, &s1);
        if (rc != BL_OK && rc != BL_E_NONFINITE) return done(rc);
        const int rc_get = bl_graph_get_coords(g, xs.data(), ys.data(), 0);
        if (rc_get != BL_OK) return done(rc_get);
        parallel_range(n, csr->nnz, [&](int64_t l0, int64_t l1) {
            for (int64_t l = l0; l < l1; ++l) {
                x[perm[l]] = xs[l];
                y[perm[l]] = ys[l];
            }
        });
        acc.iters_run += s1.iters_run;
        acc.late_overflow = std::max(acc.late_overflow, s1.late_overflow);
        acc.seconds += s1.seconds;
        acc.node_visits += s1.node_visits;
        acc.nonfinite_events += s1.nonfinite_events;
        acc.energy_last = s1.energy_last;
        es.push_back(s1.energy_last);
        if (energy_out) energy_out[t] = s1.energy_last;
        if (rc == BL_E_NONFINITE) break;
        const size_t ne = es.size();
        if (p->conv_tol > 0 && ne >= 2 && std::fabs(es[ne - 1] - es[ne - 2]) <= p->conv_tol * es[ne - 2]) break;
    }
    std::memcpy(x_out, x.data(), 8 * (size_t)n);
    std::memcpy(y_out, y.data(), 8 * (size_t)n);
    if (st) *st = acc;
    return done(rc);
}
