// Exact-mode force step (Alg. 2 semantics) for gfx950.
//
// Dataflow.  At step (k, b) the rows of batch b need the *new* coordinates of
// batches b' < b and the *old* ones (from iteration k-1) of batches b' >= b.
// Both are known as soon as the batch that owns them has moved, so after the
// update of batch b every row can consume the new coordinates of batch b at
// once: rows of later batches add them to their iteration-k sum, rows of
// batches <= b to their iteration-(k+1) sum (they will see batch b as "old").
// One "panel" launch per step therefore covers all n rows x BS columns with
// full-chip parallelism, and a row's sum is complete exactly when its batch
// comes up.  Per-row sums are built column batch by column batch in a fixed
// order (each batch: an FP32 partial, then one compensated add), so the
// result does not depend on the launch shape and a resumed run reproduces a
// continuous one bitwise.
//
// Kernels: rows_kernel (per-row sums over whole column batches: the prologue
// of a run and the one-shot force call), panel_kernel (the per-step panel),
// finalize_kernel (attraction over CSR edges with live coordinates, one wave
// per row, then the batch update by the last workgroup to finish).
#include <vector>

#include "bl_device.hpp"
#include "bl_internal.hpp"

// Only explicit fma() calls fuse: the same row arithmetic is compiled into
// several kernels (multi-workgroup steps and the one-workgroup-per-graph
// batch kernel), and must round identically in all of them.
#pragma clang fp contract(off)

namespace bl {
namespace {

template <typename T>
struct V2;
template <>
struct V2<float> {
    using type = float2;
};
template <>
struct V2<double> {
    using type = double2;
};

constexpr int kPanelThreads = 256;
constexpr int kTile = 1024;        // columns staged in LDS per pass
constexpr int kFinThreads = 256;   // 4 waves, one row per wave

// Repulsion kernel term without its constant factor -R K^2:
//   (c_j - c_i) / |c_j - c_i|^2  (Sec. 2.2 with r = -1).
// A tiny bias in d^2 makes the self pair and coincident pairs contribute an
// exact 0 (0 * huge) instead of NaN; it is below half an ulp of any d^2 of
// two distinct representable points at the coordinate scales used here.
__device__ __forceinline__ void rep_term(float xi, float yi, float2 pj, float &px, float &py) {
    float dx = pj.x - xi, dy = pj.y - yi;
    float d2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
    float inv = __builtin_amdgcn_rcpf(d2);
    px = fmaf(dx, inv, px);
    py = fmaf(dy, inv, py);
}
__device__ __forceinline__ void rep_term(double xi, double yi, double2 pj, double &px, double &py) {
    double dx = pj.x - xi, dy = pj.y - yi;
    double d2 = fma(dx, dx, fma(dy, dy, 1e-300));
    double inv = 1.0 / d2;
    px = fma(dx, inv, px);
    py = fma(dy, inv, py);
}

template <typename T>
__device__ __forceinline__ void tile_sum(T xi, T yi, const typename V2<T>::type *cols, int cnt,
                                         T &px, T &py) {
    int q = 0;
    for (; q + 4 <= cnt; q += 4) {
        rep_term(xi, yi, cols[q], px, py);
        rep_term(xi, yi, cols[q + 1], px, py);
        rep_term(xi, yi, cols[q + 2], px, py);
        rep_term(xi, yi, cols[q + 3], px, py);
    }
    for (; q < cnt; ++q) rep_term(xi, yi, cols[q], px, py);
}

// Add one column-batch partial into a row sum.
template <typename T, bool KAHAN>
__device__ __forceinline__ void acc_add(typename V2<T>::type &s, float2 &c, T px, T py) {
    if constexpr (KAHAN) {
        kahan_add(s.x, c.x, px);
        kahan_add(s.y, c.y, py);
    } else {
        s.x += px;
        s.y += py;
    }
}

// Sum of one column batch [c0, c1) for every active row of the block, staged
// through LDS in kTile chunks.  All threads of the block must call it.
template <typename T>
__device__ __forceinline__ void batch_partial(const T *__restrict__ x, const T *__restrict__ y,
                                              int c0, int c1, bool active, T xi, T yi,
                                              typename V2<T>::type *cols, T &px, T &py) {
    px = 0;
    py = 0;
    for (int t0 = c0; t0 < c1; t0 += kTile) {
        const int cnt = min(kTile, c1 - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += blockDim.x)
            cols[q] = typename V2<T>::type{x[t0 + q], y[t0 + q]};
        __syncthreads();
        if (active) tile_sum<T>(xi, yi, cols, cnt, px, py);
    }
}

// Row sums over whole column batches for the rows [first, first + blockDim)
// that are < row1.  from_own_batch = 1: batches [batch(i), nb) (the run
// prologue: everything a row sees as "old" in its first iteration); 0: all
// batches (one-shot forces).  Overwrites the sums.
template <typename T, bool KAHAN>
__device__ __forceinline__ void rows_block(int n, int BS, int nb, int first, int row1, int from_own_batch,
                                           const T *__restrict__ x, const T *__restrict__ y,
                                           typename V2<T>::type *__restrict__ accS,
                                           float2 *__restrict__ accC, typename V2<T>::type *cols) {
    using T2 = typename V2<T>::type;
    const int i = first + threadIdx.x;
    const bool active = i < row1;
    const int bi = active ? i / BS : nb;
    T xi = 0, yi = 0;
    if (active) {
        xi = x[i];
        yi = y[i];
    }
    T2 s{0, 0};
    float2 c{0.f, 0.f};
    const int bstart = from_own_batch ? first / BS : 0;
    for (int bb = bstart; bb < nb; ++bb) {
        const bool use = active && (!from_own_batch || bb >= bi);
        T px, py;
        batch_partial<T>(x, y, bb * BS, min(bb * BS + BS, n), use, xi, yi, cols, px, py);
        if (use) acc_add<T, KAHAN>(s, c, px, py);
    }
    if (active) {
        accS[i] = s;
        if constexpr (KAHAN) accC[i] = c;
    }
}

template <typename T, bool KAHAN>
__global__ __launch_bounds__(kPanelThreads) void rows_kernel(
    int n, int BS, int nb, int row0, int row1, int from_own_batch, const T *__restrict__ x,
    const T *__restrict__ y, typename V2<T>::type *__restrict__ accS, float2 *__restrict__ accC) {
    __shared__ typename V2<T>::type cols[kTile];
    rows_block<T, KAHAN>(n, BS, nb, row0 + blockIdx.x * kPanelThreads, row1, from_own_batch, x, y, accS, accC,
                         cols);
}

// The panel of step (k, b) for rows [first, first + blockDim): columns =
// batch b (just moved); rows of later batches add to their iteration-k sums,
// rows of batches <= b (when do_next) to their iteration-(k+1) sums.
template <typename T, bool KAHAN>
__device__ __forceinline__ void panel_block(int n, int BS, int b, int do_next, int first, const T *__restrict__ x,
                                            const T *__restrict__ y, typename V2<T>::type *__restrict__ accS_cur,
                                            float2 *__restrict__ accC_cur,
                                            typename V2<T>::type *__restrict__ accS_nxt,
                                            float2 *__restrict__ accC_nxt, typename V2<T>::type *cols) {
    using T2 = typename V2<T>::type;
    const int i = first + threadIdx.x;
    const int bi = i < n ? i / BS : -1;
    const bool cur = i < n && bi > b;
    const bool nxt = do_next && i < n && bi >= 0 && bi <= b;
    T xi = 0, yi = 0;
    if (i < n) {
        xi = x[i];
        yi = y[i];
    }
    T px, py;
    batch_partial<T>(x, y, b * BS, min(b * BS + BS, n), cur || nxt, xi, yi, cols, px, py);
    if (cur || nxt) {
        T2 *S = cur ? accS_cur : accS_nxt;
        float2 *Cc = cur ? accC_cur : accC_nxt;
        T2 s = S[i];
        float2 c{0.f, 0.f};
        if constexpr (KAHAN) c = Cc[i];
        acc_add<T, KAHAN>(s, c, px, py);
        S[i] = s;
        if constexpr (KAHAN) Cc[i] = c;
    }
}

template <typename T, bool KAHAN>
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(
    int n, int BS, int b, int do_next, const T *__restrict__ x, const T *__restrict__ y,
    typename V2<T>::type *__restrict__ accS_cur, float2 *__restrict__ accC_cur,
    typename V2<T>::type *__restrict__ accS_nxt, float2 *__restrict__ accC_nxt) {
    __shared__ typename V2<T>::type cols[kTile];
    const int first = blockIdx.x * kPanelThreads;
    const int i = first + threadIdx.x;
    const int bi = i < n ? i / BS : -1;
    const bool work = i < n && (bi > b || (do_next && bi <= b));
    if (!__syncthreads_or(work)) return;
    panel_block<T, KAHAN>(n, BS, b, do_next, first, x, y, accS_cur, accC_cur, accS_nxt, accC_nxt, cols);
}

template <typename T>
struct FinArgs {
    int n, BS, b;
    const int *rowptr, *colidx;
    T *x, *y;
    typename V2<T>::type *accS;
    float2 *accC;
    typename V2<T>::type *fbuf;    // [BS] net forces of the batch
    unsigned *ticket;              // last-block counter, left at 0
    double *energy_k;              // energy of iteration k (NULL: do not record)
    double *fout;                  // [2*BS] FP64 forces out (NULL: none)
    unsigned long long *nonfinite;
    T step, invK, negRK2;
    int literal;                   // subtract neighbour repulsion (Alg. 1/2 exclusion)
    int update;                    // move the batch
};

// Net force of row r of batch b by one wave: attraction over the CSR row with
// live coordinates (Sec. 2.2, a = 2: d * delta / K), plus the completed
// repulsion sum scaled by -R K^2 (literal mode: minus the neighbours'
// repulsion).  Lane 0 writes fbuf[r] and clears the row's sums.
template <typename T, bool KAHAN>
__device__ __forceinline__ void row_force_wave(const FinArgs<T> &a, int r) {
    using T2 = typename V2<T>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int i = a.b * a.BS + r;
    const T xi = a.x[i], yi = a.y[i];
    T ax = 0, ay = 0, lx = 0, ly = 0;
    const int e1 = a.rowptr[i + 1];
    for (int e = a.rowptr[i] + lane; e < e1; e += kWave) {
        const int j = a.colidx[e];
        const T dx = a.x[j] - xi, dy = a.y[j] - yi;
        const T d2 = dx * dx + dy * dy;
        const T d = sqrt(d2);
        ax += d * dx;
        ay += d * dy;
        if (a.literal) rep_term(xi, yi, T2{a.x[j], a.y[j]}, lx, ly);
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    lx = wave_sum(lx);
    ly = wave_sum(ly);
    if (lane == 0) {
        T2 s = a.accS[i];
        T rx = s.x, ry = s.y;
        if constexpr (KAHAN) {
            float2 c = a.accC[i];
            rx = s.x - c.x;
            ry = s.y - c.y;
            a.accC[i] = float2{0.f, 0.f};
        }
        a.accS[i] = T2{0, 0};
        if (a.literal) {
            rx -= lx;
            ry -= ly;
        }
        a.fbuf[r] = T2{ax * a.invK + a.negRK2 * rx, ay * a.invK + a.negRK2 * ry};
    }
}

// Move batch b (c_i += Step f_i/|f_i|, skipped for |f_i| = 0) and add
// sum |f_i|^2 to the iteration energy in a fixed order.  Called by the first
// kFinThreads threads of a workgroup (all of them must call it; the first
// kFinThreads / kWave waves do the work).
template <typename T>
__device__ __forceinline__ void move_batch(const FinArgs<T> &a, double *s_ws) {
    using T2 = typename V2<T>::type;
    const int i0 = a.b * a.BS;
    const int R = min(a.BS, a.n - i0);
    const bool worker = threadIdx.x < kFinThreads;
    double e = 0.0;
    unsigned long long bad = 0;
    for (int q = threadIdx.x; worker && q < R; q += kFinThreads) {
        const T2 f = a.fbuf[q];
        const double f2 = (double)f.x * (double)f.x + (double)f.y * (double)f.y;
        if (a.fout) {
            a.fout[2 * q] = (double)f.x;
            a.fout[2 * q + 1] = (double)f.y;
        }
        if (!isfinite(f2)) {
            ++bad;
            continue;
        }
        e += f2;
        if (a.update && f2 > 0.0) {
            const int i = i0 + q;
            const T nrm = sqrt(f.x * f.x + f.y * f.y);
            const T sc = a.step / nrm;
            a.x[i] = a.x[i] + sc * f.x;
            a.y[i] = a.y[i] + sc * f.y;
        }
    }
    if (bad) atomicAdd(a.nonfinite, bad);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    e = wave_sum(e);
    if (lane == 0 && worker) s_ws[w] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kFinThreads / kWave; ++q) t += s_ws[q];
        if (a.energy_k) *a.energy_k = (a.b == 0 ? 0.0 : *a.energy_k) + t;
    }
    __syncthreads();
}

// One wave per row of batch b, then the last workgroup to finish moves the
// batch.
template <typename T, bool KAHAN>
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(FinArgs<T> a) {
    __shared__ int s_last;
    __shared__ double s_ws[kFinThreads / kWave];
    const int r = (blockIdx.x * kFinThreads + threadIdx.x) / kWave;
    const int R = min(a.BS, a.n - a.b * a.BS);
    if (r < R) row_force_wave<T, KAHAN>(a, r);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(a.ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    move_batch<T>(a, s_ws);
    if (threadIdx.x == 0) *a.ticket = 0u;
}

// ------------------------------------------------- one workgroup per graph
// Many small graphs in one launch: each workgroup runs the whole layout of
// one graph (prologue, then per step the net forces and move of the batch and
// the panel of its new coordinates), with the same row arithmetic as the
// multi-workgroup kernels, so a graph's result does not depend on the launch.
struct ExactJob {
    int n, BS, nb, iters, start, literal;
    double step0, decay, invK, negRK2;
    const int *rowptr, *colidx;
    void *x, *y;
    void *accS[2];
    float2 *accC[2];
    void *fbuf;
    double *energy;
    unsigned long long *nonfinite;
};

template <typename T, bool KAHAN, int NT>
__global__ __launch_bounds__(NT) void exact_graph_kernel(const ExactJob *__restrict__ jobs) {
    using T2 = typename V2<T>::type;
    __shared__ T2 cols[kTile];
    __shared__ double s_ws[kFinThreads / kWave];
    const ExactJob J = jobs[blockIdx.x];
    const int n = J.n, BS = J.BS, nb = J.nb;
    T *x = (T *)J.x, *y = (T *)J.y;
    // prologue and the other parity's sums cleared
    const int p0 = J.start & 1;
    for (int first = 0; first < n; first += NT)
        rows_block<T, KAHAN>(n, BS, nb, first, n, 1, x, y, (T2 *)J.accS[p0], J.accC[p0], cols);
    for (int i = threadIdx.x; i < n; i += NT) {
        ((T2 *)J.accS[p0 ^ 1])[i] = T2{0, 0};
        if constexpr (KAHAN) J.accC[p0 ^ 1][i] = float2{0.f, 0.f};
    }
    __syncthreads();
    double step = J.step0;
    for (int t = 0; t < J.start; ++t) step *= J.decay;
    const int lane_w = threadIdx.x / kWave;
    for (int t = 0; t < J.iters; ++t) {
        const int k = J.start + t;
        const int cur = k & 1, nxt = cur ^ 1;
        const bool last = (t == J.iters - 1);
        FinArgs<T> a;
        a.n = n;
        a.BS = BS;
        a.rowptr = J.rowptr;
        a.colidx = J.colidx;
        a.x = x;
        a.y = y;
        a.accS = (T2 *)J.accS[cur];
        a.accC = J.accC[cur];
        a.fbuf = (T2 *)J.fbuf;
        a.ticket = nullptr;
        a.energy_k = J.energy + t;
        a.fout = nullptr;
        a.nonfinite = J.nonfinite;
        a.step = (T)step;
        a.invK = (T)J.invK;
        a.negRK2 = (T)J.negRK2;
        a.literal = J.literal;
        a.update = 1;
        for (int b = 0; b < nb; ++b) {
            a.b = b;
            const int R = min(BS, n - b * BS);
            for (int r = lane_w; r < R; r += NT / kWave) row_force_wave<T, KAHAN>(a, r);
            __syncthreads();
            move_batch<T>(a, s_ws);
            if ((b + 1) < nb || !last) {
                for (int first = 0; first < n; first += NT) {
                    panel_block<T, KAHAN>(n, BS, b, last ? 0 : 1, first, x, y, (T2 *)J.accS[cur], J.accC[cur],
                                          (T2 *)J.accS[nxt], J.accC[nxt], cols);
                }
                __syncthreads();
            }
        }
        step *= J.decay;
    }
}

template <typename T, bool KAHAN>
struct ExactOps {
    using T2 = typename V2<T>::type;

    static int rows(bl_graph *g, int row0, int row1, int from_own, int parity) {
        if (row1 <= row0) return BL_OK;
        const int blocks = (row1 - row0 + kPanelThreads - 1) / kPanelThreads;
        int slot;
        BL_TRY(prof_begin(g, PK_ROWS, &slot));
        hipLaunchKernelGGL((rows_kernel<T, KAHAN>), dim3(blocks), dim3(kPanelThreads), 0, g->stream,
                           g->n, g->p.batch_size, g->nb, row0, row1, from_own, (const T *)g->x,
                           (const T *)g->y, (T2 *)g->ex.accS[parity], g->ex.accC[parity]);
        BL_HIP(hipGetLastError());
        return prof_end(g, slot);
    }

    static int panel(bl_graph *g, int b, int k, int do_next) {
        const int cur = k & 1, nxt = cur ^ 1;
        const int blocks = (g->n + kPanelThreads - 1) / kPanelThreads;
        int slot;
        BL_TRY(prof_begin(g, PK_PANEL, &slot));
        hipLaunchKernelGGL((panel_kernel<T, KAHAN>), dim3(blocks), dim3(kPanelThreads), 0, g->stream,
                           g->n, g->p.batch_size, b, do_next, (const T *)g->x, (const T *)g->y,
                           (T2 *)g->ex.accS[cur], g->ex.accC[cur], (T2 *)g->ex.accS[nxt],
                           g->ex.accC[nxt]);
        BL_HIP(hipGetLastError());
        return prof_end(g, slot);
    }

    static int finalize(bl_graph *g, int b, int k, double *energy_k, double *fout, int update,
                        int parity) {
        FinArgs<T> a;
        a.n = g->n;
        a.BS = g->p.batch_size;
        a.b = b;
        a.rowptr = g->rowptr;
        a.colidx = g->colidx;
        a.x = (T *)g->x;
        a.y = (T *)g->y;
        a.accS = (T2 *)g->ex.accS[parity];
        a.accC = g->ex.accC[parity];
        a.fbuf = (T2 *)g->ex.fbuf;
        a.ticket = g->ex.ticket;
        a.energy_k = energy_k;
        a.fout = fout;
        a.nonfinite = &g->counters->nonfinite;
        a.step = (T)step_at(g->p, k);
        a.invK = (T)(1.0 / g->p.K);
        a.negRK2 = (T)(-g->p.R * g->p.K * g->p.K);
        a.literal = g->p.repulse_adjacent ? 0 : 1;
        a.update = update;
        const int R = std::min(g->p.batch_size, g->n - b * g->p.batch_size);
        const int blocks = (R + kFinThreads / kWave - 1) / (kFinThreads / kWave);
        int slot;
        BL_TRY(prof_begin(g, PK_FINALIZE, &slot));
        hipLaunchKernelGGL((finalize_kernel<T, KAHAN>), dim3(blocks), dim3(kFinThreads), 0,
                           g->stream, a);
        BL_HIP(hipGetLastError());
        return prof_end(g, slot);
    }

    static int run(bl_graph *g, int iters, int start, int stop_batch) {
        if (iters <= 0) return BL_OK;
        const int nb = g->nb;
        const size_t accBytes = sizeof(T2) * (size_t)g->n;
        BL_TRY(rows(g, 0, g->n, 1, start & 1));
        BL_HIP(hipMemsetAsync(g->ex.accS[(start + 1) & 1], 0, accBytes, g->stream));
        if (KAHAN)
            BL_HIP(hipMemsetAsync(g->ex.accC[(start + 1) & 1], 0, sizeof(float2) * g->n, g->stream));
        for (int t = 0; t < iters; ++t) {
            const int k = start + t;
            const bool last = (t == iters - 1);
            const int upto = (last && stop_batch >= 0) ? stop_batch : nb;
            for (int b = 0; b < upto; ++b) {
                BL_TRY(finalize(g, b, k, g->energy + t, nullptr, 1, k & 1));
                const bool more_rows_now = (b + 1) < nb;
                if (more_rows_now || !last) BL_TRY(panel(g, b, k, last ? 0 : 1));
            }
            if (last && stop_batch >= 0)
                BL_TRY(finalize(g, stop_batch, k, nullptr, g->fout, 0, k & 1));
        }
        return BL_OK;
    }

    static int forces(bl_graph *g, int batch) {
        const int BS = g->p.batch_size;
        const int r0 = batch * BS, r1 = std::min(g->n, r0 + BS);
        BL_TRY(rows(g, r0, r1, 0, 0));
        return finalize(g, batch, 0, nullptr, g->fout, 0, 0);
    }
};

}  // namespace

// Launch one workgroup per graph for a group of exact-mode graphs that share
// a precision.  threads: 256, 512 or 1024 (the result does not depend on it).
int exact_graph_launch(bl_graph *const *gs, int G, int threads, hipStream_t s, void *d_jobs, int iters_override) {
    if (G == 0) return BL_OK;
    std::vector<ExactJob> jobs(G);
    for (int q = 0; q < G; ++q) {
        bl_graph *g = gs[q];
        ExactJob &J = jobs[q];
        J.n = g->n;
        J.BS = g->p.batch_size;
        J.nb = g->nb;
        J.iters = iters_override >= 0 ? iters_override : g->p.iterations;
        J.start = g->p.start_iter;
        J.literal = g->p.repulse_adjacent ? 0 : 1;
        J.step0 = g->p.step0;
        J.decay = g->p.step_decay;
        J.invK = 1.0 / g->p.K;
        J.negRK2 = -g->p.R * g->p.K * g->p.K;
        J.rowptr = g->rowptr;
        J.colidx = g->colidx;
        J.x = g->x;
        J.y = g->y;
        J.accS[0] = g->ex.accS[0];
        J.accS[1] = g->ex.accS[1];
        J.accC[0] = g->ex.accC[0];
        J.accC[1] = g->ex.accC[1];
        J.fbuf = g->ex.fbuf;
        J.energy = g->energy;
        J.nonfinite = &g->counters->nonfinite;
    }
    BL_HIP(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(ExactJob) * G, hipMemcpyHostToDevice, s));
    BL_HIP(hipStreamSynchronize(s));   // the host copy of the table is freed below
    const bl_graph *g0 = gs[0];
    const ExactJob *dj = (const ExactJob *)d_jobs;
#define BL_EXACT_LAUNCH(T, K, NT) hipLaunchKernelGGL((exact_graph_kernel<T, K, NT>), dim3(G), dim3(NT), 0, s, dj)
    const bool f64 = g0->fp64, plain = g0->p.precision == BL_FP32_PLAIN;
    if (threads == 256) {
        if (f64) BL_EXACT_LAUNCH(double, false, 256); else if (plain) BL_EXACT_LAUNCH(float, false, 256); else BL_EXACT_LAUNCH(float, true, 256);
    } else if (threads == 512) {
        if (f64) BL_EXACT_LAUNCH(double, false, 512); else if (plain) BL_EXACT_LAUNCH(float, false, 512); else BL_EXACT_LAUNCH(float, true, 512);
    } else {
        if (f64) BL_EXACT_LAUNCH(double, false, 1024); else if (plain) BL_EXACT_LAUNCH(float, false, 1024); else BL_EXACT_LAUNCH(float, true, 1024);
    }
#undef BL_EXACT_LAUNCH
    BL_HIP(hipGetLastError());
    return BL_OK;
}

size_t exact_job_size() { return sizeof(ExactJob); }

int exact_alloc(bl_graph *g) {
    const size_t t2 = g->fp64 ? sizeof(double2) : sizeof(float2);
    const size_t n = (size_t)g->n;
    for (int q = 0; q < 2; ++q) {
        BL_TRY(graph_alloc(g, &g->ex.accS[q], t2 * n));
        BL_TRY(graph_alloc(g, (void **)&g->ex.accC[q], sizeof(float2) * n));
    }
    BL_TRY(graph_alloc(g, &g->ex.fbuf, t2 * (size_t)g->p.batch_size));
    BL_TRY(graph_alloc(g, (void **)&g->ex.ticket, 256));
    BL_HIP(hipMemsetAsync(g->ex.ticket, 0, 256, g->stream));
    return BL_OK;
}

int exact_run(bl_graph *g, int iters, int start_iter, int stop_batch) {
    if (g->fp64) return ExactOps<double, false>::run(g, iters, start_iter, stop_batch);
    if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false>::run(g, iters, start_iter, stop_batch);
    return ExactOps<float, true>::run(g, iters, start_iter, stop_batch);
}

int exact_forces(bl_graph *g, int batch) {
    if (g->fp64) return ExactOps<double, false>::forces(g, batch);
    if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false>::forces(g, batch);
    return ExactOps<float, true>::forces(g, batch);
}

}  // namespace bl
