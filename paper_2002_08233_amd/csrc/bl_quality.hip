// Layout quality measures of Sec. 3.7 on the GPU: stress after the best
// uniform scaling, with hop distances from a bit-parallel multi-source BFS
// (64 sources per pass, one bit each); edge energy (the attractive potential
// whose gradient is the attraction term); edge uniformity (normalised standard
// deviation of edge lengths).
//
// Every sum runs in FP64 on a fixed grid: each thread sums its grid-stride
// share in order, each block combines its waves in order into its own slot,
// and one thread adds the slots in block order.  The result depends only on
// the graph and the coordinates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "bl_device.hpp"
#include "bl_internal.hpp"

namespace bl {
namespace {

using u64 = unsigned long long;

constexpr int kQThreads = 256;
constexpr int kQBlocks = 1024;
constexpr int kSrc = 64;         // BFS sources per pass
constexpr int kLevelGroup = 4;   // BFS levels launched between checks for an empty frontier

struct Sums {
    double s[kQBlocks][3];       // per block: stress A, B (or edge sums)
    u64 c[kQBlocks];             // per block: pair or edge count
};

// Fixed-order sum over the block of three doubles and a count; the totals
// land in slot blockIdx.x of S (added when `accumulate`, else stored).
__device__ void block_slot(Sums *S, double a, double b, double c, u64 k, bool accumulate) {
    __shared__ double ws[3][kQThreads / kWave];
    __shared__ u64 wk[kQThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    k = wave_sum(k);
    if (lane == 0) {
        ws[0][w] = a;
        ws[1][w] = b;
        ws[2][w] = c;
        wk[w] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        u64 tk = 0;
        for (int q = 0; q < kQThreads / kWave; ++q) {
            t0 += ws[0][q];
            t1 += ws[1][q];
            t2 += ws[2][q];
            tk += wk[q];
        }
        double *d = S->s[blockIdx.x];
        if (accumulate) {
            d[0] += t0;
            d[1] += t1;
            d[2] += t2;
            S->c[blockIdx.x] += tk;
        } else {
            d[0] = t0;
            d[1] = t1;
            d[2] = t2;
            S->c[blockIdx.x] = tk;
        }
    }
}

__global__ void sums_clear_kernel(Sums *S) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < kQBlocks) {
        S->s[b][0] = S->s[b][1] = S->s[b][2] = 0.0;
        S->c[b] = 0;
    }
}

// Slots added in block order by one thread: out[0..2] doubles, out[3] count.
__global__ void sums_total_kernel(const Sums *S, double *out, u64 *count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    u64 tk = 0;
    for (int b = 0; b < kQBlocks; ++b) {
        t0 += S->s[b][0];
        t1 += S->s[b][1];
        t2 += S->s[b][2];
        tk += S->c[b];
    }
    out[0] = t0;
    out[1] = t1;
    out[2] = t2;
    *count = tk;
}

__global__ void pos_kernel(int n, const double *__restrict__ x, const double *__restrict__ y, double2 *p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = double2{x[i], y[i]};
}

// Row holding CSR entry e: the largest i with rp[i] <= e (rp[n] = nnz > e).
__device__ __forceinline__ int row_of(const int *rp, int n, int64_t e) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Edge lengths of the undirected edges (entries (i, j) with j > i).
// pass 0: sum d^3 / (3K), sum d, count; pass 1: sum (d - mean)^2.
__global__ __launch_bounds__(kQThreads) void edge_kernel(int n, int64_t nnz, const int *__restrict__ rp,
                                                         const int *__restrict__ ci, const double2 *__restrict__ p,
                                                         double K, int pass, double mean, Sums *S) {
    double s0 = 0.0, s1 = 0.0;
    u64 m = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        const int j = ci[e];
        const int i = row_of(rp, n, e);
        if (j <= i) continue;
        const double2 a = p[i], b = p[j];
        const double dx = b.x - a.x, dy = b.y - a.y;
        const double d = sqrt(dx * dx + dy * dy);
        if (pass == 0) {
            s0 += d * d * d / (3.0 * K);
            s1 += d;
            ++m;
        } else {
            s0 += (d - mean) * (d - mean);
        }
    }
    block_slot(S, s0, s1, 0.0, m, false);
}

__global__ void bfs_clear_kernel(int n, u64 *seen, u64 *fr) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        seen[v] = 0;
        fr[v] = 0;
    }
}

// Source k of the pass is src[k] (pivots) or base + k (all pairs).
__device__ __forceinline__ int source_of(const int *src, int base, int k) { return src ? src[k] : base + k; }

__global__ void bfs_sources_kernel(const int *src, int base, int ns, u64 *seen, u64 *fr) {
    const int k = threadIdx.x;
    if (k < ns) {
        const int s = source_of(src, base, k);
        atomicOr(&seen[s], 1ull << k);
        atomicOr(&fr[s], 1ull << k);
    }
}

__global__ void counters_clear_kernel(u64 *c, int m) {
    if (threadIdx.x < m) c[threadIdx.x] = 0;
}

// One BFS level for the pass's sources, pulled: v is reached from source k
// at `level` when a neighbour was in source k's frontier at level - 1 and v
// was not reached before.  Each new (v, source) pair adds |c_v - c_s| / d and
// |c_v - c_s|^2 / d^2 to the stress sums (for all pairs only v > s counts, so
// each unordered pair counts once).  Rows of up to kHeavyDeg entries take a
// group of 8 lanes (bfs_light_kernel); longer rows, the hubs of skewed
// graphs, take a whole workgroup (bfs_heavy_kernel), so that no lane walks a
// hub row alone.
constexpr int kHeavyDeg = 256;
constexpr int kGroup = 8;

// OR of fin[ci[e]] over e = e0, e0 + step, ... < e1, four entries per round
// so that their loads are in flight together.
__device__ __forceinline__ u64 or_row(const int *__restrict__ ci, const u64 *__restrict__ fin, int e0, int e1,
                                      int step) {
    u64 m = 0;
    for (int e = e0; e < e1; e += 4 * step) {
        int c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = e + q * step < e1 ? ci[e + q * step] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) m |= c[q] >= 0 ? fin[c[q]] : 0ull;
    }
    return m;
}

struct BfsArgs {
    int n, ns, all_pairs, level;
    const int *rp, *ci, *src;
    int base;
    const double2 *p;
    const u64 *fin;
    u64 *fout, *seen, *newcount;
    const int *heavy;
    int nheavy;
    Sums *S;
};

__device__ __forceinline__ void load_sources(const BfsArgs &a, int *ss, double2 *sp) {
    if (threadIdx.x < a.ns) {
        const int s = source_of(a.src, a.base, threadIdx.x);
        ss[threadIdx.x] = s;
        sp[threadIdx.x] = a.p[s];
    }
    __syncthreads();
}

__device__ __forceinline__ void add_pair(const BfsArgs &a, int v, double2 pv, int k, const int *ss,
                                         const double2 *sp, double &sa, double &sb, u64 &pairs) {
    if (a.all_pairs && v < ss[k]) return;
    const double dl = (double)a.level;
    const double dx = pv.x - sp[k].x, dy = pv.y - sp[k].y;
    const double g = sqrt(dx * dx + dy * dy);
    sa += g / dl;
    sb += g * g / (dl * dl);
    ++pairs;
}

__global__ __launch_bounds__(kQThreads) void bfs_light_kernel(BfsArgs a) {
    __shared__ double2 sp[kSrc];
    __shared__ int ss[kSrc];
    load_sources(a, ss, sp);
    const u64 full = a.ns == kSrc ? ~0ull : ((1ull << a.ns) - 1ull);
    const int sub = threadIdx.x & (kGroup - 1);
    const int gid = (blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
    const int ngroups = gridDim.x * blockDim.x / kGroup;
    double sa = 0.0, sb = 0.0;
    u64 pairs = 0, fresh = 0;
    for (int base = 0; base < a.n; base += ngroups) {   // the same trip count in every lane
        const int v = base + gid;
        u64 sv = 0, m = 0;
        bool light = false;
        if (v < a.n) {
            sv = a.seen[v];
            const int r0 = a.rp[v], r1 = a.rp[v + 1];
            light = r1 - r0 <= kHeavyDeg;
            if (light && sv != full) m = or_row(a.ci, a.fin, r0 + sub, r1, kGroup);
        }
        // every lane is active here: OR over the group of 8
        m |= __shfl_xor(m, 1, kWave);
        m |= __shfl_xor(m, 2, kWave);
        m |= __shfl_xor(m, 4, kWave);
        if (light) {
            u64 nw = m & ~sv;
            if (sub == 0) {
                a.fout[v] = nw;
                if (nw) a.seen[v] = sv | nw;
                fresh += (u64)__popcll(nw);
            }
            if (nw) {
                const double2 pv = a.p[v];
                nw &= 0x0101010101010101ull << sub;   // this lane's bits: k = sub mod 8
                while (nw) {
                    const int k = __builtin_ctzll(nw);
                    nw &= nw - 1ull;
                    add_pair(a, v, pv, k, ss, sp, sa, sb, pairs);
                }
            }
        }
    }
    block_slot(a.S, sa, sb, 0.0, pairs, true);
    const u64 f = wave_sum(fresh);
    if ((threadIdx.x & (kWave - 1)) == 0 && f) atomicAdd(a.newcount, f);
}

__global__ __launch_bounds__(kQThreads) void bfs_heavy_kernel(BfsArgs a) {
    __shared__ double2 sp[kSrc];
    __shared__ int ss[kSrc];
    __shared__ u64 wor[kQThreads / kWave];
    load_sources(a, ss, sp);
    const u64 full = a.ns == kSrc ? ~0ull : ((1ull << a.ns) - 1ull);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double sa = 0.0, sb = 0.0;
    u64 pairs = 0, fresh = 0;
    for (int h = blockIdx.x; h < a.nheavy; h += gridDim.x) {   // uniform over the block
        const int v = a.heavy[h];
        const u64 sv = a.seen[v];
        u64 m = 0;
        if (sv != full) m = or_row(a.ci, a.fin, a.rp[v] + threadIdx.x, a.rp[v + 1], blockDim.x);
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) m |= __shfl_xor(m, o, kWave);
        if (lane == 0) wor[w] = m;
        __syncthreads();
        m = 0;
        for (int q = 0; q < kQThreads / kWave; ++q) m |= wor[q];
        __syncthreads();
        const u64 nw = m & ~sv;
        if (threadIdx.x == 0) {
            a.fout[v] = nw;
            if (nw) a.seen[v] = sv | nw;
            fresh += (u64)__popcll(nw);
        }
        if (threadIdx.x < kSrc && ((nw >> threadIdx.x) & 1ull))
            add_pair(a, v, a.p[v], threadIdx.x, ss, sp, sa, sb, pairs);
    }
    block_slot(a.S, sa, sb, 0.0, pairs, true);
    const u64 f = wave_sum(fresh);
    if ((threadIdx.x & (kWave - 1)) == 0 && f) atomicAdd(a.newcount, f);
}

// Device buffers of one evaluation, freed on every exit path.
struct QBuffers {
    std::vector<void *> owned;
    ~QBuffers() {
        for (void *q : owned) (void)hipFree(q);
    }
    int alloc(void **out, size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) {
            (void)hipGetLastError();
            return fail_code(BL_E_NOMEM, "hipMalloc failed in bl_quality_eval");
        }
        owned.push_back(q);
        *out = q;
        return BL_OK;
    }
};

// Where one evaluation's kernels read and write: the graph and coordinates
// (device copies or the caller's device arrays) and the work buffers.
struct QWork {
    const int *rp, *ci;
    const double *dx, *dy;
    const int *src;           // device pivots (NULL: all pairs)
    const int *heavy;         // rows longer than kHeavyDeg, ascending
    int nheavy;
    double2 *p;
    u64 *seen, *fr[2];
    Sums *S;
    double *tot;
    u64 *cnt, *newc;
};

// The edge passes and the BFS passes of bl_quality_eval on prepared buffers.
int quality_compute(int n, int64_t nnz, int npivots, double K, const QWork &w, hipStream_t s, bl_quality *out) {
    const int vb = (n + 255) / 256;
    hipLaunchKernelGGL(pos_kernel, dim3(vb), dim3(256), 0, s, n, w.dx, w.dy, w.p);

    // edge energy and uniformity: two passes over the entries
    double h[4];
    u64 hc[2];
    hipLaunchKernelGGL(edge_kernel, dim3(kQBlocks), dim3(kQThreads), 0, s, n, nnz, w.rp, w.ci, w.p, K, 0, 0.0, w.S);
    hipLaunchKernelGGL(sums_total_kernel, dim3(1), dim3(1), 0, s, w.S, w.tot, w.cnt);
    BL_HIP(hipMemcpyAsync(h, w.tot, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    BL_HIP(hipMemcpyAsync(hc, w.cnt, sizeof(u64), hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    const u64 m = hc[0];
    out->edges = (int64_t)m;
    out->edge_energy = h[0];
    if (m > 0) {
        const double mean = h[1] / (double)m;
        hipLaunchKernelGGL(edge_kernel, dim3(kQBlocks), dim3(kQThreads), 0, s, n, nnz, w.rp, w.ci, w.p, K, 1, mean,
                           w.S);
        hipLaunchKernelGGL(sums_total_kernel, dim3(1), dim3(1), 0, s, w.S, w.tot, w.cnt);
        BL_HIP(hipMemcpyAsync(h, w.tot, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
        BL_HIP(hipStreamSynchronize(s));
        out->edge_uniformity = mean > 0 ? std::sqrt(h[0] / ((double)m * mean * mean)) : 0.0;
    }

    // stress: sources in passes of 64
    hipLaunchKernelGGL(sums_clear_kernel, dim3((kQBlocks + 255) / 256), dim3(256), 0, s, w.S);
    const int nsrc_total = npivots > 0 ? npivots : n;
    int levels = 0;
    for (int base = 0; base < nsrc_total; base += kSrc) {
        const int ns = std::min(kSrc, nsrc_total - base);
        const int *sp = w.src ? w.src + base : nullptr;
        hipLaunchKernelGGL(bfs_clear_kernel, dim3(vb), dim3(256), 0, s, n, w.seen, w.fr[0]);
        hipLaunchKernelGGL(bfs_sources_kernel, dim3(1), dim3(kSrc), 0, s, sp, base, ns, w.seen, w.fr[0]);
        int cur = 0;
        for (int level = 1; level < n + 1; level += kLevelGroup) {
            hipLaunchKernelGGL(counters_clear_kernel, dim3(1), dim3(kLevelGroup), 0, s, w.newc, kLevelGroup);
            for (int q = 0; q < kLevelGroup; ++q) {
                BfsArgs a;
                a.n = n;
                a.ns = ns;
                a.all_pairs = npivots > 0 ? 0 : 1;
                a.level = level + q;
                a.rp = w.rp;
                a.ci = w.ci;
                a.src = sp;
                a.base = base;
                a.p = w.p;
                a.fin = w.fr[cur];
                a.fout = w.fr[cur ^ 1];
                a.seen = w.seen;
                a.newcount = w.newc + q;
                a.heavy = w.heavy;
                a.nheavy = w.nheavy;
                a.S = w.S;
                hipLaunchKernelGGL(bfs_light_kernel, dim3(kQBlocks), dim3(kQThreads), 0, s, a);
                if (w.nheavy)
                    hipLaunchKernelGGL(bfs_heavy_kernel, dim3(std::min(w.nheavy, kQBlocks)), dim3(kQThreads), 0, s,
                                       a);
                cur ^= 1;
            }
            u64 nc[kLevelGroup];
            BL_HIP(hipMemcpyAsync(nc, w.newc, sizeof nc, hipMemcpyDeviceToHost, s));
            BL_HIP(hipStreamSynchronize(s));
            levels += kLevelGroup;
            bool done = false;
            for (int q = 0; q < kLevelGroup; ++q) done = done || nc[q] == 0;
            if (done) break;
        }
    }
    hipLaunchKernelGGL(sums_total_kernel, dim3(1), dim3(1), 0, s, w.S, w.tot, w.cnt);
    BL_HIP(hipMemcpyAsync(h, w.tot, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    BL_HIP(hipMemcpyAsync(hc, w.cnt, sizeof(u64), hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    BL_HIP(hipGetLastError());
    const double A = h[0], Bs = h[1], N = (double)hc[0];
    out->pairs = (int64_t)hc[0];
    out->bfs_levels = levels;
    if (Bs == 0.0) {
        out->stress = N;
        out->scale = 0.0;
    } else {
        out->stress = N - A * A / Bs;
        out->scale = A / Bs;
    }
    return BL_OK;
}

// Argument checks shared by both entry points (the CSR itself is checked
// separately).
int quality_args(const double *x, const double *y, int32_t npivots, const int32_t *pivots, double K,
                 bl_quality *out) {
    if (!out) return fail_code(BL_E_INVAL, "out is NULL");
    std::memset(out, 0, sizeof *out);
    if (!x || !y) return fail_code(BL_E_INVAL, "coordinate arrays are NULL");
    if (!(K > 0) || !std::isfinite(K)) return fail_code(BL_E_INVAL, "K must be > 0");
    if (npivots < 0 || (npivots > 0 && !pivots)) return fail_code(BL_E_INVAL, "bad pivot list");
    return BL_OK;
}

// ------------------------------------------------ allocation-free variant
//
// bl_quality_eval_noalloc keeps its work buffers in one static device array
// of fixed size instead of allocating them.  Its layout, for at most
// kNoAllocMaxN vertices and kNoAllocMaxPivots pivots:
//   p (double2 per vertex), seen and two frontier words (u64 per vertex),
//   the heavy-row list (int per vertex), the block slots, the totals and
//   counters, the pivots, and two ints (CSR check flag, heavy-row count);
// each piece starts on a 256-byte boundary.
constexpr int kNoAllocMaxN = 1 << 18;
constexpr int kNoAllocMaxPivots = 1 << 16;
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kScrP = 0;
constexpr size_t kScrSeen = kScrP + al256(sizeof(double2) * kNoAllocMaxN);
constexpr size_t kScrFr0 = kScrSeen + al256(sizeof(u64) * kNoAllocMaxN);
constexpr size_t kScrFr1 = kScrFr0 + al256(sizeof(u64) * kNoAllocMaxN);
constexpr size_t kScrHeavy = kScrFr1 + al256(sizeof(u64) * kNoAllocMaxN);
constexpr size_t kScrSums = kScrHeavy + al256(sizeof(int) * kNoAllocMaxN);
constexpr size_t kScrTot = kScrSums + al256(sizeof(Sums));
constexpr size_t kScrCnt = kScrTot + al256(sizeof(double) * 4);
constexpr size_t kScrNewc = kScrCnt + al256(sizeof(u64) * 2);
constexpr size_t kScrSrc = kScrNewc + al256(sizeof(u64) * kLevelGroup);
constexpr size_t kScrFlags = kScrSrc + al256(sizeof(int) * kNoAllocMaxPivots);
constexpr size_t kScratchBytes = kScrFlags + al256(sizeof(int) * 2);

}  // namespace
}  // namespace bl

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: kernels get the pointer hipGetSymbolAddress gave
// for the current device.
static __device__ __align__(256) unsigned char scratch[bl::kScratchBytes];

namespace bl {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_address(unsigned char **out) {
    int dev = 0;
    BL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail_code(BL_E_INVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail_code(BL_E_HIP, "hipGetSymbolAddress of the quality scratch array failed");
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return BL_OK;
}

__global__ void flags_clear_kernel(int *f) {
    if (threadIdx.x < 2) f[threadIdx.x] = 0;
}

// The CSR checks of check_csr without BL_VALIDATE, on device arrays:
// rowptr[0] = 0, rowptr non-decreasing, rowptr[n] = nnz, colidx in [0, n).
// Any failure sets *bad.
__global__ void csr_check_kernel(int n, int64_t nnz, const int *__restrict__ rp, const int *__restrict__ ci,
                                 int *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool b = false;
    if (t == 0) b = rp[0] != 0 || (int64_t)rp[n] != nnz;
    for (int64_t i = t; i < n; i += stride) b = b || rp[i + 1] < rp[i];
    for (int64_t e = t; e < nnz; e += stride) {
        const int j = ci[e];
        b = b || j < 0 || j >= n;
    }
    if (b) atomicOr(bad, 1);
}

// Rows with more than kHeavyDeg entries, ascending, in one workgroup of
// kQThreads threads (the list bl_quality_eval builds on the host).
__global__ __launch_bounds__(kQThreads) void heavy_list_kernel(int n, const int *__restrict__ rp, int *heavy,
                                                               int *count) {
    __shared__ int wtot[kQThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int carry = 0;
    for (int base = 0; base < n; base += kQThreads) {
        const int v = base + threadIdx.x;
        const bool f = v < n && rp[v + 1] - rp[v] > kHeavyDeg;
        const u64 bal = __ballot(f);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[w] = __popcll(bal);
        __syncthreads();
        int off = carry, tot = 0;
        for (int q = 0; q < kQThreads / kWave; ++q) {
            if (q < w) off += wtot[q];
            tot += wtot[q];
        }
        if (f) heavy[off + below] = v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

// ------------------------------------------------ neighbourhood preservation
//
// For a vertex i with k = deg(i) > 0: L(i) = the k vertices v != i nearest
// to i in the layout, ordered by the squared distance (FP64, no fused
// multiply-add) and then by id; the vertex's score is the Jaccard index
// |N(i) & L(i)| / |N(i) | L(i)| = both / (2k - both).
//
// One workgroup per sampled vertex finds the k-th smallest key (d2, id) by
// radix selection: eight 8-bit passes over the bits of d2 (non-negative
// doubles order like their bit patterns), then, if the k-th place falls
// inside a run of equal distances, four 8-bit passes over the ids of that
// run.  Each pass histograms, in LDS, the vertices whose key agrees with the
// prefix found so far.  A neighbour j is then in L(i) iff its key is at most
// the k-th key.  Every decision is on exact integers and bit patterns.
constexpr int kNpThreads = 512;

__device__ __forceinline__ u64 d2_bits(double2 a, double2 b) {
#pragma clang fp contract(off)
    const double dx = b.x - a.x, dy = b.y - a.y;
    const double d2 = dx * dx + dy * dy;
    return (u64)__double_as_longlong(d2);
}

// The bin of hist[256] holding the need-th (1-based) of the counted keys;
// need becomes the rank inside that bin and *cnt the bin's count.  Thread 0
// scans; the result is broadcast through sh[3].  Returns -1 when fewer than
// need keys were counted.
__device__ int np_pick(const int *hist, int *sh, int &need, int &cnt) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int below = 0, b = -1;
        for (int q = 0; q < 256; ++q) {
            const int c = hist[q];
            if (below + c >= need) {
                b = q;
                break;
            }
            below += c;
        }
        sh[0] = b;
        sh[1] = b >= 0 ? need - below : need;
        sh[2] = b >= 0 ? hist[b] : 0;
    }
    __syncthreads();
    const int b = sh[0];
    need = sh[1];
    cnt = sh[2];
    __syncthreads();
    return b;
}

__global__ __launch_bounds__(kNpThreads) void np_kernel(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const double2 *__restrict__ p, int ns,
                                                        const int *__restrict__ sample, int2 *res) {
    __shared__ int hist[256];
    __shared__ int sh[4];
    for (int q = blockIdx.x; q < ns; q += gridDim.x) {   // uniform over the block
        const int i = sample ? sample[q] : q;
        const int k = rp[i + 1] - rp[i];
        if (k == 0) {
            if (threadIdx.x == 0) res[q] = int2{0, 0};
            continue;
        }
        const double2 pi = p[i];
        u64 tau = ~0ull;
        int id_thr = 0x7fffffff;
        if (k <= n - 1) {
            // d2 bits, most significant byte first
            u64 pre = 0, msk = 0;
            int need = k, cnt = 0;
            for (int sft = 56; sft >= 0; sft -= 8) {
                if (threadIdx.x < 256) hist[threadIdx.x] = 0;
                __syncthreads();
                for (int v = threadIdx.x; v < n; v += blockDim.x) {
                    if (v == i) continue;
                    const u64 kb = d2_bits(pi, p[v]);
                    if ((kb & msk) == pre) atomicAdd(&hist[(int)((kb >> sft) & 255ull)], 1);
                }
                const int b = np_pick(hist, sh, need, cnt);
                pre |= (u64)b << sft;
                msk |= 255ull << sft;
            }
            tau = pre;
            if (need < cnt) {
                // only the `need` smallest ids of the run with d2 == tau are in L(i)
                int ipre = 0, imsk = 0;
                for (int sft = 24; sft >= 0; sft -= 8) {
                    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
                    __syncthreads();
                    for (int v = threadIdx.x; v < n; v += blockDim.x) {
                        if (v == i || (v & imsk) != ipre) continue;
                        if (d2_bits(pi, p[v]) == tau) atomicAdd(&hist[(v >> sft) & 255], 1);
                    }
                    const int b = np_pick(hist, sh, need, cnt);
                    ipre |= b << sft;
                    imsk |= 255 << sft;
                }
                id_thr = ipre;
            }
        }
        // neighbours inside L(i)
        if (threadIdx.x == 0) sh[3] = 0;
        __syncthreads();
        int both = 0;
        for (int e = rp[i] + threadIdx.x; e < rp[i + 1]; e += blockDim.x) {
            const int j = ci[e];
            const u64 kb = d2_bits(pi, p[j]);
            both += (kb < tau || (kb == tau && j <= id_thr)) ? 1 : 0;
        }
        both = wave_sum(both);
        if ((threadIdx.x & (kWave - 1)) == 0 && both) atomicAdd(&sh[3], both);
        __syncthreads();
        if (threadIdx.x == 0) res[q] = int2{sh[3], k};
        __syncthreads();
    }
}

// Mean of the per-vertex Jaccard indices over vertices with k > 0, in a fixed
// order: thread t sums its contiguous share in order, then thread 0 adds the
// shares in thread order.  out[0] = sum, cnt[0] = vertices counted.
__global__ __launch_bounds__(256) void np_sum_kernel(int ns, const int2 *__restrict__ res, double *out, u64 *cnt) {
    __shared__ double ps[256];
    __shared__ u64 pc[256];
    const int per = (ns + 255) / 256;
    const int q0 = threadIdx.x * per, q1 = min(ns, q0 + per);
    double sum = 0.0;
    u64 c = 0;
    for (int q = q0; q < q1; ++q) {
        const int2 r = res[q];
        if (r.y > 0) {
            sum += (double)r.x / (double)(2 * r.y - r.x);
            ++c;
        }
    }
    ps[threadIdx.x] = sum;
    pc[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        u64 tc = 0;
        for (int q = 0; q < 256; ++q) {
            t += ps[q];
            tc += pc[q];
        }
        out[0] = t;
        cnt[0] = tc;
    }
}

}  // namespace
}  // namespace bl

extern "C" int bl_quality_eval(const bl_csr *g, const double *x, const double *y, int32_t npivots,
                               const int32_t *pivots, double K, uint32_t flags, void *hip_stream,
                               bl_quality *out) {
    using namespace bl;
    BL_TRY(quality_args(x, y, npivots, pivots, K, out));
    if (flags & ~BL_DEVICE_PTRS) return fail_code(BL_E_INVAL, "unknown flags");
    hipStream_t s = (hipStream_t)hip_stream;
    BL_TRY(check_csr(g, flags, s));
    const int n = g->n;
    const int64_t nnz = g->nnz;
    for (int q = 0; q < npivots; ++q)
        if (pivots[q] < 0 || pivots[q] >= n) return fail_code(BL_E_INVAL, "pivot out of range");
    const bool dev = (flags & BL_DEVICE_PTRS) != 0;
    const hipMemcpyKind h2d = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;

    QBuffers B;
    QWork w{};
    int *rp, *ci, *src = nullptr, *heavy;
    double *dx, *dy;
    BL_TRY(B.alloc((void **)&rp, sizeof(int) * (size_t)(n + 1)));
    BL_TRY(B.alloc((void **)&ci, sizeof(int) * (size_t)nnz));
    BL_TRY(B.alloc((void **)&dx, sizeof(double) * (size_t)n));
    BL_TRY(B.alloc((void **)&dy, sizeof(double) * (size_t)n));
    BL_TRY(B.alloc((void **)&w.p, sizeof(double2) * (size_t)n));
    BL_TRY(B.alloc((void **)&w.seen, sizeof(u64) * (size_t)n));
    BL_TRY(B.alloc((void **)&w.fr[0], sizeof(u64) * (size_t)n));
    BL_TRY(B.alloc((void **)&w.fr[1], sizeof(u64) * (size_t)n));
    BL_TRY(B.alloc((void **)&w.S, sizeof(Sums)));
    BL_TRY(B.alloc((void **)&w.tot, sizeof(double) * 4));
    BL_TRY(B.alloc((void **)&w.cnt, sizeof(u64) * 2));
    BL_TRY(B.alloc((void **)&w.newc, sizeof(u64) * kLevelGroup));
    if (npivots > 0) {
        BL_TRY(B.alloc((void **)&src, sizeof(int) * (size_t)npivots));
        BL_HIP(hipMemcpyAsync(src, pivots, sizeof(int) * (size_t)npivots, hipMemcpyHostToDevice, s));
    }
    BL_HIP(hipMemcpyAsync(rp, g->rowptr, sizeof(int) * (size_t)(n + 1), h2d, s));
    if (nnz) BL_HIP(hipMemcpyAsync(ci, g->colidx, sizeof(int) * (size_t)nnz, h2d, s));
    BL_HIP(hipMemcpyAsync(dx, x, sizeof(double) * (size_t)n, h2d, s));
    BL_HIP(hipMemcpyAsync(dy, y, sizeof(double) * (size_t)n, h2d, s));
    // rows longer than kHeavyDeg, listed once for the heavy BFS kernel
    std::vector<int32_t> rph;
    const int32_t *rpv = g->rowptr;
    if (dev) {
        rph.resize((size_t)n + 1);
        BL_HIP(hipMemcpyAsync(rph.data(), g->rowptr, sizeof(int) * (size_t)(n + 1), hipMemcpyDeviceToHost, s));
        BL_HIP(hipStreamSynchronize(s));
        rpv = rph.data();
    }
    std::vector<int32_t> hv;
    for (int v = 0; v < n; ++v)
        if (rpv[v + 1] - rpv[v] > kHeavyDeg) hv.push_back(v);
    BL_TRY(B.alloc((void **)&heavy, sizeof(int) * std::max<size_t>(hv.size(), 1)));
    if (!hv.empty()) BL_HIP(hipMemcpyAsync(heavy, hv.data(), sizeof(int) * hv.size(), hipMemcpyHostToDevice, s));
    w.rp = rp;
    w.ci = ci;
    w.dx = dx;
    w.dy = dy;
    w.src = src;
    w.heavy = heavy;
    w.nheavy = (int)hv.size();
    return quality_compute(n, nnz, npivots, K, w, s, out);
}

extern "C" int bl_quality_eval_noalloc(const bl_csr *g, const double *x, const double *y, int32_t npivots,
                                       const int32_t *pivots, double K, uint32_t flags, void *hip_stream,
                                       bl_quality *out) {
    using namespace bl;
    BL_TRY(quality_args(x, y, npivots, pivots, K, out));
    if (flags != BL_DEVICE_PTRS) return fail_code(BL_E_INVAL, "flags must be exactly BL_DEVICE_PTRS");
    if (!g) return fail_code(BL_E_INVAL, "graph is NULL");
    if (g->n < 1) return fail_code(BL_E_INVAL, "n must be >= 1");
    if (g->n > kNoAllocMaxN) return fail_code(BL_E_INVAL, "n exceeds the scratch limit of 262144 vertices");
    if (npivots > kNoAllocMaxPivots) return fail_code(BL_E_INVAL, "more than 65536 pivots");
    if (g->nnz < 0 || g->nnz > 0x7fffffffLL) return fail_code(BL_E_INVAL, "nnz out of range");
    if (!g->rowptr || (g->nnz > 0 && !g->colidx)) return fail_code(BL_E_INVAL, "CSR arrays are NULL");
    const int n = g->n;
    const int64_t nnz = g->nnz;
    for (int q = 0; q < npivots; ++q)
        if (pivots[q] < 0 || pivots[q] >= n) return fail_code(BL_E_INVAL, "pivot out of range");
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned char *base = nullptr;
    BL_TRY(scratch_address(&base));
    int *fl = (int *)(base + kScrFlags);
    int hf[2] = {0, 0};
    hipLaunchKernelGGL(flags_clear_kernel, dim3(1), dim3(64), 0, s, fl);
    hipLaunchKernelGGL(csr_check_kernel, dim3(256), dim3(256), 0, s, n, nnz, g->rowptr, g->colidx, fl);
    BL_HIP(hipMemcpyAsync(hf, fl, sizeof(int), hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    if (hf[0]) return fail_code(BL_E_INVAL, "malformed CSR (rowptr not monotone from 0 to nnz, or colidx out of range)");

    QWork w{};
    w.rp = g->rowptr;
    w.ci = g->colidx;
    w.dx = x;
    w.dy = y;
    w.p = (double2 *)(base + kScrP);
    w.seen = (u64 *)(base + kScrSeen);
    w.fr[0] = (u64 *)(base + kScrFr0);
    w.fr[1] = (u64 *)(base + kScrFr1);
    w.S = (Sums *)(base + kScrSums);
    w.tot = (double *)(base + kScrTot);
    w.cnt = (u64 *)(base + kScrCnt);
    w.newc = (u64 *)(base + kScrNewc);
    int *heavy = (int *)(base + kScrHeavy);
    if (npivots > 0) {
        int *src = (int *)(base + kScrSrc);
        BL_HIP(hipMemcpyAsync(src, pivots, sizeof(int) * (size_t)npivots, hipMemcpyHostToDevice, s));
        w.src = src;
    }
    hipLaunchKernelGGL(heavy_list_kernel, dim3(1), dim3(kQThreads), 0, s, n, g->rowptr, heavy, fl + 1);
    BL_HIP(hipMemcpyAsync(hf + 1, fl + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    w.heavy = heavy;
    w.nheavy = hf[1];
    return quality_compute(n, nnz, npivots, K, w, s, out);
}

extern "C" int bl_neighborhood_preservation(const bl_csr *g, const double *x, const double *y, int32_t nsample,
                                            const int32_t *sample, uint32_t flags, void *hip_stream,
                                            double *np_out, int64_t *counted) {
    using namespace bl;
    if (!np_out) return fail_code(BL_E_INVAL, "np_out is NULL");
    *np_out = 0.0;
    if (counted) *counted = 0;
    if (!x || !y) return fail_code(BL_E_INVAL, "coordinate arrays are NULL");
    if (flags & ~BL_DEVICE_PTRS) return fail_code(BL_E_INVAL, "unknown flags");
    if (nsample < 0 || (nsample > 0 && !sample)) return fail_code(BL_E_INVAL, "bad sample list");
    hipStream_t s = (hipStream_t)hip_stream;
    BL_TRY(check_csr(g, flags, s));
    const int n = g->n;
    const int64_t nnz = g->nnz;
    for (int q = 0; q < nsample; ++q)
        if (sample[q] < 0 || sample[q] >= n) return fail_code(BL_E_INVAL, "sample vertex out of range");
    const bool dev = (flags & BL_DEVICE_PTRS) != 0;
    const hipMemcpyKind h2d = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const int ns = nsample > 0 ? nsample : n;

    QBuffers B;
    int *rp, *ci, *smp = nullptr;
    double *dx, *dy, *sum;
    double2 *p;
    int2 *res;
    u64 *cnt;
    BL_TRY(B.alloc((void **)&rp, sizeof(int) * (size_t)(n + 1)));
    BL_TRY(B.alloc((void **)&ci, sizeof(int) * (size_t)nnz));
    BL_TRY(B.alloc((void **)&dx, sizeof(double) * (size_t)n));
    BL_TRY(B.alloc((void **)&dy, sizeof(double) * (size_t)n));
    BL_TRY(B.alloc((void **)&p, sizeof(double2) * (size_t)n));
    BL_TRY(B.alloc((void **)&res, sizeof(int2) * (size_t)ns));
    BL_TRY(B.alloc((void **)&sum, sizeof(double)));
    BL_TRY(B.alloc((void **)&cnt, sizeof(u64)));
    if (nsample > 0) {
        BL_TRY(B.alloc((void **)&smp, sizeof(int) * (size_t)nsample));
        BL_HIP(hipMemcpyAsync(smp, sample, sizeof(int) * (size_t)nsample, hipMemcpyHostToDevice, s));
    }
    BL_HIP(hipMemcpyAsync(rp, g->rowptr, sizeof(int) * (size_t)(n + 1), h2d, s));
    if (nnz) BL_HIP(hipMemcpyAsync(ci, g->colidx, sizeof(int) * (size_t)nnz, h2d, s));
    BL_HIP(hipMemcpyAsync(dx, x, sizeof(double) * (size_t)n, h2d, s));
    BL_HIP(hipMemcpyAsync(dy, y, sizeof(double) * (size_t)n, h2d, s));
    hipLaunchKernelGGL(pos_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, dx, dy, p);
    hipLaunchKernelGGL(np_kernel, dim3(std::min(ns, 4096)), dim3(kNpThreads), 0, s, n, rp, ci, p, ns, smp, res);
    hipLaunchKernelGGL(np_sum_kernel, dim3(1), dim3(256), 0, s, ns, res, sum, cnt);
    double h = 0.0;
    u64 c = 0;
    BL_HIP(hipMemcpyAsync(&h, sum, sizeof h, hipMemcpyDeviceToHost, s));
    BL_HIP(hipMemcpyAsync(&c, cnt, sizeof c, hipMemcpyDeviceToHost, s));
    BL_HIP(hipStreamSynchronize(s));
    BL_HIP(hipGetLastError());
    *np_out = c ? h / (double)c : 0.0;
    if (counted) *counted = (int64_t)c;
    return BL_OK;
}
