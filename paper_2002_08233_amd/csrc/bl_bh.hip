// Barnes-Hut force step (Sec. 3.5; Alg. S1-S3) for gfx950.
//
// Per iteration (all on the device, no host round trip):
//   1. bbox_kernel     square root cell: xmin, ymin, W = max extent (Alg. S3)
//   2. morton_kernel   16-bit-per-axis Z-order keys, quantised in float32
//   3. radix sort      own LSD sort of (key, id), 4 passes of 8 bits, stable
//   4. mark_kernel     adjacent sorted keys p, p+1 first differ in 2-bit digit
//                      L: the level-L cell holding both has >= 2 children, so
//                      it is a tree cell; depth-16 runs of equal keys are
//                      buckets.  Single-child chains are never materialised.
//   5. scans           cells per start position -> pre-order indices; double-
//                      double prefix sums of the sorted coordinates
//   6. emit_kernel     nodes in DFS pre-order (the Morton order of Fig. 5) with
//                      skip links, centroid = exact mean of the members
//   7. far_kernel      one walk per vertex in Morton order against the
//                      snapshot: accepted cells (side < theta*d), and leaves
//                      whose vertex has not moved yet this iteration; leaves of
//                      already-moved vertices are listed for the chain
//   8. chain_kernel    one workgroup walks the batches in order: attraction
//                      over CSR rows and the listed leaves with live
//                      coordinates, then the batch update (Alg. 2 update loop)
#include <cfloat>

#include "bl_device.hpp"
#include "bl_internal.hpp"

namespace bl {
namespace {

constexpr int kBBoxBlocks = 256;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;     // 4096 keys per tile
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;     // 4096 values per tile
constexpr int kChainThreads = 1024;

// ------------------------------------------------------------------ bbox
__global__ __launch_bounds__(256) void bbox_kernel(int n, const float2 *__restrict__ pos, float *part,
                                                   unsigned *ticket, float *bbox) {
    __shared__ float s[4][256 / kWave];
    __shared__ int s_last;
    float mnx = FLT_MAX, mny = FLT_MAX, mxx = -FLT_MAX, mxy = -FLT_MAX;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 c = pos[i];
        const float a = c.x, b = c.y;
        mnx = fminf(mnx, a);
        mxx = fmaxf(mxx, a);
        mny = fminf(mny, b);
        mxy = fmaxf(mxy, b);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        mnx = fminf(mnx, __shfl_xor(mnx, o, kWave));
        mxx = fmaxf(mxx, __shfl_xor(mxx, o, kWave));
        mny = fminf(mny, __shfl_xor(mny, o, kWave));
        mxy = fmaxf(mxy, __shfl_xor(mxy, o, kWave));
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s[0][w] = mnx;
        s[1][w] = mxx;
        s[2][w] = mny;
        s[3][w] = mxy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 256 / kWave; ++q) {
            s[0][0] = fminf(s[0][0], s[0][q]);
            s[1][0] = fmaxf(s[1][0], s[1][q]);
            s[2][0] = fminf(s[2][0], s[2][q]);
            s[3][0] = fmaxf(s[3][0], s[3][q]);
        }
        part[4 * blockIdx.x + 0] = s[0][0];
        part[4 * blockIdx.x + 1] = s[1][0];
        part[4 * blockIdx.x + 2] = s[2][0];
        part[4 * blockIdx.x + 3] = s[3][0];
        __threadfence();
        s_last = (atomicAdd(ticket, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    __threadfence();
    float a = FLT_MAX, b = -FLT_MAX, c = FLT_MAX, d = -FLT_MAX;
    for (int q = 0; q < (int)gridDim.x; ++q) {
        a = fminf(a, part[4 * q + 0]);
        b = fmaxf(b, part[4 * q + 1]);
        c = fminf(c, part[4 * q + 2]);
        d = fmaxf(d, part[4 * q + 3]);
    }
    const float wx = b - a, wy = d - c;
    const float W = fmaxf(wx, wy);
    bbox[0] = a;
    bbox[1] = c;
    bbox[2] = W;
    // 2^16 / W rounded once to float (computed in double: double rounding is
    // innocuous for a quotient of floats since 53 >= 2*24 + 2).
    bbox[3] = W > 0.f ? (float)(65536.0 / (double)W) : 0.f;
    *ticket = 0u;
}

// ---------------------------------------------------------------- morton
__device__ __forceinline__ unsigned spread16(unsigned v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ __forceinline__ unsigned quantise(float v, float vmin, float scale) {
    const float u = v - vmin;
    const float f = u * scale;
    int q = (int)f;
    q = q < 0 ? 0 : (q > 65535 ? 65535 : q);
    return (unsigned)q;
}

__global__ void morton_kernel(int n, const float2 *__restrict__ pos,
                              const float *__restrict__ bbox, unsigned *__restrict__ key,
                              int *__restrict__ val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float xmin = bbox[0], ymin = bbox[1], scale = bbox[3];
    unsigned qx = 0, qy = 0;
    if (scale > 0.f) {
        const float2 c = pos[i];
        qx = quantise(c.x, xmin, scale);
        qy = quantise(c.y, ymin, scale);
    }
    key[i] = spread16(qx) | (spread16(qy) << 1);
    val[i] = i;
}

// ----------------------------------------------------------- radix sort
// Lanes of the wave whose 8-bit digit equals this lane's (valid lanes only).
__device__ __forceinline__ unsigned long long digit_peers(unsigned d, bool valid) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long v = __ballot(bit);
        m &= bit ? v : ~v;
    }
    return m;
}

__device__ __forceinline__ unsigned long long lanes_below() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const unsigned *__restrict__ keys,
                                                                  int n, int shift, int *hist,
                                                                  int tiles) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int base = blockIdx.x * kSortTile + w * (kSortTile / 4);
    for (int g = 0; g < kSortItems; ++g) {
        const int p = base + g * kWave + lane;
        const bool valid = p < n;
        const unsigned d = valid ? (keys[p] >> shift) & 255u : 0u;
        const unsigned long long m = digit_peers(d, valid);
        if (valid && (__ffsll((long long)m) - 1) == lane) atomicAdd(&h[d], __popcll(m));
    }
    __syncthreads();
    hist[threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const unsigned *__restrict__ kin, const int *__restrict__ vin, unsigned *__restrict__ kout,
    int *__restrict__ vout, int n, int shift, const int *__restrict__ hist, int tiles) {
    __shared__ int cnt[4][256];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int q = threadIdx.x; q < 4 * 256; q += kSortThreads) (&cnt[0][0])[q] = 0;
    __syncthreads();
    const int base = blockIdx.x * kSortTile + w * (kSortTile / 4);
    unsigned k[kSortItems];
    int v[kSortItems];
#pragma unroll
    for (int g = 0; g < kSortItems; ++g) {
        const int p = base + g * kWave + lane;
        k[g] = p < n ? kin[p] : 0u;
        v[g] = p < n ? vin[p] : 0;
    }
    // pass 1: per-wave digit counts
#pragma unroll
    for (int g = 0; g < kSortItems; ++g) {
        const bool valid = base + g * kWave + lane < n;
        const unsigned d = (k[g] >> shift) & 255u;
        const unsigned long long m = digit_peers(d, valid);
        if (valid && (__ffsll((long long)m) - 1) == lane) cnt[w][d] += __popcll(m);
    }
    __syncthreads();
    // per-wave starting offsets: tile base from the scanned histogram, then
    // earlier waves of this tile
    {
        const int d = threadIdx.x;
        int run = hist[d * tiles + blockIdx.x];
        for (int q = 0; q < 4; ++q) {
            const int c = cnt[q][d];
            cnt[q][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < kSortItems; ++g) {
        const bool valid = base + g * kWave + lane < n;
        const unsigned d = (k[g] >> shift) & 255u;
        const unsigned long long m = digit_peers(d, valid);
        const int pos = cnt[w][d] + __popcll(m & lanes_below());
        if (valid) {
            kout[pos] = k[g];
            vout[pos] = v[g];
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && (__ffsll((long long)m) - 1) == lane) cnt[w][d] += __popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
}

// Exclusive scan of `len` ints in place by one workgroup (used for the radix
// histogram, len = 256 * tiles).
__global__ __launch_bounds__(kScanThreads) void scan_single_kernel(int *data, int len) {
    __shared__ int ws[16];
    int running = 0;
    for (int b0 = 0; b0 < len; b0 += kScanTile) {
        int v[kScanItems];
        int s = 0;
        const int p0 = b0 + threadIdx.x * kScanItems;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            v[q] = (p0 + q < len) ? data[p0 + q] : 0;
            s += v[q];
        }
        int total;
        int pre = block_excl_scan(s, ws, &total) + running;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            if (p0 + q < len) data[p0 + q] = pre;
            pre += v[q];
        }
        running += total;
    }
}

// ------------------------------------------------------------ tree cells
__device__ __forceinline__ int common_levels(unsigned a, unsigned b) {
    const unsigned x = a ^ b;
    return x == 0u ? 16 : (__clz(x) >> 1);
}

// Sorted position range [lo, hi] of the level-`lvl` cell holding sorted
// position p (binary searches on the sorted keys).
__device__ __forceinline__ int cell_first(const unsigned *keys, int p, int lvl) {
    if (lvl == 0) return 0;
    const int sh = 32 - 2 * lvl;
    const unsigned pre = keys[p] >> sh;
    int lo = 0, hi = p;   // first q in [0, p] with keys[q] >> sh == pre
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((keys[mid] >> sh) < pre) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int cell_last(const unsigned *keys, int n, int p, int lvl) {
    if (lvl == 0) return n - 1;
    const int sh = 32 - 2 * lvl;
    const unsigned pre = keys[p] >> sh;
    int lo = p, hi = n - 1;   // last q in [p, n) with keys[q] >> sh == pre
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((keys[mid] >> sh) > pre) hi = mid - 1;
        else lo = mid;
    }
    return lo;
}

__global__ void mark_kernel(int n, const unsigned *__restrict__ keys, unsigned *mask) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n - 1) return;
    const int lvl = common_levels(keys[p], keys[p + 1]);
    const int s = cell_first(keys, p, lvl);
    atomicOr(&mask[s], 1u << lvl);
}

// Tile sums for the 3-phase scans.  Kind 0: popcount(mask) -> cellcnt.
// Kind 1: sorted coordinates (double-double) -> pdd.
__global__ __launch_bounds__(kScanThreads) void count_tile_kernel(int n, const unsigned *__restrict__ mask,
                                                                  int *part) {
    __shared__ int ws[16];
    const int p0 = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (p0 + q < n) s += __popc(mask[p0 + q]);
    int total;
    (void)block_excl_scan(s, ws, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void count_apply_kernel(int n, const unsigned *__restrict__ mask,
                                                                   const int *__restrict__ part,
                                                                   int *cellcnt) {
    __shared__ int ws[16];
    const int p0 = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (p0 + q < n) ? __popc(mask[p0 + q]) : 0;
        s += v[q];
    }
    int total;
    int pre = block_excl_scan(s, ws, &total) + part[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (p0 + q < n) cellcnt[p0 + q] = pre;
        pre += v[q];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) cellcnt[n] = pre;
}

// Double-double block scan helpers (x and y together).
struct dd2 {
    dd x, y;
};
__device__ __forceinline__ dd2 dd2_add(dd2 a, dd2 b) { return dd2{dd_add(a.x, b.x), dd_add(a.y, b.y)}; }

// Exclusive scan of dd2 over the block via LDS (Hillis-Steele on wave totals).
__device__ dd2 block_excl_scan_dd2(dd2 v, dd2 *ws, dd2 *total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    dd2 inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        dd2 t;
        t.x.hi = __shfl_up(inc.x.hi, o, kWave);
        t.x.lo = __shfl_up(inc.x.lo, o, kWave);
        t.y.hi = __shfl_up(inc.y.hi, o, kWave);
        t.y.lo = __shfl_up(inc.y.lo, o, kWave);
        if (lane >= o) inc = dd2_add(t, inc);
    }
    if (lane == kWave - 1) ws[w] = inc;
    __syncthreads();
    dd2 base{{0, 0}, {0, 0}}, tot{{0, 0}, {0, 0}};
    for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
        if (q < w) base = dd2_add(base, ws[q]);
        tot = dd2_add(tot, ws[q]);
    }
    __syncthreads();
    *total = tot;
    // exclusive = base + (inc - v): recompute as base + exclusive lane prefix
    dd2 ex;
    ex.x.hi = __shfl_up(inc.x.hi, 1, kWave);
    ex.x.lo = __shfl_up(inc.x.lo, 1, kWave);
    ex.y.hi = __shfl_up(inc.y.hi, 1, kWave);
    ex.y.lo = __shfl_up(inc.y.lo, 1, kWave);
    if (lane == 0) ex = dd2{{0, 0}, {0, 0}};
    return dd2_add(base, ex);
}

__global__ __launch_bounds__(kScanThreads) void coord_tile_kernel(int n, const int *__restrict__ order,
                                                                  const float2 *__restrict__ pos,
                                                                  double *part) {
    __shared__ dd2 ws[16];
    const int p0 = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    dd2 s{{0, 0}, {0, 0}};
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (p0 + q < n) {
            const int v = order[p0 + q];
            const float2 c = pos[v];
            s = dd2_add(s, dd2{{(double)c.x, 0}, {(double)c.y, 0}});
        }
    dd2 total;
    (void)block_excl_scan_dd2(s, ws, &total);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = total.x.hi;
        part[4 * blockIdx.x + 1] = total.x.lo;
        part[4 * blockIdx.x + 2] = total.y.hi;
        part[4 * blockIdx.x + 3] = total.y.lo;
    }
}

__global__ void coord_part_scan_kernel(int blocks, double *part) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    dd2 run{{0, 0}, {0, 0}};
    for (int b = 0; b < blocks; ++b) {
        dd2 v{{part[4 * b], part[4 * b + 1]}, {part[4 * b + 2], part[4 * b + 3]}};
        part[4 * b + 0] = run.x.hi;
        part[4 * b + 1] = run.x.lo;
        part[4 * b + 2] = run.y.hi;
        part[4 * b + 3] = run.y.lo;
        run = dd2_add(run, v);
    }
}

// pdd layout: [4][n+1] -> xhi, xlo, yhi, ylo;  pdd[.][p] = sum of sorted coords < p.
__global__ __launch_bounds__(kScanThreads) void coord_apply_kernel(int n, const int *__restrict__ order,
                                                                   const float2 *__restrict__ pos,
                                                                   const double *__restrict__ part,
                                                                   double *pdd) {
    __shared__ dd2 ws[16];
    const int p0 = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    dd2 v[kScanItems];
    dd2 s{{0, 0}, {0, 0}};
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = dd2{{0, 0}, {0, 0}};
        if (p0 + q < n) {
            const int id = order[p0 + q];
            const float2 c = pos[id];
            v[q] = dd2{{(double)c.x, 0}, {(double)c.y, 0}};
        }
        s = dd2_add(s, v[q]);
    }
    dd2 total;
    dd2 pre = block_excl_scan_dd2(s, ws, &total);
    const dd2 off{{part[4 * blockIdx.x], part[4 * blockIdx.x + 1]},
                  {part[4 * blockIdx.x + 2], part[4 * blockIdx.x + 3]}};
    pre = dd2_add(off, pre);
    const size_t N1 = (size_t)n + 1;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (p0 + q < n) {
            pdd[0 * N1 + p0 + q] = pre.x.hi;
            pdd[1 * N1 + p0 + q] = pre.x.lo;
            pdd[2 * N1 + p0 + q] = pre.y.hi;
            pdd[3 * N1 + p0 + q] = pre.y.lo;
        }
        pre = dd2_add(pre, v[q]);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        pdd[0 * N1 + n] = pre.x.hi;
        pdd[1 * N1 + n] = pre.x.lo;
        pdd[2 * N1 + n] = pre.y.hi;
        pdd[3 * N1 + n] = pre.y.lo;
    }
}

// Nodes in DFS pre-order.  Cells starting at sorted position p come right
// before leaf p, shallower first; a cell's subtree ends where the nodes of
// its last position + 1 begin, which gives the skip link.
__global__ void emit_kernel(int n, const unsigned *__restrict__ keys, const int *__restrict__ order,
                            const unsigned *__restrict__ mask, const int *__restrict__ cellcnt,
                            const double *__restrict__ pdd, const float2 *__restrict__ pos,
                            const float *__restrict__ bbox,
                            float4 *__restrict__ nodeA, int2 *__restrict__ nodeB,
                            int *__restrict__ leafpos, int *nnodes) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const size_t N1 = (size_t)n + 1;
    const float W = bbox[2];
    unsigned m = mask[p];
    int v = p + cellcnt[p];
    while (m) {
        const int lvl = __ffs(m) - 1;
        m &= m - 1;
        const int e = cell_last(keys, n, p, lvl);
        const int cnt = e - p + 1;
        const int skip = (e + 1) + cellcnt[e + 1];
        const dd sx = dd_add(dd{pdd[0 * N1 + e + 1], pdd[1 * N1 + e + 1]},
                             dd_neg(dd{pdd[0 * N1 + p], pdd[1 * N1 + p]}));
        const dd sy = dd_add(dd{pdd[2 * N1 + e + 1], pdd[3 * N1 + e + 1]},
                             dd_neg(dd{pdd[2 * N1 + p], pdd[3 * N1 + p]}));
        const double cx = (sx.hi + sx.lo) / (double)cnt;
        const double cy = (sy.hi + sy.lo) / (double)cnt;
        float side2;
        if (lvl == 16) {
            // A bucket (equal keys) may sit at the bottom of a chain of
            // single-child cells; any cell of that chain can be accepted with
            // the same centroid, and the deepest (level 15) is the easiest
            // to accept.  If its level-15 cell holds other points the bucket
            // is never accepted, only opened.
            const bool chain = (p == 0 || common_levels(keys[p - 1], keys[p]) < 15) &&
                               (e == n - 1 || common_levels(keys[e], keys[e + 1]) < 15);
            const float side15 = ldexpf(W, -15);
            side2 = chain ? side15 * side15 : __builtin_inff();
        } else {
            const float side = ldexpf(W, -lvl);
            side2 = side * side;
        }
        nodeA[v] = float4{(float)cx, (float)cy, side2, (float)cnt};
        nodeB[v] = int2{skip, -1};
        ++v;
    }
    const int vert = order[p];
    const float2 pv = pos[vert];
    nodeA[v] = float4{pv.x, pv.y, 0.f, 1.f};
    nodeB[v] = int2{v + 1, vert};
    leafpos[vert] = v;
    if (p == n - 1) *nnodes = v + 1;
}

// --------------------------------------------------------------- walks
struct WalkArgs {
    int n, BS;
    const int *total;       // node count, written by emit_kernel
    const float4 *nodeA;
    const int2 *nodeB;
    const int *leafpos;
    float theta2, negRK2, invK;
};

// Repulsion kernel term (c_j - c_i)/|c_j - c_i|^2 times `mult`, compensated.
__device__ __forceinline__ void rep_add(float dx, float dy, float mult, float &sx, float &cx,
                                        float &sy, float &cy) {
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
    const float inv = __builtin_amdgcn_rcpf(d2) * mult;
    kahan_add(sx, cx, dx * inv);
    kahan_add(sy, cy, dy * inv);
}

// Walk of the tree for vertex i in pre-order with skip links (Alg. S2 order).
// live == nullptr: far-field mode -- leaves of vertices j with id < late_below
// (already moved this iteration) are appended to late[] instead of summed.
// live != nullptr: every leaf uses live coordinates.
__device__ int bh_walk(const WalkArgs &a, int i, float xi, float yi, int late_below,
                       const float2 *live, float4 &acc, int *late, int &nlate, int cap) {
    const int Li = a.leafpos[i];
    const int total = *a.total;
    float sx = 0.f, cx = 0.f, sy = 0.f, cy = 0.f;
    int visits = 0;
    int v = 0;
    while (v < total) {
        const float4 A = a.nodeA[v];
        const int2 B = a.nodeB[v];
        ++visits;
        if (B.y >= 0) {
            const int j = B.y;
            if (j != i) {
                if (live) {
                    const float2 pj = live[j];
                    rep_add(pj.x - xi, pj.y - yi, 1.f, sx, cx, sy, cy);
                } else if (j < late_below) {
                    if (nlate < cap) late[nlate] = j;
                    ++nlate;
                } else {
                    rep_add(A.x - xi, A.y - yi, 1.f, sx, cx, sy, cy);
                }
            }
            ++v;
        } else if (v <= Li && Li < B.x) {
            ++v;   // the cell holds i: always opened
        } else {
            const float dx = A.x - xi, dy = A.y - yi;
            const float d2 = dx * dx + dy * dy;
            if (A.z < a.theta2 * d2) {
                rep_add(dx, dy, A.w, sx, cx, sy, cy);
                v = B.x;
            } else {
                ++v;
            }
        }
    }
    acc = float4{sx, sy, cx, cy};
    return visits;
}

__global__ __launch_bounds__(256) void far_kernel(WalkArgs a, const int *__restrict__ order,
                                                  const float2 *__restrict__ pos, int all_live,
                                                  int snapshot_leaves, float4 *__restrict__ far,
                                                  int *__restrict__ late_cnt,
                                                  int *__restrict__ late_ids, Counters *ctr) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    int visits = 0, ovf = 0;
    if (p < a.n) {
        const int i = order[p];
        const int late_below = snapshot_leaves ? 0 : (all_live ? a.n : (i / a.BS) * a.BS);
        float4 acc;
        int nlate = 0;
        const float2 pi = pos[i];
        visits = bh_walk(a, i, pi.x, pi.y, late_below, nullptr, acc,
                         late_ids + (size_t)i * kLateCap, nlate, kLateCap);
        far[i] = acc;
        late_cnt[i] = nlate;
        ovf = nlate > kLateCap;
    }
    unsigned long long vs = wave_sum((unsigned long long)visits);
    unsigned long long os = wave_sum((unsigned long long)ovf);
    unsigned long long ls = wave_sum((unsigned long long)(p < a.n ? min(late_cnt[order[p]], kLateCap) : 0));
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (vs) atomicAdd(&ctr->visits, vs);
        if (os) atomicAdd(&ctr->late_overflow, os);
        if (ls) atomicAdd(&ctr->late_total, ls);
    }
}

// ------------------------------------------------------- early attraction
// Neighbours j in batches >= batch(i) have not moved when batch(i) comes up,
// so their attraction terms (Sec. 2.2, a = 2: d * delta / K) can be summed
// for all vertices at once from the snapshot.  Sorted CSR rows make the moved
// ("late") neighbours a prefix of each row; its length is fixed per graph.
constexpr int kHeavyRow = 256;   // early entries above which a whole workgroup sums the row

__global__ void late_prefix_kernel(int n, int BS, const int *__restrict__ rowptr,
                                   const int *__restrict__ colidx, int *__restrict__ late_att,
                                   int *__restrict__ heavy, int *__restrict__ nheavy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bstart = (i / BS) * BS;
    int lo = rowptr[i], hi = rowptr[i + 1];   // first entry with colidx >= bstart
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (colidx[mid] < bstart) lo = mid + 1;
        else hi = mid;
    }
    late_att[i] = lo - rowptr[i];
    if (end - lo > kHeavyRow) heavy[atomicAdd(nheavy, 1)] = i;
}

// Light rows: 8 lanes per row.
__global__ __launch_bounds__(256) void att_early_kernel(int n, float invK, const int *__restrict__ rowptr,
                                                        const int *__restrict__ colidx,
                                                        const int *__restrict__ late_att,
                                                        const float2 *__restrict__ pos,
                                                        float2 *__restrict__ atte) {
    const int g8 = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    const int i = g8;
    if (i >= n) return;
    const int e0 = rowptr[i] + late_att[i], e1 = rowptr[i + 1];
    if (e1 - e0 > kHeavyRow) return;     // summed by att_heavy_kernel
    const float2 pi = pos[i];
    const float xi = pi.x, yi = pi.y;
    float ax = 0.f, ay = 0.f;
    for (int e = e0 + sub; e < e1; e += 8) {
        const float2 pj = pos[colidx[e]];
        const float dx = pj.x - xi, dy = pj.y - yi;
        const float d = sqrtf(dx * dx + dy * dy) * invK;
        ax = fmaf(d, dx, ax);
        ay = fmaf(d, dy, ay);
    }
    ax = group_sum<8>(ax);
    ay = group_sum<8>(ay);
    if (sub == 0) atte[i] = float2{ax, ay};
}

// Heavy rows: one workgroup per row, reduced in a fixed order.
__global__ __launch_bounds__(256) void att_heavy_kernel(const int *__restrict__ heavy, const int *__restrict__ nheavy,
                                                        float invK, const int *__restrict__ rowptr,
                                                        const int *__restrict__ colidx,
                                                        const int *__restrict__ late_att,
                                                        const float2 *__restrict__ pos,
                                                        float2 *__restrict__ atte) {
    __shared__ float wsx[4], wsy[4];
    for (int h = blockIdx.x; h < *nheavy; h += gridDim.x) {
        const int i = heavy[h];
        const int e0 = rowptr[i] + late_att[i], e1 = rowptr[i + 1];
        const float2 pi = pos[i];
        const float xi = pi.x, yi = pi.y;
        float ax = 0.f, ay = 0.f;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
            const float2 pj = pos[colidx[e]];
            const float dx = pj.x - xi, dy = pj.y - yi;
            const float d = sqrtf(dx * dx + dy * dy) * invK;
            ax = fmaf(d, dx, ax);
            ay = fmaf(d, dy, ay);
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            wsx[threadIdx.x / kWave] = ax;
            wsy[threadIdx.x / kWave] = ay;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            atte[i] = float2{((wsx[0] + wsx[1]) + wsx[2]) + wsx[3], ((wsy[0] + wsy[1]) + wsy[2]) + wsy[3]};
        __syncthreads();
    }
}

// ---------------------------------------------------------------- chain
// ------------------------------------------------------- late entry lists
// Everything a minibatch step needs that does not depend on moves is laid out
// before the chain starts: per batch, the "late" entries -- moved neighbours
// (the CSR prefix) and listed moved leaves -- of all its rows, row by row, as
// (row in batch << 32 | vertex) words, plus each row's offset in that list.
constexpr int kMaxChainRows = 2048;   // batch-size limit of the Barnes-Hut chain
constexpr int kEnt = 8;               // late entries per thread per pass (held in registers)

__device__ __forceinline__ int late_leaf_count(int lc) { return lc > kLateCap ? 0 : lc; }

// Per batch: entry counts of its rows -> exclusive offsets within the batch.
__global__ __launch_bounds__(1024) void batch_offsets_kernel(int n, int BS, const int *__restrict__ late_att,
                                                              const int *__restrict__ rowptr,
                                                              const int *__restrict__ late_cnt,
                                                              int all_late, int *__restrict__ roff,
                                                              int *__restrict__ btot) {
    __shared__ int ws[16];
    const int b = blockIdx.x;
    const int R = min(BS, n - b * BS);
    int carry = 0;
    for (int r0 = 0; r0 < R; r0 += 1024) {
        const int r = r0 + (int)threadIdx.x;
        int c = 0;
        if (r < R) {
            const int i = b * BS + r;
            const int la = all_late ? rowptr[i + 1] - rowptr[i] : late_att[i];
            c = la + late_leaf_count(late_cnt[i]);
        }
        int tot;
        const int off = block_excl_scan(c, ws, &tot);
        if (r < R) roff[b * BS + r] = carry + off;
        carry += tot;
    }
    if (threadIdx.x == 0) btot[b] = carry;
}

// 8 lanes per row copy its late entries into the batch list; listed leaves
// (repulsion terms) carry bit 31 of the vertex word, moved neighbours
// (attraction terms) do not.
__global__ __launch_bounds__(256) void late_fill_kernel(int n, int BS, const int *__restrict__ late_att,
                                                        const int *__restrict__ rowptr,
                                                        const int *__restrict__ colidx,
                                                        const int *__restrict__ late_cnt,
                                                        const int *__restrict__ late_ids, int all_late,
                                                        const int *__restrict__ roff,
                                                        const int *__restrict__ bbase,
                                                        unsigned long long *__restrict__ ent) {
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    if (i >= n) return;
    const int b = i / BS;
    const unsigned long long rbits = (unsigned long long)(i - b * BS) << 32;
    const size_t base = (size_t)bbase[b] + roff[i];
    const int rs = rowptr[i];
    const int la = all_late ? rowptr[i + 1] - rs : late_att[i];
    for (int k = sub; k < la; k += 8) ent[base + k] = rbits | (unsigned)colidx[rs + k];
    const int ll = late_leaf_count(late_cnt[i]);
    const int *lid = late_ids + (size_t)i * kLateCap;
    for (int k = sub; k < ll; k += 8) ent[base + la + k] = rbits | 0x80000000u | (unsigned)lid[k];
}

// ---------------------------------------------------------------- chain
struct ChainArgs {
    WalkArgs w;
    int nb_run;          // batches to process with updates
    int stop_batch;      // batch whose forces go to fout without update (-1: none)
    int first_batch;     // usually 0; the force call processes only `stop_batch`
    float2 *pos;
    const float4 *far;
    const float2 *atte;  // early attraction (NULL: none)
    const int *late_cnt;
    const int *roff;     // [n] offset of each row's entries in its batch list
    const int *bbase;    // [nb+1] start of each batch list in ent
    const unsigned long long *ent;
    size_t ent_cap;      // entries allocated in ent
    double *fout;        // [2*BS]
    double *energy_k;
    Counters *ctr;
    float step;
};

// Per-row data of a step, requested one step ahead.  Loads are unconditional
// with clamped indices so that a step's prefetch is straight-line code.
struct ChainRow {
    int o0, o1;          // entry range of the row in its batch list
    int ovf;             // late-leaf list overflowed: walk the whole tree live
    float x, y;
    float4 far;
    float2 atte;
};

__device__ __forceinline__ ChainRow chain_row(const ChainArgs &a, int b, int r, int R) {
    ChainRow d;
    const int rc = min(r, R - 1);
    const int i = b * a.w.BS + rc;
    const int E = a.bbase[b + 1] - a.bbase[b];
    d.o0 = a.roff[i];
    const int nxt = a.roff[min(i + 1, a.w.n - 1)];
    d.o1 = (rc + 1 < R) ? nxt : E;
    d.ovf = a.late_cnt[i] > kLateCap;
    const float2 pi = a.pos[i];
    d.x = pi.x;
    d.y = pi.y;
    d.far = a.far[i];
    d.atte = a.atte ? a.atte[i] : float2{0.f, 0.f};
    return d;
}

struct ChainShared {
    int off[2][kMaxChainRows + 1];
    float px[2][kMaxChainRows];
    float py[2][kMaxChainRows];
    float2 sum[kMaxChainRows];   // rows complete inside one thread's run
    float2 cf[kChainThreads];    // first (partial) row of each thread's run
    float2 cl[kChainThreads];    // last (partial) row of each thread's run
    double wsd[16];
};

// The minibatch chain: one workgroup walks the batches in order.  Per step b:
//   - each thread gathers the live positions of the first late entries of its
//     run (entry words were loaded one step ahead), then requests the next
//     step's row data and entry words (they do not depend on this step's
//     moves; issued after the gathers so that waiting for the gathers does
//     not wait for them), then sums its run row by row;
//   - rows cut by thread boundaries are completed from per-thread carries in
//     thread order; early attraction and the far field are added, and the
//     thread owning the row moves it (Alg. 2 update loop; Jacobi within the
//     batch because every gather of the batch precedes the barrier).
__global__ __launch_bounds__(kChainThreads) void chain_kernel(ChainArgs a) {
    __shared__ ChainShared S;
    const int tid = threadIdx.x;
    const int BS = a.w.BS, n = a.w.n;
    const int last = a.stop_batch >= 0 ? a.stop_batch : a.nb_run - 1;
    const float invK = a.w.invK, negRK2 = a.w.negRK2;
    constexpr int RPT = kMaxChainRows / kChainThreads;   // rows per thread
    const size_t entmax = a.ent_cap - 1;

    ChainRow rowd[RPT];
    unsigned long long pe[kEnt];
    auto fetch_regs = [&](int b) {
        const int R = min(BS, n - b * BS);
#pragma unroll
        for (int k = 0; k < RPT; ++k)
            if (tid + k * kChainThreads < R) rowd[k] = chain_row(a, b, tid + k * kChainThreads, R);
        const int E = a.bbase[b + 1] - a.bbase[b];
        const int chunk = (E + kChainThreads - 1) / kChainThreads;
        const int e0 = min(tid * chunk, E), e1 = min(e0 + chunk, E);
        const size_t gb = (size_t)a.bbase[b];
#pragma unroll
        for (int q = 0; q < kEnt; ++q)
            if (e0 + q < e1) pe[q] = a.ent[min(gb + (size_t)(e0 + q), entmax)];
    };
    auto fetch_lds = [&](int b, int slot) {
        const int R = min(BS, n - b * BS);
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int r = tid + k * kChainThreads;
            if (r < R) {
                S.off[slot][r] = rowd[k].o0;
                S.px[slot][r] = rowd[k].x;
                S.py[slot][r] = rowd[k].y;
            }
        }
        if (tid == 0) S.off[slot][R] = a.bbase[b + 1] - a.bbase[b];
    };
    if (a.first_batch <= last) {
        fetch_regs(a.first_batch);
        fetch_lds(a.first_batch, a.first_batch & 1);
    }
    __syncthreads();

    double e_iter = 0.0;
    unsigned long long bad = 0;
    for (int b = a.first_batch; b <= last; ++b) {
        const int slot = b & 1;
        const int R = min(BS, n - b * BS);
        const int E = S.off[slot][R];
        const int chunk = (E + kChainThreads - 1) / kChainThreads;
        const int e0 = min(tid * chunk, E), e1 = min(e0 + chunk, E);
        ChainRow cur[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) cur[k] = rowd[k];
        unsigned long long ce[kEnt];
#pragma unroll
        for (int q = 0; q < kEnt; ++q) ce[q] = pe[q];

        // gathers of the first pass (only real entries: every lane's gather
        // costs a cache-line lookup in this CU's address unit)
        const int m0 = min(kEnt, e1 - e0);
        float xj[kEnt], yj[kEnt];
#pragma unroll
        for (int q = 0; q < kEnt; ++q) {
            xj[q] = 0.f;
            yj[q] = 0.f;
            if (q < m0) {
                const float2 pj = a.pos[(int)((unsigned)ce[q] & 0x7fffffffu)];
                xj[q] = pj.x;
                yj[q] = pj.y;
            }
        }
        // next step's data (clamped to the last batch on the final step)
        fetch_regs(min(b + 1, last));

        if (e0 < e1) {
            const unsigned long long *src = a.ent + a.bbase[b];
            int r = (int)(ce[0] >> 32);
            float ax = 0.f, ay = 0.f;
            bool first = true;
            for (int base = e0; base < e1; base += kEnt) {
                const int m = min(kEnt, e1 - base);
                if (base != e0) {
#pragma unroll
                    for (int q = 0; q < kEnt; ++q)
                        if (q < m) ce[q] = src[base + q];
#pragma unroll
                    for (int q = 0; q < kEnt; ++q) {
                        if (q < m) {
                            const float2 pj = a.pos[(int)((unsigned)ce[q] & 0x7fffffffu)];
                            xj[q] = pj.x;
                            yj[q] = pj.y;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kEnt; ++q) {
                    if (q < m) {
                        const int rq = (int)(ce[q] >> 32);
                        if (rq != r) {
                            const bool full = S.off[slot][r] >= e0 && S.off[slot][r + 1] <= e1;
                            if (full) S.sum[r] = float2{ax, ay};
                            else if (first) S.cf[tid] = float2{ax, ay};
                            else S.cl[tid] = float2{ax, ay};
                            first = false;
                            ax = ay = 0.f;
                            r = rq;
                        }
                        const float dx = xj[q] - S.px[slot][r], dy = yj[q] - S.py[slot][r];
                        if (((unsigned)ce[q] & 0x80000000u) == 0u) {
                            // moved neighbour: attraction d * delta / K
                            const float d = sqrtf(dx * dx + dy * dy) * invK;
                            ax = fmaf(d, dx, ax);
                            ay = fmaf(d, dy, ay);
                        } else {
                            // moved leaf: repulsion -R K^2 delta / d^2
                            const float d2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
                            const float inv = __builtin_amdgcn_rcpf(d2) * negRK2;
                            ax = fmaf(dx, inv, ax);
                            ay = fmaf(dy, inv, ay);
                        }
                    }
                }
            }
            const bool full = S.off[slot][r] >= e0 && S.off[slot][r + 1] <= e1;
            if (full) S.sum[r] = float2{ax, ay};
            else if (first) S.cf[tid] = float2{ax, ay};
            else S.cl[tid] = float2{ax, ay};
        }
        __syncthreads();

        // complete my rows, add early attraction and far field, move them
        const bool stop = (b == a.stop_batch);
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int r = tid + k * kChainThreads;
            if (r >= R) continue;
            const int o0 = cur[k].o0, o1 = cur[k].o1;
            float2 sm{0.f, 0.f};
            if (o1 > o0) {
                const int t0 = o0 / chunk, t1 = (o1 - 1) / chunk;
                if (t0 == t1) {
                    sm = S.sum[r];
                } else {
                    sm = (o0 == t0 * chunk) ? S.cf[t0] : S.cl[t0];
                    for (int t = t0 + 1; t <= t1; ++t) {
                        sm.x += S.cf[t].x;
                        sm.y += S.cf[t].y;
                    }
                }
            }
            const int i = b * BS + r;
            float4 fr = cur[k].far;
            if (cur[k].ovf) {
                int dummy = 0;
                (void)bh_walk(a.w, i, cur[k].x, cur[k].y, 0, a.pos, fr, nullptr, dummy, 0);
            }
            const float fx = (sm.x + cur[k].atte.x) + negRK2 * (fr.x - fr.z);
            const float fy = (sm.y + cur[k].atte.y) + negRK2 * (fr.y - fr.w);
            if (stop) {
                a.fout[2 * r] = (double)fx;
                a.fout[2 * r + 1] = (double)fy;
                continue;
            }
            const double f2 = (double)fx * fx + (double)fy * fy;
            if (!isfinite(f2)) {
                ++bad;
                continue;
            }
            e_iter += f2;
            if (f2 > 0.0) {
                const float sc = a.step / sqrtf(fx * fx + fy * fy);
                a.pos[i] = float2{cur[k].x + sc * fx, cur[k].y + sc * fy};
            }
        }
        if (b + 1 <= last) fetch_lds(b + 1, slot ^ 1);
        __syncthreads();
    }
    if (bad) atomicAdd(&a.ctr->nonfinite, bad);
    const double e = block_sum_fixed(e_iter, S.wsd);
    if (tid == 0 && a.energy_k) *a.energy_k = e;
}

// ------------------------------------------------------------- host side
int build_tree(bl_graph *g, const float2 *sp) {
    BHBuffers &h = g->bh;
    const int n = g->n;
    hipStream_t s = g->stream;
    int slot;
    BL_TRY(prof_begin(g, PK_TREE, &slot));
    hipLaunchKernelGGL(bbox_kernel, dim3(kBBoxBlocks), dim3(256), 0, s, n, sp, h.bbox_part,
                       (unsigned *)(h.bbox + 8), h.bbox);
    hipLaunchKernelGGL(morton_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, sp, h.bbox,
                       h.key[0], h.val[0]);
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(radix_hist_kernel, dim3(h.tiles), dim3(kSortThreads), 0, s, h.key[cur], n,
                           shift, h.hist, h.tiles);
        hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kScanThreads), 0, s, h.hist, 256 * h.tiles);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(h.tiles), dim3(kSortThreads), 0, s, h.key[cur],
                           h.val[cur], h.key[cur ^ 1], h.val[cur ^ 1], n, shift, h.hist, h.tiles);
        cur ^= 1;
    }
    // after 4 passes the sorted data is back in buffer 0
    const unsigned *keys = h.key[0];
    const int *order = h.val[0];
    BL_HIP(hipMemsetAsync(h.mask, 0, sizeof(unsigned) * n, s));
    if (n > 1) hipLaunchKernelGGL(mark_kernel, dim3((n - 1 + 255) / 256), dim3(256), 0, s, n, keys, h.mask);
    const int sblocks = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(count_tile_kernel, dim3(sblocks), dim3(kScanThreads), 0, s, n, h.mask, h.scan_part);
    hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kScanThreads), 0, s, h.scan_part, sblocks);
    hipLaunchKernelGGL(count_apply_kernel, dim3(sblocks), dim3(kScanThreads), 0, s, n, h.mask, h.scan_part,
                       h.cellcnt);
    hipLaunchKernelGGL(coord_tile_kernel, dim3(sblocks), dim3(kScanThreads), 0, s, n, order, sp, h.pdd_part);
    hipLaunchKernelGGL(coord_part_scan_kernel, dim3(1), dim3(64), 0, s, sblocks, h.pdd_part);
    hipLaunchKernelGGL(coord_apply_kernel, dim3(sblocks), dim3(kScanThreads), 0, s, n, order, sp,
                       h.pdd_part, h.pdd);
    hipLaunchKernelGGL(emit_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, keys, order, h.mask,
                       h.cellcnt, h.pdd, sp, h.bbox, h.nodeA, h.nodeB, h.leafpos, h.nnodes);
    BL_HIP(hipGetLastError());
    return prof_end(g, slot);
}

WalkArgs walk_args(bl_graph *g) {
    WalkArgs w;
    w.n = g->n;
    w.BS = g->p.batch_size;
    w.total = g->bh.nnodes;
    w.nodeA = g->bh.nodeA;
    w.nodeB = g->bh.nodeB;
    w.leafpos = g->bh.leafpos;
    w.theta2 = (float)(g->p.theta * g->p.theta);
    w.negRK2 = (float)(-g->p.R * g->p.K * g->p.K);
    w.invK = (float)(1.0 / g->p.K);
    return w;
}

// Moved-neighbour prefix lengths (once per job) and the early attraction.
int early_pass(bl_graph *g) {
    BHBuffers &h = g->bh;
    const int n = g->n;
    if (!h.prefix_ready) {
        BL_HIP(hipMemsetAsync(h.nheavy, 0, sizeof(int), g->stream));
        hipLaunchKernelGGL(late_prefix_kernel, dim3((n + 255) / 256), dim3(256), 0, g->stream, n,
                           g->p.batch_size, g->rowptr, g->colidx, h.late_att, h.heavy, h.nheavy);
        BL_HIP(hipGetLastError());
        h.prefix_ready = true;
    }
    const float invK = (float)(1.0 / g->p.K);
    hipLaunchKernelGGL(att_early_kernel, dim3((n + 31) / 32), dim3(256), 0, g->stream, n, invK, g->rowptr,
                       g->colidx, h.late_att, (const float2 *)g->x, h.atte);
    hipLaunchKernelGGL(att_heavy_kernel, dim3(256), dim3(256), 0, g->stream, h.heavy, h.nheavy, invK,
                       g->rowptr, g->colidx, h.late_att, (const float2 *)g->x, h.atte);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

// Far-field walks of all vertices; (px, py) are the vertices' own positions.
int far_pass(bl_graph *g, const WalkArgs &w, const float2 *pp, int all_live) {
    const int snap = (g->p.flags & BL_BH_SNAPSHOT_LEAVES) ? 1 : 0;
    int slot;
    BL_TRY(prof_begin(g, PK_FAR, &slot));
    hipLaunchKernelGGL(far_kernel, dim3((g->n + 255) / 256), dim3(256), 0, g->stream, w, g->bh.val[0], pp,
                       all_live, snap && !all_live, g->bh.far, g->bh.late_cnt, g->bh.late_ids, g->counters);
    BL_HIP(hipGetLastError());
    return prof_end(g, slot);
}

// Late entry lists of all batches (needs the far pass's late-leaf counts).
int late_lists(bl_graph *g, bool all_late) {
    BHBuffers &h = g->bh;
    const int n = g->n, BS = g->p.batch_size, nb = g->nb;
    hipLaunchKernelGGL(batch_offsets_kernel, dim3(nb), dim3(1024), 0, g->stream, n, BS, h.late_att, g->rowptr,
                       h.late_cnt, all_late ? 1 : 0, h.roff, h.bbase);
    BL_HIP(hipMemsetAsync(h.bbase + nb, 0, sizeof(int), g->stream));
    hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kScanThreads), 0, g->stream, h.bbase, nb + 1);
    hipLaunchKernelGGL(late_fill_kernel, dim3((n + 31) / 32), dim3(256), 0, g->stream, n, BS, h.late_att,
                       g->rowptr, g->colidx, h.late_cnt, h.late_ids, all_late ? 1 : 0, h.roff, h.bbase,
                       h.ent);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

int chain(bl_graph *g, const WalkArgs &w, int first_batch, int nb_run, int stop_batch, int k,
          double *energy_k, bool early) {
    ChainArgs a;
    a.w = w;
    a.nb_run = nb_run;
    a.stop_batch = stop_batch;
    a.first_batch = first_batch;
    a.pos = (float2 *)g->x;
    a.far = g->bh.far;
    a.atte = early ? g->bh.atte : nullptr;
    a.late_cnt = g->bh.late_cnt;
    a.roff = g->bh.roff;
    a.bbase = g->bh.bbase;
    a.ent = g->bh.ent;
    a.ent_cap = (size_t)g->nnz + (size_t)g->n * kLateCap;
    a.fout = g->fout;
    a.energy_k = energy_k;
    a.ctr = g->counters;
    a.step = (float)step_at(g->p, k);
    int slot;
    BL_TRY(prof_begin(g, PK_CHAIN, &slot));
    hipLaunchKernelGGL(chain_kernel, dim3(1), dim3(kChainThreads), 0, g->stream, a);
    BL_HIP(hipGetLastError());
    return prof_end(g, slot);
}

}  // namespace

size_t bh_footprint(int n) {
    const size_t N = (size_t)n;
    const size_t tiles = (N + kSortTile - 1) / kSortTile;
    const size_t sblocks = (N + kScanTile - 1) / kScanTile;
    return 64 + 16 * kBBoxBlocks + 16 * N + 4 * 256 * tiles + 4 * N + 4 * (N + 1) + 4 * (sblocks + 1) +
           32 * (N + 1) + 32 * (sblocks + 1) + 2 * N * (16 + 8) + 4 * N + 16 + 16 * N + 4 * N +
           4 * N * kLateCap + 8 * N + 8 * 1024 + 16 * N + 16 + 4 * N + 4 * N + 8 * N * kLateCap;
}

int bh_alloc(bl_graph *g) {
    BHBuffers &h = g->bh;
    const size_t N = (size_t)g->n;
    h.tiles = (int)((N + kSortTile - 1) / kSortTile);
    const size_t sblocks = (N + kScanTile - 1) / kScanTile;
    BL_TRY(graph_alloc(g, (void **)&h.bbox, 64));
    BL_TRY(graph_alloc(g, (void **)&h.bbox_part, 16 * kBBoxBlocks));
    for (int q = 0; q < 2; ++q) {
        BL_TRY(graph_alloc(g, (void **)&h.key[q], 4 * N));
        BL_TRY(graph_alloc(g, (void **)&h.val[q], 4 * N));
    }
    BL_TRY(graph_alloc(g, (void **)&h.hist, 4 * 256 * (size_t)h.tiles));
    BL_TRY(graph_alloc(g, (void **)&h.mask, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.cellcnt, 4 * (N + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.scan_part, 4 * (sblocks + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.pdd, 32 * (N + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.pdd_part, 32 * (sblocks + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.nodeA, 16 * 2 * N));
    BL_TRY(graph_alloc(g, (void **)&h.nodeB, 8 * 2 * N));
    BL_TRY(graph_alloc(g, (void **)&h.leafpos, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.nnodes, 16));
    BL_TRY(graph_alloc(g, (void **)&h.far, 16 * N));
    BL_TRY(graph_alloc(g, (void **)&h.late_cnt, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.late_ids, 4 * N * kLateCap));
    BL_TRY(graph_alloc(g, (void **)&h.snap, 8 * N));
    BL_TRY(graph_alloc(g, (void **)&h.fbuf, 8 * (size_t)g->p.batch_size));
    BL_TRY(graph_alloc(g, (void **)&h.late_att, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.heavy, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.nheavy, 16));
    BL_TRY(graph_alloc(g, (void **)&h.atte, 8 * N));
    BL_TRY(graph_alloc(g, (void **)&h.roff, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.bbase, 4 * ((size_t)g->nb + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.ent, 8 * ((size_t)g->nnz + N * kLateCap)));
    h.prefix_ready = false;
    BL_HIP(hipMemsetAsync(h.bbox, 0, 64, g->stream));
    return BL_OK;
}

int bh_run(bl_graph *g, int iters, int start, int stop_batch) {
    const float2 *pos = (const float2 *)g->x;
    for (int t = 0; t < iters; ++t) {
        const int k = start + t;
        const bool last = (t == iters - 1);
        BL_TRY(build_tree(g, pos));
        const WalkArgs w = walk_args(g);
        BL_TRY(far_pass(g, w, pos, 0));
        BL_TRY(early_pass(g));
        BL_TRY(late_lists(g, false));
        const int stop = (last && stop_batch >= 0) ? stop_batch : -1;
        BL_TRY(chain(g, w, 0, stop >= 0 ? stop : g->nb, stop, k, stop >= 0 ? nullptr : g->energy + t, true));
    }
    return BL_OK;
}

// Forces of one batch from coordinates (x, y) with the tree of the snapshot
// (snap_x, snap_y); every leaf uses (x, y).
int bh_forces(bl_graph *g, int batch, const double *snap_x, const double *snap_y) {
    const float2 *sp = (const float2 *)g->x;
    if (snap_x) {
        BL_TRY(convert_to_float2(g, snap_x, snap_y, (float2 *)g->bh.snap));
        sp = (const float2 *)g->bh.snap;
    }
    BL_TRY(build_tree(g, sp));
    const WalkArgs w = walk_args(g);
    BL_TRY(far_pass(g, w, (const float2 *)g->x, 1));
    if (!g->bh.prefix_ready) BL_TRY(early_pass(g));
    BL_TRY(late_lists(g, true));
    return chain(g, w, batch, batch + 1, batch, 0, nullptr, false);
}

}  // namespace bl
