// Barnes-Hut force step (Sec. 3.5; Alg. S1-S3) for gfx950, for one or many
// layout jobs at once.
//
// Every kernel here takes the table of resident jobs and a per-kernel prefix
// of workgroups per job, so one launch serves all jobs: a single graph is the
// one-job case, and a graph's result does not depend on which other jobs
// share the launches.  Per iteration (no host round trip):
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
//   8. att_*_kernel    attraction from neighbours that have not moved yet
//   9. late lists      per batch: the moved neighbours and listed moved leaves,
//                      split into entries that refer to earlier chain segments
//                      ("old") and to the batch's own segment ("recent")
//  10. slot plan       the recent entries laid out one per lane, each row's
//                      run inside one 16-lane DPP row; one record per row
//                      (start position, force apart from recent entries)
//  11. chain_kernel    one launch: per job, one workgroup walks the batches
//                      in order -- the recent entries (the last `lag`
//                      batches) with live coordinates from an LDS ring, then
//                      the batch update (Alg. 2 update loop) -- while helper
//                      workgroups sum the older entries of later batches as
//                      soon as the batches they refer to have moved
#include <algorithm>
#include <cfloat>
#include <cstring>
#include <vector>

#include "bl_device.hpp"
#include "bl_internal.hpp"

namespace bl {

constexpr int kBBoxBlocks = 256;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;     // 2048 keys per tile
constexpr int kScanThreads = 1024;
// Up to this many sort tiles per job, each radix scatter workgroup forms its
// digit offsets from the raw histogram itself (256 x tiles reads), with no
// scan launch in between.
constexpr int kFuseTiles = 128;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;     // 4096 values per tile
constexpr int kChainThreads = 1024;
constexpr int kHeavyRow = 256;        // early entries above which a whole workgroup sums the row
constexpr int kLateHeavyRow = 256;    // moved neighbours above which a whole workgroup copies the row
constexpr int kMaxChainRows = 1024;   // batch-size limit of the Barnes-Hut chain
constexpr int kEnt = 3;               // late entries per thread per pass (held in registers)
constexpr int kMinRun = 1;            // entries per thread at least (packs a step's entries into fewer waves)
// An iteration's chain runs in one launch.  A row's late entries that refer
// to batches more than `lag` batches before its own ("old") are summed by
// helper workgroups of the same launch as soon as the chain has moved those
// batches; the chain gathers only the entries that refer to the last `lag`
// batches ("recent"), from an LDS ring holding the last lag + 1 batches'
// positions (kRing vertices at most).
constexpr int kLag = 14;
constexpr int kRelease = 4;           // the chain copies out and publishes its progress every kRelease steps
constexpr int kMinLag = kRelease + 5; // progress goes out every kRelease steps; old sums are waited for 2 steps ahead
constexpr int kRing = 16384;
constexpr int kHelpers = 32;          // helper workgroups per job, at most
constexpr int kEntH = 8;              // old entries per thread per pass in the helpers
// A batch's old list is cut into parts of whole rows, one helper item each: a
// row belongs to the part whose window of kPartEnt entries holds its first
// entry (so a part holds fewer than kPartEnt entries plus one row).
constexpr int kPartEnt = 4096;
// Per-job progress words of the chain launch: batches moved, helper batches
// claimed, then one ready flag per batch.
constexpr int kSyncMoved = 0, kSyncTicket = 1, kSyncReady = 2;
static_assert(kMaxChainRows <= 1024, "batch_offsets_kernel takes one row per thread");

// Device descriptor of one job (all pointers are device memory).
struct BHJob {
    int n, BS, nb, tiles, sblocks;
    float theta2, negRK2, invK;
    int ka, kr;                 // (a, r) model of Sec. 2.2: attraction d^ka, repulsion d^kr times (c_j - c_i)
    int general;                // 1 unless (a, r) = (2, -1): the kernels' general-model instantiations run it
    int snapshot_leaves;        // leaves use the snapshot (no late lists)
    int all_live;               // one-shot force call: every leaf and neighbour is live
    int first_batch, last_batch, stop_batch;
    int lag;                    // batches whose positions the chain gathers itself (its LDS ring)
    int helpers;                // helper workgroups of the chain launch, at most (set with the job set)
    long long spin_limit;       // polls before a wait of the chain launch gives up
    double step0, decay;
    gptr<int> kiter;            // [2]: current iteration, first iteration of the run
    gptr<const int> rowptr, colidx;
    gptr<float2> pos;           // live coordinates
    gptr<const float2> src;     // coordinates the tree is built from
    gptr<float> bbox, bbox_part;
    gptr<unsigned> ticket;
    gptr<unsigned> key0, key1;
    gptr<int> val0, val1, hist;
    gptr<unsigned> mask;
    gptr<int> cellcnt, scan_part;
    gptr<double> pdd, pdd_part;
    gptr<float4> nodeA;
    gptr<int2> nodeB;
    gptr<int> leafpos, nnodes;
    gptr<float4> far;
    gptr<int> late_cnt, late_ids, late_att, old_att, heavy, nheavy;
    gptr<float2> atte;
    gptr<int> roff, roff_old, bbase, bold;
    gptr<float4> rec;           // per vertex, for the chain: x, y and the force apart from recent entries
    gptr<int2> rmeta;           // per vertex: its recent entries' range [x, y) in its batch's recent list
    gptr<float2> oldf;          // per vertex: the sum of its old entries (helpers -> chain)
    gptr<int> sync;             // [kSyncReady + nb] progress words of the chain launch
    gptr<int> hbase;            // [nb + 1] helper parts per batch, then (scanned) the first part's item
    gptr<int2> hitem;           // helper items: (batch, part)
    gptr<unsigned long long> ent;
    size_t ent_cap;
    gptr<int> pstart;           // per vertex: first slot of its row's run within its batch's slots
    gptr<int> pbase;            // [nb + 1] slot count of each batch, then (scanned) its first slot
    gptr<unsigned long long> slots;   // the batches' slot plans (chain_kernel)
    gptr<int> pflag;            // [nb] batch flags of the slot plan (kFlag*)
    gptr<int4> bmeta;           // [nb] first slot, slot count, recent-list start, batch flags
    gptr<double> energy;        // one value per iteration of the run
    gptr<double> fout;
    Counters *ctr;
    double conv_tol;            // energy stopping rule (0: off)
};

// Workgroup -> (job, workgroup within the job) for one kernel of a launch.
struct JobBlock {
    const BHJob *J;
    int local, nblocks;
};
__device__ __forceinline__ JobBlock job_block(const BHJob *__restrict__ jobs, const int *__restrict__ pre,
                                              int G) {
    const int blk = blockIdx.x;
    int lo = 0, hi = G - 1;   // last job whose first workgroup is <= blk
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return JobBlock{&jobs[lo], blk - pre[lo], pre[lo + 1] - pre[lo]};
}

#define BH_KERNEL_ARGS const BHJob *__restrict__ jobs, const int *__restrict__ pre, int G
// The descriptor is copied into registers: stores through its pointers can
// then not force reloads of its fields.
// (a job whose energy stopping rule has held does nothing more)
#define BH_JOB()                               \
    const JobBlock jb = job_block(jobs, pre, G); \
    const BHJob J = *jb.J;                       \
    if (J.conv_tol > 0 && J.ctr->halted) return

// ------------------------------------------------------------------ bbox
__global__ __launch_bounds__(256) void bbox_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ float s[4][256 / kWave];
    __shared__ int s_last;
    float mnx = FLT_MAX, mny = FLT_MAX, mxx = -FLT_MAX, mxy = -FLT_MAX;
    for (int i = jb.local * 256 + threadIdx.x; i < J.n; i += jb.nblocks * 256) {
        const float2 c = ld<float2>(J.src, i);
        mnx = fminf(mnx, c.x);
        mxx = fmaxf(mxx, c.x);
        mny = fminf(mny, c.y);
        mxy = fmaxf(mxy, c.y);
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
        gptr<float> part = J.bbox_part + 4 * jb.local;
        part[0] = s[0][0];
        part[1] = s[1][0];
        part[2] = s[2][0];
        part[3] = s[3][0];
        __threadfence();
        s_last = (atomicAdd((unsigned *)J.ticket, 1u) == (unsigned)jb.nblocks - 1);
    }
    __syncthreads();
    if (!s_last) return;
    // the last workgroup combines the partial boxes, one per thread
    __threadfence();
    float a = FLT_MAX, b = -FLT_MAX, c = FLT_MAX, d = -FLT_MAX;
    for (int q = threadIdx.x; q < jb.nblocks; q += 256) {
        const float4 v = ld<float4>((gptr<const float4>)J.bbox_part, q);
        a = fminf(a, v.x);
        b = fmaxf(b, v.y);
        c = fminf(c, v.z);
        d = fmaxf(d, v.w);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        a = fminf(a, __shfl_xor(a, o, kWave));
        b = fmaxf(b, __shfl_xor(b, o, kWave));
        c = fminf(c, __shfl_xor(c, o, kWave));
        d = fmaxf(d, __shfl_xor(d, o, kWave));
    }
    __syncthreads();   // s[] was read by thread 0 above
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s[0][w] = a;
        s[1][w] = b;
        s[2][w] = c;
        s[3][w] = d;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 1; q < 256 / kWave; ++q) {
        a = fminf(a, s[0][q]);
        b = fmaxf(b, s[1][q]);
        c = fminf(c, s[2][q]);
        d = fmaxf(d, s[3][q]);
    }
    const float wx = b - a, wy = d - c;
    const float W = fmaxf(wx, wy);
    J.bbox[0] = a;
    J.bbox[1] = c;
    J.bbox[2] = W;
    // 2^16 / W rounded once to float (computed in double: double rounding is
    // innocuous for a quotient of floats since 53 >= 2*24 + 2).
    J.bbox[3] = W > 0.f ? (float)(65536.0 / (double)W) : 0.f;
    *J.ticket = 0u;
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

__global__ void morton_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    const int i = jb.local * blockDim.x + threadIdx.x;
    if (i >= J.n) return;
    const float xmin = J.bbox[0], ymin = J.bbox[1], scale = J.bbox[3];
    unsigned qx = 0, qy = 0;
    if (scale > 0.f) {
        const float2 c = ld<float2>(J.src, i);
        qx = quantise(c.x, xmin, scale);
        qy = quantise(c.y, ymin, scale);
    }
    J.key0[i] = spread16(qx) | (spread16(qy) << 1);
    J.val0[i] = i;
    J.mask[i] = 0u;
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

// Pass `pass` reads buffer pass&1 and writes the other one.
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(BH_KERNEL_ARGS, int pass) {
    BH_JOB();
    __shared__ int h[256];
    gptr<const unsigned> keys = (pass & 1) ? J.key1 : J.key0;
    const int shift = 8 * pass, n = J.n;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int base = jb.local * kSortTile + w * (kSortTile / 4);
    for (int g = 0; g < kSortItems; ++g) {
        const int p = base + g * kWave + lane;
        const bool valid = p < n;
        const unsigned d = valid ? (keys[p] >> shift) & 255u : 0u;
        const unsigned long long m = digit_peers(d, valid);
        if (valid && (__ffsll((long long)m) - 1) == lane) atomicAdd(&h[d], __popcll(m));
    }
    __syncthreads();
    J.hist[threadIdx.x * J.tiles + jb.local] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(BH_KERNEL_ARGS, int pass) {
    BH_JOB();
    __shared__ int cnt[4][256];
    __shared__ int s_ws[kSortThreads / kWave];
    gptr<const unsigned> kin = (pass & 1) ? J.key1 : J.key0;
    gptr<const int> vin = (pass & 1) ? J.val1 : J.val0;
    gptr<unsigned> kout = (pass & 1) ? J.key0 : J.key1;
    gptr<int> vout = (pass & 1) ? J.val0 : J.val1;
    const int shift = 8 * pass, n = J.n, tiles = J.tiles;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int q = threadIdx.x; q < 4 * 256; q += kSortThreads) (&cnt[0][0])[q] = 0;
    __syncthreads();
    const int base = jb.local * kSortTile + w * (kSortTile / 4);
    unsigned k[kSortItems];
    int v[kSortItems];
#pragma unroll
    for (int g = 0; g < kSortItems; ++g) {
        const int p = base + g * kWave + lane;
        k[g] = p < n ? kin[p] : 0u;
        v[g] = p < n ? vin[p] : 0;
    }
    // per-wave digit counts
#pragma unroll
    for (int g = 0; g < kSortItems; ++g) {
        const bool valid = base + g * kWave + lane < n;
        const unsigned d = (k[g] >> shift) & 255u;
        const unsigned long long m = digit_peers(d, valid);
        if (valid && (__ffsll((long long)m) - 1) == lane) cnt[w][d] += __popcll(m);
    }
    __syncthreads();
    // per-wave starting offsets: the tile's base for digit d (keys of lower
    // digits in every tile, then of digit d in earlier tiles), then earlier
    // waves of this tile
    {
        const int d = threadIdx.x;
        int run;
        if (tiles <= kFuseTiles) {   // the raw histogram (job-uniform branch)
            int before = 0, all = 0;
#pragma unroll 8
            for (int t = 0; t < tiles; ++t) {
                const int c = J.hist[d * tiles + t];
                all += c;
                before += t < jb.local ? c : 0;
            }
            int tot;
            run = block_excl_scan(all, s_ws, &tot) + before;
        } else {   // scanned in place by scan_single_kernel
            run = J.hist[d * tiles + jb.local];
        }
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

// Exclusive scan in place by one workgroup per job.  which: 0 radix
// histogram (256 * tiles), 1 cell-count tile sums (sblocks), 2 batch list
// sizes (nb + 1), 3 batch slot counts and helper part counts (nb + 1 each).
__global__ __launch_bounds__(kScanThreads) void scan_single_kernel(BH_KERNEL_ARGS, int which) {
    BH_JOB();
    __shared__ int ws[16];
    auto scan = [&](gptr<int> data, int len) {
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
            int pre_ = block_excl_scan(s, ws, &total) + running;
#pragma unroll
            for (int q = 0; q < kScanItems; ++q) {
                if (p0 + q < len) data[p0 + q] = pre_;
                pre_ += v[q];
            }
            running += total;
        }
    };
    if (which == 0) {
        if (J.tiles > kFuseTiles) scan(J.hist, 256 * J.tiles);   // else the scatter reads it raw
    }
    else if (which == 1) scan(J.scan_part, J.sblocks);
    else if (which == 2) scan(J.bbase, J.nb + 1);
    else {
        scan(J.pbase, J.nb + 1);
        __syncthreads();
        scan(J.hbase, J.nb + 1);
    }
}

// ------------------------------------------------------------ tree cells
__device__ __forceinline__ int common_levels(unsigned a, unsigned b) {
    const unsigned x = a ^ b;
    return x == 0u ? 16 : (__clz(x) >> 1);
}

// Sorted position range [lo, hi] of the level-`lvl` cell holding sorted
// position p (binary searches on the sorted keys).
__device__ __forceinline__ int cell_first(gptr<const unsigned> keys, int p, int lvl) {
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
__device__ __forceinline__ int cell_last(gptr<const unsigned> keys, int n, int p, int lvl) {
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

__global__ void mark_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    const int p = jb.local * blockDim.x + threadIdx.x;
    if (p >= J.n - 1) return;
    gptr<const unsigned> keys = J.key0;
    const int lvl = common_levels(keys[p], keys[p + 1]);
    const int s = cell_first(keys, p, lvl);
    atomicOr((unsigned *)(J.mask + s), 1u << lvl);
}

// Tile sums and apply of the 3-phase scan of popcount(mask) -> cellcnt.
__global__ __launch_bounds__(kScanThreads) void count_tile_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ int ws[16];
    const int p0 = jb.local * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (p0 + q < J.n) s += __popc(J.mask[p0 + q]);
    int total;
    (void)block_excl_scan(s, ws, &total);
    if (threadIdx.x == 0) J.scan_part[jb.local] = total;
}

__global__ __launch_bounds__(kScanThreads) void count_apply_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ int ws[16];
    const int n = J.n;
    const int p0 = jb.local * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (p0 + q < n) ? __popc(J.mask[p0 + q]) : 0;
        s += v[q];
    }
    int total;
    int pre_ = block_excl_scan(s, ws, &total) + J.scan_part[jb.local];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (p0 + q < n) J.cellcnt[p0 + q] = pre_;
        pre_ += v[q];
    }
    if (jb.local == jb.nblocks - 1 && threadIdx.x == kScanThreads - 1) J.cellcnt[n] = pre_;
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

__global__ __launch_bounds__(kScanThreads) void coord_tile_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ dd2 ws[16];
    const int p0 = jb.local * kScanTile + threadIdx.x * kScanItems;
    dd2 s{{0, 0}, {0, 0}};
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (p0 + q < J.n) {
            const float2 c = ld<float2>(J.src, J.val0[p0 + q]);
            s = dd2_add(s, dd2{{(double)c.x, 0}, {(double)c.y, 0}});
        }
    dd2 total;
    (void)block_excl_scan_dd2(s, ws, &total);
    if (threadIdx.x == 0) {
        gptr<double> part = J.pdd_part + 4 * jb.local;
        part[0] = total.x.hi;
        part[1] = total.x.lo;
        part[2] = total.y.hi;
        part[3] = total.y.lo;
    }
}

__global__ void coord_part_scan_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (threadIdx.x != 0) return;
    dd2 run{{0, 0}, {0, 0}};
    gptr<double> part = J.pdd_part;
    for (int b = 0; b < J.sblocks; ++b) {
        dd2 v{{part[4 * b], part[4 * b + 1]}, {part[4 * b + 2], part[4 * b + 3]}};
        part[4 * b + 0] = run.x.hi;
        part[4 * b + 1] = run.x.lo;
        part[4 * b + 2] = run.y.hi;
        part[4 * b + 3] = run.y.lo;
        run = dd2_add(run, v);
    }
}

// pdd layout: [4][n+1] -> xhi, xlo, yhi, ylo;  pdd[.][p] = sum of sorted coords < p.
__global__ __launch_bounds__(kScanThreads) void coord_apply_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ dd2 ws[16];
    const int n = J.n;
    const int p0 = jb.local * kScanTile + threadIdx.x * kScanItems;
    dd2 v[kScanItems];
    dd2 s{{0, 0}, {0, 0}};
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = dd2{{0, 0}, {0, 0}};
        if (p0 + q < n) {
            const float2 c = ld<float2>(J.src, J.val0[p0 + q]);
            v[q] = dd2{{(double)c.x, 0}, {(double)c.y, 0}};
        }
        s = dd2_add(s, v[q]);
    }
    dd2 total;
    dd2 pre_ = block_excl_scan_dd2(s, ws, &total);
    const gptr<double> part = J.pdd_part + 4 * jb.local;
    pre_ = dd2_add(dd2{{part[0], part[1]}, {part[2], part[3]}}, pre_);
    const size_t N1 = (size_t)n + 1;
    gptr<double> pdd = J.pdd;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (p0 + q < n) {
            pdd[0 * N1 + p0 + q] = pre_.x.hi;
            pdd[1 * N1 + p0 + q] = pre_.x.lo;
            pdd[2 * N1 + p0 + q] = pre_.y.hi;
            pdd[3 * N1 + p0 + q] = pre_.y.lo;
        }
        pre_ = dd2_add(pre_, v[q]);
    }
    if (jb.local == jb.nblocks - 1 && threadIdx.x == kScanThreads - 1) {
        pdd[0 * N1 + n] = pre_.x.hi;
        pdd[1 * N1 + n] = pre_.x.lo;
        pdd[2 * N1 + n] = pre_.y.hi;
        pdd[3 * N1 + n] = pre_.y.lo;
    }
}

// Bits of the bfloat16 nearest to f (round to nearest, ties to even), in the
// low 16 bits; f is finite.
__device__ __forceinline__ unsigned bf16_bits(float f) {
    const unsigned u = __builtin_bit_cast(unsigned, f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Nodes in DFS pre-order.  Cells starting at sorted position p come right
// before leaf p, shallower first; a cell's subtree ends where the nodes of
// its last position + 1 begin, which gives the skip link.
__global__ void emit_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    const int n = J.n;
    const int p = jb.local * blockDim.x + threadIdx.x;
    if (p >= n) return;
    gptr<const unsigned> keys = J.key0;
    const size_t N1 = (size_t)n + 1;
    const gptr<double> pdd = J.pdd;
    const float W = J.bbox[2];
    unsigned m = J.mask[p];
    int v = p + J.cellcnt[p];
    while (m) {
        const int lvl = __ffs(m) - 1;
        m &= m - 1;
        const int e = cell_last(keys, n, p, lvl);
        const int cnt = e - p + 1;
        const int skip = (e + 1) + J.cellcnt[e + 1];
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
        // the centroid as hi + lo: with hi = (float)c alone its rounding
        // (half an ulp of the coordinate) would be large next to the
        // distance of a nearby accepted cell; lo = c - hi goes as two
        // bfloat16 in the fourth float, the count as -count in nodeB.y
        const float hx = (float)cx, hy = (float)cy;
        const unsigned lo = bf16_bits((float)(cx - (double)hx)) | (bf16_bits((float)(cy - (double)hy)) << 16);
        st<float4>(J.nodeA, v, float4{hx, hy, side2, __builtin_bit_cast(float, lo)});
        st<int2>(J.nodeB, v, int2{skip, -(int)cnt});
        ++v;
    }
    const int vert = J.val0[p];
    const float2 pv = ld<float2>(J.src, vert);
    st<float4>(J.nodeA, v, float4{pv.x, pv.y, 0.f, 1.f});
    st<int2>(J.nodeB, v, int2{v + 1, vert});
    J.leafpos[vert] = v;
    if (p == n - 1) *J.nnodes = v + 1;
}

// --------------------------------------------------------------- walks
struct WalkArgs {
    int n, BS;
    gptr<const int> total;  // node count, written by emit_kernel
    gptr<const float4> nodeA;
    gptr<const int2> nodeB;
    gptr<const int> leafpos;
    float theta2, negRK2, invK;
    int kr;
};

// Repulsion kernel term (c_j - c_i)/|c_j - c_i|^2 times `mult`, compensated;
// under a general model (GM) the kernel is |c_j - c_i|^kr (c_j - c_i).
template <bool GM>
__device__ __forceinline__ void rep_add(float dx, float dy, float mult, int kr, float &sx, float &cx,
                                        float &sy, float &cy) {
    float inv;
    if constexpr (GM) {
        inv = dpow(dx, dy, kr) * mult;
    } else {
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
        inv = __builtin_amdgcn_rcpf(d2) * mult;
    }
    kahan_add(sx, cx, dx * inv);
    kahan_add(sy, cy, dy * inv);
}

// Walk of the tree for vertex i in pre-order with skip links (Alg. S2 order).
// live == nullptr: far-field mode -- leaves of vertices j with id < late_below
// (already moved this iteration) are appended to late[] instead of summed.
// live != nullptr: every leaf uses live coordinates.
template <bool GM>
__device__ int bh_walk(const WalkArgs &a, int i, float xi, float yi, int late_below,
                       gptr<const float2> live, float4 &acc, gptr<int> late, int &nlate, int cap,
                       int *tests = nullptr) {
    const int Li = a.leafpos[i];
    const int total = *a.total;
    float sx = 0.f, cx = 0.f, sy = 0.f, cy = 0.f;
    int visits = 0, ntest = 0;
    int v = 0;
    while (v < total) {
        const float4 A = ld<float4>(a.nodeA, v);
        const int2 B = ld<int2>(a.nodeB, v);
        ++visits;
        if (B.y >= 0) {
            const int j = B.y;
            if (j != i) {
                if (live) {
                    const float2 pj = ld<float2>(live, j);
                    rep_add<GM>(pj.x - xi, pj.y - yi, 1.f, a.kr, sx, cx, sy, cy);
                } else if (j < late_below) {
                    if (nlate < cap) late[nlate] = j;
                    ++nlate;
                } else {
                    rep_add<GM>(A.x - xi, A.y - yi, 1.f, a.kr, sx, cx, sy, cy);
                }
            }
            ++v;
        } else if (v <= Li && Li < B.x) {
            ++v;   // the cell holds i: always opened
        } else {
            // offset to the centroid hi + lo: (hi - x_i) + lo
            const unsigned lo = __builtin_bit_cast(unsigned, A.w);
            const float lox = __builtin_bit_cast(float, lo << 16), loy = __builtin_bit_cast(float, lo & 0xffff0000u);
            ++ntest;
            const float dx = (A.x - xi) + lox, dy = (A.y - yi) + loy;
            const float d2 = dx * dx + dy * dy;
            if (A.z < a.theta2 * d2) {
                rep_add<GM>(dx, dy, (float)(-B.y), a.kr, sx, cx, sy, cy);
                v = B.x;
            } else {
                ++v;
            }
        }
    }
    acc = float4{sx, sy, cx, cy};
    if (tests) *tests = ntest;
    return visits;
}

__device__ __forceinline__ WalkArgs walk_args(const BHJob &J) {
    WalkArgs w;
    w.n = J.n;
    w.BS = J.BS;
    w.total = J.nnodes;
    w.nodeA = J.nodeA;
    w.nodeB = J.nodeB;
    w.leafpos = J.leafpos;
    w.theta2 = J.theta2;
    w.negRK2 = J.negRK2;
    w.invK = J.invK;
    w.kr = J.kr;
    return w;
}

// GM: this instantiation serves the jobs with J.general == GM (the other
// instantiation's jobs leave at once).
template <bool GM>
__global__ __launch_bounds__(256) void far_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (J.general != (int)GM) return;
    const WalkArgs a = walk_args(J);
    const int p = jb.local * blockDim.x + threadIdx.x;
    int visits = 0, ovf = 0, lat = 0, tests = 0;
    if (p < a.n) {
        const int i = J.val0[p];
        const int late_below = J.snapshot_leaves ? 0 : (J.all_live ? a.n : (i / a.BS) * a.BS);
        float4 acc;
        int nlate = 0;
        const float2 pi = ld<float2>(J.pos, i);
        visits = bh_walk<GM>(a, i, pi.x, pi.y, late_below, nullptr, acc, J.late_ids + (size_t)i * kLateCap, nlate,
                             kLateCap, &tests);
        st<float4>(J.far, i, acc);
        J.late_cnt[i] = nlate;
        ovf = nlate > kLateCap;
        lat = min(nlate, kLateCap);
    }
    unsigned long long vs = wave_sum((unsigned long long)visits);
    unsigned long long os = wave_sum((unsigned long long)ovf);
    unsigned long long ls = wave_sum((unsigned long long)lat);
    unsigned long long ts = wave_sum((unsigned long long)tests);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (vs) atomicAdd(&J.ctr->visits, vs);
        if (ts) atomicAdd(&J.ctr->cell_tests, ts);
        if (os) atomicAdd(&J.ctr->late_overflow, os);
        if (ls) atomicAdd(&J.ctr->late_total, ls);
    }
}

// ------------------------------------------------------- early attraction
// Neighbours j in batches >= batch(i) have not moved when batch(i) comes up,
// so their attraction terms (Sec. 2.2, a = 2: d * delta / K) can be summed
// for all vertices at once from the snapshot.  Sorted CSR rows make the moved
// ("late") neighbours a prefix of each row; its length is fixed per job.
// The first vertex of batch b - lag: entries of batch b that refer to vertices
// below it are "old" (none in one-shot force calls, where nothing moves).
__device__ __forceinline__ int old_limit(const BHJob &J, int b) {
    return J.all_live ? 0 : max(0, b - J.lag) * J.BS;
}
// Where the chain's LDS ring keeps vertex j's position.
__device__ __forceinline__ unsigned ring_index(const BHJob &J, int j) {
    const int bj = j / J.BS;
    return (unsigned)((bj % (J.lag + 1)) * J.BS + (j - bj * J.BS));
}

__global__ void heavy_reset_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (threadIdx.x < 2) J.nheavy[threadIdx.x] = 0;
}

__global__ void late_prefix_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    const int i = jb.local * blockDim.x + threadIdx.x;
    if (i >= J.n) return;
    const int bstart = (i / J.BS) * J.BS;
    int lo = J.rowptr[i], hi = J.rowptr[i + 1];   // first entry with colidx >= bstart
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (J.colidx[mid] < bstart) lo = mid + 1;
        else hi = mid;
    }
    J.late_att[i] = lo - J.rowptr[i];
    const int olim = old_limit(J, i / J.BS);
    int ol = J.rowptr[i], oh = lo;
    while (ol < oh) {
        const int mid = (ol + oh) >> 1;
        if (J.colidx[mid] < olim) ol = mid + 1;
        else oh = mid;
    }
    J.old_att[i] = ol - J.rowptr[i];
    if (end - lo > kHeavyRow) J.heavy[atomicAdd((int *)J.nheavy, 1)] = i;
    if (lo - J.rowptr[i] > kLateHeavyRow) J.heavy[J.n + atomicAdd((int *)(J.nheavy + 1), 1)] = i;
}

// Light rows: 8 lanes per row.
// Attraction terms of one lane's entries e, e + S, e + 2S, ... below e1, in
// that order; U entries' loads are issued before their terms are added.
template <int U, int S, bool GM>
__device__ __forceinline__ void att_run(const BHJob &J, int e, int e1, float2 pi, float invK, float &ax, float &ay) {
    for (; e < e1; e += U * S) {
        int c[U];
        float2 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = e + u * S < e1 ? J.colidx[e + u * S] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) pj[u] = ld<float2>(J.pos, c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c[u] >= 0) {
                const float dx = pj[u].x - pi.x, dy = pj[u].y - pi.y;
                float d;
                if constexpr (GM) d = dpow(dx, dy, J.ka) * invK;   // d^(a-1) / K
                else d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy) * invK;   // hardware sqrt, about 1 ulp
                ax = fmaf(d, dx, ax);
                ay = fmaf(d, dy, ay);
            }
        }
    }
}

template <bool GM>
__global__ __launch_bounds__(256) void att_early_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (J.general != (int)GM) return;
    const int i = (jb.local * blockDim.x + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    if (i >= J.n) return;
    const int e0 = J.rowptr[i] + J.late_att[i], e1 = J.rowptr[i + 1];
    if (e1 - e0 > kHeavyRow) return;     // summed by att_heavy_kernel
    const float2 pi = ld<float2>(J.pos, i);
    const float invK = J.invK;
    float ax = 0.f, ay = 0.f;
    att_run<4, 8, GM>(J, e0 + sub, e1, pi, invK, ax, ay);
    ax = group_sum<8>(ax);
    ay = group_sum<8>(ay);
    if (sub == 0) st<float2>(J.atte, i, float2{ax, ay});
}

// Heavy rows: one workgroup per row, reduced in a fixed order.
template <bool GM>
__global__ __launch_bounds__(256) void att_heavy_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (J.general != (int)GM) return;
    __shared__ float wsx[4], wsy[4];
    const int nh = *J.nheavy;
    const float invK = J.invK;
    for (int h = jb.local; h < nh; h += jb.nblocks) {
        const int i = J.heavy[h];
        const int e0 = J.rowptr[i] + J.late_att[i], e1 = J.rowptr[i + 1];
        const float2 pi = ld<float2>(J.pos, i);
        float ax = 0.f, ay = 0.f;
        att_run<8, 256, GM>(J, e0 + (int)threadIdx.x, e1, pi, invK, ax, ay);
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            wsx[threadIdx.x / kWave] = ax;
            wsy[threadIdx.x / kWave] = ay;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            st<float2>(J.atte, i, float2{((wsx[0] + wsx[1]) + wsx[2]) + wsx[3], ((wsy[0] + wsy[1]) + wsy[2]) + wsy[3]});
        __syncthreads();
    }
}

// ------------------------------------------------------- late entry lists

// Everything a minibatch step needs that does not depend on moves is laid out
// before the chain starts: per batch, the "late" entries -- moved neighbours
// (the CSR prefix) and listed moved leaves -- of all its rows, row by row, as
// (row in batch << 32 | vertex) words, plus each row's offset in that list.
__device__ __forceinline__ int late_leaf_count(int lc) { return lc > kLateCap ? 0 : lc; }

// Per batch: the list holds first the old entries of all its rows, then the
// others, each part row by row.  Counts of each row -> exclusive offsets
// within each part; bold[b] = old part length, bbase[b] = list length (a scan
// turns bbase into list starts).
__global__ __launch_bounds__(1024) void batch_offsets_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ int ws[16];
    const int b = jb.local, BS = J.BS, r = (int)threadIdx.x;
    const int R = min(BS, J.n - b * BS);   // at most kMaxChainRows: one row per thread
    const int olim = old_limit(J, b);
    int co = 0, cr = 0;
    if (r < R) {
        const int i = b * BS + r;
        const int la = J.all_live ? J.rowptr[i + 1] - J.rowptr[i] : J.late_att[i];
        const int oa = J.all_live ? 0 : J.old_att[i];
        const int ll = late_leaf_count(J.late_cnt[i]);
        gptr<const int> lid = J.late_ids + (size_t)i * kLateCap;
        int ol = 0;
        for (int k = 0; k < ll; ++k) ol += lid[k] < olim ? 1 : 0;
        co = oa + ol;
        cr = (la - oa) + (ll - ol);
    }
    int tot_o, tot_r;
    const int off_o = block_excl_scan(co, ws, &tot_o);
    const int off_r = block_excl_scan(cr, ws, &tot_r);
    if (r < R) {
        J.roff_old[b * BS + r] = off_o;
        J.roff[b * BS + r] = off_r;
    }
    if (r == 0) {
        atomicAdd(&J.ctr->old_total, (unsigned long long)tot_o);
        atomicAdd(&J.ctr->recent_total, (unsigned long long)tot_r);
        J.bold[b] = tot_o;
        J.bbase[b] = tot_o + tot_r;
        if (b == 0) J.bbase[J.nb] = 0;
    }
}
__global__ __launch_bounds__(256) void late_fill_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    const int i = (jb.local * blockDim.x + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    const bool in = i < J.n;
    const int ii = in ? i : J.n - 1;
    const int b = ii / J.BS;
    const unsigned long long rbits = (unsigned long long)(ii - b * J.BS) << 32;
    const size_t bo = (size_t)J.bbase[b] + J.roff_old[ii];
    const size_t br = (size_t)J.bbase[b] + J.bold[b] + J.roff[ii];
    const int rs = J.rowptr[ii];
    const int la = J.all_live ? J.rowptr[ii + 1] - rs : J.late_att[ii];
    const int oa = J.all_live ? 0 : J.old_att[ii];
    gptr<unsigned long long> ent = J.ent;
    const bool heavy = !J.all_live && la > kLateHeavyRow;   // copied by late_fill_heavy_kernel
    if (in && !heavy) {
        for (int k = sub; k < oa; k += 8) ent[bo + k] = rbits | (unsigned)J.colidx[rs + k];
        for (int k = oa + sub; k < la; k += 8) {
            const int c = J.colidx[rs + k];
            ent[br + (k - oa)] = rbits | (J.all_live ? (unsigned)c : ring_index(J, c));
        }
    }
    // leaves: stable split by the ballot of this row's eight lanes
    const int ll = in ? late_leaf_count(J.late_cnt[ii]) : 0;
    const int olim = old_limit(J, b);
    gptr<const int> lid = J.late_ids + (size_t)ii * kLateCap;
    const int gshift = (threadIdx.x & (kWave - 1)) & ~7;
    int no = 0, nr = 0;
    int mx = ll;
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, kWave));
    for (int k0 = 0; k0 < mx; k0 += 8) {
        const int k = k0 + sub;
        const bool have = k < ll;
        const int v = have ? lid[k] : 0;
        const bool isold = have && v < olim;
        const unsigned mo = (unsigned)(__ballot(isold) >> gshift) & 0xffu;
        const unsigned mh = (unsigned)(__ballot(have) >> gshift) & 0xffu;
        const unsigned below = (1u << sub) - 1u;
        const int ro = __popc(mo & below), rr = __popc(mh & ~mo & below);
        if (have) {
            if (isold) ent[bo + oa + no + ro] = rbits | 0x80000000u | (unsigned)v;
            else ent[br + (la - oa) + nr + rr] = rbits | 0x80000000u | (J.all_live ? (unsigned)v : ring_index(J, v));
        }
        no += __popc(mo);
        nr += __popc(mh & ~mo);
    }
}

// Rows with many moved neighbours: one workgroup per row copies them.
__global__ __launch_bounds__(256) void late_fill_heavy_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (J.all_live) return;
    const int nh = J.nheavy[1];
    for (int h = jb.local; h < nh; h += jb.nblocks) {
        const int i = J.heavy[J.n + h];
        const int b = i / J.BS;
        const unsigned long long rbits = (unsigned long long)(i - b * J.BS) << 32;
        const size_t bo = (size_t)J.bbase[b] + J.roff_old[i];
        const size_t br = (size_t)J.bbase[b] + J.bold[b] + J.roff[i];
        const int rs = J.rowptr[i], la = J.late_att[i], oa = J.old_att[i];
#pragma unroll 4
        for (int k = threadIdx.x; k < la; k += 256) {
            const int c = J.colidx[rs + k];
            J.ent[k < oa ? bo + k : br + (k - oa)] = rbits | (k < oa ? (unsigned)c : ring_index(J, c));
        }
    }
}

// ---------------------------------------------------------------- chain
// A thread's run [e0, e1) of a batch list (entries ordered by row): rows
// wholly inside the run go to sum[r], the run's first and last (cut) rows to
// cf/cl[thread].  The first min(KE, e1 - e0) entry words and their gathered
// live positions come in (w, xj, yj).  Terms: a moved neighbour adds the
// attraction d * delta / K, a listed leaf the repulsion -R K^2 delta / d^2
// (Sec. 2.2).
// Where a run's gathers read positions: global memory, or the chain's LDS
// window of the vertices its segment has moved (vertex base .. base + size).
struct PosG {
    gptr<const float2> p;
    __device__ __forceinline__ float2 operator()(int j) const { return ld<float2>(p, j); }
};
struct PosL {
    const float2 *w;
    int base;
    __device__ __forceinline__ float2 operator()(int j) const { return w[j - base]; }
};

// Under a general model (GM) the terms are d^ka delta / K and -R K^2 d^kr delta.
template <bool GM>
__device__ __forceinline__ void entry_term(unsigned long long w, float dx, float dy, float invK, float negRK2,
                                           int ka, int kr, float &ax, float &ay) {
    if ((((unsigned)w) & 0x80000000u) == 0u) {
        float d;
        if constexpr (GM) d = dpow(dx, dy, ka) * invK;
        else d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy)) * invK;   // hardware sqrt, about 1 ulp
        ax = fmaf(d, dx, ax);
        ay = fmaf(d, dy, ay);
    } else {
        float inv;
        if constexpr (GM) {
            inv = dpow(dx, dy, kr) * negRK2;
        } else {
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
            inv = __builtin_amdgcn_rcpf(d2) * negRK2;
        }
        ax = fmaf(dx, inv, ax);
        ay = fmaf(dy, inv, ay);
    }
}

template <int KE, typename P, bool GM>
__device__ __forceinline__ void run_sum(gptr<const unsigned long long> src, P pos, int e0, int e1, int rbase,
                                        unsigned long long (&w)[KE], float (&xj)[KE], float (&yj)[KE],
                                        const int *off, const float *px, const float *py, float2 *sum,
                                        float2 &first, float2 *cl, float invK, float negRK2, int ka, int kr) {
    first = float2{0.f, 0.f};
    if (e0 >= e1) return;
    const int tid = threadIdx.x;
    int r = (int)(w[0] >> 32) - rbase;
    float ax = 0.f, ay = 0.f;
    bool firstseg = true;
    for (int base = e0; base < e1; base += KE) {
        const int m = min(KE, e1 - base);
        if (base != e0) {
#pragma unroll
            for (int q = 0; q < KE; ++q)
                if (q < m) w[q] = src[base + q];
#pragma unroll
            for (int q = 0; q < KE; ++q) {
                if (q < m) {
                    const float2 pj = pos((int)((unsigned)w[q] & 0x7fffffffu));
                    xj[q] = pj.x;
                    yj[q] = pj.y;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KE; ++q) {
            if (q < m) {
                const int rq = (int)(w[q] >> 32) - rbase;
                if (rq != r) {
                    const bool full = off[r] >= e0 && off[r + 1] <= e1;
                    if (full) sum[r] = float2{ax, ay};
                    else if (firstseg) first = float2{ax, ay};
                    else cl[tid] = float2{ax, ay};
                    firstseg = false;
                    ax = ay = 0.f;
                    r = rq;
                }
                const float dx = xj[q] - px[r], dy = yj[q] - py[r];
                entry_term<GM>(w[q], dx, dy, invK, negRK2, ka, kr, ax, ay);
            }
        }
    }
    const bool full = off[r] >= e0 && off[r + 1] <= e1;
    if (full) sum[r] = float2{ax, ay};
    else if (firstseg) first = float2{ax, ay};
    else cl[tid] = float2{ax, ay};
}

// Sums of the runs' first partial rows over consecutive threads that start
// in the same row (a segmented inclusive scan in thread order), in two
// halves around the barrier that follows: before it, each wave scans its
// threads by shuffles and publishes its total and first/last keys; after
// it, scan_at(t) adds the carry of earlier waves.  key: the row of the
// thread's first entry (unique per thread when it has none); v: its first
// partial row (0 when that row is complete inside the run).
// One step of the wave's segmented scan by a DPP lane move: v takes the
// value of the source lane when that lane exists for the move and has the
// same key (keys are sorted over the threads that have entries, and unique
// elsewhere, so equal keys enclose only equal keys).
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_dpp(float2 &v, int key) {
    const int uk = __builtin_amdgcn_update_dpp((int)0x80000000, key, CTRL, ROWS, 0xf, false);
    const float ux = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v.x), CTRL, ROWS, 0xf, false));
    const float uy = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v.y), CTRL, ROWS, 0xf, false));
    if (uk == key) {
        v.x += ux;
        v.y += uy;
    }
}

__device__ __forceinline__ void carry_scan_wave(float2 v, int key, float2 *loc, int *keys, float2 *wv, int *wk,
                                                int *wkf) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    // within rows of 16 lanes (shift right by 1, 2, 4, 8), then lane 15 of
    // rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3
    seg_dpp<0x111, 0xf>(v, key);
    seg_dpp<0x112, 0xf>(v, key);
    seg_dpp<0x114, 0xf>(v, key);
    seg_dpp<0x118, 0xf>(v, key);
    seg_dpp<0x142, 0xa>(v, key);
    seg_dpp<0x143, 0xc>(v, key);
    loc[tid] = v;
    keys[tid] = key;
    if (lane == kWave - 1) {
        wv[w] = v;
        wk[w] = key;
    }
    if (lane == 0) wkf[w] = key;
}

__device__ __forceinline__ float2 scan_at(int t, const float2 *loc, const int *keys, const float2 *wv, const int *wk,
                                          const int *wkf) {
    const int w = t / kWave;
    float2 v = loc[t];
    const int K = wkf[w];
    if (keys[t] == K) {
        float2 c{0.f, 0.f};
        for (int u = w - 1; u >= 0 && wk[u] == K; --u) {
            c.x += wv[u].x;
            c.y += wv[u].y;
            if (wkf[u] != K) break;
        }
        v.x += c.x;
        v.y += c.y;
    }
    return v;
}

// A row's total over its entries [o0, o1) from the runs' results, runs of
// `chunk` entries: one run's sum, or the part in the run it starts in plus
// the scanned first parts of the following runs.
__device__ __forceinline__ float2 row_total(int r, int o0, int o1, int chunk, const float2 *sum, const float2 *cl,
                                            const float2 *loc, const int *keys, const float2 *wv, const int *wk,
                                            const int *wkf) {
    float2 sm{0.f, 0.f};
    if (o1 > o0) {
        const int t0 = o0 / chunk, t1 = (o1 - 1) / chunk;
        if (t0 == t1) {
            sm = sum[r];
        } else {
            sm = scan_at(t1, loc, keys, wv, wk, wkf);
            if (o0 != t0 * chunk) {
                sm.x = cl[t0].x + sm.x;
                sm.y = cl[t0].y + sm.y;
            }
        }
    }
    return sm;
}

// ------------------------------------------------ chain over a slot plan
// Before the chain, the recent entries of each batch are laid out as "slots",
// one per lane of the chain's workgroup, and a batch never takes more than one
// pass of the workgroup's lanes.  With k entries per lane (the smallest k for
// which the batch fits), a row with cr recent entries takes
// l = max(1, ceil(cr / k)) lanes: lane j holds entries j, j + l, j + 2l, ...
// When l <= kRunLanes the lanes are one run inside a 16-lane row of a wave
// (the row's slots rounded up to a power of two, so that runs stay inside
// 16-lane rows); a longer row is split into 16-lane runs (its lane count
// rounded up to a multiple of 16).  A step then forms each lane's terms, a DPP suffix sum
// inside each run brings the run's sum to its first lane, and that lane
// completes and moves the row; the first run of a split row adds the other
// runs' sums, which they leave in LDS, in run order after a second barrier.
// With k = 1 every entry is in its slot word, loaded steps ahead; with k > 1
// the lane reads its entries from the batch list.  One barrier per step
// (two with split rows) makes the moved positions visible to the next.
constexpr int kRunLanes = 16;
constexpr int kMoreLoads = 8;         // list words a lane with several entries loads at once
// Slot word: bits 0-31 the entry word's low half (vertex | leaf bit 31), or
// for a lane with several entries its lane index in the row (bits 0-15) and
// the row's lane count (bits 16-31); 32-41 the row in its batch; 42-45 lanes
// after this one in its run; 46 holds one entry; 47 first lane of a run; 48
// several entries from the list; 49 padding (no row); 50 the row's late-leaf
// list overflowed (its far field comes from a full walk when it moves); 51
// first lane of the row (moves it); 52-57 the row's further runs.
constexpr unsigned long long kSlotHas = 1ull << 46, kSlotLead = 1ull << 47, kSlotMulti = 1ull << 48,
                             kSlotPad = 1ull << 49, kSlotWalk = 1ull << 50, kSlotRow = 1ull << 51;
constexpr int kSlotRunsShift = 52;
// Batch flags (pflag): bit 0 a row overflowed its leaf list, bit 1 the batch
// has split rows, bits 8-15 the index of its entries per lane in kPlanK, bits
// 16 and up the slots its rows use.
constexpr int kFlagOvf = 1, kFlagSplit = 2, kFlagKShift = 8, kFlagUsedShift = 16;
static_assert(kMaxChainRows <= 1024, "slot words hold the row in 10 bits");

// Recent entries of row r of batch b (R rows); bbase holds list starts.
__device__ __forceinline__ int recent_count(const BHJob &J, int b, int r, int R) {
    const int i = b * J.BS + r;
    const int rend = (r + 1 < R) ? J.roff[i + 1] : (J.bbase[b + 1] - J.bbase[b] - J.bold[b]);
    return rend - J.roff[i];
}
// Lanes a row with cr recent entries takes at k entries per lane.
__device__ __forceinline__ int row_lanes(int cr, int k) {
    const int l = max(1, (cr + k - 1) / k);
    return l > kRunLanes ? (l + kRunLanes - 1) & ~(kRunLanes - 1) : l;
}
// Slot capacity of a batch of R rows (a row alone never needs more than
// 2 kRunLanes lanes at k = cr).
__device__ __host__ __forceinline__ int plan_cap(int R) { return min(kChainThreads, 2 * kRunLanes * R + kRunLanes); }

// Entries per lane the planner may choose.
__constant__ int kPlanK[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128, 192, 256, 384, 512, 1 << 30};
constexpr int kPlanKs = 23;

// Lanes a row's slots occupy: its lane count rounded up to a power of two
// when it is one run, as it is when split.
__device__ __forceinline__ int row_span(int l) {
    return l > kRunLanes ? l : (l == 1 ? 1 : 1 << (32 - __builtin_clz((unsigned)(l - 1))));
}

// Sum over the workgroup (1024 threads) of v, returned to every thread.
__device__ __forceinline__ int plan_block_sum(int v, int *wsum) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();   // wsum free from the previous sum
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = v;
    __syncthreads();
    int s = 0;
    for (int w = 0; w < kChainThreads / kWave; ++w) s += wsum[w];
    return s;
}
// Number of earlier threads (in thread order) with pred set, and the total.
__device__ __forceinline__ int plan_block_rank(bool pred, int *wsum, int &total) {
    const unsigned long long m = __ballot(pred);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int in_wave = __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int before = 0;
    total = 0;
    for (int q = 0; q < kChainThreads / kWave; ++q) {
        before += q < w ? wsum[q] : 0;
        total += wsum[q];
    }
    return before + in_wave;
}

// One workgroup per batch (1024 threads, one row each): the batch's entries
// per lane k -- the first of kPlanK whose plan fits the batch's slot capacity,
// found by bisection (a row's span does not grow with k, and the last k, one
// lane per row, always fits) -- and each row's first slot.  The plan places
// split rows first, then one-run rows by span (16, 8, 4, 2, 1 lanes), each
// group in row order, so that every position is a prefix count and no run
// crosses a 16-lane row.  pbase[b] gets the batch's slot count (a padding
// slot last unless the slots fill whole passes), pflag[b] its flags, the
// index of k and the slots its rows use.
__global__ __launch_bounds__(1024) void plan_count_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    __shared__ int wsum[kChainThreads / kWave];
    const int b = jb.local, r = (int)threadIdx.x;
    const int R = min(J.BS, J.n - b * J.BS);
    const bool row = r < R;
    const int cr = row ? recent_count(J, b, r, R) : 0;
    const int ovf = plan_block_sum(row && J.late_cnt[b * J.BS + r] > kLateCap ? 1 : 0, wsum) > 0;
    const int cap = plan_cap(R);
    auto total_at = [&](int c) {
        const int pos = plan_block_sum(row ? row_span(row_lanes(cr, kPlanK[c])) : 0, wsum);
        return (pos % kChainThreads) == 0 ? pos : (pos + kRunLanes) & ~(kRunLanes - 1);
    };
    int lo = 0, hi = kPlanKs - 1;
    if (total_at(0) <= cap) hi = 0;
    else lo = 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (total_at(mid) <= cap) hi = mid;
        else lo = mid + 1;
    }
    const int c = lo, k = kPlanK[c];
    const int l = row ? row_lanes(cr, k) : 0;
    const int span = row ? row_span(l) : 0;
    // split rows first: an exclusive scan of their spans (multiples of 16)
    int start = 0, base = 0, split = 0;
    {
        const int v = row && l > kRunLanes ? span : 0;
        int x = v;
        const int lane = r & (kWave - 1), w = r / kWave;
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        __syncthreads();
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        int before = 0, tot = 0;
        for (int q = 0; q < kChainThreads / kWave; ++q) {
            before += q < w ? wsum[q] : 0;
            tot += wsum[q];
        }
        if (v) start = before + x - v;
        base = tot;
        split = tot > 0;
    }
    for (int s = kRunLanes; s >= 1; s >>= 1) {
        int cnt = 0;
        const int rk = plan_block_rank(row && l <= kRunLanes && span == s, wsum, cnt);
        if (row && l <= kRunLanes && span == s) start = base + rk * s;
        base += cnt * s;
    }
    if (row) J.pstart[b * J.BS + r] = start;
    // the chain launch's progress words for this iteration, and the batch's
    // helper parts (batches above lag in the launch's range; the ready word
    // counts the parts done up from 1 - parts, ready at 1)
    if (r == 0) {
        const bool helped = !J.all_live && b >= max(J.first_batch, J.lag + 1) && b <= J.last_batch;
        const int parts = helped ? max(1, (J.bold[b] + kPartEnt - 1) / kPartEnt) : 0;
        J.hbase[b] = parts;
        J.sync[kSyncReady + b] = 1 - parts;
        if (b == 0) {
            J.sync[kSyncMoved] = J.first_batch;
            J.sync[kSyncTicket] = 0;
            J.hbase[J.nb] = 0;
        }
    }
    if (r == 0) {
        const int total = (base % kChainThreads) == 0 ? base : (base + kRunLanes) & ~(kRunLanes - 1);
        J.pbase[b] = total;
        J.pflag[b] = (ovf ? kFlagOvf : 0) | (split ? kFlagSplit : 0) | (c << kFlagKShift) | (base << kFlagUsedShift);
        if (b == 0) J.pbase[J.nb] = 0;
    }
}

// One thread per row: its slot words (padding to its span), and for the
// batch's first row the padding after the last row's slots.
__global__ __launch_bounds__(256) void plan_fill_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    const int i = jb.local * blockDim.x + threadIdx.x;
    if (i >= J.n) return;
    const int b = i / J.BS, r = i - b * J.BS, R = min(J.BS, J.n - b * J.BS);
    const int cr = recent_count(J, b, r, R);
    const int flags = J.pflag[b];
    const int k = kPlanK[(flags >> kFlagKShift) & 255];
    const int l = row_lanes(cr, k);
    const bool split = l > kRunLanes;
    const int s0 = J.pstart[i];
    const size_t base = (size_t)J.pbase[b];
    const size_t list = (size_t)J.bbase[b] + J.bold[b] + J.roff[i];
    const unsigned long long rb = (unsigned long long)r << 32;
    const unsigned long long rowlead = kSlotRow | (J.late_cnt[i] > kLateCap ? kSlotWalk : 0ull) |
                                       ((unsigned long long)(split ? l / kRunLanes - 1 : 0) << kSlotRunsShift);
    for (int j = 0; j < l; ++j) {
        const int rem = split ? (kRunLanes - 1) - (j & (kRunLanes - 1)) : l - 1 - j;
        unsigned long long w = rb | ((unsigned long long)rem << 42);
        if (k > 1) w |= kSlotMulti | (unsigned long long)j | ((unsigned long long)l << 16);
        else if (j < cr) w |= kSlotHas | (J.ent[list + j] & 0xffffffffull);
        if (split ? (j & (kRunLanes - 1)) == 0 : j == 0) w |= kSlotLead;
        if (j == 0) w |= rowlead;
        J.slots[base + s0 + j] = w;
    }
    for (int q = l; q < row_span(l); ++q) J.slots[base + s0 + q] = kSlotPad;
    if (r == 0)
        for (int q = flags >> kFlagUsedShift; q < J.pbase[b + 1] - J.pbase[b]; ++q) J.slots[base + q] = kSlotPad;
    // the row's record: position at the iteration's start, and its force apart
    // from recent entries -- early attraction and far field (a row whose leaf
    // list overflowed takes its far field from a full walk when it moves); the
    // segment kernel adds the old entries
    const int lc = J.late_cnt[i];
    const float2 p = ld<float2>(J.pos, i);
    float2 bs = J.all_live ? float2{0.f, 0.f} : ld<float2>(J.atte, i);
    if (lc <= kLateCap) {
        const float4 fr = ld<float4>(J.far, i);
        bs.x += J.negRK2 * (fr.x - fr.z);
        bs.y += J.negRK2 * (fr.y - fr.w);
    }
    st<float4>(J.rec, i, float4{p.x, p.y, bs.x, bs.y});
    st<int2>(J.rmeta, i, int2{J.roff[i], J.roff[i] + cr});
    if (r == 0) {
        st<int4>(J.bmeta, b, int4{J.pbase[b], J.pbase[b + 1] - J.pbase[b], J.bbase[b] + J.bold[b], flags});
        for (int q = J.hbase[b]; q < J.hbase[b + 1]; ++q) st<int2>(J.hitem, q, int2{b, q - J.hbase[b]});
    }
}

struct ChainShared {
    float2 xpart[kChainThreads / kRunLanes];   // run totals of split rows' later runs
    double wsd[16];
    double step;
    int go;                                    // 0: a bounded wait ran out, leave
};

// The helpers' workspace: one batch's old entries summed by runs of equal
// length, the runs' cut rows combined by a carry scan.
struct HelperShared {
    int off[kMaxChainRows + 1];
    float px[kMaxChainRows], py[kMaxChainRows];
    float2 sum[kMaxChainRows];
    float2 cl[kChainThreads], loc[kChainThreads];
    int keys[kChainThreads];
    float2 wv[kChainThreads / kWave];
    int wk[kChainThreads / kWave], wkf[kChainThreads / kWave];
    int item, go;
};

// Barrier for LDS traffic only: every wave's LDS stores are complete and
// visible after it, while global loads and stores stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum of v over this lane and the `rem` lanes after it in its 16-lane row
// (a Hillis-Steele suffix sum whose steps stay inside the lane's run).
__device__ __forceinline__ float run_suffix_sum(float v, int rem) {
#define BL_RUN_STEP(O)                                                                                            \
    {                                                                                                             \
        const float t = __builtin_bit_cast(                                                                       \
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x100 + (O), 0xf, 0xf, false));     \
        if ((O) <= rem) v += t;                                                                                   \
    }
    BL_RUN_STEP(1)
    BL_RUN_STEP(2)
    BL_RUN_STEP(4)
    BL_RUN_STEP(8)
#undef BL_RUN_STEP
    return v;
}

// Uniform loads through the scalar unit (the address is the same for every
// lane): the chain's per-batch records (first slot, slot count, recent-list
// start, flags).
__device__ __forceinline__ int4 sld4(gptr<const int4> p, int i) {
    using B = RawBits<16>::type;
    return __builtin_bit_cast(int4, ((const __attribute__((address_space(4))) B *)p)[__builtin_amdgcn_readfirstlane(i)]);
}
__device__ __forceinline__ int2 sld2(gptr<const int4> p, int i) {   // the first two fields
    using B = RawBits<8>::type;
    return __builtin_bit_cast(int2,
                              ((const __attribute__((address_space(4))) B *)p)[2 * __builtin_amdgcn_readfirstlane(i)]);
}

// Values that workgroups of one launch exchange across the chip: positions
// the chain moves, the helpers' old sums, the progress counters.  A writer
// stores plainly, waits for its stores, and raises a counter with an
// agent-scope release (which writes its die's L2 back); a reader polls the
// counter and reads the values with agent-scope loads, which bypass its own
// die's L2.
__device__ __forceinline__ float2 ld_coh(gptr<const float2> p, size_t i) {
    const unsigned long long v =
        __hip_atomic_load((gptr<unsigned long long>)(p + i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, v);
}
__device__ __forceinline__ int ld_flag(gptr<int> p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
struct PosC {
    gptr<const float2> p;
    __device__ __forceinline__ float2 operator()(int j) const { return ld_coh(p, j); }
};

// Thread 0: wait until *flag >= need.  Returns 0 when the launch is being
// abandoned (this wait or another one ran out of polls).
__device__ __forceinline__ int bh_wait(gptr<int> flag, int need, gptr<unsigned long long> abort, long long limit) {
    for (long long it = 0;; ++it) {
        if (ld_flag(flag) >= need) return 1;
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0;
        if (it >= limit) {
            __hip_atomic_store(abort, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // (complete here: a store left in flight would cost the chain's
            // loads their completion count)
            __builtin_amdgcn_s_waitcnt(0x0F70);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Two paths of the chain off its common case: the terms of a lane with
// several entries (list entries e0, e0 + stride, ... below e1 from base,
// kMoreLoads list words in flight at a time), and the far field of a row
// whose late-leaf list overflowed, from a full walk over the live positions.
// The walk reads its job fields through a pointer that an empty asm statement
// hands it inside the branch, so that the compiler cannot hoist those reads
// into the hot loop's scalar registers.
using JobC = const __attribute__((address_space(4))) BHJob *;
__device__ __forceinline__ JobC launder(const BHJob *p) {
    JobC q = (JobC)p;
    asm volatile("" : "+s"(q));
    return q;
}

template <bool GM, bool WIN>
__device__ __forceinline__ float2 lane_terms(gptr<const unsigned long long> ent, const float2 *win,
                                             gptr<const float2> pos, size_t base, int e0, int e1, int stride, float x,
                                             float y, float invK, float negRK2, int ka, int kr) {
    float ax = 0.f, ay = 0.f;
    for (int e = e0; e < e1; e += kMoreLoads * stride) {
        unsigned long long we[kMoreLoads];
#pragma unroll
        for (int u = 0; u < kMoreLoads; ++u) we[u] = e + u * stride < e1 ? ent[base + e + u * stride] : 0ull;
#pragma unroll
        for (int u = 0; u < kMoreLoads; ++u) {
            if (e + u * stride < e1) {
                const int j = (int)((unsigned)we[u] & 0x7fffffffu);
                const float2 pj = WIN ? win[j] : ld<float2>(pos, j);
                entry_term<GM>(we[u], pj.x - x, pj.y - y, invK, negRK2, ka, kr, ax, ay);
            }
        }
    }
    return float2{ax, ay};
}

template <bool GM>
__device__ __forceinline__ float2 overflow_far(JobC Jp, int i, float x, float y) {
    WalkArgs wa;
    wa.n = Jp->n;
    wa.BS = Jp->BS;
    wa.total = Jp->nnodes;
    wa.nodeA = Jp->nodeA;
    wa.nodeB = Jp->nodeB;
    wa.leafpos = Jp->leafpos;
    wa.theta2 = Jp->theta2;
    wa.negRK2 = Jp->negRK2;
    wa.invK = Jp->invK;
    wa.kr = Jp->kr;
    float4 fr;
    int dummy = 0;
    (void)bh_walk<GM>(wa, i, x, y, 0, Jp->pos, fr, nullptr, dummy, 0);
    return float2{wa.negRK2 * (fr.x - fr.z), wa.negRK2 * (fr.y - fr.w)};
}


// A helper workgroup: items (batch b, part p) of the chain, claimed in order.
// Once the chain has moved the batches below b - lag, the helper sums the old
// entries of the part's rows with their final positions -- the part's list
// split into equal runs, summed per row, the runs' cut rows combined by the
// carry scan -- stores the sums in oldf and counts the part done in the
// batch's ready word.
template <bool GM>
__device__ __forceinline__ void chain_helper(const BHJob &J, HelperShared &H) {
    const int tid = threadIdx.x, BS = J.BS;
    const int items = J.hbase[J.nb];
    for (;;) {
        if (tid == 0) H.item = __hip_atomic_fetch_add(J.sync + kSyncTicket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        // (scalar copies: the loop's barriers stay in uniform control flow)
        const int t = __builtin_amdgcn_readfirstlane(H.item);
        if (t >= items) return;
        const int2 it = ld<int2>(J.hitem, t);
        const int b = __builtin_amdgcn_readfirstlane(it.x), part = __builtin_amdgcn_readfirstlane(it.y);
        // What does not depend on moves is loaded before the wait: the part's
        // rows and list words, and the batch's own positions (its rows move
        // only at step b).
        const int R = min(BS, J.n - b * BS);
        gptr<const int> ro = J.roff_old + (size_t)b * BS;
        const int E = J.bold[b];
        const int parts = J.hbase[b + 1] - J.hbase[b];
        const int myoff = tid < R ? ro[tid] : E;
        const int mypart = tid < R ? min(myoff / kPartEnt, parts - 1) : parts;
        const int r_lo = __syncthreads_count(mypart < part);
        const int r_hi = __syncthreads_count(mypart <= part);
        const int E0 = r_lo < R ? ro[r_lo] : E, E1 = r_hi < R ? ro[r_hi] : E;
        const int len = E1 - E0, nr = r_hi - r_lo;
        const size_t base = (size_t)J.bbase[b] + E0;
        const int chunk = max(1, (len + kChainThreads - 1) / kChainThreads);
        const int e0 = min(tid * chunk, len), e1 = min(e0 + chunk, len);
        unsigned long long w[kEntH];
        float xj[kEntH], yj[kEntH];
        const int m0 = min(kEntH, e1 - e0);
#pragma unroll
        for (int q = 0; q < kEntH; ++q) {
            w[q] = 0;
            xj[q] = 0.f;
            yj[q] = 0.f;
            if (q < m0) w[q] = J.ent[base + e0 + q];
        }
        if (tid >= r_lo && tid < r_hi) {
            H.off[tid - r_lo] = myoff - E0;
            const float2 p = ld<float2>(J.pos, b * BS + tid);
            H.px[tid - r_lo] = p.x;
            H.py[tid - r_lo] = p.y;
        }
        if (tid == 0) {
            H.off[nr] = len;
            H.go = bh_wait(J.sync + kSyncMoved, b - J.lag, (gptr<unsigned long long>)&J.ctr->wait_abort, J.spin_limit);
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(H.go)) return;
        const PosC pc{J.pos};
#pragma unroll
        for (int q = 0; q < kEntH; ++q) {
            if (q < m0) {
                const float2 pj = pc((int)((unsigned)w[q] & 0x7fffffffu));
                xj[q] = pj.x;
                yj[q] = pj.y;
            }
        }
        const int key0 = e0 < e1 ? (int)(w[0] >> 32) - r_lo : -1 - tid;
        float2 firstp;
        run_sum<kEntH, PosC, GM>(J.ent + base, pc, e0, e1, r_lo, w, xj, yj, H.off, H.px, H.py, H.sum, firstp, H.cl,
                                 J.invK, J.negRK2, J.ka, J.kr);
        carry_scan_wave(firstp, key0, H.loc, H.keys, H.wv, H.wk, H.wkf);
        __syncthreads();
        for (int j = tid; j < nr; j += kChainThreads) {
            const float2 s2 = row_total(j, H.off[j], H.off[j + 1], chunk, H.sum, H.cl, H.loc, H.keys, H.wv, H.wk,
                                        H.wkf);
            st<float2>(J.oldf, (size_t)b * BS + r_lo + j, s2);
        }
        // every wave's sums complete, then their release with the count
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(0);
            (void)__hip_atomic_fetch_add(J.sync + kSyncReady + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// The minibatch chain: one workgroup per job walks the job's batches in
// order, one step per batch, over the slot plan.  A lane's slot word is
// loaded four steps before its batch comes up and its row's record and old
// sum two steps before (their address is the slot word's row); batch records
// come through the scalar unit a step ahead.  A step loads the ready flag of
// the batch whose old sums the next step loads, the record and the old sum two
// batches ahead and the slot word four batches ahead, and stores nothing to
// memory: moved positions go to the ring, and a copy every kRelease steps
// takes them to memory and waits for its stores.  (A store in flight among
// loads leaves the compiler no count of the loads that have completed, so that
// it would wait for all of them where a loaded value is used.)  A barrier on
// LDS traffic alone ends the step.  The rows' terms use the positions their batch sees:
// moved ones from an LDS ring of the last lag + 1 batches (WIN; Jacobi within
// the batch, Gauss-Seidel across batches) or from memory (one-shot force
// calls, where nothing moves).  The chain publishes how many batches it has
// moved for the helpers, and waits for a batch's old sums before loading
// them.
template <bool GM, bool WIN>
__device__ __forceinline__ void chain_run(const BHJob &J, const BHJob *Jg, ChainShared &S, float2 *win) {
    const int tid = threadIdx.x;
    const int BS = J.BS, first = J.first_batch, last = J.last_batch, lag = J.lag;
    const float invK = J.invK, negRK2 = J.negRK2;
    const int k_it = J.kiter[0];
    const gptr<const int4> p_bmeta = J.bmeta;
    const gptr<const unsigned long long> p_slots = J.slots, p_ent = J.ent;
    const gptr<const float4> p_rec = J.rec;
    const gptr<const float2> p_oldf = J.oldf;
    const gptr<const int2> p_rmeta = J.rmeta;
    const gptr<float2> p_pos = J.pos;
    const gptr<int> p_sync = J.sync;
    const bool helped = !J.all_live && last > lag;   // batches above lag have old entries
    // this lane's slot word of a batch with first slot pb0 and sc slots
    // (lanes past the last slot read the last one, which is padding)
    auto slot_load = [&](int pb0, int sc) -> unsigned long long {
        return p_slots[(size_t)pb0 + min(tid, sc - 1)];
    };
    auto rec_load = [&](int b, unsigned long long w) -> float4 {
        return ld<float4>(p_rec, (size_t)b * BS + (int)((w >> 32) & 1023u));
    };
    // the old-entry sum of the lane's row (batches up to lag have none: the
    // load is issued all the same, so that every step has the same loads, and
    // its value is dropped where it is used)
    auto old_load = [&](int b, unsigned long long w) -> float2 {
        if (!helped) return float2{0.f, 0.f};
        return ld_coh(p_oldf, (size_t)b * BS + (int)((w >> 32) & 1023u));
    };
    // the recent-entry range of the row of a lane with several entries
    // (other lanes: none)
    auto range_load = [&](int b, unsigned long long w) -> int2 {
        return (w & kSlotMulti) ? ld<int2>(p_rmeta, (size_t)b * BS + (int)((w >> 32) & 1023u)) : int2{0, 0};
    };
    auto bq = [&](int q) { return min(q, last); };
    // the old sums of batch q are there (or the launch is being left)
    auto needs = [&](int q) { return helped && q > lag && q <= last; };
    auto ready = [&](int q) -> int {
        return !needs(q) || bh_wait(p_sync + kSyncReady + q, 1, (gptr<unsigned long long>)&J.ctr->wait_abort, J.spin_limit);
    };

    if (tid == 0) {
        double st = J.step0;
        for (int t = 0; t < k_it; ++t) st *= J.decay;
        S.step = st;
        S.go = ready(first) && ready(first + 1);
    }
    if (WIN)   // the ring's batches moved before this launch
        for (int v = max(0, first - lag) * BS + tid; v < first * BS; v += kChainThreads)
            win[((v / BS) % (lag + 1)) * BS + v % BS] = ld<float2>(J.pos, v);
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(S.go)) return;
    // every wave's copy of the ready flag of the batch whose old sums the next
    // step loads (it checks it itself; a wait that gives up clears S.go,
    // which all waves read after each group of four steps).  It is loaded
    // ahead of the prologue's other loads, as each step loads it ahead of its
    // others, so that the step's partial wait covers it on the first step too.
    int fl = helped ? ld_flag(p_sync + kSyncReady + bq(first + 2)) : 1;
    // prologue: slot words of the first four batches, records, old sums and
    // ranges of the first two
    unsigned long long W0, W1, W2, W3;
    float4 R0{}, R1{}, R2{}, R3{};
    float2 F0{}, F1{}, F2{}, F3{};
    int2 O0{}, O1{}, O2{}, O3{};
    {
        int2 q = sld2(p_bmeta, bq(first));
        W0 = slot_load(q.x, q.y);
        q = sld2(p_bmeta, bq(first + 1));
        W1 = slot_load(q.x, q.y);
        q = sld2(p_bmeta, bq(first + 2));
        W2 = slot_load(q.x, q.y);
        q = sld2(p_bmeta, bq(first + 3));
        W3 = slot_load(q.x, q.y);
        R0 = rec_load(bq(first), W0);
        R1 = rec_load(bq(first + 1), W1);
        F0 = old_load(bq(first), W0);
        F1 = old_load(bq(first + 1), W1);
        O0 = range_load(bq(first), W0);
        O1 = range_load(bq(first + 1), W1);
    }
    // scalar state: this batch's record, batch b + 4's first slot and slot
    // count, the ring slot of this batch
    int4 bm = sld4(p_bmeta, first);
    int2 q4 = sld2(p_bmeta, bq(first + 4));
    static_assert(kRelease % 4 == 0, "the step loop takes four steps at a time");
    int ring = first % (lag + 1);
    const float step = (float)S.step;

    double e_iter = 0.0;
    unsigned long long bad = 0;
    // Moved positions stay in the ring; every kRelease steps the workgroup
    // copies the batches moved since the last copy to memory (cp: the first
    // batch not copied yet), with agent-scope stores that the helpers' loads
    // see, and waits for them, so that the steps in between store nothing.
    int cp = first;
    // the old value the last progress update returned, used by the next one
    // (an update that returns a value is a load for the compiler's counter
    // waits, and a store in flight would cost the chain's loads their count)
    int relv = 0;
    auto copy_out = [&](int c1) __attribute__((always_inline)) {   // batches cp .. c1
        const int cnt = (c1 - cp + 1) * BS;
        for (int t = tid; t < cnt; t += kChainThreads) {
            const int q = t / BS, r = t - q * BS;
            const int v = (cp + q) * BS + r;
            if (v < J.n) {
                const float2 pv = win[((cp + q) % (lag + 1)) * BS + r];
                __hip_atomic_store((gptr<unsigned long long>)(p_pos + v), __builtin_bit_cast(unsigned long long, pv),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        cp = c1 + 1;
    };

    // The terms of this lane's slot and its run's suffix sum (the run's total
    // at its first lane).
    auto run_total = [&](unsigned long long w, const float4 &rc, const int2 &om, int lst)
                         __attribute__((always_inline)) -> float2 {
        const bool pad = (w & kSlotPad) != 0;
        float ax = 0.f, ay = 0.f;
        if (!__any(!pad)) return float2{ax, ay};   // a wave of padding only
        const int rem = pad ? 0 : (int)((w >> 42) & 15u);
        if (!pad) {
            if (w & kSlotHas) {
                const int j = (int)((unsigned)w & 0x7fffffffu);
                const float2 pj = WIN ? win[j] : ld<float2>(p_pos, j);
                entry_term<GM>(w, pj.x - rc.x, pj.y - rc.y, invK, negRK2, J.ka, J.kr, ax, ay);
            }
            if (w & kSlotMulti) {
                const float2 t = lane_terms<GM, WIN>(p_ent, win, p_pos, (size_t)lst + om.x, (int)(w & 0xffffu),
                                                     om.y - om.x, (int)((w >> 16) & 0xffffu), rc.x, rc.y, invK,
                                                     negRK2, J.ka, J.kr);
                ax += t.x;
                ay += t.y;
            }
        }
        if (__any(rem > 0)) {
            ax = run_suffix_sum(ax, rem);
            ay = run_suffix_sum(ay, rem);
        }
        return float2{ax, ay};
    };
    // The row's move by its first lane, from the total of its recent entries.
    auto move_row = [&](int b, unsigned long long w, const float4 &rc, float2 f, bool stop)
                        __attribute__((always_inline)) {
        const int r = (int)((w >> 32) & 1023u);
        const int i = b * BS + r;
        float fx = f.x + rc.z, fy = f.y + rc.w;
        if (w & kSlotWalk) {
            const float2 t = overflow_far<GM>(launder(Jg), i, rc.x, rc.y);
            fx += t.x;
            fy += t.y;
        }
        if (stop) {
            J.fout[2 * r] = (double)fx;
            J.fout[2 * r + 1] = (double)fy;
            __builtin_amdgcn_s_waitcnt(0x0F70);   // no store left in flight among the chain's loads
            if (WIN) win[ring * BS + r] = float2{rc.x, rc.y};   // unmoved (the ring is copied out)
            return;
        }
        float2 np{rc.x, rc.y};
        const double f2 = (double)fx * fx + (double)fy * fy;
        if (!isfinite(f2)) {
            ++bad;
        } else {
            e_iter += f2;
            if (f2 > 0.0) {
                // step / |f| with the hardware reciprocal square root (about 1 ulp)
                const float sc = step * __builtin_amdgcn_rsqf(fx * fx + fy * fy);
                np = float2{rc.x + sc * fx, rc.y + sc * fy};
            }
        }
        if (WIN) win[ring * BS + r] = np;
        else st<float2>(p_pos, i, np);
    };

    // step b: wc / rc / fc / oc hold batch b's slot word, record, old sum and
    // row range; w2 holds batch b + 2's slot word, and r2 / f2 / o2 receive its
    // record, old sum and range; wc receives batch b + 4's slot word.
    auto chain_step = [&](int b, unsigned long long &wc, const float4 &rc, const float2 &fc, const int2 &oc,
                          const unsigned long long &w2, float4 &r2, float2 &f2, int2 &o2)
                          __attribute__((always_inline)) {
        const bool stop = (b == J.stop_batch);
        // Every kRelease steps the batches moved since the last copy go from
        // the ring to memory (the last step's barrier completed the ring).
        // The earlier steps' loads are complete first, so that the stores in
        // flight leave the compiler no loaded value to wait for in this step;
        // the stores complete at its end, and the helpers get the batches.
        const bool copy = WIN && helped && b > first && ((b - first) & (kRelease - 1)) == 0;
        if (copy) {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            copy_out(b - 1);
        }
        // the old sums this step loads (batch b + 2): the flag loaded a step ago
        // (their helper needs batches below b + 2 - lag, published by now as
        // lag >= kMinLag)
        if (__any(fl < 1) && needs(b + 2) && !ready(b + 2)) S.go = 0;
        // next step's scalar state (its loads complete at this step's barrier)
        const int4 bmn = sld4(p_bmeta, bq(b + 1));
        const int2 q5 = sld2(p_bmeta, bq(b + 5));
        if (helped) fl = ld_flag(p_sync + kSyncReady + bq(b + 3));
        r2 = rec_load(bq(b + 2), w2);
        f2 = old_load(bq(b + 2), w2);
        o2 = range_load(bq(b + 2), w2);
        float2 f = run_total(wc, rc, oc, bm.z);
        const bool lead = !(wc & kSlotPad) && (wc & kSlotLead);
        const bool first_lane = lead && (wc & kSlotRow);
        if (bm.w & kFlagSplit) {
            // split rows: the later runs' totals through LDS, added in run order
            if (lead && !first_lane) S.xpart[tid / kRunLanes] = f;
            lds_barrier();
            if (first_lane) {
                const int runs = (int)((wc >> kSlotRunsShift) & 63u);
                for (int q = 1; q <= runs; ++q) {
                    const float2 t = S.xpart[tid / kRunLanes + q];
                    f.x += t.x;
                    f.y += t.y;
                }
            }
        }
        if (first_lane) {
            if (helped && b > lag) {   // the row's old entries, once
                f.x += fc.x;
                f.y += fc.y;
            }
            move_row(b, wc, rc, f, stop);
        }
        if (copy) {
            // every wave's copy stores are complete after the barrier
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __builtin_amdgcn_s_barrier();
            if (tid == 0)
                relv = __hip_atomic_fetch_max(p_sync + kSyncMoved, relv < 0 ? relv : cp, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        }
        wc = slot_load(q4.x, q4.y);
        if (WIN && b + 1 <= last && (bmn.w & kFlagOvf)) {
            // a row of the next batch walks the tree over positions in memory
            lds_barrier();
            copy_out(b);
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
        } else {
            lds_barrier();
        }
        bm = bmn;
        q4 = q5;
        ring = ring == lag ? 0 : ring + 1;
    };
    bool go = true;
    for (int b = first; b <= last && go; b += 4) {
        chain_step(b, W0, R0, F0, O0, W2, R2, F2, O2);
        if (b + 1 <= last) chain_step(b + 1, W1, R1, F1, O1, W3, R3, F3, O3);
        if (b + 2 <= last) chain_step(b + 2, W2, R2, F2, O2, W0, R0, F0, O0);
        if (b + 3 <= last) chain_step(b + 3, W3, R3, F3, O3, W1, R1, F1, O1);
        go = __builtin_amdgcn_readfirstlane(S.go) != 0;
    }
    if (!go) return;
    if (WIN) copy_out(last);   // the last step's barrier made the ring complete
    if (bad) atomicAdd(&J.ctr->nonfinite, bad);
    const double e = block_sum_fixed(e_iter, S.wsd);
    if (tid == 0 && J.stop_batch < 0) {
        const int slot_e = k_it - J.kiter[1];
        J.energy[slot_e] = e;
        J.kiter[0] = k_it + 1;
        if (J.conv_tol > 0 && slot_e >= 1) {
            const double ep = J.energy[slot_e - 1];
            if (fabs(e - ep) <= J.conv_tol * ep) J.ctr->halted = (unsigned long long)(slot_e + 1);
        }
    }
}

// One launch per iteration: per job, workgroup 0 runs the chain and the
// others are its helpers.
template <bool GM>
__global__ __launch_bounds__(kChainThreads) void chain_kernel(BH_KERNEL_ARGS) {
    BH_JOB();
    if (J.general != (int)GM) return;
    extern __shared__ double lds_raw[];
    if (jb.local > 0) {
        chain_helper<GM>(J, *reinterpret_cast<HelperShared *>(lds_raw));
        return;
    }
    ChainShared &S = *reinterpret_cast<ChainShared *>(lds_raw);
    float2 *win = reinterpret_cast<float2 *>(lds_raw + (sizeof(ChainShared) + 7) / 8);
    if (!J.all_live)
        chain_run<GM, true>(J, jb.J, S, win);
    else
        chain_run<GM, false>(J, jb.J, S, win);
}

// ------------------------------------------------------------- host side
namespace {

enum PreType { PT_BBOX = 0, PT_VERT, PT_SORT, PT_ONE, PT_MARK, PT_SCAN, PT_VERT8, PT_HEAVY, PT_BATCH, PT_CHAIN, PT_COUNT };

// Helper workgroups of a job's chain launch: none in one-shot force calls or
// when no batch of the run has old entries.
int chain_helpers(const BHJob &J) {
    if (J.all_live || J.last_batch <= J.lag) return 0;
    return std::min(J.helpers, J.last_batch - std::max(J.first_batch, J.lag + 1) + 1);
}

int blocks_for(int type, const BHJob &J) {
    const int n = J.n;
    switch (type) {
        case PT_BBOX: return std::max(1, std::min(kBBoxBlocks, (n + 255) / 256));
        case PT_VERT: return (n + 255) / 256;
        case PT_SORT: return J.tiles;
        case PT_ONE: return 1;
        case PT_MARK: return std::max(1, (n - 1 + 255) / 256);
        case PT_SCAN: return J.sblocks;
        case PT_VERT8: return (n + 31) / 32;
        case PT_HEAVY: return std::max(16, std::min(256, n / 512));
        case PT_BATCH: return J.nb;
        case PT_CHAIN: return 1 + chain_helpers(J);
    }
    return 0;
}

}  // namespace

// Device tables of the resident jobs, double-buffered so that a new job set
// can be uploaded while launches that read the previous one are in flight.
struct BHEngine {
    hipStream_t stream = nullptr;
    int G = 0, cap = 0, cur = 0;
    BHJob *d_jobs[2] = {nullptr, nullptr};
    int *d_pre[2] = {nullptr, nullptr};
    BHJob *h_jobs[2] = {nullptr, nullptr};   // pinned staging
    int *h_pre[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ev_used[2] = {false, false};
    int total[PT_COUNT] = {};
    int nkind[2] = {0, 0};              // jobs of the (2, -1) model, jobs of other (a, r) models
    int sort_scans = 0;                 // jobs with more than kFuseTiles sort tiles
    size_t lds_bytes = 0;               // dynamic LDS of the chain launch
    hipGraph_t graph = nullptr;         // one captured iteration of the current set
    hipGraphExec_t exec = nullptr;
};

// Dynamic LDS of the chain launch for a ring of `ring` vertices: the chain's
// shared block and ring, or the helpers' workspace, whichever is larger.
static size_t chain_lds_bytes(size_t ring) {
    return std::max((sizeof(ChainShared) + 7) / 8 * 8 + sizeof(float2) * ring, sizeof(HelperShared));
}

// Drop the captured iteration (after the stream has drained).
static void engine_drop_graph(BHEngine *e) {
    if (!e->exec && !e->graph) return;
    (void)hipStreamSynchronize(e->stream);
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->exec = nullptr;
    e->graph = nullptr;
}

int bh_engine_create(hipStream_t s, BHEngine **out) {
    BHEngine *e = new BHEngine();
    e->stream = s;
    for (int q = 0; q < 2; ++q) {
        hipError_t r = hipEventCreateWithFlags(&e->ev[q], hipEventDisableTiming);
        if (r != hipSuccess) {
            bh_engine_destroy(e);
            set_error("hipEventCreate failed: %s", hipGetErrorString(r));
            return BL_E_HIP;
        }
    }
    // the chain's window is dynamic LDS beyond the 64 KB default
    const void *chains[2] = {(const void *)chain_kernel<false>, (const void *)chain_kernel<true>};
    for (int kind = 0; kind < 2; ++kind) {
        hipError_t r = hipFuncSetAttribute(chains[kind], hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)chain_lds_bytes(kRing));
        if (r != hipSuccess) {
            bh_engine_destroy(e);
            set_error("hipFuncSetAttribute(chain_kernel) failed: %s", hipGetErrorString(r));
            return BL_E_HIP;
        }
    }
    *out = e;
    return BL_OK;
}

void bh_engine_destroy(BHEngine *e) {
    if (!e) return;
    engine_drop_graph(e);
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    for (int q = 0; q < 2; ++q) {
        if (e->d_jobs[q]) (void)hipFree(e->d_jobs[q]);
        if (e->d_pre[q]) (void)hipFree(e->d_pre[q]);
        if (e->h_jobs[q]) (void)hipHostFree(e->h_jobs[q]);
        if (e->h_pre[q]) (void)hipHostFree(e->h_pre[q]);
        if (e->ev[q]) (void)hipEventDestroy(e->ev[q]);
    }
    delete e;
}

// Descriptor of a job from its buffers.
int bh_fill_job(bl_graph *g, BHJob *J, const BHRunSpec &spec) {
    BHBuffers &h = g->bh;
    std::memset(J, 0, sizeof *J);
    J->n = (decltype(J->n))(g->n);
    J->BS = (decltype(J->BS))(g->p.batch_size);
    J->nb = (decltype(J->nb))(g->nb);
    J->tiles = (decltype(J->tiles))((g->n + kSortTile - 1) / kSortTile);
    J->sblocks = (decltype(J->sblocks))((g->n + kScanTile - 1) / kScanTile);
    J->theta2 = (decltype(J->theta2))((float)(g->p.theta * g->p.theta));
    J->negRK2 = (decltype(J->negRK2))((float)(-g->p.R * g->p.K * g->p.K));
    J->invK = (decltype(J->invK))((float)(1.0 / g->p.K));
    J->ka = (decltype(J->ka))(g->p.model_a - 1);
    J->kr = (decltype(J->kr))(g->p.model_r - 1);
    J->general = (decltype(J->general))(model_general(g->p) ? 1 : 0);
    J->snapshot_leaves = (decltype(J->snapshot_leaves))((g->p.flags & BL_BH_SNAPSHOT_LEAVES) ? 1 : 0);
    J->all_live = (decltype(J->all_live))(spec.all_live);
    J->first_batch = (decltype(J->first_batch))(spec.first_batch);
    J->last_batch = (decltype(J->last_batch))(spec.last_batch);
    J->stop_batch = (decltype(J->stop_batch))(spec.stop_batch);
    {
        // The chain's LDS ring holds lag + 1 batches.  A chain the ring holds
        // whole needs no helpers (no entry refers to a batch more than lag
        // back); a longer one keeps the last kLag batches and hands the rest
        // to helpers.  BL_BH_LAG caps the lag (tests, measurements).
        const int lmax = kRing / (int)g->p.batch_size - 1;
        if (lmax < kMinLag) {
            set_error("batch size %d above the chain's ring", (int)g->p.batch_size);
            return BL_E_INVAL;
        }
        int lag = (int)g->nb - 1 <= lmax ? std::max(1, (int)g->nb - 1) : std::min(kLag, lmax);
        if (const char *v = getenv("BL_BH_LAG")) lag = std::min(lag, std::max(kMinLag, atoi(v)));
        J->lag = (decltype(J->lag))lag;
        long long limit = 1ll << 18;   // polls of a microsecond or two each
        if (const char *v = getenv("BL_BH_SPIN_LIMIT")) limit = atoll(v);
        J->spin_limit = (decltype(J->spin_limit))limit;
    }
    J->step0 = (decltype(J->step0))(g->p.step0);
    J->decay = (decltype(J->decay))(g->p.step_decay);
    J->kiter = (decltype(J->kiter))(h.kiter);
    J->rowptr = (decltype(J->rowptr))(g->rowptr);
    J->colidx = (decltype(J->colidx))(g->colidx);
    J->pos = (decltype(J->pos))((float2 *)g->x);
    J->src = (decltype(J->src))(spec.src ? spec.src : (const float2 *)g->x);
    J->bbox = (decltype(J->bbox))(h.bbox);
    J->bbox_part = (decltype(J->bbox_part))(h.bbox_part);
    J->ticket = (decltype(J->ticket))((unsigned *)(h.bbox + 8));
    J->key0 = (decltype(J->key0))(h.key[0]);
    J->key1 = (decltype(J->key1))(h.key[1]);
    J->val0 = (decltype(J->val0))(h.val[0]);
    J->val1 = (decltype(J->val1))(h.val[1]);
    J->hist = (decltype(J->hist))(h.hist);
    J->mask = (decltype(J->mask))(h.mask);
    J->cellcnt = (decltype(J->cellcnt))(h.cellcnt);
    J->scan_part = (decltype(J->scan_part))(h.scan_part);
    J->pdd = (decltype(J->pdd))(h.pdd);
    J->pdd_part = (decltype(J->pdd_part))(h.pdd_part);
    J->nodeA = (decltype(J->nodeA))(h.nodeA);
    J->nodeB = (decltype(J->nodeB))(h.nodeB);
    J->leafpos = (decltype(J->leafpos))(h.leafpos);
    J->nnodes = (decltype(J->nnodes))(h.nnodes);
    J->far = (decltype(J->far))(h.far);
    J->late_cnt = (decltype(J->late_cnt))(h.late_cnt);
    J->late_ids = (decltype(J->late_ids))(h.late_ids);
    J->late_att = (decltype(J->late_att))(h.late_att);
    J->old_att = (decltype(J->old_att))(h.old_att);
    J->roff_old = (decltype(J->roff_old))(h.roff_old);
    J->bold = (decltype(J->bold))(h.bold);
    J->rec = (decltype(J->rec))(h.rec);
    J->rmeta = (decltype(J->rmeta))(h.rmeta);
    J->oldf = (decltype(J->oldf))(h.oldf);
    J->sync = (decltype(J->sync))(h.sync);
    J->hbase = (decltype(J->hbase))(h.hbase);
    J->hitem = (decltype(J->hitem))(h.hitem);
    J->heavy = (decltype(J->heavy))(h.heavy);
    J->nheavy = (decltype(J->nheavy))(h.nheavy);
    J->atte = (decltype(J->atte))(h.atte);
    J->roff = (decltype(J->roff))(h.roff);
    J->bbase = (decltype(J->bbase))(h.bbase);
    J->ent = (decltype(J->ent))(h.ent);
    J->ent_cap = (decltype(J->ent_cap))((size_t)g->nnz + (size_t)g->n * kLateCap);
    J->pstart = (decltype(J->pstart))(h.pstart);
    J->pbase = (decltype(J->pbase))(h.pbase);
    J->slots = (decltype(J->slots))(h.slots);
    J->pflag = (decltype(J->pflag))(h.pflag);
    J->bmeta = (decltype(J->bmeta))(h.bmeta);
    J->energy = (decltype(J->energy))(g->energy);
    J->fout = (decltype(J->fout))(g->fout);
    J->ctr = (decltype(J->ctr))(g->counters);
    J->conv_tol = (decltype(J->conv_tol))(spec.all_live || spec.stop_batch >= 0 ? 0.0 : g->p.conv_tol);
    return BL_OK;
}

// Make `jobs` the resident set (descriptors already filled).
int bh_engine_set(BHEngine *e, const BHJob *jobs, int G) {
    engine_drop_graph(e);
    const int s = e->cur ^ 1;
    if (e->ev_used[s]) BL_HIP(hipEventSynchronize(e->ev[s]));
    if (G > e->cap) {
        BL_HIP(hipStreamSynchronize(e->stream));
        const int cap = std::max(G, 2 * e->cap);
        for (int q = 0; q < 2; ++q) {
            if (e->d_jobs[q]) BL_HIP(hipFree(e->d_jobs[q]));
            if (e->d_pre[q]) BL_HIP(hipFree(e->d_pre[q]));
            if (e->h_jobs[q]) BL_HIP(hipHostFree(e->h_jobs[q]));
            if (e->h_pre[q]) BL_HIP(hipHostFree(e->h_pre[q]));
            e->d_jobs[q] = nullptr;
            e->d_pre[q] = nullptr;
            BL_HIP(hipMalloc((void **)&e->d_jobs[q], sizeof(BHJob) * cap));
            BL_HIP(hipMalloc((void **)&e->d_pre[q], sizeof(int) * PT_COUNT * (cap + 1)));
            BL_HIP(hipHostMalloc((void **)&e->h_jobs[q], sizeof(BHJob) * cap, hipHostMallocDefault));
            BL_HIP(hipHostMalloc((void **)&e->h_pre[q], sizeof(int) * PT_COUNT * (cap + 1), hipHostMallocDefault));
        }
        e->cap = cap;
        e->ev_used[0] = e->ev_used[1] = false;
    }
    std::memcpy(e->h_jobs[s], jobs, sizeof(BHJob) * G);
    // helpers: up to kHelpers per job, fewer when many jobs share the chip
    // (every job keeps one)
    for (int j = 0; j < G; ++j) e->h_jobs[s][j].helpers = std::max(1, std::min(kHelpers, 512 / std::max(1, G) - 1));
    for (int t = 0; t < PT_COUNT; ++t) {
        int *pre = e->h_pre[s] + t * (e->cap + 1);
        pre[0] = 0;
        for (int j = 0; j < G; ++j) pre[j + 1] = pre[j] + blocks_for(t, e->h_jobs[s][j]);
        e->total[t] = pre[G];
    }
    e->lds_bytes = sizeof(HelperShared);
    e->nkind[0] = e->nkind[1] = 0;
    e->sort_scans = 0;
    for (int j = 0; j < G; ++j) {
        const BHJob &J = jobs[j];
        ++e->nkind[J.general ? 1 : 0];
        if (J.tiles > kFuseTiles) ++e->sort_scans;
        e->lds_bytes = std::max(e->lds_bytes, chain_lds_bytes((size_t)J.BS * (J.all_live ? 0 : J.lag + 1)));
    }
    BL_HIP(hipMemcpyAsync(e->d_jobs[s], e->h_jobs[s], sizeof(BHJob) * G, hipMemcpyHostToDevice, e->stream));
    BL_HIP(hipMemcpyAsync(e->d_pre[s], e->h_pre[s], sizeof(int) * PT_COUNT * (e->cap + 1),
                          hipMemcpyHostToDevice, e->stream));
    // launches that read the previous tables are all enqueued before this point
    BL_HIP(hipEventRecord(e->ev[e->cur], e->stream));
    e->ev_used[e->cur] = true;
    e->cur = s;
    e->G = G;
    return BL_OK;
}

#define BH_LAUNCH(kernel, type, threads, ...)                                                       \
    do {                                                                                            \
        if (e->total[type] > 0)                                                                     \
            hipLaunchKernelGGL(kernel, dim3(e->total[type]), dim3(threads), 0, e->stream, jobs,     \
                               e->d_pre[e->cur] + (type) * (e->cap + 1), e->G, ##__VA_ARGS__);      \
    } while (0)

// A kernel with an instantiation per model kind: each kind present in the
// set gets its launch (the other kind's workgroups leave at once).
#define BH_LAUNCH_M(kernel, type, threads, ...)                  \
    do {                                                         \
        if (e->nkind[0]) BH_LAUNCH(kernel<false>, type, threads, ##__VA_ARGS__); \
        if (e->nkind[1]) BH_LAUNCH(kernel<true>, type, threads, ##__VA_ARGS__);  \
    } while (0)

// Once per job set: lengths of the moved-neighbour CSR prefixes, heavy rows.
int bh_engine_setup(BHEngine *e) {
    if (e->G == 0) return BL_OK;
    const BHJob *jobs = e->d_jobs[e->cur];
    BH_LAUNCH(heavy_reset_kernel, PT_ONE, 64);
    BH_LAUNCH(late_prefix_kernel, PT_VERT, 256);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

// One layout iteration of every job of the set.
int bh_engine_iteration(BHEngine *e, bl_graph *prof) {
    if (e->G == 0) return BL_OK;
    const BHJob *jobs = e->d_jobs[e->cur];
    int slot = -1;
    if (prof) BL_TRY(prof_begin(prof, PK_TREE, &slot));
    BH_LAUNCH(bbox_kernel, PT_BBOX, 256);
    BH_LAUNCH(morton_kernel, PT_VERT, 256);
    for (int pass = 0; pass < 4; ++pass) {
        BH_LAUNCH(radix_hist_kernel, PT_SORT, kSortThreads, pass);
        if (e->sort_scans) BH_LAUNCH(scan_single_kernel, PT_ONE, kScanThreads, 0);
        BH_LAUNCH(radix_scatter_kernel, PT_SORT, kSortThreads, pass);
    }
    BH_LAUNCH(mark_kernel, PT_MARK, 256);
    BH_LAUNCH(count_tile_kernel, PT_SCAN, kScanThreads);
    BH_LAUNCH(scan_single_kernel, PT_ONE, kScanThreads, 1);
    BH_LAUNCH(count_apply_kernel, PT_SCAN, kScanThreads);
    BH_LAUNCH(coord_tile_kernel, PT_SCAN, kScanThreads);
    BH_LAUNCH(coord_part_scan_kernel, PT_ONE, 64);
    BH_LAUNCH(coord_apply_kernel, PT_SCAN, kScanThreads);
    BH_LAUNCH(emit_kernel, PT_VERT, 256);
    if (prof) BL_TRY(prof_end(prof, slot));
    if (prof) BL_TRY(prof_begin(prof, PK_FAR, &slot));
    BH_LAUNCH_M(far_kernel, PT_VERT, 256);
    if (prof) BL_TRY(prof_end(prof, slot));
    BH_LAUNCH_M(att_early_kernel, PT_VERT8, 256);
    BH_LAUNCH_M(att_heavy_kernel, PT_HEAVY, 256);
    BH_LAUNCH(batch_offsets_kernel, PT_BATCH, 1024);
    BH_LAUNCH(scan_single_kernel, PT_ONE, kScanThreads, 2);
    BH_LAUNCH(late_fill_kernel, PT_VERT8, 256);
    BH_LAUNCH(late_fill_heavy_kernel, PT_HEAVY, 256);
    BH_LAUNCH(plan_count_kernel, PT_BATCH, 1024);
    BH_LAUNCH(scan_single_kernel, PT_ONE, kScanThreads, 3);
    BH_LAUNCH(plan_fill_kernel, PT_VERT, 256);
    if (prof) BL_TRY(prof_begin(prof, PK_CHAIN, &slot));
    for (int kind = 0; kind < 2; ++kind) {
        if (e->total[PT_CHAIN] == 0 || !e->nkind[kind]) continue;
        const int *pre = e->d_pre[e->cur] + PT_CHAIN * (e->cap + 1);
        hipLaunchKernelGGL(kind ? chain_kernel<true> : chain_kernel<false>, dim3(e->total[PT_CHAIN]),
                           dim3(kChainThreads), e->lds_bytes, e->stream, jobs, pre, e->G);
    }
    if (prof) BL_TRY(prof_end(prof, slot));
    BL_HIP(hipGetLastError());
    return BL_OK;
}

size_t bh_job_size() { return sizeof(BHJob); }

// `iters` iterations of the current job set.  With use_graph, one iteration's
// launches are captured once into a hipGraph and replayed (the iteration
// number lives on the device, so every replay is identical).
int bh_engine_run(BHEngine *e, int iters, bool use_graph) {
    if (e->G == 0 || iters <= 0) return BL_OK;
    if (!use_graph || iters == 1) {
        for (int t = 0; t < iters; ++t) BL_TRY(bh_engine_iteration(e, nullptr));
        return BL_OK;
    }
    if (!e->exec) {
        BL_HIP(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        int rc = bh_engine_iteration(e, nullptr);
        hipGraph_t graph = nullptr;
        hipError_t ce = hipStreamEndCapture(e->stream, &graph);
        if (rc != BL_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ce != hipSuccess) {
            set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ce));
            return BL_E_HIP;
        }
        hipGraphExec_t exec = nullptr;
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(graph);
            set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
            return BL_E_HIP;
        }
        e->graph = graph;
        e->exec = exec;
    }
    hipError_t le = hipSuccess;
    for (int t = 0; t < iters && le == hipSuccess; ++t) le = hipGraphLaunch(e->exec, e->stream);
    if (le != hipSuccess) {
        set_error("hipGraphLaunch failed: %s", hipGetErrorString(le));
        return BL_E_HIP;
    }
    return BL_OK;
}

// Helper items of an iteration at most: a part per batch, and one more per
// kPartEnt entries of the old lists (at most every list entry).
static size_t help_items(size_t nb, size_t ent) { return nb + ent / kPartEnt + 1; }

size_t bh_footprint(int n, int64_t nnz, int BS) {
    const size_t N = (size_t)n;
    const size_t tiles = (N + kSortTile - 1) / kSortTile;
    const size_t sblocks = (N + kScanTile - 1) / kScanTile;
    const size_t nb = (N + BS - 1) / BS;
    return 64 + 16 * kBBoxBlocks + 16 * N + 4 * 256 * tiles + 4 * N + 4 * (N + 1) + 4 * (sblocks + 1) +
           32 * (N + 1) + 32 * (sblocks + 1) + 2 * N * (16 + 8) + 4 * N + 16 + 16 * N + 4 * N +
           4 * N * kLateCap + 8 * N + 8 * (size_t)BS + 4 * N + 4 * N + 16 + 8 * N + 4 * N + 4 * (nb + 1) +
           8 * ((size_t)nnz + N * kLateCap) + 64 + 4 * N + 16 * N + 4 * (nb + 1) + 8 * N + 4 * (nb + kSyncReady) +
           4 * N + 4 * (nb + 1) + 8 * nb * (size_t)plan_cap(BS) + 4 * nb + 16 * N + 16 * nb + 4 * (nb + 1) +
           8 * help_items(nb, (size_t)nnz + N * kLateCap);
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
    BL_TRY(graph_alloc(g, (void **)&h.late_att, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.old_att, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.roff_old, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.bold, 4 * ((size_t)g->nb + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.rec, 16 * N));
    BL_TRY(graph_alloc(g, (void **)&h.rmeta, 8 * N));
    BL_TRY(graph_alloc(g, (void **)&h.oldf, 8 * N));
    BL_TRY(graph_alloc(g, (void **)&h.sync, 4 * ((size_t)g->nb + kSyncReady)));
    BL_TRY(graph_alloc(g, (void **)&h.hbase, 4 * ((size_t)g->nb + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.hitem, 8 * help_items(g->nb, (size_t)g->nnz + N * kLateCap)));
    BL_TRY(graph_alloc(g, (void **)&h.heavy, 8 * N));
    BL_TRY(graph_alloc(g, (void **)&h.nheavy, 16));
    BL_TRY(graph_alloc(g, (void **)&h.atte, 8 * N));
    BL_TRY(graph_alloc(g, (void **)&h.roff, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.bbase, 4 * ((size_t)g->nb + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.ent, 8 * ((size_t)g->nnz + N * kLateCap)));
    // slot plans: a batch's runs (at most kRunLanes lanes per row) packed into
    // 16-lane rows take fewer than twice their lanes, plus the last row's padding
    BL_TRY(graph_alloc(g, (void **)&h.pstart, 4 * N));
    BL_TRY(graph_alloc(g, (void **)&h.pbase, 4 * ((size_t)g->nb + 1)));
    BL_TRY(graph_alloc(g, (void **)&h.slots, 8 * (size_t)g->nb * plan_cap(g->p.batch_size)));
    BL_TRY(graph_alloc(g, (void **)&h.pflag, 4 * (size_t)g->nb));
    BL_TRY(graph_alloc(g, (void **)&h.bmeta, 16 * (size_t)g->nb));
    BL_TRY(graph_alloc(g, (void **)&h.kiter, 16));
    BL_HIP(hipMemsetAsync(h.bbox, 0, 64, g->stream));
    BL_HIP(hipMemsetAsync(h.kiter, 0, 16, g->stream));
    return BL_OK;
}

// Start a run of job g at iteration k (device-side iteration counter).
int bh_set_iteration(bl_graph *g, int k) {
    g->bh.host_kiter[0] = k;
    g->bh.host_kiter[1] = k;
    BL_HIP(hipMemcpyAsync(g->bh.kiter, g->bh.host_kiter, 2 * sizeof(int), hipMemcpyHostToDevice, g->stream));
    return BL_OK;
}

static int single_engine(bl_graph *g, const BHRunSpec &spec) {
    if (!g->bh.engine) BL_TRY(bh_engine_create(g->stream, &g->bh.engine));
    BHJob J;
    BL_TRY(bh_fill_job(g, &J, spec));
    BL_TRY(bh_engine_set(g->bh.engine, &J, 1));
    return BL_OK;
}

int bh_run(bl_graph *g, int iters, int start, int stop_batch) {
    if (iters <= 0) return BL_OK;
    BL_TRY(bh_set_iteration(g, start));
    BHRunSpec spec;
    spec.last_batch = g->nb - 1;
    BL_TRY(single_engine(g, spec));
    if (!g->bh.prefix_ready) {
        BL_TRY(bh_engine_setup(g->bh.engine));
        g->bh.prefix_ready = true;
    }
    for (int t = 0; t < iters; ++t) {
        if (t == iters - 1 && stop_batch >= 0) {
            BHRunSpec st;
            st.last_batch = stop_batch;
            st.stop_batch = stop_batch;
            BL_TRY(single_engine(g, st));
        }
        BL_TRY(bh_engine_iteration(g->bh.engine, g));
    }
    return BL_OK;
}

// Forces of one batch from coordinates (x, y) with the tree of the snapshot
// (snap_x, snap_y); every leaf and neighbour uses (x, y).
int bh_forces(bl_graph *g, int batch, const double *snap_x, const double *snap_y) {
    BHRunSpec spec;
    spec.all_live = 1;
    spec.first_batch = batch;
    spec.last_batch = batch;
    spec.stop_batch = batch;
    if (snap_x) {
        BL_TRY(convert_to_float2(g, snap_x, snap_y, (float2 *)g->bh.snap));
        spec.src = (const float2 *)g->bh.snap;
    }
    BL_TRY(bh_set_iteration(g, 0));
    BL_TRY(single_engine(g, spec));
    if (!g->bh.prefix_ready) {
        BL_TRY(bh_engine_setup(g->bh.engine));
        g->bh.prefix_ready = true;
    }
    return bh_engine_iteration(g->bh.engine, g);
}

}  // namespace bl
