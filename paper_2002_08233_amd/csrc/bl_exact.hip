// Exact-mode force step (Sec. 2.2 and 3.3, Alg. 2) for gfx950.
//
// Dataflow.  At step (k, b) the rows of batch b need the *new* coordinates of
// batches b' < b and the *old* ones (from iteration k-1) of batches b' >= b.
// Both are final as soon as the batch that owns them has moved, so once batch
// c has moved, every row can take in its contribution from batch c at once:
// rows of later batches add it to their iteration-k sum, rows of batches
// <= c to their iteration-(k+1) sum (they will see batch c as "old").  The
// contribution of a column batch to a row holds the repulsion from all of
// its columns and the attraction from the row's neighbours inside it (their
// positions are the same ones), so a row's net force is complete exactly
// when its batch comes up.
//
// One launch per step therefore does the panel of the batch that just moved
// over all n rows (full-chip parallelism) and, in the workgroups that hold
// the rows of the next batch, finishes those rows and moves them: their last
// contribution is the one this very launch adds.  The critical path of a
// step is one launch.
//
// Arithmetic (the same in every kernel here, so a graph's result does not
// depend on the launch shape, and a resumed run equals a continuous one
// bitwise).  Per row and column batch: the repulsion of the batch's columns
// in four interleaved partial sums (column q to sum q mod 4, ascending), the
// attraction (and, in literal mode, the neighbour repulsion) of the row's
// CSR entries inside the batch in a fixed order (four round-robin partials
// for entries 0..15, a pairwise tree over 64 lane sums for the rest),
// combined into one partial,
// then one compensated (Kahan) add into the row's sum.  Energy: per batch,
// each kRows-row chunk (aligned to absolute row ids) is summed by wave
// butterflies and then its wave sums in order; the chunk sums are added in
// row order; iteration energies add the batch sums in batch order.
//
// Kernels: rows_kernel (whole-column-batch sums: the prologue of a run and
// the one-shot force call), steps_kernel (all steps of a run in one
// cooperative launch: workgroups own fixed rows and wait only for the batch
// whose columns they add next), step_kernel (one step: panel + fused finish
// of the next batch; probes, and jobs that share the device),
// finalize_kernel (finish only: first batch of a run, probes, and
// single-batch graphs), exact_graph_kernel (one workgroup runs a whole small
// layout; many graphs per launch).
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "bl_device.hpp"
#include "bl_internal.hpp"

// Only explicit fma() calls fuse: the same row arithmetic is compiled into
// several kernels and must round identically in all of them.
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

constexpr int kRows = 128;     // rows per workgroup of the multi-workgroup kernels (= energy chunk)
constexpr int kChunkWaves = kRows / kWave;   // waves of one energy chunk at one lane per row
constexpr int kTile = 1024;    // columns staged in LDS per pass
constexpr int kSimds = 256 * 4;   // SIMDs of the chip (256 compute units x 4)
constexpr int kPre = 4;        // CSR entries of a row prefetched per column batch
// Graphs with n * BS up to this many pairs per step run alone in the
// one-workgroup kernel: one compute unit finishes such a step faster than
// a chain of full-chip launches.
constexpr long long kOneWGPairs = 3LL << 13;      // pairs per step up to which a graph runs in one workgroup
constexpr long long kOneWGMaxPairs = 1LL << 18;   // ... and up to which BL_EXACT_ONE_WG=1 may force it

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

// One CSR entry's terms, each rounded on its own so that they can be formed
// in any lane and then added in the fixed order: the attraction d * (c_j - c_i)
// without its factor 1/K (Sec. 2.2 with a = 2: magnitude d^2 / K along the
// unit vector), and the repulsion kernel (c_j - c_i) / d^2 that literal mode
// takes back out for a neighbour.
struct EntryTerms {
    template <typename T, typename T2>
    __device__ __forceinline__ static void att(T xi, T yi, T2 pj, T &tx, T &ty) {
        const T dx = pj.x - xi, dy = pj.y - yi;
        const T d = sqrt(fma(dx, dx, dy * dy));
        tx = d * dx;
        ty = d * dy;
    }
    __device__ __forceinline__ static void rep(float xi, float yi, float2 pj, float &ux, float &uy) {
        const float dx = pj.x - xi, dy = pj.y - yi;
        const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1e-30f)));
        ux = dx * inv;
        uy = dy * inv;
    }
    __device__ __forceinline__ static void rep(double xi, double yi, double2 pj, double &ux, double &uy) {
        const double dx = pj.x - xi, dy = pj.y - yi;
        const double inv = 1.0 / fma(dx, dx, fma(dy, dy, 1e-300));
        ux = dx * inv;
        uy = dy * inv;
    }
};

// Pair terms for model M: 0 = (2, -1) (Fruchterman-Reingold, the paths above
// unchanged), 1 = the general integer (a, r) of the view, 2 = general a with
// r = -1 (the repulsion of the (2, -1) paths, e.g. (1, -1) and (0, -1)).
template <int M, typename T, typename T2>
__device__ __forceinline__ void rep_pair(int kr, T xi, T yi, T2 pj, T &px, T &py) {
    if constexpr (M != 1) {
        rep_term(xi, yi, pj, px, py);
    } else {
        const T dx = pj.x - xi, dy = pj.y - yi;
        const T f = dpow(dx, dy, kr);
        px = fma(dx, f, px);
        py = fma(dy, f, py);
    }
}
template <int M, typename T, typename T2>
__device__ __forceinline__ void ent_att(int ka, T xi, T yi, T2 pj, T &tx, T &ty) {
    if constexpr (M == 0) {
        EntryTerms::att(xi, yi, pj, tx, ty);
    } else {
        const T dx = pj.x - xi, dy = pj.y - yi;
        const T f = dpow(dx, dy, ka);
        tx = f * dx;
        ty = f * dy;
    }
}
template <int M, typename T, typename T2>
__device__ __forceinline__ void ent_rep(int kr, T xi, T yi, T2 pj, T &ux, T &uy) {
    if constexpr (M != 1) {
        EntryTerms::rep(xi, yi, pj, ux, uy);
    } else {
        const T dx = pj.x - xi, dy = pj.y - yi;
        const T f = dpow(dx, dy, kr);
        ux = dx * f;
        uy = dy * f;
    }
}

// Four interleaved repulsion partials of one row.
template <typename T>
struct Rep4 {
    T x0, y0, x1, y1, x2, y2, x3, y3;
    __device__ void zero() { x0 = y0 = x1 = y1 = x2 = y2 = x3 = y3 = 0; }
};

// Columns [lo, hi) of the staged tile (lo a multiple of 4; the tile starts at
// a multiple of 4 columns from the batch start, so column q goes to sum q&3).
template <typename T>
__device__ __forceinline__ void rep_range(T xi, T yi, const typename V2<T>::type *cols, int lo, int hi, Rep4<T> &P) {
    int q = lo;
    for (; q + 4 <= hi; q += 4) {
        rep_term(xi, yi, cols[q], P.x0, P.y0);
        rep_term(xi, yi, cols[q + 1], P.x1, P.y1);
        rep_term(xi, yi, cols[q + 2], P.x2, P.y2);
        rep_term(xi, yi, cols[q + 3], P.x3, P.y3);
    }
    if (q < hi) rep_term(xi, yi, cols[q], P.x0, P.y0);
    if (q + 1 < hi) rep_term(xi, yi, cols[q + 1], P.x1, P.y1);
    if (q + 2 < hi) rep_term(xi, yi, cols[q + 2], P.x2, P.y2);
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

// Everything a kernel needs of one graph.
template <typename T>
struct GView {
    using T2 = typename V2<T>::type;
    int n, BS, nb, literal;
    T invK, negRK2;
    const int *rowptr, *colidx;
    const int2 *segs;
    const int *segoff;
    int *cursor;
    T *x, *y;
    T2 *accS[2];
    float2 *accC[2];
    int ka, kr;   // (a, r) model: the terms are d^(a-1) and d^(r-1) times (c_j - c_i)
    // by parity, without dynamic indexing (keeps a local view out of scratch)
    __device__ __forceinline__ T2 *S(int par) const { return par ? accS[1] : accS[0]; }
    __device__ __forceinline__ float2 *C(int par) const { return par ? accC[1] : accC[0]; }
};

// Order of the CSR terms of one row in one column batch.  Entry u of 0..15
// goes to partial u % 4; each partial adds its entries in order and the four
// meet as (V0 + V1) + (V2 + V3).  Entries 16.. (hub rows) are
// dealt round a wave: "lane" l in [0, 64) sums the terms of entries
// 16 + l, 16 + l + 64, 16 + l + 128, ... in that order, the 64 lane sums
// meet in a balanced pairwise tree over the lanes in order ((l0 + l1) +
// (l2 + l3)) + ..., and the tree's total is added last.  On a wave the tree
// is four data-parallel-primitive exchanges inside each 16-lane row (pairs at
// distance 1 and 2, then the row's half and whole mirror images, which pair
// equal quads and equal octets) and the four row totals read into scalars;
// the paths that take a row's entries one lane at a time evaluate the same
// tree with lane_tree.
template <typename T>
struct Sum4 {
    T ax, ay, lx, ly;
};
// The pairwise tree's total of leaf(0..63) (a 2-vector) evaluated by one
// lane: a stack of one subtree per level pairs each finished subtree with its
// left sibling.
template <typename T2, typename F>
__device__ __forceinline__ T2 lane_tree(const F &leaf) {
    T2 stk[6];
    T2 v{0, 0};
    for (int i = 0; i < kWave; ++i) {
        v = leaf(i);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int low = (1 << k) - 1;
            if ((i & low) != low) continue;   // a lower level kept the subtree
            if ((i >> k) & 1) {
#pragma clang fp contract(off)
                v = T2{stk[k].x + v.x, stk[k].y + v.y};
            } else {
                stk[k] = v;
            }
        }
    }
    return v;
}

// v + (v of the lane that DPP control CTRL selects), every lane active.
template <int CTRL>
__device__ __forceinline__ float dpp_pair(float v) {
    const int o = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false);
    float r;
    {
#pragma clang fp contract(off)
        r = v + __builtin_bit_cast(float, o);
    }
    return r;
}
template <int CTRL>
__device__ __forceinline__ double dpp_pair(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    const long long ob = ((long long)hi << 32) | (long long)(unsigned)lo;
    double r;
    {
#pragma clang fp contract(off)
        r = v + __builtin_bit_cast(double, ob);
    }
    return r;
}
__device__ __forceinline__ float lane_read(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
// The pairwise tree's total of the wave's 64 values (all lanes active; the
// result is uniform).  quad_perm [1,0,3,2] and [2,3,0,1] pair lanes at
// distance 1 and 2; once quads hold equal values the row half mirror pairs
// quad 0 with quad 1 of each octet, and once octets do the row mirror pairs
// the two octets of a row.  Each pair's two lanes add the same two values,
// so they hold the same bits.
template <typename T>
__device__ __forceinline__ T wave_tree(T v) {
    v = dpp_pair<0xB1>(v);    // quad_perm [1,0,3,2]
    v = dpp_pair<0x4E>(v);    // quad_perm [2,3,0,1]
    v = dpp_pair<0x141>(v);   // row_half_mirror
    v = dpp_pair<0x140>(v);   // row_mirror
    const T r0 = lane_read(v, 0), r1 = lane_read(v, 16), r2 = lane_read(v, 32), r3 = lane_read(v, 48);
    T t;
    {
#pragma clang fp contract(off)
        t = (r0 + r1) + (r2 + r3);
    }
    return t;
}

// Contribution of column batch c = [c0, c1) to row i (all threads of the
// workgroup call it; `active` rows compute).  `s` is the row's candidate
// segment (its next unconsumed CSR run), `send` the row's segment end.  On
// return (qx, qy) is the combined partial and `used` tells whether segment s
// belonged to batch c.  The row's CSR segment is prefetched halfway through
// the first column tile so that its latency hides behind the repulsion.
template <typename T>
__device__ __forceinline__ void batch_contrib(const GView<T> &G, int c, bool active, int i, T xi, T yi, int s,
                                              int send, typename V2<T>::type *cols, T &qx, T &qy, bool &used) {
    using T2 = typename V2<T>::type;
    const int c0 = c * G.BS, c1 = min(c0 + G.BS, G.n);
    const bool cand = active && s < send;
    int2 sg = make_int2(-1, 0);
    int eend = 0;
    if (cand) {
        sg = G.segs[s];
        eend = (s + 1 < send) ? G.segs[s + 1].y : G.rowptr[i + 1];
    }
    Rep4<T> P;
    P.zero();
    int pre[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) pre[u] = 0;
    int cnt = 0;
    used = false;
    for (int t0 = c0; t0 < c1; t0 += kTile) {
        const int m = min(kTile, c1 - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += blockDim.x) cols[q] = T2{G.x[t0 + q], G.y[t0 + q]};
        __syncthreads();
        if (active) {
            const int half = (t0 == c0) ? ((m / 2) & ~3) : 0;
            rep_range<T>(xi, yi, cols, 0, half, P);
            if (t0 == c0) {
                used = cand && sg.x == c;
                cnt = used ? eend - sg.y : 0;
#pragma unroll
                for (int u = 0; u < kPre; ++u)
                    if (u < cnt) pre[u] = G.colidx[sg.y + u];
            }
            rep_range<T>(xi, yi, cols, half, m, P);
        }
    }
    T ax = 0, ay = 0, lx = 0, ly = 0;
    if (active && cnt > 0) {
        const bool in_lds = (c1 - c0) <= kTile;   // the whole batch is staged
        // entries 0..15: entry u into partial u % 4, met as (V0 + V1) + (V2 + V3)
        Sum4<T> V[4] = {};
        auto one = [&](int j, int t) {
            const T2 pj = in_lds ? cols[j - c0] : T2{G.x[j], G.y[j]};
            T tx, ty, ux = 0, uy = 0;
            EntryTerms::att(xi, yi, pj, tx, ty);
            if (G.literal) EntryTerms::rep(xi, yi, pj, ux, uy);
            {
#pragma clang fp contract(off)
                V[t].ax += tx;
                V[t].ay += ty;
                if (G.literal) {
                    V[t].lx += ux;
                    V[t].ly += uy;
                }
            }
        };
#pragma unroll
        for (int u = 0; u < kPre; ++u)
            if (u < cnt) one(pre[u], u & 3);
        const int c16 = min(cnt, 16);
        for (int u = kPre; u < c16; u += 4) {
            int jj[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) jj[v] = (u + v < c16) ? G.colidx[sg.y + u + v] : 0;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (u + v < c16) one(jj[v], v);   // u is a multiple of 4
        }
        {
#pragma clang fp contract(off)
            ax = (V[0].ax + V[1].ax) + (V[2].ax + V[3].ax);
            ay = (V[0].ay + V[1].ay) + (V[2].ay + V[3].ay);
            lx = (V[0].lx + V[1].lx) + (V[2].lx + V[3].lx);
            ly = (V[0].ly + V[1].ly) + (V[2].ly + V[3].ly);
        }
        if (cnt > 16) {
            // entries 16.., one lane's share at a time, in the lanes' tree
            // (the attraction, then the literal repulsion in a second pass)
            const int st = sg.y;
            auto share = [&](bool rep_term) {
                return lane_tree<T2>([&](int l) {
                    T2 q{0, 0};
                    for (int e = 16 + l; e < cnt; e += kWave) {
                        const int j = G.colidx[st + e];
                        const T2 pj = in_lds ? cols[j - c0] : T2{G.x[j], G.y[j]};
                        T tx, ty;
                        if (rep_term) EntryTerms::rep(xi, yi, pj, tx, ty);
                        else EntryTerms::att(xi, yi, pj, tx, ty);
                        {
#pragma clang fp contract(off)
                            q.x += tx;
                            q.y += ty;
                        }
                    }
                    return q;
                });
            };
            const T2 ta = share(false);
            ax += ta.x;
            ay += ta.y;
            if (G.literal) {
                const T2 tl = share(true);
                lx += tl.x;
                ly += tl.y;
            }
        }
    }
    const T rx = (P.x0 + P.x1) + (P.x2 + P.x3);
    const T ry = (P.y0 + P.y1) + (P.y2 + P.y3);
    qx = G.invK * ax + G.negRK2 * (rx - lx);
    qy = G.invK * ay + G.negRK2 * (ry - ly);
}

// First segment of row i whose column batch is >= b (binary search).
__device__ __forceinline__ int first_seg_from(const int2 *segs, int s0, int s1, int b) {
    while (s0 < s1) {
        const int mid = (s0 + s1) >> 1;
        if (segs[mid].x < b) s0 = mid + 1;
        else s1 = mid;
    }
    return s0;
}

// Whole-column-batch sums for the rows [first, first + blockDim) below row1.
// from_own = 1: batches [batch(i), nb) (the run prologue: what a row sees as
// "old" in its first iteration); 0: all batches (one-shot forces).  Writes
// the sums of parity p, clears parity p^1 when asked, and points each row's
// cursor at its first segment (the next column batch to arrive is batch 0).
template <typename T, bool KAHAN>
__device__ __forceinline__ void rows_block(const GView<T> &G, int first, int row1, int from_own, int p, int clear_other,
                                           typename V2<T>::type *cols) {
    using T2 = typename V2<T>::type;
    const int i = first + threadIdx.x;
    const bool in = i < row1;
    const int bi = in ? i / G.BS : G.nb;
    T xi = 0, yi = 0;
    int s = 0, send = 0, srow = 0;
    if (in) {
        xi = G.x[i];
        yi = G.y[i];
        srow = G.segoff[i];
        send = G.segoff[i + 1];
        s = from_own ? first_seg_from(G.segs, srow, send, bi) : srow;
    }
    T2 acc{0, 0};
    float2 cc{0.f, 0.f};
    const int bstart = from_own ? min(first / G.BS, G.nb) : 0;
    for (int bb = bstart; bb < G.nb; ++bb) {
        const bool use = in && (!from_own || bb >= bi);
        T qx, qy;
        bool used;
        batch_contrib<T>(G, bb, use, i, xi, yi, s, send, cols, qx, qy, used);
        if (use) {
            acc_add<T, KAHAN>(acc, cc, qx, qy);
            if (used) ++s;
        }
    }
    if (in) {
        G.S(p)[i] = acc;
        if constexpr (KAHAN) G.C(p)[i] = cc;
        if (clear_other) {
            G.S(p ^ 1)[i] = T2{0, 0};
            if constexpr (KAHAN) G.C(p ^ 1)[i] = float2{0.f, 0.f};
        }
        G.cursor[i] = srow;
    }
}

// The same contribution with L lanes per row (L = 1, 2 or 4 consecutive
// lanes; lane h holds the partial sums m = h, h + L, ... and the lead lane
// h = 0 gets the combined partial).  The combine (P0 + P1) + (P2 + P3) and
// the CSR segment's order defined above make the bits those of
// batch_contrib.  The column loop runs on a wave-uniform counter.  The
// segment's first 16 entries are prefetched by the row's lanes halfway
// through the first tile and summed in the four round-robin partials; entries
// 16.. of longer segments (hub rows) are summed by all lanes of the wave, one
// row at a time, in the lane-sum and pairwise-tree order defined above.
// A coordinate that another workgroup of a running launch may have written:
// an agent-scope load, coherent across the chip's L2 caches.
template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// COH: the column batch was moved by another workgroup of the same launch
// (persistent run), so its coordinates are read with agent-scope loads.
template <typename T, int L, bool COH = false, int M = 0>
__device__ __forceinline__ void batch_contribL(const GView<T> &G, int c, bool active, bool lead, int i, T xi, T yi,
                                               int s, int send, typename V2<T>::type *cols, T &qx, T &qy,
                                               bool &used) {
    using T2 = typename V2<T>::type;
    constexpr int A = 4 / L;               // partial sums per lane
    constexpr int NP = 16 / L;             // prefetched entries per lane
    const int lane = threadIdx.x & (kWave - 1);
    const int h = threadIdx.x & (L - 1);
    const int c0 = c * G.BS, c1 = min(c0 + G.BS, G.n);
    const bool cand = active && s < send;
    int2 sg = make_int2(-1, 0);
    int eend = 0;
    if (cand) {
        sg = G.segs[s];
        eend = (s + 1 < send) ? G.segs[s + 1].y : G.rowptr[i + 1];
    }
    T px[A], py[A];
#pragma unroll
    for (int t = 0; t < A; ++t) px[t] = py[t] = 0;
    int pre[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) pre[k] = 0;
    int big[4] = {0, 0, 0, 0};     // entries 16.. of the wave's first long segment
    int cnt = 0, st0 = 0, ct0 = 0, src0 = -1;
    used = false;
    // columns [4 k0, 4 k1) of the staged tile; column 4k + h + L t -> sum t.
    // UG groups per loop round give every lane eight pairs a round at any L.
    constexpr int UG = 2 * L;
    auto group_range = [&](int k0, int k1) {
        int k = k0;
        for (; k + UG <= k1; k += UG) {
#pragma unroll
            for (int u = 0; u < UG; ++u) {
#pragma unroll
                for (int t = 0; t < A; ++t)
                    rep_pair<M>(G.kr, xi, yi, cols[4 * (k + u) + h + L * t], px[t], py[t]);
            }
        }
        for (; k < k1; ++k) {
#pragma unroll
            for (int t = 0; t < A; ++t) rep_pair<M>(G.kr, xi, yi, cols[4 * k + h + L * t], px[t], py[t]);
        }
    };
    for (int t0 = c0; t0 < c1; t0 += kTile) {
        const int m = min(kTile, c1 - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += blockDim.x) {
            if constexpr (COH) cols[q] = T2{ld_agent(G.x + t0 + q), ld_agent(G.y + t0 + q)};
            else cols[q] = T2{G.x[t0 + q], G.y[t0 + q]};
        }
        __syncthreads();
        const int groups = m >> 2;
        const int hg = (t0 == c0) ? (groups >> 1) : 0;
        if (active) group_range(0, hg);
        if (t0 == c0) {
            // CSR prefetch, in flight during the rest of the tile
            used = cand && sg.x == c;
            cnt = used ? eend - sg.y : 0;
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (h + L * k < cnt) pre[k] = G.colidx[sg.y + h + L * k];
            const unsigned long long longm = __ballot(lead && cnt > 16);
            if (longm) {
                src0 = __ffsll((long long)longm) - 1;
                st0 = __shfl(sg.y, src0, kWave);
                ct0 = __shfl(cnt, src0, kWave);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e = 16 + lane + kWave * k;
                    if (e < ct0) big[k] = G.colidx[st0 + e];
                }
            }
        }
        if (active) {
            group_range(hg, groups);
            // the last m % 4 columns
#pragma unroll
            for (int t = 0; t < A; ++t) {
                const int q = 4 * groups + h + L * t;
                if (q < m) rep_pair<M>(G.kr, xi, yi, cols[q], px[t], py[t]);
            }
        }
    }
    // (P0 + P1) + (P2 + P3)
    T rx, ry;
    if constexpr (L == 1) {
        rx = (px[0] + px[1]) + (px[2] + px[3]);
        ry = (py[0] + py[1]) + (py[2] + py[3]);
    } else if constexpr (L == 2) {
        const T a0 = px[0] + __shfl_xor(px[0], 1, kWave), b0 = py[0] + __shfl_xor(py[0], 1, kWave);
        const T a1 = px[1] + __shfl_xor(px[1], 1, kWave), b1 = py[1] + __shfl_xor(py[1], 1, kWave);
        rx = a0 + a1;
        ry = b0 + b1;
    } else {
        rx = px[0] + __shfl_xor(px[0], 1, kWave);
        ry = py[0] + __shfl_xor(py[0], 1, kWave);
        rx += __shfl_xor(rx, 2, kWave);
        ry += __shfl_xor(ry, 2, kWave);
    }
    T ax = 0, ay = 0, lx = 0, ly = 0;
    const bool in_lds = (c1 - c0) <= kTile;
    auto pos = [&](int j) {
        if (in_lds) return cols[j - c0];
        if constexpr (COH) return T2{ld_agent(G.x + j), ld_agent(G.y + j)};
        else return T2{G.x[j], G.y[j]};
    };
    // entries 0..15, held by the row's lanes (entry u in lane u % L, slot
    // u / L): entry u goes to partial u % 4, which lane h = u % L holds as its
    // partial t = (u / L) % A, as the repulsion's partials are held.  Each
    // partial adds its entries in order; the partials meet as (V0 + V1) +
    // (V2 + V3) by the repulsion's combine.
    Sum4<T> V[A];
#pragma unroll
    for (int t = 0; t < A; ++t) V[t] = Sum4<T>{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < NP; k0 += A) {
        if (!__ballot(lead && L * k0 < cnt)) break;
#pragma unroll
        for (int q = 0; q < A; ++q) {
            if (h + L * (k0 + q) < cnt) {
                const T2 pj = pos(pre[k0 + q]);
                T tx, ty, ux = 0, uy = 0;
                ent_att<M>(G.ka, xi, yi, pj, tx, ty);
                if (G.literal) ent_rep<M>(G.kr, xi, yi, pj, ux, uy);
                {
#pragma clang fp contract(off)
                    V[q].ax += tx;
                    V[q].ay += ty;
                    if (G.literal) {
                        V[q].lx += ux;
                        V[q].ly += uy;
                    }
                }
            }
        }
    }
    auto meet = [&](auto get) -> T {
        T r;
        {
#pragma clang fp contract(off)
            if constexpr (L == 1) {
                r = (get(V[0]) + get(V[1])) + (get(V[2]) + get(V[3]));
            } else if constexpr (L == 2) {
                const T a0 = get(V[0]) + __shfl_xor(get(V[0]), 1, kWave);
                const T a1 = get(V[1]) + __shfl_xor(get(V[1]), 1, kWave);
                r = a0 + a1;
            } else {
                r = get(V[0]) + __shfl_xor(get(V[0]), 1, kWave);
                r += __shfl_xor(r, 2, kWave);
            }
        }
        return r;
    };
    ax = meet([](const Sum4<T> &v) { return v.ax; });
    ay = meet([](const Sum4<T> &v) { return v.ay; });
    if (G.literal) {
        lx = meet([](const Sum4<T> &v) { return v.lx; });
        ly = meet([](const Sum4<T> &v) { return v.ly; });
    }
    // entries 16.. of long segments (hub rows), one row at a time: lane l of
    // the wave sums the terms of entries 16 + l + 64 g in order of g, the
    // lane sums meet in the wave's pairwise tree, and the row's lead lane adds
    // the total
    unsigned long long longm = __ballot(lead && cnt > 16);
    bool first_long = true;
    while (longm) {
        const int src = __ffsll((long long)longm) - 1;
        longm &= longm - 1;
        const int st = lane_read(sg.y, src), ct = lane_read(cnt, src);
        const T rxi = lane_read(xi, src), ryi = lane_read(yi, src);
        const bool have = first_long && src == src0;
        first_long = false;
        Sum4<T> q{0, 0, 0, 0};
        for (int b = 16; b < ct; b += 4 * kWave) {
            int jj[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = b + lane + kWave * k;
                jj[k] = have && b == 16 ? big[k] : (e < ct ? G.colidx[st + e] : c0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = b + lane + kWave * k;
                if (e < ct) {
                    const T2 pj = pos(jj[k]);
                    T tx, ty, ux = 0, uy = 0;
                    ent_att<M>(G.ka, rxi, ryi, pj, tx, ty);
                    if (G.literal) ent_rep<M>(G.kr, rxi, ryi, pj, ux, uy);
                    {
#pragma clang fp contract(off)
                        q.ax += tx;
                        q.ay += ty;
                        if (G.literal) {
                            q.lx += ux;
                            q.ly += uy;
                        }
                    }
                }
            }
        }
        const T sx = wave_tree(q.ax), sy = wave_tree(q.ay);
        T ux = 0, uy = 0;
        if (G.literal) {
            ux = wave_tree(q.lx);
            uy = wave_tree(q.ly);
        }
        if (lane == src) {
            ax += sx;
            ay += sy;
            lx += ux;
            ly += uy;
        }
    }
    qx = G.invK * ax + G.negRK2 * (rx - lx);
    qy = G.invK * ay + G.negRK2 * (ry - ly);
}

// rows_block with L lanes per row (workgroups of kRows * L; rows
// [first, first + kRows)).
template <typename T, bool KAHAN, int L, int M = 0>
__device__ __forceinline__ void rows_blockL(const GView<T> &G, int first, int row1, int from_own, int p, int clear_other,
                                            typename V2<T>::type *cols) {
    using T2 = typename V2<T>::type;
    const bool lead = (threadIdx.x & (L - 1)) == 0;
    const int i = first + threadIdx.x / L;
    const bool in = i < row1;
    const int bi = in ? i / G.BS : G.nb;
    T xi = 0, yi = 0;
    int s = 0, send = 0, srow = 0;
    if (in) {
        xi = G.x[i];
        yi = G.y[i];
        srow = G.segoff[i];
        send = G.segoff[i + 1];
        s = from_own ? first_seg_from(G.segs, srow, send, bi) : srow;
    }
    T2 acc{0, 0};
    float2 cc{0.f, 0.f};
    const int bstart = from_own ? min(first / G.BS, G.nb) : 0;
    for (int bb = bstart; bb < G.nb; ++bb) {
        const bool use = in && (!from_own || bb >= bi);
        T qx, qy;
        bool used;
        batch_contribL<T, L, false, M>(G, bb, use, lead, i, xi, yi, s, send, cols, qx, qy, used);
        if (use) {
            if (lead) acc_add<T, KAHAN>(acc, cc, qx, qy);
            if (used) ++s;
        }
    }
    if (in && lead) {
        G.S(p)[i] = acc;
        if constexpr (KAHAN) G.C(p)[i] = cc;
        if (clear_other) {
            G.S(p ^ 1)[i] = T2{0, 0};
            if constexpr (KAHAN) G.C(p ^ 1)[i] = float2{0.f, 0.f};
        }
        G.cursor[i] = srow;
    }
}

// Chunks of kRows rows; with `pair` (the run prologue, where chunk c sums the
// batches from its own on, so the work falls with c) workgroup b takes chunk b
// and chunk nblk - 1 - b, which evens out the workgroups' work.  A row's sums
// do not depend on which workgroup forms them.
template <typename T, bool KAHAN, int L, int M>
__global__ __launch_bounds__(kRows * L) void rows_kernel(GView<T> G, int row0, int row1, int from_own, int p,
                                                         int clear_other, int nblk, int pair) {
    __shared__ typename V2<T>::type cols[kTile];
    const int c = blockIdx.x;
    rows_blockL<T, KAHAN, L, M>(G, row0 + c * kRows, row1, from_own, p, clear_other, cols);
    if (pair && nblk - 1 - c > c)
        rows_blockL<T, KAHAN, L, M>(G, row0 + (nblk - 1 - c) * kRows, row1, from_own, p, clear_other, cols);
}

// The panel of column batch c for the rows [first, first + blockDim): rows of
// later batches add it to their parity-pc sums, rows of batches <= c (when
// do_next) to their parity-(pc^1) sums.  A row of batch `fin` keeps its
// completed sum in (fx, fy) (and its sums are cleared) instead of storing it.
template <typename T, bool KAHAN>
__device__ __forceinline__ void panel_rows(const GView<T> &G, int first, int c, int pc, int do_next, int fin,
                                           typename V2<T>::type *cols, T &xi, T &yi, T &fx, T &fy) {
    using T2 = typename V2<T>::type;
    const int i = first + threadIdx.x;
    const int bi = i < G.n ? i / G.BS : -1;
    const bool cur = i < G.n && bi > c;
    const bool nxt = do_next && i < G.n && bi >= 0 && bi <= c;
    const bool act = cur || nxt;
    int s = 0, send = 0;
    if (act) {
        xi = G.x[i];
        yi = G.y[i];
        s = G.cursor[i];
        send = G.segoff[i + 1];
    }
    T qx, qy;
    bool used;
    batch_contrib<T>(G, c, act, i, xi, yi, s, send, cols, qx, qy, used);
    if (act) {
        const int par = cur ? pc : (pc ^ 1);
        T2 acc = G.S(par)[i];
        float2 cc{0.f, 0.f};
        if constexpr (KAHAN) cc = G.C(par)[i];
        acc_add<T, KAHAN>(acc, cc, qx, qy);
        if (bi == fin) {
            fx = acc.x;
            fy = acc.y;
            if constexpr (KAHAN) {
                fx = acc.x - cc.x;
                fy = acc.y - cc.y;
            }
            G.S(par)[i] = T2{0, 0};
            if constexpr (KAHAN) G.C(par)[i] = float2{0.f, 0.f};
        } else {
            G.S(par)[i] = acc;
            if constexpr (KAHAN) G.C(par)[i] = cc;
        }
        G.cursor[i] = (c == G.nb - 1) ? G.segoff[i] : s + (used ? 1 : 0);
    }
}

// panel_rows with L lanes per row (workgroups of kRows * L, rows [first,
// first + kRows)); the completed sum of a row of batch `fin` lands in the
// lead lane's (fx, fy).
template <typename T, bool KAHAN, int L, bool COH = false, int M = 0>
__device__ __forceinline__ void panel_rowsL(const GView<T> &G, int first, int c, int pc, int do_next, int fin,
                                            typename V2<T>::type *cols, T &xi, T &yi, T &fx, T &fy) {
    using T2 = typename V2<T>::type;
    const bool lead = (threadIdx.x & (L - 1)) == 0;
    const int i = first + threadIdx.x / L;
    const int bi = i < G.n ? i / G.BS : -1;
    const bool cur = i < G.n && bi > c;
    const bool nxt = do_next && i < G.n && bi >= 0 && bi <= c;
    const bool act = cur || nxt;
    const int par = cur ? pc : (pc ^ 1);
    int s = 0, send = 0;
    T2 acc{0, 0};
    float2 cc{0.f, 0.f};
    if (act) {
        xi = G.x[i];
        yi = G.y[i];
        s = G.cursor[i];
        send = G.segoff[i + 1];
        if (lead) {
            acc = G.S(par)[i];
            if constexpr (KAHAN) cc = G.C(par)[i];
        }
    }
    T qx, qy;
    bool used;
    batch_contribL<T, L, COH, M>(G, c, act, lead, i, xi, yi, s, send, cols, qx, qy, used);
    if (act && lead) {
        acc_add<T, KAHAN>(acc, cc, qx, qy);
        if (bi == fin) {
            fx = acc.x;
            fy = acc.y;
            if constexpr (KAHAN) {
                fx = acc.x - cc.x;
                fy = acc.y - cc.y;
            }
            G.S(par)[i] = T2{0, 0};
            if constexpr (KAHAN) G.C(par)[i] = float2{0.f, 0.f};
        } else {
            G.S(par)[i] = acc;
            if constexpr (KAHAN) G.C(par)[i] = cc;
        }
        G.cursor[i] = (c == G.nb - 1) ? G.segoff[i] : s + (used ? 1 : 0);
    }
}

// Completed force of row i of the batch being finished, from memory.
template <typename T, bool KAHAN>
__device__ __forceinline__ void load_force(const GView<T> &G, int i, int pf, T &fx, T &fy) {
    using T2 = typename V2<T>::type;
    const T2 acc = G.S(pf)[i];
    fx = acc.x;
    fy = acc.y;
    if constexpr (KAHAN) {
        const float2 cc = G.C(pf)[i];
        fx = acc.x - cc.x;
        fy = acc.y - cc.y;
        G.C(pf)[i] = float2{0.f, 0.f};
    }
    G.S(pf)[i] = T2{0, 0};
}

// Move row i (c_i += Step f_i/|f_i|, none for |f_i| = 0; Alg. 2 update) and
// return |f_i|^2 in FP64 (0 for a non-finite force, which is counted).
template <typename T>
__device__ __forceinline__ double finish_row(const GView<T> &G, int i, int r, T xi, T yi, T fx, T fy, T step,
                                             int update, double *fout, unsigned long long &bad) {
    const double f2 = (double)fx * (double)fx + (double)fy * (double)fy;
    if (fout) {
        fout[2 * r] = (double)fx;
        fout[2 * r + 1] = (double)fy;
    }
    if (!isfinite(f2)) {
        ++bad;
        return 0.0;
    }
    if (update && f2 > 0.0) {
        const T nrm = sqrt(fx * fx + fy * fy);
        const T sc = step / nrm;
        G.x[i] = xi + sc * fx;
        G.y[i] = yi + sc * fy;
    }
    return f2;
}

// Sum over one kRows-row chunk held by kChunkWaves consecutive waves: wave
// butterflies, then the wave sums in order.  `ws` is LDS of one double per
// wave; `w0` the chunk's first wave.  Valid in the chunk's first thread; all
// threads of the workgroup call it.
__device__ __forceinline__ double chunk_sum(double e, double *ws, int w0) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    e = wave_sum(e);
    if (lane == 0) ws[w] = e;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == w0 * kWave) {
        r = ws[w0];
#pragma unroll
        for (int q = 1; q < kChunkWaves; ++q) r += ws[w0 + q];
    }
    __syncthreads();
    return r;
}

template <typename T>
struct FinArgs {
    int fin;              // batch to finish (-1: none)
    int pf;               // its iteration parity
    int update;           // move it (0: forces only)
    T step;
    double *energy_k;     // energy of its iteration (NULL: not recorded)
    double *fout;         // [2 * BS] FP64 forces out (NULL: none)
    double *epart;        // chunk partials of the batch
    unsigned *ticket;
    unsigned long long *nonfinite_count;
    // energy stopping rule: applied when the run's iteration ending with this
    // batch is not its first (energy_k > energy0)
    double conv_tol;      // 0: off
    const double *energy0;
    unsigned long long *halted;
};

// After the last batch of an iteration: the energy stopping rule, relative
// change against the run's previous iteration (COH: that energy was written
// by another workgroup of the same launch).
template <typename T, bool COH>
__device__ __forceinline__ void energy_rule(const FinArgs<T> &a, int nb, double ek) {
    if (a.conv_tol > 0 && a.fin == nb - 1 && a.energy_k > a.energy0) {
        const double ep = COH ? ld_agent(a.energy_k - 1) : a.energy_k[-1];
        if (fabs(ek - ep) <= a.conv_tol * ep) *a.halted = (unsigned long long)(a.energy_k - a.energy0) + 1;
    }
}
__device__ __forceinline__ bool halted_run(double conv_tol, const unsigned long long *h) {
    return conv_tol > 0 && h && *h;
}

// Finishing of batch a.fin by the workgroup holding rows [first, first +
// kRows): each row's force (already in (fx, fy) when `have`, else from
// memory), the move, and the batch energy, combined over the batch's chunks
// by the last workgroup to finish.
template <typename T, bool KAHAN>
__device__ __forceinline__ void finish_chunk(const GView<T> &G, const FinArgs<T> &a, int first, bool have, T xi, T yi,
                                             T fx, T fy, double *ws) {
    __shared__ int s_last;
    const int i = first + threadIdx.x;
    const int b0 = a.fin * G.BS, b1 = min(b0 + G.BS, G.n);
    const bool mine = i >= b0 && i < b1;
    double e = 0.0;
    unsigned long long bad = 0;
    if (mine) {
        if (!have) {
            xi = G.x[i];
            yi = G.y[i];
            load_force<T, KAHAN>(G, i, a.pf, fx, fy);
        }
        e = finish_row<T>(G, i, i - b0, xi, yi, fx, fy, a.step, a.update, a.fout, bad);
    }
    if (bad) atomicAdd(a.nonfinite_count, bad);
    const double cs = chunk_sum(e, ws, 0);
    if (!a.energy_k) return;
    const int ch0 = b0 / kRows, ch1 = (b1 - 1) / kRows, nch = ch1 - ch0 + 1;
    if (nch == 1) {
        if (threadIdx.x == 0) {
            const double ek = (a.fin == 0) ? cs : *a.energy_k + cs;
            *a.energy_k = ek;
            energy_rule<T, false>(a, G.nb, ek);
        }
        return;
    }
    if (threadIdx.x == 0) {
        a.epart[first / kRows - ch0] = cs;
        __threadfence();
        s_last = (atomicAdd(a.ticket, 1u) == (unsigned)(nch - 1));
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        const volatile double *ep = a.epart;
        double bs = ep[0];
        for (int q = 1; q < nch; ++q) bs += ep[q];
        const double ek = (a.fin == 0) ? bs : *a.energy_k + bs;
        *a.energy_k = ek;
        energy_rule<T, false>(a, G.nb, ek);   // (after the fence above)
        *a.ticket = 0u;
    }
}

// finish_chunk for the lead lanes of a kRows * L workgroup: the rows' |f|^2
// go through LDS to the first kRows threads, which sum them with the same tree
// as finish_chunk.
// The rows' moves and the chunk's energy sum (valid in thread 0).
template <typename T, bool KAHAN, int L>
__device__ __forceinline__ double finish_rowsL(const GView<T> &G, const FinArgs<T> &a, int first, T xi, T yi, T fx,
                                               T fy, double *e2, double *ws) {
    const bool lead = (threadIdx.x & (L - 1)) == 0;
    const int r = threadIdx.x / L;
    const int i = first + r;
    const int b0 = a.fin * G.BS, b1 = min(b0 + G.BS, G.n);
    const bool mine = lead && i >= b0 && i < b1;
    unsigned long long bad = 0;
    if (lead) e2[r] = mine ? finish_row<T>(G, i, i - b0, xi, yi, fx, fy, a.step, a.update, a.fout, bad) : 0.0;
    if (bad) atomicAdd(a.nonfinite_count, bad);
    __syncthreads();
    return chunk_sum(threadIdx.x < kRows ? e2[threadIdx.x] : 0.0, ws, 0);
}

template <typename T, bool KAHAN, int L, bool COH = false>
__device__ __forceinline__ void finish_chunkL(const GView<T> &G, const FinArgs<T> &a, int first, T xi, T yi, T fx,
                                              T fy, double *e2, double *ws) {
    __shared__ int s_last;
    const int b0 = a.fin * G.BS, b1 = min(b0 + G.BS, G.n);
    const double cs = finish_rowsL<T, KAHAN, L>(G, a, first, xi, yi, fx, fy, e2, ws);
    if (!a.energy_k) return;
    const int ch0 = b0 / kRows, ch1 = (b1 - 1) / kRows, nch = ch1 - ch0 + 1;
    // (COH: the running energy was written by another workgroup of the
    // same launch)
    if (nch == 1) {
        if (threadIdx.x == 0) {
            double prev = 0.0;
            if (a.fin != 0) prev = COH ? ld_agent(a.energy_k) : *a.energy_k;
            const double ek = (a.fin == 0) ? cs : prev + cs;
            *a.energy_k = ek;
            energy_rule<T, COH>(a, G.nb, ek);
        }
        return;
    }
    if (threadIdx.x == 0) {
        a.epart[first / kRows - ch0] = cs;
        __threadfence();
        s_last = (atomicAdd(a.ticket, 1u) == (unsigned)(nch - 1));
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        const volatile double *ep = a.epart;
        double bs = ep[0];
        for (int q = 1; q < nch; ++q) bs += ep[q];
        const double ek = (a.fin == 0) ? bs : *a.energy_k + bs;
        *a.energy_k = ek;
        energy_rule<T, false>(a, G.nb, ek);   // (after the fence above)
        *a.ticket = 0u;
    }
}

// Panel of column batch c (moved in an iteration of parity pc) over all rows,
// fused with the finish of batch fa.fin (whose last contribution is this
// panel's).  Needs nb > 1: the finished rows are read by no other workgroup.
template <typename T, bool KAHAN, int L, int M>
__global__ __launch_bounds__(kRows * L) void step_kernel(GView<T> G, int c, int pc, int do_next, FinArgs<T> fa) {
    if (halted_run(fa.conv_tol, fa.halted)) return;   // the energy stopping rule ended the run
    __shared__ typename V2<T>::type cols[kTile];
    __shared__ double ws[kRows * L / kWave];
    __shared__ double e2[kRows];
    const int first = blockIdx.x * kRows;
    const int i = first + threadIdx.x / L;
    const int bi = i < G.n ? i / G.BS : -1;
    const bool work = i < G.n && (bi > c || (do_next && bi <= c));
    const bool fin_row = fa.fin >= 0 && bi == fa.fin;
    if (!__syncthreads_or(work || fin_row)) return;
    T xi = 0, yi = 0, fx = 0, fy = 0;
    panel_rowsL<T, KAHAN, L, false, M>(G, first, c, pc, do_next, fa.fin, cols, xi, yi, fx, fy);
    if (fa.fin >= 0 && __syncthreads_or(fin_row)) finish_chunkL<T, KAHAN, L>(G, fa, first, xi, yi, fx, fy, e2, ws);
}

// ------------------------------------------------- persistent whole run
// A run as one launch of co-resident workgroups (cooperative launch).  Each
// workgroup owns fixed kRows-row chunks and walks the steps in order; a step
// waits only until the batch whose columns it adds has moved, and the
// workgroups holding the next batch's rows move them and count the move.
// Every wait is for an earlier step, so the launch always progresses; a wait
// that runs out sets a flag that makes every workgroup leave, and the run
// reports a time-out.  The arithmetic is that of step_kernel.
struct StepsArgs {
    int e0, e1;            // steps [e0, e1) of the run; step e adds batch (e-1) % nb, finishes batch e % nb
    int start, lastk;      // first and last iteration of the run
    double step_start;     // step length of iteration `start`
    double decay;
    double *energy;        // energy[k - start]
    unsigned *moved;       // [nb] chunk moves of each batch since the run started
    unsigned long long *abort;
    long long spin_limit;  // polls before a wait gives up
    // energies combined after the release (no stopping rule): per iteration
    // parity, chunk sums [nb][maxch], batch sums [nb], tickets [nb + 1]
    int deferred, maxch;
    double *echunk, *ebatch;
    unsigned *eticket;
};

// The iteration energy off the chain's critical path (thread 0 of a
// finishing workgroup, after its release): the chunk sum goes to its slot;
// the batch's last chunk adds the batch's chunk sums in order; the last
// batch's, once every batch of the iteration has its sum, adds the batch sums
// in batch order.  The same additions in the same order as the finish that
// combines them before the release.  Batch 0 of the run's first iteration was
// finished before the launch, its sum already in energy_k.
__device__ __forceinline__ void energy_deferred(const StepsArgs &A, int nb, int BS, int n, int fin, int kf, int first,
                                                double cs, double *energy_k) {
    const int p = kf & 1;
    const int b0 = fin * BS, b1 = min(b0 + BS, n);
    const int ch0 = b0 / kRows, nch = (b1 - 1) / kRows - ch0 + 1;
    double *ec = A.echunk + ((size_t)p * nb + fin) * A.maxch;
    unsigned *tk = A.eticket + (size_t)p * (nb + 1);
    ec[first / kRows - ch0] = cs;
    if (__hip_atomic_fetch_add(tk + fin, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) != (unsigned)(nch - 1)) return;
    double bs = ec[0];   // (after the acquire above)
    for (int q = 1; q < nch; ++q) bs += ec[q];
    __hip_atomic_store(tk + fin, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    A.ebatch[(size_t)p * nb + fin] = bs;
    const unsigned need = (kf == A.start) ? (unsigned)(nb - 1) : (unsigned)nb;
    if (__hip_atomic_fetch_add(tk + nb, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u == need) {
        // (after the acquire above, plain loads see every batch's sum; eight
        // in flight at a time, added in batch order)
        const double *eb = A.ebatch + (size_t)p * nb;
        double ek = (kf == A.start) ? *energy_k : eb[0];
        for (int b = 1; b < nb; b += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = b + u < nb ? eb[b + u] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (b + u < nb) ek += v[u];
        }
        *energy_k = ek;
        __hip_atomic_store(tk + nb, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Thread 0: wait until *cnt >= need (the caller then acquires).  Returns 0
// when the launch is being abandoned.
__device__ __forceinline__ int wait_moved(unsigned *cnt, unsigned need, unsigned long long *abort,
                                          long long limit) {
    for (long long it = 0;; ++it) {
        if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return 1;
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0;
        if (it >= limit) {
            __hip_atomic_store(abort, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__device__ __forceinline__ int batch_chunks(int b, int BS, int n) {
    const int b0 = b * BS, b1 = min(b0 + BS, n);
    return (b1 - 1) / kRows - b0 / kRows + 1;
}

template <typename T, bool KAHAN, int L, int M>
__global__ __launch_bounds__(kRows * L) void steps_kernel(GView<T> G, StepsArgs A, FinArgs<T> fa0) {
    __shared__ typename V2<T>::type cols[kTile];
    __shared__ double ws[kRows * L / kWave];
    __shared__ double e2[kRows];
    __shared__ int s_go[2];   // by step parity: thread 0 cannot be two steps ahead of a wave reading it
    const int nb = G.nb, nch = (G.n + kRows - 1) / kRows;
    int kf_cur = A.start;
    double st_cur = A.step_start;   // step length of iteration kf_cur (the host's sequential product)
    for (int e = A.e0; e < A.e1; ++e) {
        const int c = (e - 1) % nb, pk = A.start + (e - 1) / nb;
        const int fin = e % nb, kf = A.start + e / nb;
        const int do_next = pk < A.lastk ? 1 : 0;
        while (kf_cur < kf) {
            st_cur *= A.decay;
            ++kf_cur;
        }
        // batch c has moved in iteration pk
        const int fb0 = fin * G.BS, fb1 = min(fb0 + G.BS, G.n);
        const int fch0 = fb0 / kRows, fch1 = (fb1 - 1) / kRows;
        // What other workgroups of this launch wrote is read with agent-scope
        // loads: the moved columns and the running energy (the batch
        // partials of a batch of several chunks behind a fence of their
        // own), so no acquire has to drop this workgroup's cached rows.
        if (threadIdx.x == 0) {
            const unsigned need = (unsigned)(pk - A.start + 1) * (unsigned)batch_chunks(c, G.BS, G.n);
            int go = wait_moved(A.moved + c, need, A.abort, A.spin_limit);
            // the energy stopping rule held at the end of the previous step
            if (go && fa0.conv_tol > 0 && ld_agent(fa0.halted)) go = 0;
            s_go[e & 1] = go;
        }
        __syncthreads();
        if (!s_go[e & 1]) return;
        // the chunks of the batch to finish first: the next step waits for them
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = blockIdx.x; q < nch; q += gridDim.x) {
                const bool is_fin = q >= fch0 && q <= fch1;
                if ((pass == 0) != is_fin) continue;
                const int first = q * kRows, last = min(first + kRows, G.n) - 1;
                const bool work = last / G.BS > c || (do_next && first / G.BS <= c) || is_fin;
                if (!work) continue;
                T xi = 0, yi = 0, fx = 0, fy = 0;
                // the rows every workgroup waits for next go first on their SIMDs
                if (is_fin) __builtin_amdgcn_s_setprio(3);
                panel_rowsL<T, KAHAN, L, true, M>(G, first, c, pk & 1, do_next, fin, cols, xi, yi, fx, fy);
                if (is_fin) {
                    FinArgs<T> fa = fa0;
                    fa.fin = fin;
                    fa.pf = kf & 1;
                    fa.step = (T)st_cur;
                    fa.energy_k = A.energy + (kf - A.start);
                    double cs = 0.0;
                    if (A.deferred) cs = finish_rowsL<T, KAHAN, L>(G, fa, first, xi, yi, fx, fy, e2, ws);
                    else finish_chunkL<T, KAHAN, L, true>(G, fa, first, xi, yi, fx, fy, e2, ws);
                    // every wave's stores complete, then one release of them and the count
                    __builtin_amdgcn_s_waitcnt(0);
                    __syncthreads();
                    if (threadIdx.x == 0)
                        __hip_atomic_fetch_add(A.moved + fin, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_s_setprio(0);
                    if (A.deferred && threadIdx.x == 0 && fa.energy_k)
                        energy_deferred(A, nb, G.BS, G.n, fin, kf, first, cs, fa.energy_k);
                }
            }
        }
    }
}

// Move counters of a persistent run: batch 0 of its first iteration was
// finished before the launch.
__global__ void moved_init_kernel(unsigned *moved, int nb, unsigned first_chunks, unsigned *eticket) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) moved[b] = b == 0 ? first_chunks : 0u;
    for (int q = threadIdx.x; q < 2 * (nb + 1); q += blockDim.x) eticket[q] = 0u;
}


// Finish of batch fa.fin only (its sums are complete in memory).
template <typename T, bool KAHAN>
__global__ __launch_bounds__(kRows) void finalize_kernel(GView<T> G, FinArgs<T> fa) {
    if (halted_run(fa.conv_tol, fa.halted)) return;
    __shared__ double ws[kRows / kWave];
    const int first = (fa.fin * G.BS) / kRows * kRows + blockIdx.x * kRows;
    finish_chunk<T, KAHAN>(G, fa, first, false, 0, 0, 0, 0, ws);
}

// ------------------------------------------------- one workgroup per graph
// Many small graphs in one launch: each workgroup runs the whole layout of
// one graph, the steps in order with workgroup barriers between them, in
// passes of NT rows aligned to absolute row ids (so waves and kRows-row chunks
// cover the same rows as in the multi-workgroup kernels, and the result is
// the same bitwise).
struct ExactJob {
    int n, BS, nb, iters, start, literal;
    double step0, decay, invK, negRK2;
    const int *rowptr, *colidx;
    const int2 *segs;
    const int *segoff;
    int *cursor;
    void *x, *y;
    void *accS[2];
    float2 *accC[2];
    double *energy;
    unsigned long long *nonfinite;
    double conv_tol;                 // energy stopping rule (0: off)
    unsigned long long *halted;
};

template <typename T, bool KAHAN, int NT>
__global__ __launch_bounds__(NT) void exact_graph_kernel(const ExactJob *__restrict__ jobs) {
    using T2 = typename V2<T>::type;
    __shared__ T2 cols[kTile];
    __shared__ double ws[NT / kWave];
    __shared__ double s_batch;
    __shared__ int s_stop;
    const ExactJob &J0 = jobs[blockIdx.x];
    GView<T> G;
    G.n = J0.n;
    G.BS = J0.BS;
    G.nb = J0.nb;
    G.literal = J0.literal;
    G.ka = 1;    // this kernel runs the (2, -1) model only
    G.kr = -2;
    G.invK = (T)J0.invK;
    G.negRK2 = (T)J0.negRK2;
    G.rowptr = J0.rowptr;
    G.colidx = J0.colidx;
    G.segs = J0.segs;
    G.segoff = J0.segoff;
    G.cursor = J0.cursor;
    G.x = (T *)J0.x;
    G.y = (T *)J0.y;
    G.accS[0] = (T2 *)J0.accS[0];
    G.accS[1] = (T2 *)J0.accS[1];
    G.accC[0] = J0.accC[0];
    G.accC[1] = J0.accC[1];
    const int iters = J0.iters, start = J0.start;
    double *energy = J0.energy;
    unsigned long long *nonfinite = J0.nonfinite;
    if (iters <= 0) return;
    const int n = G.n, nb = G.nb, BS = G.BS;
    const int p0 = start & 1;
    for (int first = 0; first < n; first += NT) rows_block<T, KAHAN>(G, first, n, 1, p0, 1, cols);
    __syncthreads();
    double step = J0.step0;
    for (int t = 0; t < start; ++t) step *= J0.decay;
    const int lastk = start + iters - 1;
    const int w = threadIdx.x / kWave;
    unsigned long long bad = 0;
    // finish batch b of iteration k from memory
    auto finish = [&](int k, int b, double stepk) {
        const int b0 = b * BS, b1 = min(b0 + BS, n);
        const int f0 = b0 / NT * NT;
        for (int first = f0; first < b1; first += NT) {
            const int i = first + threadIdx.x;
            double e = 0.0;
            if (i >= b0 && i < b1) {
                T fx, fy;
                const T xi = G.x[i], yi = G.y[i];
                load_force<T, KAHAN>(G, i, k & 1, fx, fy);
                e = finish_row<T>(G, i, i - b0, xi, yi, fx, fy, (T)stepk, 1, nullptr, bad);
            }
            e = wave_sum(e);
            if ((threadIdx.x & (kWave - 1)) == 0) ws[w] = e;
            __syncthreads();
            if (threadIdx.x == 0) {
                double bs = (first == f0) ? 0.0 : s_batch;
                for (int ch = 0; ch < NT / kRows; ++ch) {
                    const int cf = first + ch * kRows;
                    if (cf + kRows <= b0 || cf >= b1) continue;
                    double cs = ws[kChunkWaves * ch];
#pragma unroll
                    for (int q = 1; q < kChunkWaves; ++q) cs += ws[kChunkWaves * ch + q];
                    bs = (cf <= b0) ? cs : bs + cs;
                }
                s_batch = bs;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double *ek = energy + (k - start);
            *ek = (b == 0) ? s_batch : *ek + s_batch;
        }
    };
    finish(start, 0, step);
    __syncthreads();
    for (int k = start; k <= lastk; ++k) {
        const double stepk = step;
        for (int b = 0; b < nb; ++b) {
            // the panel of batch b (moved in iteration k), then the next batch
            const bool has_next = (b + 1 < nb) || (k < lastk);
            if (!has_next) break;
            if (b == nb - 1 && J0.conv_tol > 0 && k > start) {
                // E_k is final: the energy stopping rule before batch 0 of k + 1 moves
                if (threadIdx.x == 0) {
                    const double ek = energy[k - start], ep = energy[k - start - 1];
                    s_stop = fabs(ek - ep) <= J0.conv_tol * ep;
                    if (s_stop) *J0.halted = (unsigned long long)(k - start + 1);
                }
                __syncthreads();
                if (s_stop) {
                    if (bad) atomicAdd(nonfinite, bad);
                    return;
                }
            }
            const int do_next = k < lastk ? 1 : 0;
            for (int first = 0; first < n; first += NT) {
                T xi = 0, yi = 0, fx = 0, fy = 0;
                panel_rows<T, KAHAN>(G, first, b, k & 1, do_next, -1, cols, xi, yi, fx, fy);
            }
            __syncthreads();
            if (b + 1 < nb) finish(k, b + 1, stepk);
            else finish(k + 1, 0, stepk * J0.decay);
            __syncthreads();
        }
        step *= J0.decay;
    }
    if (bad) atomicAdd(nonfinite, bad);
}

template <typename T, bool KAHAN, int M>
struct ExactOps {
    using T2 = typename V2<T>::type;

    static GView<T> view(bl_graph *g) {
        GView<T> G;
        G.n = g->n;
        G.BS = g->p.batch_size;
        G.nb = g->nb;
        G.literal = g->p.repulse_adjacent ? 0 : 1;
        G.ka = g->p.model_a - 1;
        G.kr = g->p.model_r - 1;
        G.invK = (T)(1.0 / g->p.K);
        G.negRK2 = (T)(-g->p.R * g->p.K * g->p.K);
        G.rowptr = g->rowptr;
        G.colidx = g->colidx;
        G.segs = g->ex.segs;
        G.segoff = g->ex.segoff;
        G.cursor = g->ex.cursor;
        G.x = (T *)g->x;
        G.y = (T *)g->y;
        G.accS[0] = (T2 *)g->ex.accS[0];
        G.accS[1] = (T2 *)g->ex.accS[1];
        G.accC[0] = g->ex.accC[0];
        G.accC[1] = g->ex.accC[1];
        return G;
    }

    // Lanes per row of the multi-workgroup kernels: enough waves per SIMD to
    // hide latency, as few lanes as that allows (each lane's loop overhead is
    // shared by more pairs).  Two lanes from two one-lane waves per SIMD up:
    // with fewer, the workgroups that finish a batch -- the chain's critical
    // path -- run on too few waves (rgg64k, 1024 one-lane waves: 1.49 ms per
    // iteration at four lanes, 1.67 at two).  The result does not depend on it.
    static int lanes(bl_graph *g, int rows) {
        if (const char *e = getenv("BL_EXACT_LANES")) {
            const int v = atoi(e);
            if (v == 1 || v == 2 || v == 4) return v;
        }
        const long long waves1 = ((long long)rows + kWave - 1) / kWave;   // waves at one lane per row
        if (waves1 >= 8LL * kSimds) return 1;
        if (waves1 >= 2LL * kSimds) return 2;
        return 4;
    }

    static int rows(bl_graph *g, int row0, int row1, int from_own, int parity, int clear_other) {
        if (row1 <= row0) return BL_OK;
        const int nblk = (row1 - row0 + kRows - 1) / kRows;
        const int pair = from_own ? 1 : 0;
        const int blocks = pair ? (nblk + 1) / 2 : nblk;
        int slot;
        BL_TRY(prof_begin(g, PK_ROWS, &slot));
        // paired chunks: half as many workgroups hold the rows at a time
        const int L = lanes(g, pair ? blocks * kRows : row1 - row0);
        if (L == 1)
            hipLaunchKernelGGL((rows_kernel<T, KAHAN, 1, M>), dim3(blocks), dim3(kRows), 0, g->stream, view(g), row0,
                               row1, from_own, parity, clear_other, nblk, pair);
        else if (L == 2)
            hipLaunchKernelGGL((rows_kernel<T, KAHAN, 2, M>), dim3(blocks), dim3(kRows * 2), 0, g->stream, view(g),
                               row0, row1, from_own, parity, clear_other, nblk, pair);
        else
            hipLaunchKernelGGL((rows_kernel<T, KAHAN, 4, M>), dim3(blocks), dim3(kRows * 4), 0, g->stream, view(g),
                               row0, row1, from_own, parity, clear_other, nblk, pair);
        BL_HIP(hipGetLastError());
        return prof_end(g, slot);
    }

    static FinArgs<T> fin_args(bl_graph *g, int b, int k, double *energy_k, double *fout, int update) {
        FinArgs<T> a;
        a.fin = b;
        a.pf = k & 1;
        a.update = update;
        a.step = (T)step_at(g->p, k);
        a.energy_k = energy_k;
        a.fout = fout;
        a.epart = g->ex.epart;
        a.ticket = g->ex.ticket;
        a.nonfinite_count = &g->counters->nonfinite;
        a.conv_tol = g->p.conv_tol;
        a.energy0 = g->energy;
        a.halted = &g->counters->halted;
        return a;
    }

    static FinArgs<T> no_fin() {
        FinArgs<T> a{};
        a.fin = -1;
        return a;
    }

    static int step(bl_graph *g, int c, int pc, int do_next, const FinArgs<T> &fa) {
        const int blocks = (g->n + kRows - 1) / kRows;
        int slot;
        BL_TRY(prof_begin(g, PK_PANEL, &slot));
        const int L = lanes(g, g->n);
        if (L == 1)
            hipLaunchKernelGGL((step_kernel<T, KAHAN, 1, M>), dim3(blocks), dim3(kRows), 0, g->stream, view(g), c, pc,
                               do_next, fa);
        else if (L == 2)
            hipLaunchKernelGGL((step_kernel<T, KAHAN, 2, M>), dim3(blocks), dim3(kRows * 2), 0, g->stream, view(g), c,
                               pc, do_next, fa);
        else
            hipLaunchKernelGGL((step_kernel<T, KAHAN, 4, M>), dim3(blocks), dim3(kRows * 4), 0, g->stream, view(g), c,
                               pc, do_next, fa);
        BL_HIP(hipGetLastError());
        return prof_end(g, slot);
    }

    // Steps [e0, e1) of a run as one cooperative launch of co-resident
    // workgroups (steps_kernel).  `launched` stays 0 when the device cannot
    // hold a workgroup of it; the caller then launches step by step.
    static int steps(bl_graph *g, int e0, int e1, int start, int lastk, int &launched) {
        launched = 0;
        const int L = lanes(g, g->n);
        const void *f = L == 1 ? (const void *)steps_kernel<T, KAHAN, 1, M>
                               : (L == 2 ? (const void *)steps_kernel<T, KAHAN, 2, M> : (const void *)steps_kernel<T, KAHAN, 4, M>);
        int dev = 0, cus = 0, per_cu = 0;
        BL_HIP(hipGetDevice(&dev));
        BL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kRows * L, 0));
        const int nch = (g->n + kRows - 1) / kRows;
        const int grid = std::min(nch, per_cu * cus);
        if (grid < 1) return BL_OK;
        long long limit = 1ll << 22;   // polls of about a microsecond each
        if (const char *v = getenv("BL_EXACT_SPIN_LIMIT")) limit = atoll(v);
        const int BS = g->p.batch_size;
        const unsigned first_chunks = (unsigned)((std::min(BS, g->n) - 1) / kRows + 1);
        hipLaunchKernelGGL(moved_init_kernel, dim3(1), dim3(256), 0, g->stream, g->ex.moved, g->nb, first_chunks,
                           g->ex.eticket);
        BL_HIP(hipGetLastError());
        StepsArgs A;
        A.e0 = e0;
        A.e1 = e1;
        A.start = start;
        A.lastk = lastk;
        A.step_start = step_at(g->p, start);
        A.decay = g->p.step_decay;
        A.energy = g->energy;
        A.moved = g->ex.moved;
        A.abort = &g->counters->wait_abort;
        A.spin_limit = limit;
        A.deferred = g->p.conv_tol > 0 ? 0 : 1;   // (the stopping rule needs each energy before the next step)
        A.maxch = BS / kRows + 2;
        A.echunk = g->ex.echunk;
        A.ebatch = g->ex.ebatch;
        A.eticket = g->ex.eticket;
        FinArgs<T> fa0 = fin_args(g, 0, start, nullptr, nullptr, 1);
        GView<T> G = view(g);
        void *args[] = {&G, &A, &fa0};
        int slot;
        BL_TRY(prof_begin(g, PK_STEPS, &slot));
        BL_HIP(hipLaunchCooperativeKernel(f, dim3(grid), dim3(kRows * L), args, 0, g->stream));
        BL_TRY(prof_end(g, slot));
        launched = 1;
        return BL_OK;
    }

    static int finalize(bl_graph *g, const FinArgs<T> &fa) {
        const int BS = g->p.batch_size;
        const int b0 = fa.fin * BS, b1 = std::min(g->n, b0 + BS);
        const int blocks = (b1 - 1) / kRows - b0 / kRows + 1;
        int slot;
        BL_TRY(prof_begin(g, PK_FINALIZE, &slot));
        hipLaunchKernelGGL((finalize_kernel<T, KAHAN>), dim3(blocks), dim3(kRows), 0, g->stream, view(g), fa);
        BL_HIP(hipGetLastError());
        return prof_end(g, slot);
    }

    // iters iterations from iteration `start`; with stop_batch >= 0 the last
    // iteration ends before batch stop_batch, whose forces go to g->fout.
    static int run(bl_graph *g, int iters, int start, int stop_batch) {
        if (iters <= 0) return BL_OK;
        const int nb = g->nb;
        const long long total = (stop_batch >= 0) ? (long long)(iters - 1) * nb + stop_batch + 1
                                                  : (long long)iters * nb;
        const int lastk = start + iters - 1;
        const bool cont = g->cont_iter == start;
        g->cont_iter = -1;
        // keep: the last iteration's panels also count toward iteration lastk+1
        const bool keep = g->keep_next && stop_batch < 0 && g->p.conv_tol == 0;
        const int next_bound = keep ? lastk + 1 : lastk;
        if (!cont) BL_TRY(rows(g, 0, g->n, 1, start & 1, 1));
        auto fin_of = [&](long long e) {
            const int k = start + (int)(e / nb), b = (int)(e % nb);
            const bool probe = stop_batch >= 0 && e == total - 1;
            return fin_args(g, b, k, probe ? nullptr : g->energy + (k - start), probe ? g->fout : nullptr,
                            probe ? 0 : 1);
        };
        BL_TRY(finalize(g, fin_of(0)));
        // the rest as one persistent launch where the device may be held
        if (stop_batch < 0 && nb > 1 && total > 1 && total < (1ll << 30) && g->coop && !getenv("BL_EXACT_STEPWISE")) {
            int launched = 0;
            BL_TRY(steps(g, 1, (int)total, start, next_bound, launched));
            if (launched) return keep ? keep_last_panel(g, lastk) : BL_OK;
        }
        for (long long e = 1; e < total; ++e) {
            const int pk = start + (int)((e - 1) / nb), pb = (int)((e - 1) % nb);
            const int do_next = pk < next_bound ? 1 : 0;
            if (nb > 1) {
                BL_TRY(step(g, pb, pk & 1, do_next, fin_of(e)));
            } else {
                BL_TRY(step(g, pb, pk & 1, do_next, no_fin()));
                BL_TRY(finalize(g, fin_of(e)));
            }
        }
        return keep ? keep_last_panel(g, lastk) : BL_OK;
    }

    // The panel of the last batch moved in iteration lastk, added toward
    // iteration lastk+1 (the step a longer run would take next, without its
    // finish); the next run may then start at lastk+1 without its prologue.
    static int keep_last_panel(bl_graph *g, int lastk) {
        BL_TRY(step(g, g->nb - 1, lastk & 1, 1, no_fin()));
        g->cont_iter = lastk + 1;
        return BL_OK;
    }

    static int forces(bl_graph *g, int batch) {
        const int BS = g->p.batch_size;
        const int r0 = batch * BS, r1 = std::min(g->n, r0 + BS);
        BL_TRY(rows(g, r0, r1, 0, 0, 0));
        return finalize(g, fin_args(g, batch, 0, nullptr, g->fout, 0));
    }
};

// CSR segments: per row, the runs of neighbours that fall in one column batch.
// One wave per row (rows are sorted, so a run starts where the column batch
// changes); lane l looks at entries rowptr[i] + l + 64 k, so a hub row costs
// its length / 64 rounds.
constexpr int kSegRowsPerBlock = 4;   // waves (rows) per 256-thread workgroup

__device__ __forceinline__ bool seg_start(const int *__restrict__ colidx, int BS, int e0, int e) {
    return e == e0 || colidx[e] / BS != colidx[e - 1] / BS;
}

__global__ __launch_bounds__(256) void seg_count_kernel(int n, int BS, const int *__restrict__ rowptr,
                                                        const int *__restrict__ colidx, int *__restrict__ cnt) {
    const int i = blockIdx.x * kSegRowsPerBlock + (int)(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    if (i >= n) return;   // the whole wave
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    int c = 0;
    for (int b0 = e0; b0 < e1; b0 += kWave) {
        const int e = b0 + lane;
        c += __popcll(__ballot(e < e1 && seg_start(colidx, BS, e0, e)));
    }
    if (lane == 0) cnt[i] = c;
}

// Exclusive scan of cnt[0..n) into off[0..n] by one workgroup of 1024.
__global__ __launch_bounds__(1024) void seg_scan_kernel(int n, const int *__restrict__ cnt, int *__restrict__ off) {
    __shared__ int wsum[16];
    int base = 0;
    for (int t0 = 0; t0 < n; t0 += 1024) {
        const int i = t0 + threadIdx.x;
        const int v = i < n ? cnt[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, wsum, &tot);
        if (i < n) off[i] = base + ex;
        base += tot;
    }
    if (threadIdx.x == 0) off[n] = base;
}

__global__ __launch_bounds__(256) void seg_fill_kernel(int n, int BS, const int *__restrict__ rowptr,
                                                       const int *__restrict__ colidx, const int *__restrict__ off,
                                                       int2 *__restrict__ segs) {
    const int i = blockIdx.x * kSegRowsPerBlock + (int)(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    if (i >= n) return;   // the whole wave
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    const unsigned long long below = (1ull << lane) - 1;
    int s = off[i];
    for (int b0 = e0; b0 < e1; b0 += kWave) {
        const int e = b0 + lane;
        const bool start = e < e1 && seg_start(colidx, BS, e0, e);
        const unsigned long long m = __ballot(start);
        if (start) segs[s + __popcll(m & below)] = make_int2(colidx[e] / BS, e);
        s += __popcll(m);
    }
}

}  // namespace

#ifdef BL_EXACT_MODELS_TU
// Runs and force calls under (a, r) models other than (2, -1).  They are
// instantiated in a translation unit of their own: next to the (2, -1)
// kernels in one code object they slowed those by about 3% (placement).
int exact_run_model(bl_graph *g, int iters, int start_iter, int stop_batch) {
    if (g->p.model_r == -1) {
        if (g->fp64) return ExactOps<double, false, 2>::run(g, iters, start_iter, stop_batch);
        if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false, 2>::run(g, iters, start_iter, stop_batch);
        return ExactOps<float, true, 2>::run(g, iters, start_iter, stop_batch);
    }
    if (g->fp64) return ExactOps<double, false, 1>::run(g, iters, start_iter, stop_batch);
    if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false, 1>::run(g, iters, start_iter, stop_batch);
    return ExactOps<float, true, 1>::run(g, iters, start_iter, stop_batch);
}

int exact_forces_model(bl_graph *g, int batch) {
    if (g->p.model_r == -1) {
        if (g->fp64) return ExactOps<double, false, 2>::forces(g, batch);
        if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false, 2>::forces(g, batch);
        return ExactOps<float, true, 2>::forces(g, batch);
    }
    if (g->fp64) return ExactOps<double, false, 1>::forces(g, batch);
    if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false, 1>::forces(g, batch);
    return ExactOps<float, true, 1>::forces(g, batch);
}
#else

// Launch one workgroup per graph for a group of exact-mode graphs that share
// a precision.  threads: 256, 512 or 1024 (the result does not depend on it).
int exact_graph_launch(bl_graph *const *gs, int G, int threads, hipStream_t s, void *d_jobs, int iters_override,
                       int start_override) {
    if (G == 0) return BL_OK;
    std::vector<ExactJob> jobs(G);
    for (int q = 0; q < G; ++q) {
        bl_graph *g = gs[q];
        ExactJob &J = jobs[q];
        J.n = g->n;
        J.BS = g->p.batch_size;
        J.nb = g->nb;
        J.iters = iters_override >= 0 ? iters_override : g->p.iterations;
        J.start = start_override >= 0 ? start_override : g->p.start_iter;
        J.literal = g->p.repulse_adjacent ? 0 : 1;
        J.step0 = g->p.step0;
        J.decay = g->p.step_decay;
        J.invK = 1.0 / g->p.K;
        J.negRK2 = -g->p.R * g->p.K * g->p.K;
        J.rowptr = g->rowptr;
        J.colidx = g->colidx;
        J.segs = g->ex.segs;
        J.segoff = g->ex.segoff;
        J.cursor = g->ex.cursor;
        J.x = g->x;
        J.y = g->y;
        J.accS[0] = g->ex.accS[0];
        J.accS[1] = g->ex.accS[1];
        J.accC[0] = g->ex.accC[0];
        J.accC[1] = g->ex.accC[1];
        J.energy = g->energy;
        J.nonfinite = &g->counters->nonfinite;
        J.conv_tol = g->p.conv_tol;
        J.halted = &g->counters->halted;
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
    const int BS = g->p.batch_size;
    for (int q = 0; q < 2; ++q) {
        BL_TRY(graph_alloc(g, &g->ex.accS[q], t2 * n));
        BL_TRY(graph_alloc(g, (void **)&g->ex.accC[q], sizeof(float2) * n));
    }
    BL_TRY(graph_alloc(g, (void **)&g->ex.epart, sizeof(double) * (size_t)(BS / kRows + 2)));
    BL_TRY(graph_alloc(g, (void **)&g->ex.ticket, 256));
    BL_TRY(graph_alloc(g, (void **)&g->ex.echunk, sizeof(double) * 2 * (size_t)g->nb * (size_t)(BS / kRows + 2)));
    BL_TRY(graph_alloc(g, (void **)&g->ex.ebatch, sizeof(double) * 2 * (size_t)g->nb));
    BL_TRY(graph_alloc(g, (void **)&g->ex.eticket, sizeof(unsigned) * 2 * ((size_t)g->nb + 1)));
    BL_TRY(graph_alloc(g, &g->ex.d_job, sizeof(ExactJob)));
    BL_TRY(graph_alloc(g, (void **)&g->ex.moved, sizeof(unsigned) * (size_t)g->nb));
    BL_HIP(hipMemsetAsync(g->ex.ticket, 0, 256, g->stream));
    BL_TRY(graph_alloc(g, (void **)&g->ex.segoff, sizeof(int) * (n + 1)));
    BL_TRY(graph_alloc(g, (void **)&g->ex.cursor, sizeof(int) * n));
    return BL_OK;
}

// CSR segments by column batch; needs the uploaded CSR.
int exact_prepare(bl_graph *g) {
    const size_t n = (size_t)g->n;
    const int BS = g->p.batch_size;
    const int blocks = (g->n + kSegRowsPerBlock - 1) / kSegRowsPerBlock;
    hipLaunchKernelGGL(seg_count_kernel, dim3(blocks), dim3(256), 0, g->stream, g->n, BS, g->rowptr, g->colidx,
                       g->ex.cursor);
    hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(1024), 0, g->stream, g->n, g->ex.cursor, g->ex.segoff);
    BL_HIP(hipGetLastError());
    int nseg = 0;
    BL_HIP(hipMemcpyAsync(&nseg, g->ex.segoff + n, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    BL_HIP(hipStreamSynchronize(g->stream));
    if (!g->ex.segs || g->ex.segs_cap < (size_t)std::max(nseg, 1)) {   // (a reloaded CSR reuses the room)
        BL_TRY(graph_alloc(g, (void **)&g->ex.segs, sizeof(int2) * (size_t)std::max<int64_t>(std::max(nseg, 1), g->nnz)));
        g->ex.segs_cap = (size_t)std::max<int64_t>(std::max(nseg, 1), g->nnz);
    }
    hipLaunchKernelGGL(seg_fill_kernel, dim3(blocks), dim3(256), 0, g->stream, g->n, BS, g->rowptr, g->colidx,
                       g->ex.segoff, g->ex.segs);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

// Segment bytes of a graph (at most one per CSR entry).
size_t exact_footprint(int n, int64_t nnz, int BS, bool fp64) {
    const size_t N = (size_t)n, T2 = fp64 ? 16 : 8;
    const size_t nb = (N + BS - 1) / BS;
    return 2 * (T2 * N + 8 * N) + 8 * (size_t)(BS / kRows + 2) + 256 + sizeof(ExactJob) + 4 * nb + 4 * (N + 1) + 4 * N +
           8 * (size_t)std::max<int64_t>(nnz, 1) + 4 * 256 + 16 * nb * (size_t)(BS / kRows + 2) + 16 * nb +
           8 * (nb + 1);
}

// Small graphs run in the one-workgroup kernel (one workgroup per graph); it
// computes the same bits as the multi-workgroup kernels.  One compute unit
// forms a step's n * BS pairs, so from about 24576 pairs on the persistent
// multi-workgroup run is faster (16384 pairs: 0.022 against 0.025 ms per
// iteration in one workgroup; 32768: 0.013 against 0.016; grid32, 131072:
// 0.042 against 0.082); BL_EXACT_ONE_WG=1 forces it up to
// kOneWGMaxPairs (tests of the kernel, measurements).
// It runs the (2, -1) model only; other (a, r) models take the multi-workgroup path.
static bool use_one_wg(const bl_graph *g, int stop_batch) {
    if (stop_batch >= 0 || (g->p.flags & BL_EXACT_MULTI_WG) || model_general(g->p)) return false;
    const long long pairs = (long long)g->n * g->p.batch_size;
    const char *force = getenv("BL_EXACT_ONE_WG");
    if (force && force[0] == '1') return pairs <= kOneWGMaxPairs;
    return pairs <= kOneWGPairs;
}

int exact_run(bl_graph *g, int iters, int start_iter, int stop_batch) {
    if (iters > 0 && use_one_wg(g, stop_batch)) {
        g->cont_iter = -1;
        const int nt = g->n >= 1024 ? 1024 : (g->n >= 512 ? 512 : 256);
        int slot;
        BL_TRY(prof_begin(g, PK_GRAPH, &slot));
        BL_TRY(exact_graph_launch(&g, 1, nt, g->stream, g->ex.d_job, iters, start_iter));
        return prof_end(g, slot);
    }
    if (model_general(g->p)) return exact_run_model(g, iters, start_iter, stop_batch);
    if (g->fp64) return ExactOps<double, false, 0>::run(g, iters, start_iter, stop_batch);
    if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false, 0>::run(g, iters, start_iter, stop_batch);
    return ExactOps<float, true, 0>::run(g, iters, start_iter, stop_batch);
}

int exact_forces(bl_graph *g, int batch) {
    g->cont_iter = -1;
    if (model_general(g->p)) return exact_forces_model(g, batch);
    if (g->fp64) return ExactOps<double, false, 0>::forces(g, batch);
    if (g->p.precision == BL_FP32_PLAIN) return ExactOps<float, false, 0>::forces(g, batch);
    return ExactOps<float, true, 0>::forces(g, batch);
}

#endif  // BL_EXACT_MODELS_TU

}  // namespace bl
