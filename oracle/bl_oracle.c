/*
 * BatchLayout oracle: a plain, slow, FP64 CPU implementation of the
 * minibatch force-directed layout step (Rahman, Sujon & Azad, "BatchLayout:
 * A Batch-Parallel Force-Directed Graph Layout Algorithm in Shared Memory").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library.  It is written for a reader to check against the paper by eye:
 * one vertex at a time, j ascending, no blocking, no reordering.
 *
 * Conventions (each is a reading of the paper, listed in the design notes):
 *  - Force model, Sec. 2.2 (the (a,r)-energy model) with the (2,-1) instance
 *    of Sec. 4.1: attraction magnitude d^2/K, repulsion magnitude R*K^2/d,
 *    both applied along the unit vector (c_j - c_i)/d; repulsion with a
 *    negative sign, so it pushes i away from j.
 *  - A pair with d == 0 (i itself, or a coincident vertex) contributes 0.
 *  - Repulsion runs over every j != i by default; with repulse_adjacent = 0
 *    adjacent pairs are skipped as in Algorithms 1 and 2.
 *  - Minibatch step, Sec. 3.3 and Algorithm 2: forces of all vertices of a
 *    batch are computed from one set of positions, then the batch is moved;
 *    batches are consecutive vertex ids and later batches see earlier moves.
 *  - Update: c_i += Step * f_i / |f_i| (no move when |f_i| == 0);
 *    Energy += |f_i|^2; Step is multiplied by the decay after each iteration.
 *  - Barnes-Hut, Sec. 3.5 and Algorithms S1-S3: per iteration the snapshot is
 *    quantised on a 2^16 x 2^16 Morton grid over the square bounding box
 *    (quantisation done in float32 arithmetic), the sorted list is split
 *    recursively into quadrants, a centroid is the FP64 mean of the members,
 *    a cell is accepted when side < theta * distance, a cell holding i is
 *    always opened, leaves (single vertices, or depth-16 buckets) interact
 *    exactly using the live coordinates of their members.
 *  - Greedy initialisation, Sec. 3.6 and Algorithm 3: a stack-driven
 *    traversal from a start vertex at (0, 0); each popped vertex places its
 *    unvisited neighbours on the unit circle around itself, at angles that
 *    advance by 360 / degree degrees, with the paper's constant 3.1416 for pi.
 *
 * Threads: the per-vertex force loops of a batch and the per-pivot BFS of the
 * stress run on OpenMP threads (orc_set_threads).  Every vertex's sum, and
 * every pivot's partial sums, keep their one sequential order, and pivot
 * partials are added in pivot order, so the results are the same bits at any
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LEVELS 16

/* Threads for the parallel loops (<= 0: the OpenMP default). */
void orc_set_threads(int t)
{
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : omp_get_num_procs());
#else
    (void)t;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- pair terms
 * The (a,r)-energy model of Sec. 2.2: attraction magnitude d^a / K and
 * repulsion magnitude R K^2 d^r (the exponent r read as the power of d in the
 * force, so that (2,-1) is Fruchterman-Reingold), each along the unit vector
 * (c_j - c_i)/d, the repulsion with a negative sign.  A pair with d == 0
 * contributes 0.  (2,-1) is written out on its own. */

/* Attraction term on i from neighbour j:
 *   a = 2:   (d^2/K) * delta/d = d * delta / K;
 *   general: (d^a/K) * delta/d. */
static void pair_attraction_ar(double dx, double dy, double K, int a, double *tx, double *ty)
{
    double d = sqrt(dx * dx + dy * dy);
    if (a == 2) {
        *tx = d * dx / K;
        *ty = d * dy / K;
        return;
    }
    if (d == 0.0) { *tx = 0.0; *ty = 0.0; return; }
    double f = pow(d, (double)a) / K;
    *tx = f * dx / d;
    *ty = f * dy / d;
}

/* Repulsion term on i from j:
 *   r = -1:  (-R K^2 / d) * delta/d = -R K^2 delta / d^2;
 *   general: (-R K^2 d^r) * delta/d. */
static void pair_repulsion_ar(double dx, double dy, double K, double R, int r, double *tx, double *ty)
{
    double d2 = dx * dx + dy * dy;
    if (d2 == 0.0) { *tx = 0.0; *ty = 0.0; return; }
    if (r == -1) {
        double c = -R * K * K / d2;
        *tx = c * dx;
        *ty = c * dy;
        return;
    }
    double d = sqrt(d2);
    double f = -R * K * K * pow(d, (double)r);
    *tx = f * dx / d;
    *ty = f * dy / d;
}

/* ------------------------------------------------------------- exact forces
 * Net force on vertex i from the current coordinates (Sec. 2.2, the combined
 * force f(i,c); Algorithm 2 walks j = 0..n-1 and the sorted CSR row in step).
 * Outputs attraction and repulsion separately, plus the condition scale
 * S_i = sum of |term| over all terms. */
static void force_exact_one(int n, const int *rowptr, const int *colidx,
                            const double *x, const double *y, int i,
                            double K, double R, int repulse_adjacent, int a, int r,
                            double *ax, double *ay, double *rx, double *ry, double *scale)
{
    double sax = 0, say = 0, srx = 0, sry = 0, s = 0;
    int k = rowptr[i], kend = rowptr[i + 1];
    for (int j = 0; j < n; ++j) {
        double dx = x[j] - x[i], dy = y[j] - y[i];
        int adjacent = 0;
        while (k < kend && colidx[k] < j) ++k;
        if (k < kend && colidx[k] == j) adjacent = 1;
        if (adjacent) {
            double tx, ty;
            pair_attraction_ar(dx, dy, K, a, &tx, &ty);
            sax += tx; say += ty;
            s += sqrt(tx * tx + ty * ty);
        }
        if (j == i) continue;
        if (adjacent && !repulse_adjacent) continue;
        double tx, ty;
        pair_repulsion_ar(dx, dy, K, R, r, &tx, &ty);
        srx += tx; sry += ty;
        s += sqrt(tx * tx + ty * ty);
    }
    *ax = sax; *ay = say; *rx = srx; *ry = sry;
    if (scale) *scale = s;
}

int orc_forces_exact_ar(int n, const int *rowptr, const int *colidx,
                        const double *x, const double *y, int i0, int i1,
                        double K, double R, int repulse_adjacent, int a, int r,
                        double *ax, double *ay, double *rx, double *ry, double *scale)
{
    if (n < 1 || i0 < 0 || i1 > n || i0 > i1) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = i0; i < i1; ++i)
        force_exact_one(n, rowptr, colidx, x, y, i, K, R, repulse_adjacent, a, r,
                        &ax[i - i0], &ay[i - i0], &rx[i - i0], &ry[i - i0],
                        scale ? &scale[i - i0] : NULL);
    return 0;
}

int orc_forces_exact(int n, const int *rowptr, const int *colidx,
                     const double *x, const double *y, int i0, int i1,
                     double K, double R, int repulse_adjacent,
                     double *ax, double *ay, double *rx, double *ry, double *scale)
{
    return orc_forces_exact_ar(n, rowptr, colidx, x, y, i0, i1, K, R, repulse_adjacent, 2, -1,
                               ax, ay, rx, ry, scale);
}

/* Move the vertices of one batch along their normalised net forces
 * (Algorithm 2, the update loop after the parallel force loop).  The batch
 * is members[0..m) (consecutive ids, or a run of a permutation). */
static double move_batch(const int *members, int m, double *x, double *y,
                         const double *fx, const double *fy, double step)
{
    double energy = 0.0;
    for (int q = 0; q < m; ++q) {
        int i = members[q];
        double f2 = fx[q] * fx[q] + fy[q] * fy[q];
        double norm = sqrt(f2);
        if (norm > 0.0) {
            x[i] += step * fx[q] / norm;
            y[i] += step * fy[q] / norm;
        }
        energy += f2;
    }
    return energy;
}

/* The members of batch b: order[b*bs ...] when an order is given (batch
 * randomisation, Sec. 4.3.3), else the id range [b*bs, min((b+1)*bs, n)). */
static int batch_members(int n, int bs, int b, const int *order, int *members)
{
    int i0 = b * bs, i1 = i0 + bs < n ? i0 + bs : n;
    for (int q = i0; q < i1; ++q) members[q - i0] = order ? order[q] : q;
    return i1 - i0;
}

/* Step length at iteration k: Step_0 multiplied by the decay once per
 * completed iteration (Algorithm 2, Step = Step * 0.999 after each loop). */
double orc_step_at(double step0, double decay, int k)
{
    double s = step0;
    for (int t = 0; t < k; ++t) s *= decay;
    return s;
}

/* Exact BatchLayout (Algorithm 2 without the cache blocking).
 * Runs iterations [start_iter, start_iter + iters).  When stop_batch >= 0 the
 * last iteration stops after that many batches (used to dump a mid-iteration
 * state).  energy[t] receives the energy of iteration start_iter + t.
 * order (may be NULL): a permutation of the ids whose consecutive runs of bs
 * entries are the batches of every iteration run by this call. */
int orc_layout_exact_ord(int n, const int *rowptr, const int *colidx,
                         double *x, double *y, int bs, int iters, int start_iter,
                         double step0, double decay, double K, double R,
                         int repulse_adjacent, int a, int r, int stop_batch,
                         const int *order, double *energy)
{
    if (n < 1 || bs < 1 || iters < 0) return -1;
    int nb = (n + bs - 1) / bs;
    double *fx = malloc(sizeof(double) * bs), *fy = malloc(sizeof(double) * bs);
    int *mem = malloc(sizeof(int) * bs);
    if (!fx || !fy || !mem) { free(fx); free(fy); free(mem); return -2; }
    for (int t = 0; t < iters; ++t) {
        double step = orc_step_at(step0, decay, start_iter + t);
        double e = 0.0;
        int last = (t == iters - 1 && stop_batch >= 0) ? stop_batch : nb;
        for (int b = 0; b < last; ++b) {
            int m = batch_members(n, bs, b, order, mem);
#pragma omp parallel for schedule(dynamic, 4)
            for (int q = 0; q < m; ++q) {
                double ax, ay, rx, ry;
                force_exact_one(n, rowptr, colidx, x, y, mem[q], K, R, repulse_adjacent, a, r,
                                &ax, &ay, &rx, &ry, NULL);
                fx[q] = ax + rx;
                fy[q] = ay + ry;
            }
            e += move_batch(mem, m, x, y, fx, fy, step);
        }
        if (energy) energy[t] = e;
    }
    free(fx); free(fy); free(mem);
    return 0;
}

int orc_layout_exact_ar(int n, const int *rowptr, const int *colidx,
                        double *x, double *y, int bs, int iters, int start_iter,
                        double step0, double decay, double K, double R,
                        int repulse_adjacent, int a, int r, int stop_batch, double *energy)
{
    return orc_layout_exact_ord(n, rowptr, colidx, x, y, bs, iters, start_iter, step0, decay, K, R,
                                repulse_adjacent, a, r, stop_batch, NULL, energy);
}

int orc_layout_exact(int n, const int *rowptr, const int *colidx,
                     double *x, double *y, int bs, int iters, int start_iter,
                     double step0, double decay, double K, double R,
                     int repulse_adjacent, int stop_batch, double *energy)
{
    return orc_layout_exact_ar(n, rowptr, colidx, x, y, bs, iters, start_iter, step0, decay, K, R,
                               repulse_adjacent, 2, -1, stop_batch, energy);
}

/* ------------------------------------------------------------- Barnes-Hut */

typedef struct {
    int level;        /* 0 = root square of side W */
    int lo, hi;       /* members: sorted positions [lo, hi) */
    int nchild;
    int child[4];     /* node indices, Morton order */
    int bucket;       /* 1: depth-16 cell holding >= 2 members */
    double cx, cy;    /* FP64 centroid of the members' snapshot coordinates */
} onode;

typedef struct {
    int n;
    int nnodes, cap;
    onode *nodes;
    uint32_t *key;    /* key of sorted position p */
    int *order;       /* vertex at sorted position p */
    int *pos;         /* sorted position of vertex i */
    double W;         /* side of the root square (float32 value) */
    float xmin, ymin;
    const double *sx, *sy;   /* snapshot (copied) */
    double *sxbuf, *sybuf;
} otree;

/* Morton key of a point, quantised in float32 arithmetic on a 2^16 grid over
 * the square [xmin, xmin+W] x [ymin, ymin+W]; bit 2b holds x bit b and bit
 * 2b+1 holds y bit b.  Cells of the quadtree are the key prefixes (Fig. 5). */
static uint32_t morton_key(float px, float py, float xmin, float ymin, float W)
{
    uint32_t qx = 0, qy = 0;
    if (W > 0.0f) {
        volatile float scale = 65536.0f / W;
        volatile float ux = px - xmin, uy = py - ymin;
        volatile float fx = ux * scale, fy = uy * scale;
        long lx = (long)fx, ly = (long)fy;
        if (lx < 0) lx = 0;
        if (ly < 0) ly = 0;
        if (lx > 65535) lx = 65535;
        if (ly > 65535) ly = 65535;
        qx = (uint32_t)lx; qy = (uint32_t)ly;
    }
    uint32_t k = 0;
    for (int b = 0; b < 16; ++b) {
        k |= ((qx >> b) & 1u) << (2 * b);
        k |= ((qy >> b) & 1u) << (2 * b + 1);
    }
    return k;
}

static otree *g_sort_tree;
static int cmp_sorted(const void *a, const void *b)
{
    int i = *(const int *)a, j = *(const int *)b;
    /* keys stored per vertex in tree->pos temporarily */
    uint32_t ki = (uint32_t)g_sort_tree->pos[i], kj = (uint32_t)g_sort_tree->pos[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j);
}

static int new_node(otree *t)
{
    if (t->nnodes == t->cap) {
        int nc = t->cap ? 2 * t->cap : 64;
        onode *nn = realloc(t->nodes, sizeof(onode) * nc);
        if (!nn) return -1;
        t->nodes = nn; t->cap = nc;
    }
    memset(&t->nodes[t->nnodes], 0, sizeof(onode));
    return t->nnodes++;
}

/* Algorithm S1 (constructBHT): split the Morton-sorted members of a cell into
 * its four quadrants, build each non-empty one, then form the centroid from
 * the children.  Recursion stops at a single member or at depth 16. */
static int build_cell(otree *t, int lo, int hi, int level)
{
    int id = new_node(t);
    if (id < 0) return -1;
    t->nodes[id].level = level;
    t->nodes[id].lo = lo;
    t->nodes[id].hi = hi;
    if (hi - lo == 1) {
        int v = t->order[lo];
        t->nodes[id].cx = t->sx[v];
        t->nodes[id].cy = t->sy[v];
        return id;
    }
    if (level == ORC_LEVELS) {
        double sx = 0, sy = 0;
        for (int p = lo; p < hi; ++p) { sx += t->sx[t->order[p]]; sy += t->sy[t->order[p]]; }
        t->nodes[id].bucket = 1;
        t->nodes[id].cx = sx / (hi - lo);
        t->nodes[id].cy = sy / (hi - lo);
        return id;
    }
    int shift = 2 * (ORC_LEVELS - 1 - level);
    int start = lo;
    int kids[4], nk = 0;
    for (uint32_t q = 0; q < 4; ++q) {
        int end = start;
        while (end < hi && ((t->key[end] >> shift) & 3u) == q) ++end;
        if (end > start) {
            int c = build_cell(t, start, end, level + 1);
            if (c < 0) return -1;
            kids[nk++] = c;
        }
        start = end;
    }
    /* centroid from the children: count-weighted mean of their centroids */
    double sx = 0, sy = 0;
    for (int c = 0; c < nk; ++c) {
        onode *ch = &t->nodes[kids[c]];
        int cnt = ch->hi - ch->lo;
        sx += cnt * ch->cx;
        sy += cnt * ch->cy;
    }
    onode *nd = &t->nodes[id];
    nd->nchild = nk;
    for (int c = 0; c < nk; ++c) nd->child[c] = kids[c];
    nd->cx = sx / (hi - lo);
    nd->cy = sy / (hi - lo);
    return id;
}

void orc_tree_free(void *tp)
{
    otree *t = (otree *)tp;
    if (!t) return;
    free(t->nodes); free(t->key); free(t->order); free(t->pos);
    free(t->sxbuf); free(t->sybuf);
    free(t);
}

/* Build the quadtree of a snapshot (Algorithm S3: bounding box, Morton sort,
 * D = max extent, constructBHT).  Returns an opaque handle. */
void *orc_tree_build(int n, const double *sx, const double *sy)
{
    if (n < 1) return NULL;
    otree *t = calloc(1, sizeof(otree));
    if (!t) return NULL;
    t->n = n;
    t->key = malloc(sizeof(uint32_t) * n);
    t->order = malloc(sizeof(int) * n);
    t->pos = malloc(sizeof(int) * n);
    t->sxbuf = malloc(sizeof(double) * n);
    t->sybuf = malloc(sizeof(double) * n);
    if (!t->key || !t->order || !t->pos || !t->sxbuf || !t->sybuf) { orc_tree_free(t); return NULL; }
    memcpy(t->sxbuf, sx, sizeof(double) * n);
    memcpy(t->sybuf, sy, sizeof(double) * n);
    t->sx = t->sxbuf; t->sy = t->sybuf;

    float xmin = (float)sx[0], xmax = xmin, ymin = (float)sy[0], ymax = ymin;
    for (int i = 1; i < n; ++i) {
        float fx = (float)sx[i], fy = (float)sy[i];
        if (fx < xmin) xmin = fx;
        if (fx > xmax) xmax = fx;
        if (fy < ymin) ymin = fy;
        if (fy > ymax) ymax = fy;
    }
    volatile float wx = xmax - xmin, wy = ymax - ymin;
    float W = wx > wy ? wx : wy;
    t->xmin = xmin; t->ymin = ymin; t->W = (double)W;

    for (int i = 0; i < n; ++i) {
        t->pos[i] = (int)morton_key((float)sx[i], (float)sy[i], xmin, ymin, W);
        t->order[i] = i;
    }
    g_sort_tree = t;
    qsort(t->order, n, sizeof(int), cmp_sorted);
    for (int p = 0; p < n; ++p) t->key[p] = (uint32_t)t->pos[t->order[p]];
    for (int p = 0; p < n; ++p) t->pos[t->order[p]] = p;

    if (build_cell(t, 0, n, 0) < 0) { orc_tree_free(t); return NULL; }
    return t;
}

/* Tree inspection for the tests. */
int orc_tree_nnodes(void *tp) { return ((otree *)tp)->nnodes; }
double orc_tree_width(void *tp) { return ((otree *)tp)->W; }
int orc_tree_node(void *tp, int id, int *level, int *lo, int *hi, int *nchild,
                  int *child4, int *bucket, double *cx, double *cy)
{
    otree *t = (otree *)tp;
    if (id < 0 || id >= t->nnodes) return -1;
    onode *nd = &t->nodes[id];
    *level = nd->level; *lo = nd->lo; *hi = nd->hi; *nchild = nd->nchild;
    for (int c = 0; c < 4; ++c) child4[c] = c < nd->nchild ? nd->child[c] : -1;
    *bucket = nd->bucket; *cx = nd->cx; *cy = nd->cy;
    return 0;
}
int orc_tree_order(void *tp, int *order, uint32_t *keys)
{
    otree *t = (otree *)tp;
    for (int p = 0; p < t->n; ++p) { order[p] = t->order[p]; keys[p] = t->key[p]; }
    return 0;
}

typedef struct {
    const otree *t;
    const double *x, *y;     /* live coordinates */
    int i, posi;
    double xi, yi;
    double K, R, theta;
    int r;            /* repulsion exponent of the (a, r) model */
    int leaf_live;
    double rx, ry, scale;
    long visits;
    int near_tie;
} walk_ctx;

static void add_rep(walk_ctx *w, double px, double py, double mult)
{
    double tx, ty;
    pair_repulsion_ar(px - w->xi, py - w->yi, w->K, w->R, w->r, &tx, &ty);
    w->rx += mult * tx;
    w->ry += mult * ty;
    w->scale += mult * sqrt(tx * tx + ty * ty);
}

static void add_member(walk_ctx *w, int v)
{
    if (v == w->i) return;
    const double *px = w->leaf_live ? w->x : w->t->sx;
    const double *py = w->leaf_live ? w->y : w->t->sy;
    add_rep(w, px[v], py[v], 1.0);
}

/* Algorithm S2 (calcRepulsiveForce): accept a cell when side < theta * d,
 * otherwise descend into its children in Morton order; leaves interact
 * exactly; a cell that holds i is always opened. */
static void walk(walk_ctx *w, int id)
{
    const otree *t = w->t;
    const onode *nd = &t->nodes[id];
    w->visits++;
    if (nd->hi - nd->lo == 1) { add_member(w, t->order[nd->lo]); return; }
    if (nd->bucket) {
        for (int p = nd->lo; p < nd->hi; ++p) add_member(w, t->order[p]);
        return;
    }
    int holds_i = (w->posi >= nd->lo && w->posi < nd->hi);
    if (!holds_i) {
        double side = ldexp(t->W, -nd->level);
        double dx = nd->cx - w->xi, dy = nd->cy - w->yi;
        double d = sqrt(dx * dx + dy * dy);
        if (fabs(side - w->theta * d) <= 1e-5 * w->theta * d) w->near_tie = 1;
        if (side < w->theta * d) {
            add_rep(w, nd->cx, nd->cy, (double)(nd->hi - nd->lo));
            return;
        }
    }
    for (int c = 0; c < nd->nchild; ++c) walk(w, nd->child[c]);
}

/* Barnes-Hut force on vertex i (Algorithm S3, force loop): attraction over
 * its CSR neighbours with live coordinates, repulsion through the tree of
 * the snapshot, under the (a, r) model (an accepted cell adds count times the
 * repulsion from its centroid).  leaf_live = 1 makes leaves use live
 * coordinates. */
static void force_bh_one(const int *rowptr, const int *colidx, const double *x, const double *y,
                         const otree *t, int i, double K, double R, double theta, int leaf_live,
                         int a, int r, double *ax, double *ay, double *rx, double *ry,
                         double *scale, long *visits, int *near_tie)
{
    double sax = 0, say = 0, s = 0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        int j = colidx[k];
        double tx, ty;
        pair_attraction_ar(x[j] - x[i], y[j] - y[i], K, a, &tx, &ty);
        sax += tx; say += ty;
        s += sqrt(tx * tx + ty * ty);
    }
    walk_ctx w;
    memset(&w, 0, sizeof w);
    w.t = t; w.x = x; w.y = y; w.i = i; w.posi = t->pos[i];
    w.xi = x[i]; w.yi = y[i];
    w.K = K; w.R = R; w.theta = theta; w.r = r; w.leaf_live = leaf_live;
    walk(&w, 0);
    *ax = sax; *ay = say;
    *rx = w.rx; *ry = w.ry;
    if (scale) *scale = s + w.scale;
    if (visits) *visits = w.visits;
    if (near_tie) *near_tie = w.near_tie;
}

/* Barnes-Hut forces for vertices [i0, i1) under the (a, r) model. */
int orc_forces_bh_ar(int n, const int *rowptr, const int *colidx,
                     const double *x, const double *y, void *tp, int i0, int i1,
                     double K, double R, double theta, int leaf_live, int a, int r,
                     double *ax, double *ay, double *rx, double *ry, double *scale,
                     long *visits, int *near_tie)
{
    otree *t = (otree *)tp;
    if (!t || t->n != n || i0 < 0 || i1 > n || i0 > i1) return -1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = i0; i < i1; ++i)
        force_bh_one(rowptr, colidx, x, y, t, i, K, R, theta, leaf_live, a, r,
                     &ax[i - i0], &ay[i - i0], &rx[i - i0], &ry[i - i0],
                     scale ? &scale[i - i0] : NULL, visits ? &visits[i - i0] : NULL,
                     near_tie ? &near_tie[i - i0] : NULL);
    return 0;
}

int orc_forces_bh(int n, const int *rowptr, const int *colidx,
                  const double *x, const double *y, void *tp, int i0, int i1,
                  double K, double R, double theta, int leaf_live,
                  double *ax, double *ay, double *rx, double *ry, double *scale,
                  long *visits, int *near_tie)
{
    return orc_forces_bh_ar(n, rowptr, colidx, x, y, tp, i0, i1, K, R, theta, leaf_live, 2, -1,
                            ax, ay, rx, ry, scale, visits, near_tie);
}

/* BatchLayoutBH (Algorithm S3) with the step decay of Algorithm 2, under the
 * (a, r) model.  When snap_x/snap_y are given they receive the snapshot of
 * the last (possibly partial, see stop_batch) iteration.  visits_total
 * accumulates the node visits of all force evaluations.  order (may be
 * NULL): a permutation whose runs of bs entries are the batches. */
int orc_layout_bh_ord(int n, const int *rowptr, const int *colidx,
                      double *x, double *y, int bs, int iters, int start_iter,
                      double step0, double decay, double K, double R, double theta,
                      int leaf_live, int a, int r, int stop_batch, const int *order, double *energy,
                      double *snap_x, double *snap_y, long *visits_total)
{
    if (n < 1 || bs < 1 || iters < 0 || theta < 0) return -1;
    int nb = (n + bs - 1) / bs;
    double *fx = malloc(sizeof(double) * bs), *fy = malloc(sizeof(double) * bs);
    long *vis = malloc(sizeof(long) * bs);
    int *mem = malloc(sizeof(int) * bs);
    if (!fx || !fy || !vis || !mem) {
        free(fx); free(fy); free(vis); free(mem);
        return -2;
    }
    long vt = 0;
    int rc = 0;
    for (int t = 0; t < iters && rc == 0; ++t) {
        double step = orc_step_at(step0, decay, start_iter + t);
        otree *tree = orc_tree_build(n, x, y);
        if (!tree) { rc = -2; break; }
        if (t == iters - 1 && snap_x && snap_y) {
            memcpy(snap_x, x, sizeof(double) * n);
            memcpy(snap_y, y, sizeof(double) * n);
        }
        double e = 0.0;
        int last = (t == iters - 1 && stop_batch >= 0) ? stop_batch : nb;
        for (int b = 0; b < last; ++b) {
            int m = batch_members(n, bs, b, order, mem);
#pragma omp parallel for schedule(dynamic, 8)
            for (int q = 0; q < m; ++q) {
                double ax, ay, rx, ry;
                force_bh_one(rowptr, colidx, x, y, tree, mem[q], K, R, theta, leaf_live, a, r,
                             &ax, &ay, &rx, &ry, NULL, &vis[q], NULL);
                fx[q] = ax + rx;
                fy[q] = ay + ry;
            }
            for (int q = 0; q < m; ++q) vt += vis[q];
            e += move_batch(mem, m, x, y, fx, fy, step);
        }
        if (energy) energy[t] = e;
        orc_tree_free(tree);
    }
    if (visits_total) *visits_total = vt;
    free(fx); free(fy); free(vis); free(mem);
    return rc;
}

int orc_layout_bh(int n, const int *rowptr, const int *colidx,
                  double *x, double *y, int bs, int iters, int start_iter,
                  double step0, double decay, double K, double R, double theta,
                  int leaf_live, int stop_batch, double *energy,
                  double *snap_x, double *snap_y, long *visits_total)
{
    return orc_layout_bh_ord(n, rowptr, colidx, x, y, bs, iters, start_iter, step0, decay, K, R, theta,
                             leaf_live, 2, -1, stop_batch, NULL, energy, snap_x, snap_y, visits_total);
}

/* ------------------------------------------------------- quality measures */

/* Edge energy: the attractive potential whose gradient is the attraction
 * term, summed once per undirected edge: sum d^3 / (3K). */
double orc_edge_energy(int n, const int *rowptr, const int *colidx,
                       const double *x, const double *y, double K)
{
    double e = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = colidx[k];
            if (j <= i) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i];
            double d = sqrt(dx * dx + dy * dy);
            e += d * d * d / (3.0 * K);
        }
    return e;
}

/* Edge uniformity (Sec. 3.7): normalised standard deviation of edge lengths. */
double orc_edge_uniformity(int n, const int *rowptr, const int *colidx,
                           const double *x, const double *y)
{
    double s = 0.0;
    long m = 0;
    for (int i = 0; i < n; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = colidx[k];
            if (j <= i) continue;
            s += hypot(x[j] - x[i], y[j] - y[i]);
            m++;
        }
    if (m == 0) return 0.0;
    double mean = s / m, v = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = colidx[k];
            if (j <= i) continue;
            double l = hypot(x[j] - x[i], y[j] - y[i]);
            v += (l - mean) * (l - mean);
        }
    return sqrt(v / ((double)m * mean * mean));
}

/* Stress (Sec. 3.7) after the best uniform scaling of the layout:
 *   sum w_ij (s |c_i - c_j| - d_ij)^2 with w_ij = d_ij^-2, minimised over s,
 * d_ij = BFS hop distance, unreachable pairs skipped.  With pivots == NULL the
 * sum runs over unordered pairs i < j; otherwise over pivot p and all j != p.
 * The minimum over s is N - A^2/B with A = sum |.|/d, B = sum |.|^2/d^2. */
double orc_stress(int n, const int *rowptr, const int *colidx,
                  const double *x, const double *y, int npivots, const int *pivots,
                  double *scale_out)
{
    int np = pivots ? npivots : n;
    /* per-pivot partial sums, added in pivot order below */
    double *pA = calloc(np > 0 ? np : 1, sizeof(double));
    double *pB = calloc(np > 0 ? np : 1, sizeof(double));
    double *pN = calloc(np > 0 ? np : 1, sizeof(double));
    int failed = 0;
    if (!pA || !pB || !pN) { free(pA); free(pB); free(pN); return -1.0; }
#pragma omp parallel
    {
        int *dist = malloc(sizeof(int) * n), *queue = malloc(sizeof(int) * n);
        if (!dist || !queue) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < np; ++q) {
            if (!dist || !queue) continue;
            int p = pivots ? pivots[q] : q;
            for (int i = 0; i < n; ++i) dist[i] = -1;
            int head = 0, tail = 0;
            dist[p] = 0; queue[tail++] = p;
            while (head < tail) {
                int u = queue[head++];
                for (int k = rowptr[u]; k < rowptr[u + 1]; ++k) {
                    int v = colidx[k];
                    if (dist[v] < 0) { dist[v] = dist[u] + 1; queue[tail++] = v; }
                }
            }
            double A = 0.0, B = 0.0, N = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == p || dist[j] <= 0) continue;
                if (!pivots && j < p) continue;
                double dij = dist[j];
                double g = hypot(x[j] - x[p], y[j] - y[p]);
                A += g / dij;
                B += g * g / (dij * dij);
                N += 1.0;
            }
            pA[q] = A; pB[q] = B; pN[q] = N;
        }
        free(dist); free(queue);
    }
    double A = 0.0, B = 0.0, N = 0.0;
    for (int q = 0; q < np; ++q) { A += pA[q]; B += pB[q]; N += pN[q]; }
    free(pA); free(pB); free(pN);
    if (failed) return -1.0;
    if (B == 0.0) { if (scale_out) *scale_out = 0.0; return N; }
    if (scale_out) *scale_out = A / B;
    return N - A * A / B;
}

/* Neighbourhood preservation (Sec. 3.7, the measure tsNET and Maxent use),
 * read as the mean over vertices i with deg(i) = k > 0 of the Jaccard index
 * |N(i) & L(i)| / |N(i) | L(i)|, N(i) the graph neighbours of i and L(i) the k
 * vertices nearest to i in the layout (squared Euclidean distance in FP64,
 * computed without fused operations; equal distances ordered by vertex id).
 * With sample != NULL only the listed vertices are averaged (repeats count
 * again); isolated vertices are skipped.  *counted receives the number of
 * vertices averaged.  Returns 0 when none is counted. */
typedef struct { double d2; int v; } ord_dv;

static int cmp_dv(const void *a, const void *b)
{
    const ord_dv *p = (const ord_dv *)a, *q = (const ord_dv *)b;
    if (p->d2 != q->d2) return p->d2 < q->d2 ? -1 : 1;
    return p->v < q->v ? -1 : (p->v > q->v);
}

double orc_neighborhood_preservation(int n, const int *rowptr, const int *colidx,
                                     const double *x, const double *y,
                                     int nsample, const int *sample, long *counted)
{
    int ns = sample ? nsample : n;
    double *jac = calloc(ns > 0 ? ns : 1, sizeof(double));
    char *use = calloc(ns > 0 ? ns : 1, 1);
    int failed = 0;
    if (!jac || !use) { free(jac); free(use); return -1.0; }
#pragma omp parallel
    {
        ord_dv *buf = malloc(sizeof(ord_dv) * (n > 1 ? n - 1 : 1));
        char *near = calloc(n, 1);
        if (!buf || !near) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < ns; ++q) {
            if (!buf || !near) continue;
            int i = sample ? sample[q] : q;
            int k = rowptr[i + 1] - rowptr[i];
            if (k == 0) continue;
            int m = 0;
            for (int v = 0; v < n; ++v) {
                if (v == i) continue;
                double dx = x[v] - x[i], dy = y[v] - y[i];
                buf[m].d2 = dx * dx + dy * dy;
                buf[m].v = v;
                ++m;
            }
            qsort(buf, m, sizeof(ord_dv), cmp_dv);
            for (int t = 0; t < k; ++t) near[buf[t].v] = 1;
            int both = 0;
            for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) both += near[colidx[e]];
            for (int t = 0; t < k; ++t) near[buf[t].v] = 0;
            jac[q] = (double)both / (double)(2 * k - both);
            use[q] = 1;
        }
        free(buf); free(near);
    }
    double sum = 0.0;
    long cnt = 0;
    for (int q = 0; q < ns; ++q)
        if (use[q]) { sum += jac[q]; ++cnt; }
    free(jac); free(use);
    if (counted) *counted = cnt;
    if (failed) return -1.0;
    return cnt ? sum / (double)cnt : 0.0;
}

/* ------------------------------------------------- greedy initialisation */

/* Greedy initialisation, Sec. 3.6 and Algorithm 3.  The start vertex sits at
 * (0, 0) and is pushed on an empty stack.  While the stack is not empty, pop
 * U; with d = 360 / deg(U) (all neighbours counted) and D = 0, every
 * neighbour u of U, in row order, that is not yet visited is placed at
 * U + (cos(PI*D/180), sin(PI*D/180)) with PI = 3.1416, marked visited and
 * pushed, and D grows by d.  Vertices the start cannot reach (the paper is
 * silent): the lowest-id unvisited vertex starts a new traversal from its
 * given position (xr, yr), repeated until every vertex is placed.
 * parent[v] is the vertex that placed v (-1 for the start and the roots). */
int orc_greedy_init(int n, const int *rowptr, const int *colidx, int start,
                    const double *xr, const double *yr, double *x, double *y, int *parent)
{
    const double PI = 3.1416;
    if (n < 1 || start < 0 || start >= n) return -1;
    int *stack = malloc(sizeof(int) * n);
    char *visited = calloc(n, 1);
    if (!stack || !visited) { free(stack); free(visited); return -2; }
    int root = start, next = 0;
    for (;;) {
        if (root == start) { x[root] = 0.0; y[root] = 0.0; }
        else { x[root] = xr[root]; y[root] = yr[root]; }
        visited[root] = 1;
        parent[root] = -1;
        int sp = 0;
        stack[sp++] = root;
        while (sp > 0) {
            int U = stack[--sp];
            int deg = rowptr[U + 1] - rowptr[U];
            if (deg == 0) continue;
            double d = 360.0 / deg;
            double D = 0.0;
            for (int k = rowptr[U]; k < rowptr[U + 1]; ++k) {
                int u = colidx[k];
                if (visited[u]) continue;
                x[u] = x[U] + cos(PI * D / 180.0);
                y[u] = y[U] + sin(PI * D / 180.0);
                visited[u] = 1;
                parent[u] = U;
                stack[sp++] = u;
                D = D + d;
            }
        }
        while (next < n && visited[next]) ++next;
        if (next == n) break;
        root = next;
    }
    free(stack); free(visited);
    return 0;
}
