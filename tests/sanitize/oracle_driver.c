/* Drives every entry point of the FP64 oracle on small inputs, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Inputs cover ragged batches, isolated and coincident vertices, buckets of
 * equal Morton keys, pivots with repeats and a sample for neighbourhood
 * preservation.  Exits 1 if a result is not finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_forces_exact_ar(int, const int *, const int *, const double *, const double *, int, int, double, double,
                        int, int, int, double *, double *, double *, double *, double *);
int orc_layout_exact_ord(int, const int *, const int *, double *, double *, int, int, int, double, double, double,
                         double, int, int, int, int, const int *, double *);
void *orc_tree_build(int, const double *, const double *);
void orc_tree_free(void *);
int orc_tree_nnodes(void *);
int orc_tree_order(void *, int *, unsigned *);
int orc_forces_bh_ar(int, const int *, const int *, const double *, const double *, void *, int, int, double,
                     double, double, int, int, int, double *, double *, double *, double *, double *, long *, int *);
int orc_layout_bh_ord(int, const int *, const int *, double *, double *, int, int, int, double, double, double,
                      double, double, int, int, int, int, const int *, double *, double *, double *, long *);
double orc_edge_energy(int, const int *, const int *, const double *, const double *, double);
double orc_edge_uniformity(int, const int *, const int *, const double *, const double *);
double orc_stress(int, const int *, const int *, const double *, const double *, int, const int *, double *);
double orc_neighborhood_preservation(int, const int *, const int *, const double *, const double *, int,
                                     const int *, long *);
int orc_greedy_init(int, const int *, const int *, int, const double *, const double *, double *, double *, int *);
void orc_set_threads(int);

static int bad = 0;
static void chk(const char *what, double v)
{
    if (!isfinite(v)) {
        printf("non-finite %s\n", what);
        bad = 1;
    }
}

/* a ring of n vertices plus chords i -- i + 7, vertex n - 1 isolated */
static void graph(int n, int *rp, int *ci)
{
    int e = 0;
    for (int i = 0; i < n; ++i) {
        rp[i] = e;
        if (i == n - 1) continue;
        int nb[4], k = 0;
        int cand[4] = {i - 7, i - 1, i + 1, i + 7};
        for (int q = 0; q < 4; ++q)
            if (cand[q] >= 0 && cand[q] < n - 1) nb[k++] = cand[q];
        for (int q = 0; q < k; ++q) ci[e++] = nb[q];
    }
    rp[n] = e;
}

int main(void)
{
    enum { N = 45 };
    int rp[N + 1], ci[4 * N];
    double x[N], y[N], x2[N], y2[N], ax[N], ay[N], rx[N], ry[N], sc[N], e[8], sx[N], sy[N];
    int order[N], tie[N], parent[N];
    unsigned keys[N];
    long vis[N], vt = 0, cnt = 0;
    graph(N, rp, ci);
    srand(7);
    for (int i = 0; i < N; ++i) {
        x[i] = (rand() % 1000) / 500.0 - 1.0;
        y[i] = (rand() % 1000) / 500.0 - 1.0;
        order[i] = (i * 17) % N;
    }
    x[5] = x[6];   /* coincident pair: a bucket */
    y[5] = y[6];
    for (int t = 1; t <= 3; t += 2) {
        orc_set_threads(t);
        const int models[3][2] = {{2, -1}, {1, -1}, {3, 0}};
        for (int m = 0; m < 3; ++m) {
            int a = models[m][0], r = models[m][1];
            if (orc_forces_exact_ar(N, rp, ci, x, y, 0, N, 1.0, 1.0, m & 1, a, r, ax, ay, rx, ry, sc)) return 2;
            for (int i = 0; i < N; ++i) chk("exact force", ax[i] + ay[i] + rx[i] + ry[i] + sc[i]);
            for (int i = 0; i < N; ++i) x2[i] = x[i], y2[i] = y[i];
            if (orc_layout_exact_ord(N, rp, ci, x2, y2, 8, 3, 1, 1.0, 0.999, 1.0, 1.0, 1, a, r, -1,
                                     m == 1 ? order : NULL, e)) return 3;
            for (int q = 0; q < 3; ++q) chk("exact energy", e[q]);
            void *tr = orc_tree_build(N, x, y);
            if (!tr || orc_tree_nnodes(tr) < 1 || orc_tree_order(tr, order, keys)) return 4;
            if (orc_forces_bh_ar(N, rp, ci, x, y, tr, 3, 40, 1.0, 1.0, 0.8, 1, a, r, ax, ay, rx, ry, sc, vis, tie))
                return 5;
            for (int i = 0; i < 37; ++i) chk("bh force", ax[i] + ay[i] + rx[i] + ry[i]);
            orc_tree_free(tr);
            for (int i = 0; i < N; ++i) {
                x2[i] = x[i], y2[i] = y[i];
                order[i] = (i * 17) % N;
            }
            if (orc_layout_bh_ord(N, rp, ci, x2, y2, 7, 2, 0, 1.0, 0.999, 1.0, 1.0, 1.2, m != 2, a, r, -1,
                                  m == 2 ? order : NULL, e, sx, sy, &vt)) return 6;
            chk("bh energy", e[0] + e[1]);
        }
    }
    int piv[5] = {0, 3, 3, 44, 20};
    double s = 0.0;
    chk("edge energy", orc_edge_energy(N, rp, ci, x, y, 1.0));
    chk("edge uniformity", orc_edge_uniformity(N, rp, ci, x, y));
    chk("stress", orc_stress(N, rp, ci, x, y, 0, NULL, &s));
    chk("stress pivots", orc_stress(N, rp, ci, x, y, 5, piv, &s));
    chk("np", orc_neighborhood_preservation(N, rp, ci, x, y, 0, NULL, &cnt));
    chk("np sample", orc_neighborhood_preservation(N, rp, ci, x, y, 5, piv, &cnt));
    if (orc_greedy_init(N, rp, ci, 3, x, y, x2, y2, parent)) return 7;
    for (int i = 0; i < N; ++i) chk("greedy", x2[i] + y2[i]);
    printf("oracle driver done\n");
    return bad;
}
