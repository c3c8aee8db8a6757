/* Drives the host-side paths of libbatchlayout that run without a GPU --
 * argument and CSR checks, the greedy initialisation (Sec. 3.6), the
 * footprint model, error messages -- for a build of the library's host code
 * with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py).  Every call here returns before any device
 * work.  Exits non-zero on an unexpected status. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "batchlayout.h"

static int fails = 0;
static void expect(const char *what, int got, int want)
{
    if (got != want) {
        printf("%s: status %d, expected %d (%s)\n", what, got, want, bl_last_error());
        fails = 1;
    }
}

int main(void)
{
    /* path 0-1-2-3-4 and a vertex 5 with no edges */
    int rp[7] = {0, 1, 3, 5, 7, 8, 8};
    int ci[8] = {1, 0, 2, 1, 3, 2, 4, 3};
    bl_csr g = {6, 8, rp, ci};
    double x[6] = {0.1, -0.3, 0.7, 0.2, -0.9, 0.5}, y[6] = {0.4, 0.2, -0.6, 0.8, 0.0, -0.1};
    double xo[6], yo[6], en[4];
    bl_params p;
    bl_stats st;
    expect("params_init", bl_params_init(&p), BL_OK);
    expect("params_init NULL", bl_params_init(NULL), BL_E_INVAL);

    /* greedy initialisation, host only */
    double gx[6], gy[6];
    memcpy(gx, x, sizeof x);
    memcpy(gy, y, sizeof y);
    expect("greedy", bl_greedy_init(&g, 2, gx, gy), BL_OK);
    for (int i = 0; i < 6; ++i)
        if (!isfinite(gx[i]) || !isfinite(gy[i])) expect("greedy finite", 1, 0);
    expect("greedy start out of range", bl_greedy_init(&g, 6, gx, gy), BL_E_INVAL);

    /* parameter checks */
    const struct { const char *what; int field; double v; } bad[] = {
        {"batch 0", 0, 0}, {"iterations -1", 1, -1}, {"step0 0", 2, 0}, {"decay 1.5", 3, 1.5},
        {"K 0", 4, 0}, {"R -1", 5, -1}, {"theta -1", 6, -1}, {"conv_tol -1", 7, -1}, {"model (1,2)", 8, 0}};
    for (unsigned q = 0; q < sizeof bad / sizeof bad[0]; ++q) {
        bl_params b = p;
        switch (bad[q].field) {
            case 0: b.batch_size = (int)bad[q].v; break;
            case 1: b.iterations = (int)bad[q].v; break;
            case 2: b.step0 = bad[q].v; break;
            case 3: b.step_decay = bad[q].v; break;
            case 4: b.K = bad[q].v; break;
            case 5: b.R = bad[q].v; break;
            case 6: b.theta = bad[q].v; break;
            case 7: b.conv_tol = bad[q].v; break;
            case 8: b.model_a = 1; b.model_r = 2; break;
        }
        expect(bad[q].what, bl_layout(&g, x, y, &b, NULL, xo, yo, en, &st), BL_E_INVAL);
        if (!strlen(bl_last_error())) expect("error message", 1, 0);
    }

    /* CSR checks */
    int rp_bad[7] = {0, 1, 3, 2, 7, 8, 8};
    bl_csr gb = {6, 8, rp_bad, ci};
    expect("rowptr decreasing", bl_layout(&gb, x, y, &p, NULL, xo, yo, en, &st), BL_E_INVAL);
    int ci_bad[8] = {1, 0, 2, 1, 3, 2, 9, 3};
    bl_csr gc = {6, 8, rp, ci_bad};
    expect("colidx out of range", bl_layout(&gc, x, y, &p, NULL, xo, yo, en, &st), BL_E_INVAL);
    bl_params v = p;
    v.flags = BL_VALIDATE;
    int ci_asym[8] = {1, 0, 2, 1, 3, 2, 4, 2};
    bl_csr ga = {6, 8, rp, ci_asym};
    expect("asymmetric (validate)", bl_layout(&ga, x, y, &v, NULL, xo, yo, en, &st), BL_E_INVAL);
    /* the shuffled layout checks in-degrees against row lengths itself */
    int rp_s[3] = {0, 1, 1}, ci_s[1] = {1};
    bl_csr gs = {2, 1, rp_s, ci_s};
    double xs[2] = {0, 1}, ys[2] = {0, 0}, xso[2], yso[2], es[2];
    bl_params ps = p;
    ps.iterations = 1;
    ps.batch_size = 1;
    expect("shuffled asymmetric", bl_layout_shuffled(&gs, xs, ys, &ps, 1, NULL, xso, yso, es, &st), BL_E_INVAL);

    /* quality, neighbourhood preservation and the allocation-free call reject bad arguments */
    bl_quality q;
    expect("quality NULL out", bl_quality_eval(&g, x, y, 0, NULL, 1.0, 0, NULL, NULL), BL_E_INVAL);
    expect("quality K", bl_quality_eval(&g, x, y, 0, NULL, 0.0, 0, NULL, &q), BL_E_INVAL);
    int piv[2] = {0, 6};
    expect("quality pivot", bl_quality_eval(&g, x, y, 2, piv, 1.0, 0, NULL, &q), BL_E_INVAL);
    expect("noalloc host pointers", bl_quality_eval_noalloc(&g, x, y, 0, NULL, 1.0, 0, NULL, &q), BL_E_INVAL);
    double npv;
    long long cnt;
    expect("np sample", bl_neighborhood_preservation(&g, x, y, 2, piv, 0, NULL, &npv, (int64_t *)&cnt), BL_E_INVAL);

    /* footprint model */
    if (bl_footprint_bytes(1000, 8000, &p) == 0 || bl_footprint_bytes(0, 0, &p) != 0) expect("footprint", 1, 0);
    bl_params pb = p;
    pb.mode = BL_BH;
    if (bl_footprint_bytes(100000, 1600000, &pb) <= bl_footprint_bytes(1000, 16000, &pb)) expect("footprint bh", 1, 0);
    if (!bl_version() || !strlen(bl_version())) expect("version", 1, 0);
    printf("abi driver done\n");
    return fails;
}
