// Greedy initial layout (Sec. 3.6, Algorithm 3), a host routine of the
// library.
//
// The traversal is sequential by definition: which neighbours a popped vertex
// still finds unvisited, and so every angle, depends on the exact pop order of
// the stack.  On the GPU each pop would be a chain of dependent memory round
// trips (row bounds, then the row, then the visited flags), about a
// microsecond or more, for up to n pops; on one host core the whole traversal
// is O(n + m) with cache-resident state and takes milliseconds at 10^5
// vertices.  It runs once, before the iterations, on the caller's host arrays.
#include <cmath>
#include <cstdint>
#include <vector>

#include "bl_internal.hpp"

namespace {

// The paper's value for pi in the placement angle.
constexpr double kPaperPi = 3.1416;

// One traversal from `root` (already placed): pop a vertex, put its unvisited
// neighbours on the unit circle around it, in row order, 360/deg degrees
// apart starting at angle 0, and push them.
void place_from(int root, const int32_t *rp, const int32_t *ci, std::vector<uint8_t> &seen,
                std::vector<int32_t> &stack, double *x, double *y) {
    stack.clear();
    stack.push_back(root);
    seen[root] = 1;
    while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        const int r0 = rp[u], r1 = rp[u + 1];
        if (r1 == r0) continue;
        const double step_deg = 360.0 / (r1 - r0);
        double ang_deg = 0.0;
        const double ux = x[u], uy = y[u];
        for (int e = r0; e < r1; ++e) {
            const int v = ci[e];
            if (seen[v]) continue;
            seen[v] = 1;
            const double a = kPaperPi * ang_deg / 180.0;
            x[v] = ux + std::cos(a);
            y[v] = uy + std::sin(a);
            stack.push_back(v);
            ang_deg = ang_deg + step_deg;
        }
    }
}

}  // namespace

extern "C" int bl_greedy_init(const bl_csr *g, int32_t start, double *x, double *y) {
    using namespace bl;
    if (!g) return fail_code(BL_E_INVAL, "graph is NULL");
    if (g->n < 1) return fail_code(BL_E_INVAL, "n must be >= 1");
    if (g->nnz < 0 || g->nnz > 0x7fffffffLL) return fail_code(BL_E_INVAL, "nnz out of range");
    if (!g->rowptr || (g->nnz > 0 && !g->colidx)) return fail_code(BL_E_INVAL, "CSR arrays are NULL");
    if (!x || !y) return fail_code(BL_E_INVAL, "coordinate arrays are NULL");
    if (start < 0 || start >= g->n) return fail_code(BL_E_INVAL, "start vertex out of range");
    int rc = check_csr_host(g->n, g->nnz, g->rowptr, g->colidx, false);
    if (rc != BL_OK) return rc;
    const int n = g->n;
    std::vector<uint8_t> seen;
    std::vector<int32_t> stack;
    try {
        seen.assign(n, 0);
        stack.reserve(n);
    } catch (...) {
        return fail_code(BL_E_NOMEM, "host allocation failed");
    }
    x[start] = 0.0;
    y[start] = 0.0;
    place_from(start, g->rowptr, g->colidx, seen, stack, x, y);
    // vertices the start does not reach: each further component grows from
    // its lowest id, which keeps the position given on entry
    for (int v = 0; v < n; ++v)
        if (!seen[v]) place_from(v, g->rowptr, g->colidx, seen, stack, x, y);
    return BL_OK;
}
