// Coordinate conversion between the FP64 ABI and the device state, and the
// step-length schedule.
#include "bl_device.hpp"
#include "bl_internal.hpp"

namespace bl {
namespace {

template <typename T>
__global__ void coords_in_kernel(int n, const double *__restrict__ x, const double *__restrict__ y,
                                 T *__restrict__ ox, T *__restrict__ oy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        ox[i] = (T)x[i];
        oy[i] = (T)y[i];
    }
}

template <typename T>
__global__ void coords_out_kernel(int n, const T *__restrict__ x, const T *__restrict__ y,
                                  double *__restrict__ ox, double *__restrict__ oy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        ox[i] = (double)x[i];
        oy[i] = (double)y[i];
    }
}

__global__ void coords_in_aos_kernel(int n, const double *__restrict__ x, const double *__restrict__ y,
                                     float2 *__restrict__ o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = float2{(float)x[i], (float)y[i]};
}

__global__ void coords_out_aos_kernel(int n, const float2 *__restrict__ p, double *__restrict__ ox,
                                      double *__restrict__ oy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float2 c = p[i];
        ox[i] = (double)c.x;
        oy[i] = (double)c.y;
    }
}

}  // namespace

// Step length of iteration k: step0 multiplied by the decay once per finished
// iteration (Alg. 2: Step = Step * 0.999 at the end of every iteration).
double step_at(const bl_params &p, int k) {
    double s = p.step0;
    for (int t = 0; t < k; ++t) s *= p.step_decay;
    return s;
}

int convert_coords_in(bl_graph *g, const double *x, const double *y) {
    g->cont_iter = -1;
    const int blocks = (g->n + 255) / 256;
    if (g->aos)
        hipLaunchKernelGGL(coords_in_aos_kernel, dim3(blocks), dim3(256), 0, g->stream, g->n, x, y, (float2 *)g->x);
    else if (g->fp64)
        hipLaunchKernelGGL(coords_in_kernel<double>, dim3(blocks), dim3(256), 0, g->stream, g->n, x, y,
                           (double *)g->x, (double *)g->y);
    else
        hipLaunchKernelGGL(coords_in_kernel<float>, dim3(blocks), dim3(256), 0, g->stream, g->n, x, y,
                           (float *)g->x, (float *)g->y);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

int convert_coords_out(bl_graph *g, double *x, double *y) {
    const int blocks = (g->n + 255) / 256;
    if (g->aos)
        hipLaunchKernelGGL(coords_out_aos_kernel, dim3(blocks), dim3(256), 0, g->stream, g->n,
                           (const float2 *)g->x, x, y);
    else if (g->fp64)
        hipLaunchKernelGGL(coords_out_kernel<double>, dim3(blocks), dim3(256), 0, g->stream, g->n,
                           (const double *)g->x, (const double *)g->y, x, y);
    else
        hipLaunchKernelGGL(coords_out_kernel<float>, dim3(blocks), dim3(256), 0, g->stream, g->n,
                           (const float *)g->x, (const float *)g->y, x, y);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

int prof_begin(bl_graph *g, int kid, int *slot) {
    *slot = -1;
    if (!g->prof || !g->prof->on) return BL_OK;
    Prof &P = *g->prof;
    if (P.used == kProfPool) BL_TRY(prof_collect(g));
    *slot = P.used;
    P.kid[P.used] = kid;
    BL_HIP(hipEventRecord(P.ev[2 * P.used], g->stream));
    return BL_OK;
}

int prof_end(bl_graph *g, int slot) {
    if (slot < 0 || !g->prof) return BL_OK;
    Prof &P = *g->prof;
    BL_HIP(hipEventRecord(P.ev[2 * slot + 1], g->stream));
    P.used = slot + 1;
    return BL_OK;
}

int prof_collect(bl_graph *g) {
    if (!g->prof) return BL_OK;
    Prof &P = *g->prof;
    if (P.used == 0) return BL_OK;
    BL_HIP(hipStreamSynchronize(g->stream));
    for (int q = 0; q < P.used; ++q) {
        float ms = 0.f;
        BL_HIP(hipEventElapsedTime(&ms, P.ev[2 * q], P.ev[2 * q + 1]));
        P.ms[P.kid[q]] += ms;
        P.launches[P.kid[q]] += 1;
    }
    P.used = 0;
    return BL_OK;
}

int convert_to_float2(bl_graph *g, const double *x, const double *y, float2 *o) {
    const int blocks = (g->n + 255) / 256;
    hipLaunchKernelGGL(coords_in_aos_kernel, dim3(blocks), dim3(256), 0, g->stream, g->n, x, y, o);
    BL_HIP(hipGetLastError());
    return BL_OK;
}

}  // namespace bl
