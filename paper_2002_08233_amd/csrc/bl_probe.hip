// Instruction issue-rate probe (a diagnostic beside the layout path): how many
// FP32 fused multiply-adds and hardware reciprocals (v_rcp_f32) the device
// issues per second, alone and in the repulsion term's mix of six FMA-class
// operations per reciprocal.  The exact kernel's instruction-bound ceiling is
// stated from these rates.
#include "bl_internal.hpp"

namespace bl {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;   // independent dependency chains per thread

// op 0: v_fma_f32 chains; op 1: v_rcp_f32 chains; op 2: per chain one
// v_rcp_f32 and six v_fma_f32 of other chains, all independent.
__global__ __launch_bounds__(kProbeThreads) void issue_probe_kernel(int op, int iters, float seed, float *out) {
    float a[kProbeChains], b[kProbeChains], c[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
        a[k] = seed + 1e-3f * (float)(threadIdx.x + k);
        b[k] = a[k] * 0.5f;
        c[k] = a[k] * 0.25f;
    }
    if (op == 0) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kProbeChains; ++k) a[k] = fmaf(a[k], 0.9999f, 1e-4f);
        }
    } else if (op == 1) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kProbeChains; ++k) a[k] = __builtin_amdgcn_rcpf(a[k]);
        }
    } else {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kProbeChains; ++k) {
                a[k] = __builtin_amdgcn_rcpf(a[k]);
                b[k] = fmaf(b[k], 0.9999f, 1e-4f);
                c[k] = fmaf(c[k], 0.9999f, 1e-4f);
                b[k] = fmaf(b[k], 0.9999f, 1e-4f);
                c[k] = fmaf(c[k], 0.9999f, 1e-4f);
                b[k] = fmaf(b[k], 0.9999f, 1e-4f);
                c[k] = fmaf(c[k], 0.9999f, 1e-4f);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += a[k] + b[k] + c[k];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = s;   // keeps every chain live
}

}  // namespace
}  // namespace bl

extern "C" int bl_probe_issue_rate(int32_t op, int32_t blocks, int32_t iters, void *hip_stream, double *ms,
                                   double *lane_ops) {
    using namespace bl;
    if (op < 0 || op > 2 || blocks <= 0 || iters <= 0 || !ms) {
        set_error("bl_probe_issue_rate: op must be 0, 1 or 2 and blocks, iters positive, ms non-null");
        return BL_E_INVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BL_OK;
    if (hipMalloc((void **)&out, sizeof(float) * (size_t)blocks * kProbeThreads) != hipSuccess) {
        set_error("bl_probe_issue_rate: device allocation failed");
        return BL_E_NOMEM;
    }
    float t = 0.f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = BL_E_HIP;
    if (rc == BL_OK) {
        // one untimed launch, then the timed one
        hipLaunchKernelGGL(issue_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, op, iters, 1.25f, out);
        if (hipEventRecord(e0, s) != hipSuccess) rc = BL_E_HIP;
        hipLaunchKernelGGL(issue_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, op, iters, 1.5f, out);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            rc = BL_E_HIP;
    }
    if (rc != BL_OK) set_error("bl_probe_issue_rate: HIP launch or event failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc != BL_OK) return rc;
    *ms = (double)t;
    if (lane_ops) {
        const double per = op == 2 ? 7.0 : 1.0;   // instructions per chain and round
        *lane_ops = (double)blocks * kProbeThreads * (double)iters * kProbeChains * per;
    }
    return BL_OK;
}
