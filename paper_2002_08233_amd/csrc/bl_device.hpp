// Device-side helpers shared by the BatchLayout kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bl {

constexpr int kWave = 64;

// Pointer to device global memory.  Kernels that read pointers out of a
// descriptor in memory would otherwise see generic pointers and emit flat
// instructions, which also count against the LDS wait counter (so every LDS
// wait would wait for the gathers in flight too).
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <int N>
struct RawBits;
template <>
struct RawBits<4> {
    using type = unsigned;
};
template <>
struct RawBits<8> {
    using type = unsigned long long;
};
template <>
struct RawBits<16> {
    using type = unsigned __attribute__((ext_vector_type(4)));
};

// Element i of a global array of a vector type (HIP's vector types have no
// constructors from other address spaces, so they move as raw bits).
template <typename T>
__device__ __forceinline__ T ld(gptr<const T> p, size_t i) {
    using B = typename RawBits<sizeof(T)>::type;
    return __builtin_bit_cast(T, ((gptr<const B>)p)[i]);
}
template <typename T>
__device__ __forceinline__ void st(gptr<T> p, size_t i, T v) {
    using B = typename RawBits<sizeof(T)>::type;
    ((gptr<B>)p)[i] = __builtin_bit_cast(B, v);
}

// Kahan-compensated FP32 accumulation: (s, c) represents s - c.
__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Double-double value hi + lo (Knuth two-sum; no products, so no FMA concerns).
struct dd {
    double hi, lo;
};
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    double s = a.hi + b.hi;
    double v = s - a.hi;
    double e = (a.hi - (s - v)) + (b.hi - v);
    e += a.lo + b.lo;
    double hi = s + e;
    double lo = e - (hi - s);
    return dd{hi, lo};
}
__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

// Butterfly sums over a wave.  Lane 0's result is the one used, so the order
// of additions is fixed and the result is reproducible run to run.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over groups of G consecutive lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Inclusive scan of an int over a wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of an int over the whole block (blockDim.x <= 1024, multiple
// of 64).  `wsum` is __shared__ scratch of >= 16 ints.  Returns the exclusive
// prefix; *total receives the block total.  Contains two __syncthreads().
__device__ __forceinline__ int block_excl_scan(int v, int *wsum, int *total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
    for (int q = 0; q < nw; ++q) {
        int s = wsum[q];
        if (q < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Sum of a double over the block in a fixed order: wave butterflies, then
// lane 0 of thread 0 adds the wave results in wave order.  Result valid in
// thread 0 only.  `ws` is __shared__ scratch of >= 16 doubles.
__device__ __forceinline__ double block_sum_fixed(double v, double *ws) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) r += ws[q];
    __syncthreads();
    return r;
}

// The (a, r) model of Sec. 2.2 for integer exponents: |c_j - c_i|^k with
// k = a - 1 (attraction) or r - 1 (repulsion kernel), from d^2 by k/2
// multiplications (or their reciprocal: the hardware one in FP32, as in the
// (2, -1) terms) and one square root for odd k; 0 for a coincident pair.  k
// is uniform across the workgroup.
template <typename T>
__device__ __forceinline__ T dpow(T dx, T dy, int k) {
    const T d2 = fma(dx, dx, dy * dy);
    if (d2 == (T)0) return (T)0;
    const int h = k >> 1;   // floor(k / 2)
    const int m = h < 0 ? -h : h;
    T p = 1;
    for (int q = 0; q < m; ++q) p *= d2;
    if (h < 0) {
        if constexpr (sizeof(T) == 4) p = __builtin_amdgcn_rcpf(p);
        else p = 1.0 / p;
    }
    if (k & 1) p *= sqrt(d2);
    return p;
}

}  // namespace bl
