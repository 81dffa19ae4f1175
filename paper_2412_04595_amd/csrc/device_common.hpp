// Device helpers shared by the kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace sog {

// a complex value on its natural 8 (float) / 16 (double) byte boundary
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }

// four reals on their natural 16 (float) / 32 (double) byte boundary, so a record moves
// with one vector load or store
template <typename T>
struct alignas(4 * sizeof(T)) vec4 {
    T x, y, z, w;
};

template <typename T>
__device__ __forceinline__ T dexp(T v);
template <>
__device__ __forceinline__ float dexp<float>(float v) { return __expf(v); }
template <>
__device__ __forceinline__ double dexp<double>(double v) { return exp(v); }

template <typename T>
__device__ __forceinline__ T drsqrt(T v);
template <>
__device__ __forceinline__ float drsqrt<float>(float v) { return rsqrtf(v); }
template <>
__device__ __forceinline__ double drsqrt<double>(double v) { return rsqrt(v); }

template <typename T>
__device__ __forceinline__ void dsincos(T v, T* s, T* c);
template <>
__device__ __forceinline__ void dsincos<float>(float v, float* s, float* c) { sincosf(v, s, c); }
template <>
__device__ __forceinline__ void dsincos<double>(double v, double* s, double* c) { sincos(v, s, c); }

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).  Give each
// XCD a contiguous range of logical work items so that neighbouring tiles share an L2.
// Launch 8 * ceil(nwork / 8) blocks; returns -1 for the spare blocks.
__device__ __forceinline__ int xcd_logical_block(int nwork) {
    const int per = (nwork + 7) >> 3;
    const int b = blockIdx.x;
    const int logical = (b & 7) * per + (b >> 3);
    return logical < nwork ? logical : -1;
}
inline int xcd_grid(int nwork) { return ((nwork + 7) / 8) * 8; }

// x wrapped into [0, L)
__device__ __forceinline__ double wrap_periodic(double x, double L) {
    double w = x - L * floor(x / L);
    if (w >= L) w -= L;
    if (w < 0) w = 0;
    return w;
}

__device__ __forceinline__ int imod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Sum of a double over a block (blockDim.x <= 1024, multiple of 64); result valid in thread 0.
__device__ __forceinline__ double block_sum_double(double v, double* lds /* >= 16 */) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r += lds[i];
    }
    return r;
}

}  // namespace sog
