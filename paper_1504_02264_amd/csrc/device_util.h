// Device helpers: XCD-aware block numbering and wavefront/block reductions
// in float64.  Reductions are two-kernel: every block stores one partial,
// then a single-block finalize kernel sums them in a fixed order (no
// atomics, no cross-block fences, deterministic).
#pragma once

#include <hip/hip_runtime.h>

#include "les_impl.h"

namespace les {

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs,
// each with a private L2.  Renumber so that every XCD owns one contiguous
// range of logical blocks: stencil neighbours (the k-1 and k+1 planes) are
// then fetched into the same L2 instead of into three different ones.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned q = nb / kNumXcd, r = nb % kNumXcd;
    const unsigned x = b % kNumXcd, l = b / kNumXcd;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// A copy of a block-uniform object whose every 32-bit word passes through
// readfirstlane, so that the compiler keeps it (and what is computed from it,
// such as buffer offsets) in scalar registers even when it was loaded from
// memory the compiler cannot prove unchanged.
template <class T>
__device__ __forceinline__ T uniform_copy(const T& src) {
    static_assert(sizeof(T) % 4 == 0, "uniform_copy: whole 32-bit words");
    T dst;
    const int* s = reinterpret_cast<const int*>(&src);
    int* d = reinterpret_cast<int*>(&dst);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return dst;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over a block of kBlock threads in a fixed order (deterministic).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) t += red[i];
    }
    __syncthreads();
    return t;   // valid in thread 0
}

__device__ __forceinline__ double block_max(double v) {
    __shared__ double redm[kBlock / 64];
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) redm[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) t = fmax(t, redm[i]);
    }
    __syncthreads();
    return t;
}

// Block-wide reductions of the single-block finalize kernel (kFinBlock
// threads, fixed order: deterministic for a given partial count).
constexpr int kFinBlock = 256;

__device__ __forceinline__ double fin_sum(double v) {
    __shared__ double red[kFinBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kFinBlock / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double fin_max(double v) {
    __shared__ double redm[kFinBlock / 64];
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) redm[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kFinBlock / 64; ++i) t = fmax(t, redm[i]);
    __syncthreads();
    return t;
}

// Sum of n partials with stride (result valid in thread 0).
__device__ __forceinline__ double sum_partials(const double* part, int n, int stride = 1) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kFinBlock) s += part[(long long)i * stride];
    return fin_sum(s);
}

__device__ __forceinline__ double max_partials(const double* part, int n, int stride = 1) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kFinBlock) s = fmax(s, part[(long long)i * stride]);
    return fin_max(s);
}

}  // namespace les
