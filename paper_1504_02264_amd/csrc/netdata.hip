// Training-set preparation for the learned warm start, on the device: the
// pairs the LES captures are cut into windows (optionally reflected in y),
// gathered into mini-batches and scaled by their RMS here, so the learned
// part's data path runs in the library's own kernels (the caller's
// framework only provides the memory).  Declared in include/lesnet.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lesnet.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxGather = 64;   // mini-batch items per lesnet_gather call

struct GatherIdx {
    int32_t v[kMaxGather];
};

// dst[r][c][e][k] = src[z + r][y + (mirror ? ch - 1 - c : c)][x + e][k]
__global__ __launch_bounds__(kThreads) void k_crop(const float* __restrict__ src, int H, int W, int C, int z,
                                                   int y, int x, int cd, int ch, int cw, int mirror,
                                                   float* __restrict__ dst) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long n = (long long)cd * ch * cw * C;
    if (t >= n) return;
    const int k = (int)(t % C);
    long long r = t / C;
    const int e = (int)(r % cw);
    r /= cw;
    const int c = (int)(r % ch);
    const int d = (int)(r / ch);
    const int sy = y + (mirror ? ch - 1 - c : c);
    dst[t] = src[(((long long)(z + d) * H + sy) * W + (x + e)) * C + k];
}

__global__ __launch_bounds__(kThreads) void k_gather(const float* __restrict__ src, long long item, GatherIdx idx,
                                                     int n, float* __restrict__ dst) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= item * n) return;
    const int b = (int)(t / item);
    const long long o = t - (long long)b * item;
    dst[t] = src[(long long)idx.v[b] * item + o];
}

// One block, fixed order: thread i sums elements i, i + 1024, ... in
// float64, then a tree over the block; the result is deterministic.
__global__ __launch_bounds__(1024) void k_sum_squares(const float* __restrict__ x, long long n,
                                                      double* __restrict__ out) {
    __shared__ double part[1024];
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += 1024) {
        const double v = (double)x[i];
        s += v * v;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

__global__ __launch_bounds__(kThreads) void k_scale_div(const float* __restrict__ x, long long n, float s,
                                                        float* __restrict__ y) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t < n) y[t] = x[t] / s;
}

unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

int launch_status() { return hipGetLastError() == hipSuccess ? LES_OK : LES_EDEVICE; }

}  // namespace

extern "C" int lesnet_crop(const float* d_src, int32_t D, int32_t H, int32_t W, int32_t C, int32_t z,
                           int32_t y, int32_t x, int32_t cd, int32_t ch, int32_t cw, int32_t mirror_y,
                           float* d_dst, void* stream) {
    if (!d_src || !d_dst || D < 1 || H < 1 || W < 1 || C < 1 || cd < 1 || ch < 1 || cw < 1) return LES_EINVAL;
    if (z < 0 || y < 0 || x < 0 || z + cd > D || y + ch > H || x + cw > W) return LES_EINVAL;
    const long long n = (long long)cd * ch * cw * C;
    if (n / C / cw / ch != cd || (long long)blocks_for(n) >= (1LL << 31)) return LES_EINVAL;
    hipLaunchKernelGGL(k_crop, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, d_src, H, W, C, z, y,
                       x, cd, ch, cw, mirror_y ? 1 : 0, d_dst);
    return launch_status();
}

extern "C" int lesnet_gather(const float* d_src, int64_t item, int64_t count, const int32_t* idx, int32_t n,
                             float* d_dst, void* stream) {
    if (!d_src || !d_dst || !idx || item < 1 || count < 1 || n < 1 || n > kMaxGather) return LES_EINVAL;
    GatherIdx g{};
    for (int b = 0; b < n; ++b) {
        if (idx[b] < 0 || idx[b] >= count) return LES_EINVAL;
        g.v[b] = idx[b];
    }
    const long long m = item * n;
    if ((long long)blocks_for(m) >= (1LL << 31)) return LES_EINVAL;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(m)), dim3(kThreads), 0, (hipStream_t)stream, d_src,
                       (long long)item, g, (int)n, d_dst);
    return launch_status();
}

extern "C" int lesnet_sum_squares(const float* d_x, int64_t n, double* d_out, void* stream) {
    if (!d_out || n < 0 || (n > 0 && !d_x)) return LES_EINVAL;
    hipLaunchKernelGGL(k_sum_squares, dim3(1), dim3(1024), 0, (hipStream_t)stream, d_x, (long long)n, d_out);
    return launch_status();
}

extern "C" int lesnet_scale_div(const float* d_x, int64_t n, float s, float* d_y, void* stream) {
    if (n < 0 || (n > 0 && (!d_x || !d_y)) || !(s > 0.f) || !(s < 3.0e38f)) return LES_EINVAL;
    if (n == 0) return LES_OK;
    if ((long long)blocks_for(n) >= (1LL << 31)) return LES_EINVAL;
    hipLaunchKernelGGL(k_scale_div, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, d_x,
                       (long long)n, s, d_y);
    return launch_status();
}
