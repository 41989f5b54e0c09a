// Twinned double-buffer relaxation (section 2.6): the paper's GPU
// alternative to the red-black scheme, built here as a measured comparison
// solver beside the red-black SOR of the time step.
//
// p is held as a pair (p_0, p_1) per cell in one interleaved float2 array
// with a zero ghost ring, natural order ((nz+2) planes of (ny+2) rows of
// nx+2 pairs).  The first half of an iteration sets every cell's p_1 from
// the p_0 values (own and six neighbours), the second half p_0 from p_1,
// each with the SOR point formula (sor_point, the same rounding as the
// red-black sweeps).  Every neighbour therefore comes from the previous
// half: a relaxed Jacobi iteration, not red-black SOR.
//
// 64 consecutive cells of a row per wavefront, 4 rows per block, each
// thread marching up 8 planes of its column.  Per half: the pair of the
// cell (8 bytes; neighbours from registers, lanes and the cache), rhs (4
// bytes) and one component written (4 bytes), 16 bytes per cell at best.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "les_bodies.h"

using namespace les;

namespace {

constexpr int kTwRows = kBlock / 64;

__device__ __forceinline__ long long tw_index(const Geo& g, int i0, int j0, int k0) {
    return ((long long)(k0 + 1) * (g.ny + 2) + (j0 + 1)) * (g.nx + 2) + (i0 + 1);
}

__device__ __forceinline__ bool tw_cell(const Geo& g, int& i0, int& j0, int& k0) {
    i0 = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    j0 = (int)blockIdx.y * kTwRows + (int)(threadIdx.x >> 6);
    k0 = (int)blockIdx.z;
    return i0 < g.nx && j0 < g.ny;
}

__global__ __launch_bounds__(kBlock) void k_twin_load(Geo g, const float* __restrict__ p,
                                                      float2* __restrict__ q) {
    int i0, j0, k0;
    if (!tw_cell(g, i0, j0, k0)) return;
    const float v = p[((long long)k0 * g.ny + j0) * g.nx + i0];
    q[tw_index(g, i0, j0, k0)] = make_float2(v, v);
}

// Half-iteration: component SRC of every cell's pair -> component 1 - SRC.
// A thread marches up kt planes of its (i, j) column keeping the values of
// planes k-1, k, k+1 in registers; east and west come from the adjacent
// lanes (a wavefront holds 64 consecutive cells of a row), the row ends and
// the last cell of the grid row from memory.  Lanes past the row end take
// part in the shuffles only.
// kt: at most 8, fewer when the grid would otherwise have under 1024
// blocks (4 per compute unit; measured: at 150x150x90, 8 planes in 1368
// blocks beat 2 planes in 5130).
constexpr int kTwPlanesMax = 8;
constexpr long long kTwMinBlocks = 1024;

template <int SRC>
__global__ __launch_bounds__(kBlock) void k_twin_sweep(Geo g, float2* q, const float* __restrict__ rhs,
                                                       float omega, int kt) {
    const int lane = (int)(threadIdx.x & 63);
    const int i0 = (int)blockIdx.x * 64 + lane;
    const int j0 = (int)blockIdx.y * kTwRows + (int)(threadIdx.x >> 6);
    if (j0 >= g.ny) return;                      // a whole wavefront
    const int kb = (int)blockIdx.z * kt;
    const int ke = min(g.nz, kb + kt);
    const bool live = i0 < g.nx;
    const float* src = reinterpret_cast<const float*>(q) + SRC;
    float* dst = reinterpret_cast<float*>(q) + (1 - SRC);
    const long long X = g.nx + 2, P = X * (g.ny + 2);
    long long e = tw_index(g, i0, j0, kb);
    const long long rrow = (long long)j0 * g.nx + i0, rplane = (long long)g.ny * g.nx;
    const float dxy = diag_x(g, i0) + diag_y(g, j0);
    float pb = live ? src[2 * (e - P)] : 0.f;
    float pc = live ? src[2 * e] : 0.f;
    for (int k0 = kb; k0 < ke; ++k0) {
        const float pt = live ? src[2 * (e + P)] : 0.f;
        float pe = __shfl_down(pc, 1, 64);
        float pw = __shfl_up(pc, 1, 64);
        if (live) {
            if (lane == 63 || i0 == g.nx - 1) pe = src[2 * (e + 1)];
            if (lane == 0) pw = src[2 * (e - 1)];
            const float ps = src[2 * (e - X)], pn = src[2 * (e + X)];
            const float r = rhs[(long long)k0 * rplane + rrow];
            float reltmp;
            dst[2 * e] = sor_point(pw, pe, ps, pn, pb, pt, g.cx, g.cy, g.cz, dxy + diag_z(g, k0), r, pc,
                                   omega, reltmp);
        }
        pb = pc;
        pc = pt;
        e += P;
    }
}

__global__ __launch_bounds__(kBlock) void k_twin_store(Geo g, const float2* __restrict__ q,
                                                       float* __restrict__ p) {
    int i0, j0, k0;
    if (!tw_cell(g, i0, j0, k0)) return;
    p[((long long)k0 * g.ny + j0) * g.nx + i0] = q[tw_index(g, i0, j0, k0)].x;
}

// Per-block float64 partials of sum (rhs - A p_0)^2 and sum rhs^2, A p =
// sum_nb cn_nb p_nb - diag p, elementwise in float64 from the float32
// values; fixed order within the block.
__global__ __launch_bounds__(kBlock) void k_twin_resid(Geo g, const float2* __restrict__ q,
                                                       const float* __restrict__ rhs,
                                                       double* __restrict__ part) {
    int i0, j0, k0;
    double r2 = 0.0, b2 = 0.0;
    if (tw_cell(g, i0, j0, k0)) {
        const long long e = tw_index(g, i0, j0, k0);
        const long long X = g.nx + 2, P = X * (g.ny + 2);
        const double nb = (double)g.cx * ((double)q[e - 1].x + (double)q[e + 1].x) +
                          (double)g.cy * ((double)q[e - X].x + (double)q[e + X].x) +
                          (double)g.cz * ((double)q[e - P].x + (double)q[e + P].x);
        const double ap = nb - (double)diag_of(g, i0, j0, k0) * (double)q[e].x;
        const double b = (double)rhs[((long long)k0 * g.ny + j0) * g.nx + i0];
        r2 = (b - ap) * (b - ap);
        b2 = b * b;
    }
    const long long lb = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const double s = block_sum(r2);
    if (threadIdx.x == 0) part[2 * lb] = s;
    const double t = block_sum(b2);
    if (threadIdx.x == 0) part[2 * lb + 1] = t;
}

int tw_err(les_handle* h, int code, const char* what, hipError_t e = hipSuccess) {
    char buf[512];
    if (e != hipSuccess)
        std::snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    else
        std::snprintf(buf, sizeof buf, "%s", what);
    h->err = buf;
    return code;
}

}  // namespace

namespace les {
void twinned_free(les_handle* h) {
    if (h->tw_q) (void)hipFree(h->tw_q);
    if (h->tw_part) (void)hipFree(h->tw_part);
    h->tw_q = nullptr;
    h->tw_part = nullptr;
}
}  // namespace les

extern "C" int les_pressure_solve_twinned(les_handle* h, const float* d_rhs, float* d_p, double omega,
                                          int32_t iters, les_solve_stats* st, double* ms,
                                          void* stream) {
    if (!h) return LES_EINVAL;
    if (!d_rhs || !d_p) return tw_err(h, LES_EINVAL, "NULL rhs or p");
    if (iters < 0) return tw_err(h, LES_EINVAL, "iters < 0");
    if (!(omega > 0.0 && omega <= 1.0)) return tw_err(h, LES_EINVAL, "omega outside (0, 1]");
    if (h->g.stretched) return tw_err(h, LES_EINVAL, "uniform grids only");
    const Geo& g = h->g;
    const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + kTwRows - 1) / kTwRows),
                    (unsigned)g.nz);
    const size_t nblocks = (size_t)grid.x * grid.y * grid.z;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    if (!h->tw_q) {
        // installed in the handle only once both buffers exist and the
        // ghost ring is zero
        const size_t npair = (size_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
        void* qa = nullptr;
        void* pa = nullptr;
        hipError_t e = hipMalloc(&qa, npair * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&pa, 2 * nblocks * sizeof(double));
        if (e == hipSuccess) e = hipMemsetAsync(qa, 0, npair * sizeof(float2), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            if (qa) (void)hipFree(qa);
            if (pa) (void)hipFree(pa);
            return tw_err(h, e == hipErrorOutOfMemory ? LES_ENOMEM : LES_EDEVICE, "twinned workspace", e);
        }
        h->tw_q = qa;
        h->tw_part = (double*)pa;
    }
    float2* q = (float2*)h->tw_q;
    double* part = h->tw_part;
    const dim3 block(kBlock);
    const long long per_plane = (long long)grid.x * grid.y;
    int kt = (int)std::min<long long>(kTwPlanesMax, std::max<long long>(1, (long long)g.nz * per_plane / kTwMinBlocks));
    const dim3 sweep_grid(grid.x, grid.y, (unsigned)((g.nz + kt - 1) / kt));
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto fin = [&](int rc) {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        return rc;
    };
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "hipEventCreate"));
    hipLaunchKernelGGL(k_twin_load, grid, block, 0, s, g, d_p, q);
    if (hipGetLastError() != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "k_twin_load"));
    if (hipEventRecord(ev[0], s) != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "event"));
    const float om = (float)omega;
    for (int m = 0; m < iters; ++m) {
        hipLaunchKernelGGL(k_twin_sweep<0>, sweep_grid, block, 0, s, g, q, d_rhs, om, kt);
        hipLaunchKernelGGL(k_twin_sweep<1>, sweep_grid, block, 0, s, g, q, d_rhs, om, kt);
    }
    if (hipGetLastError() != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "k_twin_sweep"));
    if (hipEventRecord(ev[1], s) != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "event"));
    hipLaunchKernelGGL(k_twin_store, grid, block, 0, s, g, q, d_p);
    hipLaunchKernelGGL(k_twin_resid, grid, block, 0, s, g, q, d_rhs, part);
    if (hipGetLastError() != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "k_twin_resid"));
    std::vector<double> hp(2 * nblocks);
    hipError_t e = hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fin(tw_err(h, LES_EDEVICE, "twinned solve", e));
    double r2 = 0.0, b2 = 0.0;
    for (size_t b = 0; b < nblocks; ++b) {
        r2 += hp[2 * b];
        b2 += hp[2 * b + 1];
    }
    float dt_ms = 0.f;
    if (hipEventElapsedTime(&dt_ms, ev[0], ev[1]) != hipSuccess) dt_ms = -1.f;
    if (ms) *ms = dt_ms;
    if (st) {
        st->iters = iters;
        st->rhs_norm = std::sqrt(b2);
        st->resid = b2 > 0.0 ? std::sqrt(r2 / b2) : 0.0;
        st->converged = st->resid <= h->prm.tol ? 1 : 0;
        st->reltmp2 = 0.0;
    }
    if (!std::isfinite(r2)) return fin(tw_err(h, LES_ENONFINITE, "non-finite residual"));
    return fin(LES_OK);
}
