// Single-instance launches of the stencil kernels of one LES time step on
// gfx950.  The per-cell arithmetic lives in les_bodies.h; these wrappers
// map the launch onto logical blocks (XCD-aware) and size the grids.
#include "les_bodies.h"

namespace les {
namespace {

__device__ __forceinline__ unsigned lblock() { return xcd_block(blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(kTileThreads) void k_step_tile(Geo g, TendArgs a, float* __restrict__ nut,
                                                          float c2, int kt) {
    __shared__ TileShared sh;
    step_tile_body(g, a, nut, c2, kt, lblock(), sh);
}

// stretched grids (per-axis metric tables in g)
__global__ __launch_bounds__(kBlock) void k_nut_str(Geo g, const float* __restrict__ u,
                                                    const float* __restrict__ v,
                                                    const float* __restrict__ w,
                                                    float* __restrict__ nut, float cs2) {
    nut_body_str(g, u, v, w, nut, cs2, lblock());
}

__global__ __launch_bounds__(kBlock) void k_tendency_str(Geo g, TendArgs a) {
    tendency_body_str(g, a, lblock());
}

__global__ __launch_bounds__(kBlock) void k_rhs_str(Geo g, const float* __restrict__ us,
                                                    const float* __restrict__ vs,
                                                    const float* __restrict__ ws, float* rhs0,
                                                    float* rhs1, double* __restrict__ part) {
    rhs_body_str(g, us, vs, ws, rhs0, rhs1, part, lblock());
}

__global__ __launch_bounds__(kBlock) void k_project_str(Geo g, float* __restrict__ us,
                                                        float* __restrict__ vs,
                                                        float* __restrict__ ws, PBufs P) {
    project_body_str(g, us, vs, ws, P, lblock());
}

__global__ __launch_bounds__(kBlock) void k_inflow(Geo g, float* __restrict__ us,
                                                   const float* __restrict__ prof,
                                                   const float* __restrict__ prof1, float wt,
                                                   const uint8_t* __restrict__ flags, float amp,
                                                   uint64_t seed, long long step) {
    inflow_body(g, us, prof, prof1, wt, flags, amp, seed, step, blockIdx.x);
}

__global__ void k_ctl_init(Ctl* ctl, double tol, int max_iter, int K) {
    ctl_init_body(ctl, tol, max_iter, K);
}

__global__ __launch_bounds__(kBlock) void k_rhs(Geo g, const float* __restrict__ us,
                                                const float* __restrict__ vs,
                                                const float* __restrict__ ws, float* rhs0,
                                                float* rhs1, double* __restrict__ part,
                                                int singular) {
    rhs_body(g, us, vs, ws, rhs0, rhs1, part, singular, lblock());
}

__global__ __launch_bounds__(kBlock) void k_rhs_mean(Geo g, float* rhs0, float* rhs1,
                                                     double* __restrict__ part, const Ctl* ctl) {
    rhs_mean_body(g, rhs0, rhs1, part, ctl, lblock());
}

__global__ __launch_bounds__(kBlock) void k_project(Geo g, float* __restrict__ us,
                                                    float* __restrict__ vs, float* __restrict__ ws,
                                                    PBufs P) {
    project_body(g, us, vs, ws, P, lblock());
}

__global__ __launch_bounds__(kBlock) void k_bc(Geo g, float* u, float* v, float* w) {
    bc_body(g, u, v, w, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_diag(Geo g, const float* __restrict__ u,
                                                 const float* __restrict__ v,
                                                 const float* __restrict__ w,
                                                 double* __restrict__ part) {
    diag_body(g, u, v, w, part, lblock());
}

// --------------------------------------------------- layout conversions
__global__ __launch_bounds__(kBlock) void k_cells_to_colour(Geo g, const float* __restrict__ src,
                                                            float* dst0, float* dst1) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
    float* dst = ((i0 + j0 + k0) & 1) ? dst1 : dst0;
    dst[g.col(i0 >> 1, j0, k0)] = src[t];
}

__global__ __launch_bounds__(kBlock) void k_colour_to_cells(Geo g, const float* __restrict__ a0,
                                                            const float* __restrict__ a1,
                                                            const float* __restrict__ b0,
                                                            const float* __restrict__ b1,
                                                            float* __restrict__ dst) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
    const int c = (i0 + j0 + k0) & 1;
    const long long e = g.col(i0 >> 1, j0, k0);
    float x = (c ? a1 : a0)[e];
    if (b0) x += (c ? b1 : b0)[e];
    dst[t] = x;
}

__global__ __launch_bounds__(kBlock) void k_fill(float* p, long long n, float v) {
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) p[t] = v;
}

inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t launch_nut_str(const Geo& g, hipStream_t st, const float* u, const float* v,
                          const float* w, float* nut, float cs2) {
    if (!g.stretched) return hipErrorInvalidValue;   // uniform grids: launch_step_tile
    hipLaunchKernelGGL(k_nut_str, dim3(box_blocks(g)), dim3(kBlock), 0, st, g, u, v, w, nut, cs2);
    return hipGetLastError();
}

hipError_t launch_tendency_str(const Geo& g, hipStream_t st, const float* u, const float* v,
                               const float* w, const float* nut, float* fu, float* fv, float* fw,
                               float* su, float* sv, float* sw, const uint8_t* flags, float* us,
                               float* vs, float* ws, float nu, float alpha, float beta, int first) {
    if (!g.stretched) return hipErrorInvalidValue;   // uniform grids: launch_step_tile
    TendArgs a{u, v, w, nut, fu, fv, fw, su, sv, sw, flags, us, vs, ws, nu, alpha, beta, first};
    hipLaunchKernelGGL(k_tendency_str, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, a);
    return hipGetLastError();
}

hipError_t launch_step_tile(const Geo& g, hipStream_t st, const float* u, const float* v,
                            const float* w, float* nut, float* fu, float* fv, float* fw, float* su,
                            float* sv, float* sw, const uint8_t* flags, float* us, float* vs,
                            float* ws, float c2, float nu, float alpha, float beta, int first) {
    if (g.stretched) return hipErrorInvalidValue;   // uniform spacing only
    TendArgs a{u, v, w, nut, fu, fv, fw, su, sv, sw, flags, us, vs, ws, nu, alpha, beta, first};
    hipLaunchKernelGGL(k_step_tile, dim3(tile_blocks(g)), dim3(kTileThreads), 0, st, g, a, nut, c2,
                       tile_kt(g));
    return hipGetLastError();
}

hipError_t launch_inflow(const Geo& g, hipStream_t st, float* us, const float* prof,
                         const float* prof1, float wt, const uint8_t* flags, float amp,
                         uint64_t seed, int64_t step) {
    hipLaunchKernelGGL(k_inflow, dim3(nblocks((long long)g.ny * g.nz)), dim3(kBlock), 0, st, g,
                       us, prof, prof1, wt, flags, amp, seed, (long long)step);
    return hipGetLastError();
}

hipError_t launch_ctl_init(hipStream_t st, Ctl* ctl, double tol, int max_iter, int K) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, ctl, tol, max_iter, K);
    return hipGetLastError();
}

hipError_t launch_rhs(const Geo& g, hipStream_t st, const float* us, const float* vs,
                      const float* ws, float* const rhs[2], double* part, Ctl* ctl,
                      int singular) {
    if (g.stretched) {   // stretched grids have an outflow face: never singular
        if (singular) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_rhs_str, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, us, vs, ws,
                           rhs[0], rhs[1], part);
    } else {
        hipLaunchKernelGGL(k_rhs, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, us, vs, ws, rhs[0],
                           rhs[1], part, singular);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, singular ? FIN_RHS_SUM : FIN_RHS2, part, (int)cell_blocks(g),
                           nullptr, nullptr, 0, ctl);
}

hipError_t launch_remove_mean_rhs(const Geo& g, hipStream_t st, float* const rhs[2],
                                  double* part, Ctl* ctl) {
    hipLaunchKernelGGL(k_rhs_mean, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, rhs[0], rhs[1],
                       part, (const Ctl*)ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, FIN_RHS2, part, (int)cell_blocks(g), nullptr, nullptr, 0, ctl);
}

hipError_t launch_project(const Geo& g, hipStream_t st, float* us, float* vs, float* ws,
                          const PBufs& P) {
    if (g.stretched)
        hipLaunchKernelGGL(k_project_str, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, us, vs, ws, P);
    else
        hipLaunchKernelGGL(k_project, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, us, vs, ws, P);
    return hipGetLastError();
}

hipError_t launch_bc(const Geo& g, hipStream_t st, float* u, float* v, float* w) {
    hipLaunchKernelGGL(k_bc, dim3(bc_blocks(g)), dim3(kBlock), 0, st, g, u, v, w);
    return hipGetLastError();
}

hipError_t launch_diag(const Geo& g, hipStream_t st, const float* u, const float* v,
                       const float* w, double* part, Ctl* ctl) {
    hipLaunchKernelGGL(k_diag, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, u, v, w, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, FIN_DIAG, part, (int)cell_blocks(g), nullptr, nullptr, 0, ctl);
}

hipError_t launch_cells_to_colour(const Geo& g, hipStream_t st, const float* src,
                                  float* const dst[2]) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_cells_to_colour, dim3(nblocks(n)), dim3(kBlock), 0, st, g, src, dst[0],
                       dst[1]);
    return hipGetLastError();
}

hipError_t launch_pair_to_cells(const Geo& g, hipStream_t st, const PBufs& P, float* dst) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_colour_to_cells, dim3(nblocks(n)), dim3(kBlock), 0, st, g, P.ph[0],
                       P.ph[1], P.pd[0], P.pd[1], dst);
    return hipGetLastError();
}

hipError_t launch_colour_to_cells(const Geo& g, hipStream_t st, float* const src[2], float* dst) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_colour_to_cells, dim3(nblocks(n)), dim3(kBlock), 0, st, g, src[0],
                       src[1], (const float*)nullptr, (const float*)nullptr, dst);
    return hipGetLastError();
}

hipError_t launch_fill(hipStream_t st, float* p, long long n, float v) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace les
