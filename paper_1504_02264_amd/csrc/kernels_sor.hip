// Red-black SOR for the pressure Poisson equation (section 2.6), gfx950.
//
// The cells of one colour are stored contiguously (colour-split layout,
// les_impl.h), so a half-sweep reads the other colour's array and its own
// arrays with unit stride and writes its own: 8 bytes per cell per
// half-sweep, 16 per iteration.  Within a colour every update only reads
// the other colour, so the parallel half-sweep equals the sequential one
// of the paper exactly.
//
// Precision.  p is held as a float32 base ph plus a float32 correction pd.
// The sweeps relax pd against r0 = rhs - A ph (evaluated in float64,
// stored in float32): since SOR is affine, the iterates ph + pd are those
// of plain SOR on p, but each update now rounds relative to |pd| instead
// of |p|, so float32 storage does not stall the iteration.  Every few
// checks the correction is folded into the base (TwoSum, no loss) and r0
// recomputed.  Residuals ||rhs - A p|| are accumulated in float64.
#include "device_util.h"
#include "les_impl.h"

namespace les {
namespace {

inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Diagonal of A at 0-based cell (i0, j0, k0): 1/h^2 per interior neighbour,
// nothing across a wall or the inflow face (Neumann), 2/h^2 across the
// outflow face (p = 0 on the face).
__device__ __forceinline__ float diag_of(const Geo& g, int i0, int j0, int k0) {
    const float dxx = (i0 > 0 ? g.cx : 0.f) + (i0 < g.nx - 1 ? g.cx : (g.outflow ? 2.f * g.cx : 0.f));
    const float dyy = (j0 > 0 ? g.cy : 0.f) + (j0 < g.ny - 1 ? g.cy : 0.f);
    const float dzz = (k0 > 0 ? g.cz : 0.f) + (k0 < g.nz - 1 ? g.cz : 0.f);
    return dxx + dyy + dzz;
}

// Thread -> colour-array coordinates (ii, j0, k0) for a launch over
// H * ny * nz half-cells.
__device__ __forceinline__ bool half_cell(const Geo& g, long long t, int& ii, int& j0, int& k0) {
    const long long hy = (long long)g.H * g.ny;
    if (t >= hy * g.nz) return false;
    k0 = (int)(t / hy);
    const long long r = t - (long long)k0 * hy;
    j0 = (int)(r / g.H);
    ii = (int)(r - (long long)j0 * g.H);
    return true;
}

// ---------------------------------------------------------- half-sweep
// Colour c: for every cell of colour c,
//   reltmp = omega (cn1 (sum_nb cn_nb p_nb - rhs) - p);  p += reltmp
// with cn1 = 1/diag.  Outside the domain the other colour's array holds
// zeros, so the neighbour sum needs no boundary branches.  Skipped when the
// solve is done or max_iter is reached; on the last iteration of a check
// interval it also leaves float64 partials of sum reltmp^2.
__global__ __launch_bounds__(kBlock) void k_sor(Geo g, int c, float* __restrict__ pself,
                                                const float* __restrict__ poth,
                                                const float* __restrict__ rself, float omega,
                                                int local_iter, double* __restrict__ rel_part,
                                                const Ctl* __restrict__ ctl) {
    const int done = ctl->done, m = ctl->m, K = ctl->K, mx = ctl->max_iter;
    if (done || m + local_iter >= mx) return;
    const bool acc = (rel_part != nullptr) && (m + local_iter + 1 == min(m + K, mx));
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    int ii, j0, k0;
    double r2 = 0.0;
    if (half_cell(g, t, ii, j0, k0)) {
        const int s = (c + j0 + k0) & 1;
        const int i0 = 2 * ii + s;
        if (i0 < g.nx) {
            const long long e = g.col(ii, j0, k0);
            const float pw = poth[e - 1 + s], pe = poth[e + s];
            const float ps = poth[e - g.S], pn = poth[e + g.S];
            const float pb = poth[e - g.SP], pt = poth[e + g.SP];
            const float nb = g.cx * (pw + pe) + g.cy * (ps + pn) + g.cz * (pb + pt);
            const float inv = 1.0f / diag_of(g, i0, j0, k0);
            const float p = pself[e];
            const float reltmp = omega * (inv * (nb - rself[e]) - p);
            pself[e] = p + reltmp;
            r2 = (double)reltmp * (double)reltmp;
        }
    }
    if (acc) {
        const double bs = block_sum(r2);
        if (threadIdx.x == 0) rel_part[lb] = bs;
    }
}

// ------------------------------------------------------------- fold
// ph <- fl(ph + pd), pd <- exact remainder (Knuth's TwoSum), pointwise over
// the whole colour arrays (padding stays 0 + 0 = 0).
__global__ __launch_bounds__(kBlock) void k_fold(long long n, float* __restrict__ ph0,
                                                 float* __restrict__ pd0, float* __restrict__ ph1,
                                                 float* __restrict__ pd1, const Ctl* ctl) {
    if (ctl->done) return;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 2 * n) return;
    float* ph = t < n ? ph0 : ph1;
    float* pd = t < n ? pd0 : pd1;
    const long long e = t < n ? t : t - n;
    const float a = ph[e], b = pd[e];
    const float s = a + b;
    const float bb = s - a;
    const float err = (a - (s - bb)) + (b - bb);
    ph[e] = s;
    pd[e] = err;
}

// (A x) at a cell in float64 from the float32 colour arrays x_own/x_oth.
__device__ __forceinline__ double apply_A64(const Geo& g, const float* xo, const float* xn,
                                            long long e, int s, double d) {
    const double nb = (double)g.cx * ((double)xn[e - 1 + s] + (double)xn[e + s]) +
                      (double)g.cy * ((double)xn[e - g.S] + (double)xn[e + g.S]) +
                      (double)g.cz * ((double)xn[e - g.SP] + (double)xn[e + g.SP]);
    return nb - d * (double)xo[e];
}

// Shared decision of a residual check, run by the last block.
__device__ void decide(Ctl* ctl, double sum_r2, double rel) {
    if (ctl->done) return;
    const int m = min(ctl->m + ctl->K, ctl->max_iter);
    ctl->m = m;
    const double R = sqrt(sum_r2) / sqrt(ctl->rhs2);
    ctl->resid = R;
    ctl->reltmp2 = rel;
    if (!isfinite(R)) ctl->done = 3;
    else if (R <= ctl->tol) ctl->done = 1;
    else if (m >= ctl->max_iter) ctl->done = 2;
}

// ------------------------------------------------------------ rebase
// After a fold: r0 = rhs - A ph in float64, stored in float32, and the
// float64 residual of the iterate, rhs - A (ph + pd).  A launch over
// H * ny * nz threads, each handling its two cells (one per colour).
// decide = 0: the set-up at the start of a solve (no check counted; an
// rhs of zero, or a non-finite one, ends the solve here).
// decide = 1: this is the check after the current chunk of iterations.
__global__ __launch_bounds__(kBlock) void k_rebase(Geo g, const float* __restrict__ ph0,
                                                   const float* __restrict__ ph1,
                                                   const float* __restrict__ pd0,
                                                   const float* __restrict__ pd1,
                                                   const float* __restrict__ rhs0,
                                                   const float* __restrict__ rhs1,
                                                   float* __restrict__ r00, float* __restrict__ r01,
                                                   double* __restrict__ part, const double* rel0,
                                                   const double* rel1, int nrel, Ctl* ctl,
                                                   int decide_flag) {
    if (ctl->done) return;   // uniform over the grid: the last-block count stays consistent
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    int ii, j0, k0;
    double acc = 0.0;
    if (half_cell(g, t, ii, j0, k0)) {
        const long long e = g.col(ii, j0, k0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int s = (c + j0 + k0) & 1;
            const int i0 = 2 * ii + s;
            if (i0 < g.nx) {
                const float* pho = c ? ph1 : ph0;
                const float* phn = c ? ph0 : ph1;
                const float* pdo = c ? pd1 : pd0;
                const float* pdn = c ? pd0 : pd1;
                const float* rh = c ? rhs1 : rhs0;
                float* r0 = c ? r01 : r00;
                const double d = (double)diag_of(g, i0, j0, k0);
                const double rb = (double)rh[e] - apply_A64(g, pho, phn, e, s, d);
                r0[e] = (float)rb;
                const double rt = rb - apply_A64(g, pdo, pdn, e, s, d);
                acc += rt * rt;
            }
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
    if (last_block(&ctl->cnt[1], gridDim.x)) {
        const double s = sum_partials(part, gridDim.x);
        double rel = 0.0;
        if (decide_flag && rel0) {
            const double a = sum_partials(rel0, nrel);
            const double b = sum_partials(rel1, nrel);
            rel = a + b;
        }
        if (threadIdx.x == 0) {
            if (decide_flag) {
                decide(ctl, s, rel);
            } else {
                if (!isfinite(ctl->rhs2)) {
                    ctl->done = 3;
                } else if (ctl->rhs2 == 0.0) {
                    ctl->done = 1;
                    ctl->resid = 0.0;
                } else {
                    ctl->resid = sqrt(s) / sqrt(ctl->rhs2);
                    if (!isfinite(ctl->resid)) ctl->done = 3;
                }
            }
        }
    }
}

// ------------------------------------------------------------- check
// Residual of the iterate from the correction: r = r0 - A pd (float64).
__global__ __launch_bounds__(kBlock) void k_check(Geo g, const float* __restrict__ pd0,
                                                  const float* __restrict__ pd1,
                                                  const float* __restrict__ r00,
                                                  const float* __restrict__ r01,
                                                  double* __restrict__ part, const double* rel0,
                                                  const double* rel1, int nrel, Ctl* ctl) {
    if (ctl->done) return;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    int ii, j0, k0;
    double acc = 0.0;
    if (half_cell(g, t, ii, j0, k0)) {
        const long long e = g.col(ii, j0, k0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int s = (c + j0 + k0) & 1;
            const int i0 = 2 * ii + s;
            if (i0 < g.nx) {
                const float* pdo = c ? pd1 : pd0;
                const float* pdn = c ? pd0 : pd1;
                const float* r0 = c ? r01 : r00;
                const double d = (double)diag_of(g, i0, j0, k0);
                const double rt = (double)r0[e] - apply_A64(g, pdo, pdn, e, s, d);
                acc += rt * rt;
            }
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
    if (last_block(&ctl->cnt[2], gridDim.x)) {
        const double s = sum_partials(part, gridDim.x);
        double rel = 0.0;
        if (rel0) rel = sum_partials(rel0, nrel) + sum_partials(rel1, nrel);
        if (threadIdx.x == 0) decide(ctl, s, rel);
    }
}

// ------------------------------------------------- singular: p mean
__global__ __launch_bounds__(kBlock) void k_p_sum(Geo g, const float* __restrict__ ph0,
                                                  const float* __restrict__ ph1,
                                                  const float* __restrict__ pd0,
                                                  const float* __restrict__ pd1,
                                                  double* __restrict__ part, Ctl* ctl) {
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    int ii, j0, k0;
    double acc = 0.0;
    if (half_cell(g, t, ii, j0, k0)) {
        const long long e = g.col(ii, j0, k0);
        for (int c = 0; c < 2; ++c) {
            const int i0 = 2 * ii + ((c + j0 + k0) & 1);
            if (i0 < g.nx) acc += (double)(c ? ph1 : ph0)[e] + (double)(c ? pd1 : pd0)[e];
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
    if (last_block(&ctl->cnt[1], gridDim.x)) {
        const double s = sum_partials(part, gridDim.x);
        if (threadIdx.x == 0) ctl->rhs_sum = s;   // reused slot: sum of p
    }
}

__global__ __launch_bounds__(kBlock) void k_p_sub(Geo g, float* ph0, float* ph1, float* pd0,
                                                  float* pd1, const Ctl* ctl) {
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    int ii, j0, k0;
    if (!half_cell(g, t, ii, j0, k0)) return;
    const double mean = ctl->rhs_sum / ((double)g.nx * g.ny * g.nz);
    const long long e = g.col(ii, j0, k0);
    for (int c = 0; c < 2; ++c) {
        const int i0 = 2 * ii + ((c + j0 + k0) & 1);
        if (i0 < g.nx) {
            float* ph = c ? ph1 : ph0;
            float* pd = c ? pd1 : pd0;
            // subtract the mean from the (base + correction) pair, keeping
            // the correction's precision: the float32-rounded mean goes out
            // of the base, its rounding error out of the correction
            const float mh = (float)mean;
            const float ml = (float)(mean - (double)mh);
            ph[e] = ph[e] - mh;
            pd[e] = pd[e] - ml;
        }
    }
}

// Sum over the cells of a colour-array pair: mode 0 stores sum x^2 in
// ctl->rhs2, mode 1 stores sum x in ctl->rhs_sum.
__global__ __launch_bounds__(kBlock) void k_colour_norm(Geo g, const float* __restrict__ a0,
                                                        const float* __restrict__ a1,
                                                        double* __restrict__ part, Ctl* ctl,
                                                        int mode) {
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    int ii, j0, k0;
    double acc = 0.0;
    if (half_cell(g, t, ii, j0, k0)) {
        const long long e = g.col(ii, j0, k0);
        for (int c = 0; c < 2; ++c) {
            const int i0 = 2 * ii + ((c + j0 + k0) & 1);
            if (i0 < g.nx) {
                const double x = (double)(c ? a1 : a0)[e];
                acc += mode ? x : x * x;
            }
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
    if (last_block(&ctl->cnt[0], gridDim.x)) {
        const double s = sum_partials(part, gridDim.x);
        if (threadIdx.x == 0) {
            if (mode) ctl->rhs_sum = s;
            else ctl->rhs2 = s;
        }
    }
}

}  // namespace

int sor_blocks(const Geo& g) { return (int)nblk((long long)g.H * g.ny * g.nz); }

hipError_t launch_sor(const Geo& g, hipStream_t st, const PBufs& P, int colour, float omega,
                      int local_iter, double* rel_part, const Ctl* ctl) {
    hipLaunchKernelGGL(k_sor, dim3(sor_blocks(g)), dim3(kBlock), 0, st, g, colour, P.pd[colour],
                       P.pd[1 - colour], P.r0[colour], omega, local_iter, rel_part, ctl);
    return hipGetLastError();
}

hipError_t launch_fold(const Geo& g, hipStream_t st, const PBufs& P, const Ctl* ctl) {
    hipLaunchKernelGGL(k_fold, dim3(nblk(2 * g.ctot)), dim3(kBlock), 0, st, g.ctot, P.ph[0],
                       P.pd[0], P.ph[1], P.pd[1], ctl);
    return hipGetLastError();
}

hipError_t launch_rebase(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                         const double* rel0, const double* rel1, int nrel, Ctl* ctl, int decide) {
    hipLaunchKernelGGL(k_rebase, dim3(sor_blocks(g)), dim3(kBlock), 0, st, g, P.ph[0], P.ph[1],
                       P.pd[0], P.pd[1], P.rhs[0], P.rhs[1], P.r0[0], P.r0[1], part, rel0, rel1,
                       nrel, ctl, decide);
    return hipGetLastError();
}

hipError_t launch_colour_norm(const Geo& g, hipStream_t st, float* const a[2], double* part,
                              Ctl* ctl, int mode) {
    hipLaunchKernelGGL(k_colour_norm, dim3(sor_blocks(g)), dim3(kBlock), 0, st, g, a[0], a[1],
                       part, ctl, mode);
    return hipGetLastError();
}

hipError_t launch_check(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                        const double* rel0, const double* rel1, int nrel, Ctl* ctl) {
    hipLaunchKernelGGL(k_check, dim3(sor_blocks(g)), dim3(kBlock), 0, st, g, P.pd[0], P.pd[1],
                       P.r0[0], P.r0[1], part, rel0, rel1, nrel, ctl);
    return hipGetLastError();
}

hipError_t launch_remove_mean_p(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                                Ctl* ctl) {
    hipLaunchKernelGGL(k_p_sum, dim3(sor_blocks(g)), dim3(kBlock), 0, st, g, P.ph[0], P.ph[1],
                       P.pd[0], P.pd[1], part, ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_p_sub, dim3(sor_blocks(g)), dim3(kBlock), 0, st, g, P.ph[0], P.ph[1],
                       P.pd[0], P.pd[1], ctl);
    return hipGetLastError();
}

}  // namespace les
