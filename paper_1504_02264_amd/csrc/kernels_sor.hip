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
#include <algorithm>

#include "device_util.h"
#include "les_impl.h"

namespace les {
namespace {

inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Reductions over the H * ny * nz half-cells use at most kRedBlocks blocks;
// block L owns one contiguous chunk of half-cells, walked by its threads
// with unit stride, so the finalize kernel sums few partials.
constexpr unsigned kRedBlocks = 2048;
inline unsigned red_blocks(const Geo& g) {
    const long long n = (long long)g.H * g.ny * g.nz;
    return (unsigned)std::min<long long>(kRedBlocks, (n + kBlock - 1) / kBlock);
}
__device__ __forceinline__ void red_chunk(const Geo& g, unsigned lb, unsigned nb, long long& t0,
                                          long long& t1) {
    const long long n = (long long)g.H * g.ny * g.nz;
    const long long chunk = ((n + nb - 1) / nb + kBlock - 1) / kBlock * kBlock;
    t0 = (long long)lb * chunk;
    t1 = (t0 + chunk < n) ? t0 + chunk : n;
}

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
    const unsigned hy = (unsigned)g.H * (unsigned)g.ny;   // H ny nz < 2^31
    if (t >= (long long)hy * g.nz) return false;
    const unsigned tt = (unsigned)t;
    const unsigned kk = tt / hy;
    const unsigned r = tt - kk * hy;
    const unsigned jj = r / (unsigned)g.H;
    ii = (int)(r - jj * (unsigned)g.H);
    j0 = (int)jj;
    k0 = (int)kk;
    return true;
}

// ---------------------------------------------------------- half-sweep
// Colour c: for every cell of colour c,
//   reltmp = omega (cn1 (sum_nb cn_nb p_nb - rhs) - p);  p += reltmp
// with cn1 = 1/diag.  Outside the domain the other colour's array holds
// zeros, so the neighbour sum needs no boundary branches.  Skipped when the
// solve is done or max_iter is reached; on the last iteration of a check
// interval it also leaves one float64 partial of sum reltmp^2 per block.
//
// Tiling: a block is 4 wavefronts; a wavefront covers TX consecutive
// half-cells of 64/TX rows, and the block marches up KT planes (KT = 1:
// one cell per thread, the most memory-level parallelism).  The
// other colour's values at (ii, j0) are kept in registers across k (the
// top neighbour of plane k is the in-row value of plane k+1 and the bottom
// one of plane k+2), east/west neighbours come from the adjacent lanes by
// cross-lane shuffles, north/south ones from the cache.  Within a row the
// cell parity is uniform, so the wave needs no divergent branch.
template <int TX, int KT>
__global__ __launch_bounds__(kBlock) void k_sor(Geo g, int c, float* __restrict__ pself,
                                                const float* __restrict__ poth,
                                                const float* __restrict__ rself, float omega,
                                                int local_iter, double* __restrict__ rel_part,
                                                const Ctl* __restrict__ ctl) {
    const int done = ctl->done, m = ctl->m, K = ctl->K, mx = ctl->max_iter;
    if (done || m + local_iter >= mx) return;
    const bool acc = (rel_part != nullptr) && (m + local_iter + 1 == min(m + K, mx));
    constexpr int RPW = 64 / TX;            // rows per wavefront
    constexpr int TY = RPW * (kBlock / 64); // rows per block
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned nbx = (unsigned)(g.H + TX - 1) / TX;
    const unsigned nby = (unsigned)(g.ny + TY - 1) / TY;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int tx = lane % TX;
    const int ii = (int)bx * TX + tx;
    const int j0 = (int)by * TY + (threadIdx.x >> 6) * RPW + lane / TX;
    const int k_begin = (int)bk * KT;
    const int k_end = min(g.nz, k_begin + KT);
    const bool col_ok = ii < g.H && j0 < g.ny;
    const float cx = g.cx, cy = g.cy, cz = g.cz;
    // diagonal parts that do not depend on k
    const float dyy = (j0 > 0 ? cy : 0.f) + (j0 < g.ny - 1 ? cy : 0.f);
    long long e = col_ok ? g.col(ii, j0, k_begin) : 0;
    float pb = col_ok ? poth[e - g.SP] : 0.f;
    float pc = col_ok ? poth[e] : 0.f;
    double r2 = 0.0, dr2 = 0.0;
    for (int k0 = k_begin; k0 < k_end; ++k0) {
        const float pt = col_ok ? poth[e + g.SP] : 0.f;
        // neighbours along the row from the adjacent lanes
        float pe = __shfl_down(pc, 1, TX);
        float pw = __shfl_up(pc, 1, TX);
        if (tx == TX - 1 && col_ok) pe = poth[e + 1];
        if (tx == 0 && col_ok) pw = poth[e - 1];
        const int s = (c + j0 + k0) & 1;
        const int i0 = 2 * ii + s;
        if (col_ok && i0 < g.nx) {
            // cell i0 = 2 ii + s: west neighbour at half-index ii - 1 + s,
            // east at ii + s
            const float west = s ? pc : pw;
            const float east = s ? pe : pc;
            const float ps = poth[e - g.S], pn = poth[e + g.S];
            const float nb = cx * (west + east) + cy * (ps + pn) + cz * (pb + pt);
            const float dxx = (i0 > 0 ? cx : 0.f) + (i0 < g.nx - 1 ? cx : (g.outflow ? 2.f * cx : 0.f));
            const float dzz = (k0 > 0 ? cz : 0.f) + (k0 < g.nz - 1 ? cz : 0.f);
            const float diag = dxx + dyy + dzz;
            const float inv = 1.0f / diag;
            const float p = pself[e];
            const float reltmp = omega * (inv * (nb - rself[e]) - p);
            pself[e] = p + reltmp;
            if (acc) {
                const double rt = (double)reltmp;
                r2 += rt * rt;
                dr2 += ((double)diag * rt) * ((double)diag * rt);
            }
        }
        pb = pc;
        pc = pt;
        e += g.SP;
    }
    if (acc) {
        // [sum reltmp^2, sum (diag reltmp)^2] per block; after the colour-1
        // half-sweep, diag (omega-1)/omega reltmp is exactly the residual of
        // the colour-1 cells, so the second sum bounds ||r|| from below
        const double bs = block_sum(r2);
        const double bd = block_sum(dr2);
        if (threadIdx.x == 0) {
            rel_part[2 * lb] = bs;
            rel_part[2 * lb + 1] = bd;
        }
    }
}

}  // namespace

// Sweep variants (row width TX, planes per block KT), chosen per grid.
const SorVariant kSorVariants[kNumSorVariants] = {
    {64, 1}, {32, 1}, {64, 2}, {32, 2}, {64, 4}, {32, 4}, {64, 8}, {32, 8}};

int sor_default_variant(const Geo& g) {
    const int w64 = ((g.H + 63) / 64) * 64 - g.H;
    const int w32 = ((g.H + 31) / 32) * 32 - g.H;
    return (w32 < w64) ? 1 : 0;   // one cell per thread, the row width that wastes fewer lanes
}

unsigned sor_sweep_blocks(const Geo& g, int variant) {
    const int tx = kSorVariants[variant].tx, kt = kSorVariants[variant].kt;
    const int ty = (64 / tx) * (kBlock / 64);
    return (unsigned)((g.H + tx - 1) / tx) * (unsigned)((g.ny + ty - 1) / ty) *
           (unsigned)((g.nz + kt - 1) / kt);
}

namespace {

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
__device__ void decide(Ctl* ctl, double sum_r2) {
    if (ctl->done) return;
    const int m = min(ctl->m + ctl->K, ctl->max_iter);
    ctl->m = m;
    ctl->skip = 0;
    const double R = sqrt(sum_r2) / sqrt(ctl->rhs2);
    ctl->resid = R;
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
                                                   double* __restrict__ part, const Ctl* ctl) {
    if (ctl->done) return;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    long long t0, t1;
    red_chunk(g, lb, gridDim.x, t0, t1);
    double acc = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
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
}

// ------------------------------------------------------------- check
// Residual of the iterate from the correction: r = r0 - A pd (float64).
__global__ __launch_bounds__(kBlock) void k_check(Geo g, const float* __restrict__ pd0,
                                                  const float* __restrict__ pd1,
                                                  const float* __restrict__ r00,
                                                  const float* __restrict__ r01,
                                                  double* __restrict__ part, const Ctl* ctl) {
    if (ctl->done || ctl->skip) return;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    long long t0, t1;
    red_chunk(g, lb, gridDim.x, t0, t1);
    double acc = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
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
}

// ------------------------------------------------- singular: p mean
__global__ __launch_bounds__(kBlock) void k_p_sum(Geo g, const float* __restrict__ ph0,
                                                  const float* __restrict__ ph1,
                                                  const float* __restrict__ pd0,
                                                  const float* __restrict__ pd1,
                                                  double* __restrict__ part) {
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    long long t0, t1;
    red_chunk(g, lb, gridDim.x, t0, t1);
    double acc = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
        const long long e = g.col(ii, j0, k0);
        for (int c = 0; c < 2; ++c) {
            const int i0 = 2 * ii + ((c + j0 + k0) & 1);
            if (i0 < g.nx) acc += (double)(c ? ph1 : ph0)[e] + (double)(c ? pd1 : pd0)[e];
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
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
                                                        double* __restrict__ part, int mode) {
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    long long t0, t1;
    red_chunk(g, lb, gridDim.x, t0, t1);
    double acc = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
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
}

// One block of kFinBlock threads: fixed-order sums of the partials of the
// preceding reduction kernel, then the bookkeeping of op.
//   FIN_BOUND  after the sweeps of a check interval: sum reltmp^2 for the
//              report, and the colour-1 residual lower bound
//              |omega-1|/omega sqrt(sum (diag reltmp)^2) <= ||r||; if it
//              exceeds 1.5 tol the coming check cannot succeed and is
//              skipped (never the last check before max_iter)
//   FIN_CHECK  decide on the residual (or just count a skipped check)
//   FIN_CHECK_FULL  decide on the residual (rebase checks never skip)
__global__ __launch_bounds__(kFinBlock) void k_finalize(int op, const double* __restrict__ part,
                                                        int n, const double* __restrict__ rel0,
                                                        const double* __restrict__ rel1, int nrel,
                                                        Ctl* ctl, double omega) {
    const bool sor_op = op == FIN_CHECK || op == FIN_CHECK_FULL || op == FIN_SETUP || op == FIN_BOUND;
    if (sor_op && ctl->done) return;
    if (op == FIN_DIAG) {
        const double a = sum_partials(part, n, 2);
        const double b = max_partials(part + 1, n, 2);
        if (threadIdx.x == 0) {
            ctl->div2 = a;
            ctl->cfl = b;
        }
        return;
    }
    if (op == FIN_BOUND) {
        const double r0s = sum_partials(rel0, nrel, 2);
        const double r1s = sum_partials(rel1, nrel, 2);
        const double d1s = sum_partials(rel1 + 1, nrel, 2);
        if (threadIdx.x == 0) {
            ctl->reltmp2 = r0s + r1s;
            const double lb = fabs(omega - 1.0) / omega * sqrt(d1s) / sqrt(ctl->rhs2);
            const int m_next = min(ctl->m + ctl->K, ctl->max_iter);
            ctl->skip = (m_next < ctl->max_iter && lb > 1.5 * ctl->tol) ? 1 : 0;
        }
        return;
    }
    if (op == FIN_CHECK && ctl->skip) {
        if (threadIdx.x == 0) {
            ctl->m = min(ctl->m + ctl->K, ctl->max_iter);
            ctl->skip = 0;
        }
        return;
    }
    const double s = sum_partials(part, n);
    if (threadIdx.x != 0) return;
    switch (op) {
        case FIN_RHS2: ctl->rhs2 = s; break;
        case FIN_RHS_SUM: ctl->rhs_sum = s; break;
        case FIN_PSUM: ctl->rhs_sum = s; break;   // reused slot: sum of p
        case FIN_SETUP:
            if (!isfinite(ctl->rhs2)) {
                ctl->done = 3;
            } else if (ctl->rhs2 == 0.0) {
                ctl->done = 1;
                ctl->resid = 0.0;
            } else {
                ctl->resid = sqrt(s) / sqrt(ctl->rhs2);
                if (!isfinite(ctl->resid)) ctl->done = 3;
            }
            break;
        case FIN_CHECK:
        case FIN_CHECK_FULL: decide(ctl, s); break;
        default: break;
    }
}

}  // namespace

hipError_t launch_finalize(hipStream_t st, int op, const double* part, int n, const double* rel0,
                           const double* rel1, int nrel, Ctl* ctl, double omega) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, st, op, part, n, rel0, rel1,
                       nrel, ctl, omega);
    return hipGetLastError();
}

hipError_t launch_sor(const Geo& g, hipStream_t st, const PBufs& P, int colour, float omega,
                      int local_iter, double* rel_part, const Ctl* ctl, int variant) {
    const dim3 grid(sor_sweep_blocks(g, variant)), block(kBlock);
    float* ps = P.pd[colour];
    const float* po = P.pd[1 - colour];
    const float* rs = P.r0[colour];
#define LES_SOR_CASE(V, TX, KT)                                                                 \
    case V:                                                                                    \
        hipLaunchKernelGGL((k_sor<TX, KT>), grid, block, 0, st, g, colour, ps, po, rs, omega, \
                           local_iter, rel_part, ctl);                                         \
        break;
    switch (variant) {
        LES_SOR_CASE(0, 64, 1)
        LES_SOR_CASE(1, 32, 1)
        LES_SOR_CASE(2, 64, 2)
        LES_SOR_CASE(3, 32, 2)
        LES_SOR_CASE(4, 64, 4)
        LES_SOR_CASE(5, 32, 4)
        LES_SOR_CASE(6, 64, 8)
        LES_SOR_CASE(7, 32, 8)
        default: return hipErrorInvalidValue;
    }
#undef LES_SOR_CASE
    return hipGetLastError();
}

hipError_t launch_fold(const Geo& g, hipStream_t st, const PBufs& P, const Ctl* ctl) {
    hipLaunchKernelGGL(k_fold, dim3(nblk(2 * g.ctot)), dim3(kBlock), 0, st, g.ctot, P.ph[0],
                       P.pd[0], P.ph[1], P.pd[1], ctl);
    return hipGetLastError();
}

hipError_t launch_rebase(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                         const double* rel0, const double* rel1, int nrel, Ctl* ctl, int decide) {
    hipLaunchKernelGGL(k_rebase, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, P.ph[0], P.ph[1],
                       P.pd[0], P.pd[1], P.rhs[0], P.rhs[1], P.r0[0], P.r0[1], part,
                       (const Ctl*)ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, decide ? FIN_CHECK_FULL : FIN_SETUP, part, (int)red_blocks(g), rel0,
                           rel1, nrel, ctl);
}

hipError_t launch_colour_norm(const Geo& g, hipStream_t st, float* const a[2], double* part,
                              Ctl* ctl, int mode) {
    hipLaunchKernelGGL(k_colour_norm, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, a[0], a[1],
                       part, mode);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, mode ? FIN_RHS_SUM : FIN_RHS2, part, (int)red_blocks(g), nullptr,
                           nullptr, 0, ctl);
}

hipError_t launch_check(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                        const double* rel0, const double* rel1, int nrel, Ctl* ctl) {
    hipLaunchKernelGGL(k_check, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, P.pd[0], P.pd[1],
                       P.r0[0], P.r0[1], part, (const Ctl*)ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, FIN_CHECK, part, (int)red_blocks(g), rel0, rel1, nrel, ctl);
}

hipError_t launch_remove_mean_p(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                                Ctl* ctl) {
    hipLaunchKernelGGL(k_p_sum, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, P.ph[0], P.ph[1],
                       P.pd[0], P.pd[1], part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_finalize(st, FIN_PSUM, part, (int)red_blocks(g), nullptr, nullptr, 0, ctl);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_p_sub, dim3(nblk((long long)g.H * g.ny * g.nz)), dim3(kBlock), 0, st, g, P.ph[0], P.ph[1],
                       P.pd[0], P.pd[1], ctl);
    return hipGetLastError();
}

}  // namespace les
