// Single-instance launches of the red-black SOR machinery (section 2.6):
// half-sweeps in eight tile variants, fused red-black iterations in four,
// fold, rebase, residual check, p mean and the single-block finalize.
// Bodies in les_bodies.h.
#include "les_bodies.h"

namespace les {
namespace {

__device__ __forceinline__ unsigned lblock() { return xcd_block(blockIdx.x, gridDim.x); }

template <int TX, int KT, bool STR>
__global__ __launch_bounds__(kBlock) void k_sor(Geo g, int c, float* __restrict__ pself,
                                                const float* __restrict__ poth,
                                                const float* __restrict__ rself, float omega,
                                                int local_iter, double* __restrict__ rel_part,
                                                const Ctl* __restrict__ ctl) {
    bool acc;
    if (!sweep_active(ctl, local_iter, acc)) return;
    sor_body<TX, KT, STR>(g, c, pself, poth, rself, omega, acc && rel_part != nullptr, rel_part,
                          lblock());
}

template <int TX, int NW, int KT, bool STR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(8))) void k_sor_rb(Geo g, const float* __restrict__ a0,
                                                    const float* __restrict__ a1,
                                                    const float* __restrict__ r0c,
                                                    const float* __restrict__ r1c,
                                                    float* __restrict__ b0, float* __restrict__ b1,
                                                    float omega, int local_iter,
                                                    double* __restrict__ rel0,
                                                    double* __restrict__ rel1,
                                                    const Ctl* __restrict__ ctl, int kt) {
    bool acc;
    const bool active = sweep_active(ctl, local_iter, acc);
    if (!active && ctl->done) return;
    if constexpr (!STR) {
        if (!active)
            sor_rb_copy_u<TX, NW, KT>(g, a0, a1, b0, b1, lblock(), kt);
        else if (acc && rel0 != nullptr)
            sor_rb_body_u<TX, NW, KT, true>(g, a0, a1, r0c, r1c, b0, b1, omega, rel0, rel1, lblock(), kt);
        else
            sor_rb_body_u<TX, NW, KT, false>(g, a0, a1, r0c, r1c, b0, b1, omega, rel0, rel1, lblock(), kt);
    } else {
        sor_rb_body<TX, NW, KT, STR>(g, a0, a1, r0c, r1c, b0, b1, omega,
                                     active && acc && rel0 != nullptr, !active, rel0, rel1, lblock(), kt);
    }
}

// Uniform grids too large for the lean form's 32-bit buffer offsets.
template <int TX, int NW, int KT>
__global__ __launch_bounds__(64 * NW) void k_sor_rb_wide(Geo g, const float* __restrict__ a0,
                                                         const float* __restrict__ a1,
                                                         const float* __restrict__ r0c,
                                                         const float* __restrict__ r1c,
                                                         float* __restrict__ b0, float* __restrict__ b1,
                                                         float omega, int local_iter,
                                                         double* __restrict__ rel0,
                                                         double* __restrict__ rel1,
                                                         const Ctl* __restrict__ ctl, int kt) {
    bool acc;
    const bool active = sweep_active(ctl, local_iter, acc);
    if (!active && ctl->done) return;
    sor_rb_body<TX, NW, KT, false>(g, a0, a1, r0c, r1c, b0, b1, omega, active && acc && rel0 != nullptr,
                                   !active, rel0, rel1, lblock(), kt);
}

template <bool STR>
__global__ __launch_bounds__(1024) void k_sor_rb2(Geo g, const float* __restrict__ a0,
                                                 const float* __restrict__ a1,
                                                 const float* __restrict__ r0c,
                                                 const float* __restrict__ r1c,
                                                 float* __restrict__ b0, float* __restrict__ b1,
                                                 float omega, int local_iter,
                                                 double* __restrict__ rel0,
                                                 double* __restrict__ rel1,
                                                 const Ctl* __restrict__ ctl, int kt) {
    bool acc1, acc2;
    const bool act1 = sweep_active(ctl, local_iter, acc1);
    const bool act2 = sweep_active(ctl, local_iter + 1, acc2);
    if (!act1 && ctl->done) return;
    const bool part = rel0 != nullptr;
    const bool p1 = part && act1 && acc1 && !act2, p2 = part && act1 && act2 && acc2;
    if constexpr (!STR) {
        __shared__ Rb2Smem sm;
        if (!act1)
            sor_rb2_copy_u(g, a0, a1, b0, b1, lblock(), kt);
        else if (p1 || p2)
            sor_rb2_body_u<true>(sm, g, a0, a1, r0c, r1c, b0, b1, omega, act2, p1, p2, rel0, rel1, lblock(), kt);
        else
            sor_rb2_body_u<false>(sm, g, a0, a1, r0c, r1c, b0, b1, omega, act2, false, false, rel0, rel1,
                                  lblock(), kt);
    } else {
        sor_rb2_body<STR>(g, a0, a1, r0c, r1c, b0, b1, omega, act1, act1 && act2, p1, p2, rel0, rel1, lblock(),
                          kt);
    }
}

// Uniform grids too large for the lean form's 32-bit buffer offsets.
__global__ __launch_bounds__(1024) void k_sor_rb2_wide(Geo g, const float* __restrict__ a0,
                                                      const float* __restrict__ a1,
                                                      const float* __restrict__ r0c,
                                                      const float* __restrict__ r1c,
                                                      float* __restrict__ b0, float* __restrict__ b1,
                                                      float omega, int local_iter,
                                                      double* __restrict__ rel0,
                                                      double* __restrict__ rel1,
                                                      const Ctl* __restrict__ ctl, int kt) {
    bool acc1, acc2;
    const bool act1 = sweep_active(ctl, local_iter, acc1);
    const bool act2 = sweep_active(ctl, local_iter + 1, acc2);
    if (!act1 && ctl->done) return;
    const bool part = rel0 != nullptr;
    sor_rb2_body<false>(g, a0, a1, r0c, r1c, b0, b1, omega, act1, act1 && act2, part && act1 && acc1 && !act2,
                        part && act1 && act2 && acc2, rel0, rel1, lblock(), kt);
}

__global__ __launch_bounds__(kBlock) void k_fold(long long n, float* __restrict__ ph0,
                                                 float* __restrict__ pd0, float* __restrict__ ph1,
                                                 float* __restrict__ pd1, const Ctl* ctl) {
    if (ctl->done) return;
    fold_body(n, ph0, pd0, ph1, pd1, (long long)blockIdx.x * kBlock + threadIdx.x);
}

template <bool STR>
__global__ __launch_bounds__(kBlock) void k_rebase(Geo g, PBufs P, double* __restrict__ part,
                                                   const Ctl* ctl) {
    if (ctl->done) return;
    rebase_body<STR>(g, P, part, lblock(), gridDim.x);
}

template <bool STR>
__global__ __launch_bounds__(kBlock) void k_check(Geo g, PBufs P, double* __restrict__ part,
                                                  const Ctl* ctl) {
    if (ctl->done || ctl->skip) return;
    check_body<STR>(g, P, part, lblock(), gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_colour_sum(Geo g, const float* a0, const float* a1,
                                                       const float* b0, const float* b1, int mode,
                                                       double* __restrict__ part) {
    colour_sum_body(g, a0, a1, b0, b1, mode, part, lblock(), gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_p_sub(Geo g, PBufs P, const Ctl* ctl) {
    p_sub_body(g, P, ctl, blockIdx.x);
}

__global__ __launch_bounds__(kFinBlock) void k_finalize(int op, const double* __restrict__ part,
                                                        int n, const double* __restrict__ rel0,
                                                        const double* __restrict__ rel1, int nrel,
                                                        Ctl* ctl, double omega) {
    finalize_body<kFinBlock>(op, part, n, rel0, rel1, nrel, ctl, omega);
}

inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// Sweep variants, chosen per grid: half-sweeps (row width TX, planes per
// block KT) and fused iterations (TX, KT, NW wavefronts per block).
const SorVariant kSorVariants[kNumSorVariants] = {
    {64, 1, 0}, {32, 1, 0}, {64, 2, 0}, {32, 2, 0}, {64, 4, 0}, {32, 4, 0}, {64, 8, 0}, {32, 8, 0},
    {32, 12, 16}, {64, 16, 16}, {32, 0, 16}, {64, 0, 16},
    // two iterations per launch (64 lanes x 32 rows, 16 wavefronts); kt
    // planes chosen per grid for one (12) or two (13) resident blocks per CU
    {64, 1, 16}, {64, 2, 16}};

int sor_default_variant(const Geo& g) {
    const int w64 = ((g.H + 63) / 64) * 64 - g.H;
    const int w32 = ((g.H + 31) / 32) * 32 - g.H;
    return (w32 < w64) ? 1 : 0;   // one cell per thread, the row width that wastes fewer lanes
}

unsigned sor_sweep_blocks(const Geo& g, int variant) {
    const int tx = kSorVariants[variant].tx, kt = kSorVariants[variant].kt;
    if (sor_fused2(variant)) {
        const int k = rb2_kt(g, kt);
        return (unsigned)((g.H + kRb2TXO - 1) / kRb2TXO) * (unsigned)((g.ny + kRb2TYO - 1) / kRb2TYO) *
               (unsigned)((g.nz + k - 1) / k);
    }
    if (sor_fused(variant)) {
        const int nw = kSorVariants[variant].nw;
        const int txo = tx - 2, tyo = (64 / tx) * nw - 2, k = fused_kt(g, tx, nw, kt);
        return (unsigned)((g.H + txo - 1) / txo) * (unsigned)((g.ny + tyo - 1) / tyo) *
               (unsigned)((g.nz + k - 1) / k);
    }
    const int ty = (64 / tx) * (kBlock / 64);
    return (unsigned)((g.H + tx - 1) / tx) * (unsigned)((g.ny + ty - 1) / ty) *
           (unsigned)((g.nz + kt - 1) / kt);
}

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
#define LES_SOR_CASE(V, TX, KT)                                                                  \
    case V:                                                                                     \
        if (g.stretched)                                                                        \
            hipLaunchKernelGGL((k_sor<TX, KT, true>), grid, block, 0, st, g, colour, ps, po, rs,  \
                               omega, local_iter, rel_part, ctl);                               \
        else                                                                                    \
            hipLaunchKernelGGL((k_sor<TX, KT, false>), grid, block, 0, st, g, colour, ps, po, rs, \
                               omega, local_iter, rel_part, ctl);                               \
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

hipError_t launch_sor_rb(const Geo& g, hipStream_t st, const PBufs& P, int parity, float omega,
                         int local_iter, double* rel0, double* rel1, const Ctl* ctl, int variant) {
    const dim3 grid(sor_sweep_blocks(g, variant));
    const float* a0 = parity ? P.pa[0] : P.pd[0];
    const float* a1 = parity ? P.pa[1] : P.pd[1];
    float* b0 = parity ? P.pd[0] : P.pa[0];
    float* b1 = parity ? P.pd[1] : P.pa[1];
    const SorVariant& sv = kSorVariants[variant];
    const int kt = fused_kt(g, sv.tx, sv.nw, sv.kt);
#define LES_RB_CASE(V, TX, NW, KT)                                                                   \
    case V:                                                                                         \
        if (g.stretched)                                                                            \
            hipLaunchKernelGGL((k_sor_rb<TX, NW, KT, true>), grid, dim3(64 * NW), 0, st, g, a0, a1,   \
                               P.r0[0], P.r0[1], b0, b1, omega, local_iter, rel0, rel1, ctl, kt);   \
        else if (rb_lean_fits(g))                                                                   \
            hipLaunchKernelGGL((k_sor_rb<TX, NW, KT, false>), grid, dim3(64 * NW), 0, st, g, a0, a1,  \
                               P.r0[0], P.r0[1], b0, b1, omega, local_iter, rel0, rel1, ctl, kt);   \
        else                                                                                        \
            hipLaunchKernelGGL((k_sor_rb_wide<TX, NW, KT>), grid, dim3(64 * NW), 0, st, g, a0, a1,    \
                               P.r0[0], P.r0[1], b0, b1, omega, local_iter, rel0, rel1, ctl, kt);   \
        break;
    switch (variant) {
        LES_RB_CASE(8, 32, 16, 12)
        LES_RB_CASE(9, 64, 16, 16)
        LES_RB_CASE(10, 32, 16, 0)
        LES_RB_CASE(11, 64, 16, 0)
        default: return hipErrorInvalidValue;
    }
#undef LES_RB_CASE
    return hipGetLastError();
}

hipError_t launch_sor_rb2(const Geo& g, hipStream_t st, const PBufs& P, int parity, float omega,
                          int local_iter, double* rel0, double* rel1, const Ctl* ctl, int variant) {
    if (!sor_fused2(variant)) return hipErrorInvalidValue;
    const dim3 grid(sor_sweep_blocks(g, variant));
    const float* a0 = parity ? P.pa[0] : P.pd[0];
    const float* a1 = parity ? P.pa[1] : P.pd[1];
    float* b0 = parity ? P.pd[0] : P.pa[0];
    float* b1 = parity ? P.pd[1] : P.pa[1];
    const int kt = rb2_kt(g, kSorVariants[variant].kt);
    if (g.stretched)
        hipLaunchKernelGGL(k_sor_rb2<true>, grid, dim3(1024), 0, st, g, a0, a1, P.r0[0], P.r0[1], b0, b1,
                           omega, local_iter, rel0, rel1, ctl, kt);
    else if (rb_lean_fits(g))
        hipLaunchKernelGGL(k_sor_rb2<false>, grid, dim3(1024), 0, st, g, a0, a1, P.r0[0], P.r0[1], b0, b1,
                           omega, local_iter, rel0, rel1, ctl, kt);
    else
        hipLaunchKernelGGL(k_sor_rb2_wide, grid, dim3(1024), 0, st, g, a0, a1, P.r0[0], P.r0[1], b0, b1,
                           omega, local_iter, rel0, rel1, ctl, kt);
    return hipGetLastError();
}

hipError_t launch_fold(const Geo& g, hipStream_t st, const PBufs& P, const Ctl* ctl) {
    hipLaunchKernelGGL(k_fold, dim3(nblk(2 * g.ctot)), dim3(kBlock), 0, st, g.ctot, P.ph[0],
                       P.pd[0], P.ph[1], P.pd[1], ctl);
    return hipGetLastError();
}

hipError_t launch_rebase(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                         const double* rel0, const double* rel1, int nrel, Ctl* ctl, int decide) {
    if (g.stretched)
        hipLaunchKernelGGL(k_rebase<true>, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, P, part,
                           (const Ctl*)ctl);
    else
        hipLaunchKernelGGL(k_rebase<false>, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, P, part,
                           (const Ctl*)ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, decide ? FIN_CHECK_FULL : FIN_SETUP, part, (int)red_blocks(g), rel0,
                           rel1, nrel, ctl);
}

hipError_t launch_colour_norm(const Geo& g, hipStream_t st, float* const a[2], double* part,
                              Ctl* ctl, int mode) {
    hipLaunchKernelGGL(k_colour_sum, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, a[0], a[1],
                       (const float*)nullptr, (const float*)nullptr, mode, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, mode ? FIN_RHS_SUM : FIN_RHS2, part, (int)red_blocks(g), nullptr,
                           nullptr, 0, ctl);
}

hipError_t launch_check(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                        const double* rel0, const double* rel1, int nrel, Ctl* ctl) {
    if (g.stretched)
        hipLaunchKernelGGL(k_check<true>, dim3(check_blocks(g)), dim3(kBlock), 0, st, g, P, part,
                           (const Ctl*)ctl);
    else
        hipLaunchKernelGGL(k_check<false>, dim3(check_blocks(g)), dim3(kBlock), 0, st, g, P, part,
                           (const Ctl*)ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, FIN_CHECK, part, (int)check_blocks(g), rel0, rel1, nrel, ctl);
}

hipError_t launch_remove_mean_p(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                                Ctl* ctl) {
    hipLaunchKernelGGL(k_colour_sum, dim3(red_blocks(g)), dim3(kBlock), 0, st, g, P.ph[0],
                       P.ph[1], P.pd[0], P.pd[1], 1, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_finalize(st, FIN_PSUM, part, (int)red_blocks(g), nullptr, nullptr, 0, ctl);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_p_sub, dim3(nblk((long long)g.H * g.ny * g.nz)), dim3(kBlock), 0, st, g,
                       P, (const Ctl*)ctl);
    return hipGetLastError();
}

}  // namespace les
