// Batched ensemble: several LES instances of uneven grids advanced together.
//
// Per step, every stage is ONE launch over an (instance, block) work list
// (XCD-aware numbering, then a lookup of the owning instance), and the
// whole pressure solve of all instances is ONE persistent cooperative
// launch: its blocks walk the sweep work list of all unfinished instances,
// meet at grid barriers between half-sweeps, evaluate each instance's
// stopping test on the device and leave instances as they converge.  The
// per-step stage sequences before and after the solve are captured once in
// HIP graphs and replayed (two pairs, for the two velocity-buffer parities).
// The per-cell arithmetic is the single-instance one (les_bodies.h), so an
// ensemble step is bitwise identical to stepping each member alone.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "les_bodies.h"

namespace cg = cooperative_groups;

namespace les {

// Device descriptor of one member.
struct EnsInst {
    Geo g;
    float* u[2];
    float* v[2];
    float* w[2];
    float* nut;
    float* fu; float* fv; float* fw;
    float* su; float* sv; float* sw;
    uint8_t* flags;
    float* prof;
    float* prof1;       // second inflow sample (prof itself without a pair)
    double t0, t1, dt;  // times of the samples, time step
    int interp;         // inflow interpolated between prof and prof1
    PBufs P;
    double* part;       // rhs / check / rebase partials
    double* rel0;       // sweep partials, colour 0 and 1
    double* rel1;
    Ctl* ctl;
    float c2, nu, alpha, beta, omega, amp;
    uint64_t seed;
    double tol;
    int max_iter, K, R, variant, singular, inflow;
    unsigned nsweep, nred;
    int kt_tile;        // planes per block of the fused tendency pass
    int kt_rb2;         // planes per block of a two-iteration sweep launch
};

// Per-member state that changes from step to step (device memory).
struct EnsDyn {
    int cur;            // index of u^n
    int first;          // next step is the first (forward Euler)
    long long step;     // completed steps
    int last_iters;
    int done;
    double resid;
    double reltmp2;
    double rhs2;
};

// Offsets of each member's blocks in a stage's work list.
struct EnsOffsets {
    unsigned tile[kMaxEnsemble + 1];
    unsigned cell[kMaxEnsemble + 1];
    unsigned half[kMaxEnsemble + 1];
    unsigned red[kMaxEnsemble + 1];
    unsigned bc[kMaxEnsemble + 1];
    unsigned inflow[kMaxEnsemble + 1];
    unsigned sweep[kMaxEnsemble + 1];
    unsigned fold[kMaxEnsemble + 1];
};

namespace {

// Control-block fields that steer the persistent solve are written by one
// block and read by all after a grid barrier: read them coherently.
__device__ __forceinline__ int ld(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool member_active(const Ctl* c, int it, bool& acc) {
    const int done = ld(&c->done), m = ld(&c->m), K = ld(&c->K), mx = ld(&c->max_iter);
    acc = (m + it + 1 == min(m + K, mx));
    return !(done || m + it >= mx);
}

__device__ __forceinline__ int owner(const unsigned* off, int n, unsigned L) {
    int lo = 0, hi = n - 1;   // largest q with off[q] <= L
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= L) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------- batched stages
__global__ __launch_bounds__(kTileThreads) void k_ens_step_tile(const EnsInst* I, const EnsDyn* D,
                                                              int n, const EnsOffsets* O) {
    __shared__ TileShared sh;
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = owner(O->tile, n, L);
    const EnsInst& d = I[q];
    const int a = D[q].cur, b = 1 - a;
    TendArgs A{d.u[a], d.v[a], d.w[a], d.nut, d.fu, d.fv, d.fw, d.su, d.sv, d.sw, d.flags,
               d.u[b], d.v[b], d.w[b], d.nu, d.alpha, d.beta, D[q].first};
    step_tile_body(d.g, A, d.nut, d.c2, d.kt_tile, L - O->tile[q], sh);
}

__global__ __launch_bounds__(kBlock) void k_ens_inflow(const EnsInst* I, const EnsDyn* D, int n,
                                                       const EnsOffsets* O) {
    const unsigned L = blockIdx.x;
    const int q = owner(O->inflow, n, L);
    const EnsInst& d = I[q];
    if (!d.inflow) return;
    const float wt = d.interp ? inflow_weight_at(D[q].step, d.dt, d.t0, d.t1) : 0.f;
    inflow_body(d.g, d.u[1 - D[q].cur], d.prof, d.prof1, wt, d.flags, d.amp, d.seed, D[q].step + 1,
                L - O->inflow[q]);
}

__global__ __launch_bounds__(kBlock) void k_ens_rhs(const EnsInst* I, const EnsDyn* D, int n,
                                                    const EnsOffsets* O) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = owner(O->cell, n, L);
    const EnsInst& d = I[q];
    const int b = 1 - D[q].cur;
    rhs_body(d.g, d.u[b], d.v[b], d.w[b], d.P.rhs[0], d.P.rhs[1], d.part, d.singular,
             L - O->cell[q]);
}

__global__ __launch_bounds__(kBlock) void k_ens_rhs_mean(const EnsInst* I, int n,
                                                         const EnsOffsets* O) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = owner(O->cell, n, L);
    const EnsInst& d = I[q];
    if (!d.singular) return;
    rhs_mean_body(d.g, d.P.rhs[0], d.P.rhs[1], d.part, d.ctl, L - O->cell[q]);
}

// One block per member: initialise the control block, then (op) finalize.
__global__ __launch_bounds__(kBlock) void k_ens_ctl_init(const EnsInst* I) {
    const EnsInst& d = I[blockIdx.x];
    ctl_init_body(d.ctl, d.tol, d.max_iter, d.K);
}

// After k_ens_rhs: rhs2 (or the rhs sum of a singular member).
__global__ __launch_bounds__(kBlock) void k_ens_fin_rhs(const EnsInst* I, const EnsOffsets* O) {
    const int q = blockIdx.x;
    const EnsInst& d = I[q];
    finalize_body<kBlock>(d.singular ? FIN_RHS_SUM : FIN_RHS2, d.part, (int)(O->cell[q + 1] - O->cell[q]),
                          nullptr, nullptr, 0, d.ctl, d.omega);
}

__global__ __launch_bounds__(kBlock) void k_ens_fin_rhs_mean(const EnsInst* I, const EnsOffsets* O) {
    const int q = blockIdx.x;
    const EnsInst& d = I[q];
    if (!d.singular) return;
    finalize_body<kBlock>(FIN_RHS2, d.part, (int)(O->cell[q + 1] - O->cell[q]), nullptr, nullptr, 0,
                          d.ctl, d.omega);
}

__global__ __launch_bounds__(kBlock) void k_ens_p_sum(const EnsInst* I, int n, const EnsOffsets* O) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = owner(O->red, n, L);
    const EnsInst& d = I[q];
    if (!d.singular) return;
    colour_sum_body(d.g, d.P.ph[0], d.P.ph[1], d.P.pd[0], d.P.pd[1], 1, d.part, L - O->red[q], d.nred);
}

__global__ __launch_bounds__(kBlock) void k_ens_fin_p_sum(const EnsInst* I) {
    const EnsInst& d = I[blockIdx.x];
    if (!d.singular) return;
    finalize_body<kBlock>(FIN_PSUM, d.part, (int)d.nred, nullptr, nullptr, 0, d.ctl, d.omega);
}

__global__ __launch_bounds__(kBlock) void k_ens_p_sub(const EnsInst* I, int n, const EnsOffsets* O) {
    const unsigned L = blockIdx.x;
    const int q = owner(O->half, n, L);
    const EnsInst& d = I[q];
    if (!d.singular) return;
    p_sub_body(d.g, d.P, d.ctl, L - O->half[q]);
}

__global__ __launch_bounds__(kBlock) void k_ens_project(const EnsInst* I, const EnsDyn* D, int n,
                                                        const EnsOffsets* O) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = owner(O->cell, n, L);
    const EnsInst& d = I[q];
    const int b = 1 - D[q].cur;
    project_body(d.g, d.u[b], d.v[b], d.w[b], d.P, L - O->cell[q]);
}

__global__ __launch_bounds__(kBlock) void k_ens_bc(const EnsInst* I, const EnsDyn* D, int n,
                                                   const EnsOffsets* O) {
    const unsigned L = blockIdx.x;
    const int q = owner(O->bc, n, L);
    const EnsInst& d = I[q];
    const int b = 1 - D[q].cur;
    bc_body(d.g, d.u[b], d.v[b], d.w[b], L - O->bc[q]);
}

// End of a step: flip the buffers, count the step, record the solve.
__global__ void k_ens_advance(const EnsInst* I, EnsDyn* D, int n) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const Ctl* c = I[q].ctl;
    EnsDyn& s = D[q];
    s.cur = 1 - s.cur;
    s.first = 0;
    s.step += 1;
    s.last_iters = c->m;
    s.done = c->done;
    s.resid = c->resid;
    s.reltmp2 = c->reltmp2;
    s.rhs2 = c->rhs2;
}

// Outside the graphs: copy this step's [iterations, status] per member.
__global__ void k_ens_record(const EnsDyn* D, int n, int* out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    out[2 * q] = D[q].last_iters;
    out[2 * q + 1] = D[q].done;
}

// ------------------------------------------------- persistent SOR solve
// Half-sweeps of items [a, b) of one member, the tile variant resolved once.
template <int TX, int KT>
__device__ __forceinline__ void sweep_items(const EnsInst& d, int c, bool acc, unsigned a, unsigned b) {
    float* ps = d.P.pd[c];
    const float* po = d.P.pd[1 - c];
    const float* rs = d.P.r0[c];
    double* rel = c ? d.rel1 : d.rel0;
    for (unsigned lb = a; lb < b; ++lb) sor_body<TX, KT>(d.g, c, ps, po, rs, d.omega, acc, rel, lb);
}

__device__ __forceinline__ void sweep_range(const EnsInst& d, int c, bool acc, unsigned a, unsigned b) {
    switch (d.variant) {
        case 0: sweep_items<64, 1>(d, c, acc, a, b); break;
        case 1: sweep_items<32, 1>(d, c, acc, a, b); break;
        case 2: sweep_items<64, 2>(d, c, acc, a, b); break;
        case 3: sweep_items<32, 2>(d, c, acc, a, b); break;
        case 4: sweep_items<64, 4>(d, c, acc, a, b); break;
        case 5: sweep_items<32, 4>(d, c, acc, a, b); break;
        case 6: sweep_items<64, 8>(d, c, acc, a, b); break;
        default: sweep_items<32, 8>(d, c, acc, a, b); break;
    }
}

// Block b owns the contiguous items [b chunk, (b+1) chunk) of a work list
// (offsets in LDS) and visits them member by member: f(q, a, b) for the
// member-local item range [a, b).
template <class F>
__device__ __forceinline__ void walk_items(const unsigned* s_off, int n, F&& f) {
    const unsigned total = s_off[n];
    const unsigned chunk = (total + gridDim.x - 1) / gridDim.x;
    const unsigned L0 = blockIdx.x * chunk;
    const unsigned L1 = min(total, L0 + chunk);
    if (L0 >= L1) return;
    int q = owner(s_off, n, L0);
    unsigned L = L0;
    while (L < L1 && q < n) {
        const unsigned end = min(L1, s_off[q + 1]);
        if (end > L) f(q, L - s_off[q], end - s_off[q]);
        L = end;
        ++q;
    }
}

// The whole solve of every member in one cooperative launch.  Check
// interval c (K iterations) is the same for all members; every loop trip
// count between grid barriers depends only on kernel arguments or on data
// read after a barrier, so all blocks meet every barrier, and the outer
// loop is bounded by max_checks.  A member leaves the work once its
// stopping test succeeds or it reaches its max_iter.
__global__ __launch_bounds__(kBlock, 6) void k_ens_solve(const EnsInst* __restrict__ I, int n,
                                                      const EnsOffsets* __restrict__ O, int K,
                                                      int max_checks) {
    cg::grid_group grid = cg::this_grid();
    __shared__ unsigned s_sweep[kMaxEnsemble + 1], s_red[kMaxEnsemble + 1], s_fold[kMaxEnsemble + 1];
    for (int q = threadIdx.x; q <= n; q += kBlock) {
        s_sweep[q] = O->sweep[q];
        s_red[q] = O->red[q];
        s_fold[q] = O->fold[q];
    }
    __syncthreads();
    const unsigned nb = gridDim.x;
    // set-up: fold, sync, rebase (r0 and the initial residual), sync, finalize
    walk_items(s_fold, n, [&](int q, unsigned a, unsigned b) {
        const EnsInst& d = I[q];
        if (ld(&d.ctl->done)) return;
        for (unsigned L = a; L < b; ++L)
            fold_body(d.g.ctot, d.P.ph[0], d.P.pd[0], d.P.ph[1], d.P.pd[1],
                      (long long)L * kBlock + threadIdx.x);
    });
    grid.sync();
    walk_items(s_red, n, [&](int q, unsigned a, unsigned b) {
        const EnsInst& d = I[q];
        if (ld(&d.ctl->done)) return;
        for (unsigned L = a; L < b; ++L) rebase_body(d.g, d.P, d.part, L, d.nred);
    });
    grid.sync();
    for (int q = blockIdx.x; q < n; q += nb)
        finalize_body<kBlock>(FIN_SETUP, I[q].part, (int)I[q].nred, nullptr, nullptr, 0, I[q].ctl, I[q].omega);
    grid.sync();

    for (int c = 0; c < max_checks; ++c) {
        bool all_done = true;
        for (int q = 0; q < n; ++q) all_done = all_done && (ld(&I[q].ctl->done) != 0);
        if (all_done) break;   // uniform: every block read the same flags after the barrier
        for (int it = 0; it < K; ++it) {
            for (int colour = 0; colour < 2; ++colour) {
                walk_items(s_sweep, n, [&](int q, unsigned a, unsigned b) {
                    const EnsInst& d = I[q];
                    bool acc;
                    if (!member_active(d.ctl, it, acc)) return;
                    sweep_range(d, colour, acc, a, b);
                });
                grid.sync();
            }
        }
        for (int q = blockIdx.x; q < n; q += nb)
            finalize_body<kBlock>(FIN_BOUND, nullptr, 0, I[q].rel0, I[q].rel1, (int)I[q].nsweep,
                                  I[q].ctl, I[q].omega);
        grid.sync();
        // members whose check interval ends with a rebase fold first
        bool any_rebase = false;
        for (int q = 0; q < n; ++q) any_rebase = any_rebase || rebase_due_at(c + 1, I[q].K, I[q].R);
        if (any_rebase) {
            walk_items(s_fold, n, [&](int q, unsigned a, unsigned b) {
                const EnsInst& d = I[q];
                if (!rebase_due_at(c + 1, d.K, d.R) || ld(&d.ctl->done)) return;
                for (unsigned L = a; L < b; ++L)
                    fold_body(d.g.ctot, d.P.ph[0], d.P.pd[0], d.P.ph[1], d.P.pd[1],
                              (long long)L * kBlock + threadIdx.x);
            });
            grid.sync();
        }
        walk_items(s_red, n, [&](int q, unsigned a, unsigned b) {
            const EnsInst& d = I[q];
            if (ld(&d.ctl->done)) return;
            if (rebase_due_at(c + 1, d.K, d.R)) {
                for (unsigned L = a; L < b; ++L) rebase_body(d.g, d.P, d.part, L, d.nred);
            } else if (!ld(&d.ctl->skip)) {
                for (unsigned L = a; L < b; ++L) check_body(d.g, d.P, d.part, L, d.nred);
            }
        });
        grid.sync();
        for (int q = blockIdx.x; q < n; q += nb) {
            const EnsInst& d = I[q];
            finalize_body<kBlock>(rebase_due_at(c + 1, d.K, d.R) ? FIN_CHECK_FULL : FIN_CHECK, d.part,
                                  (int)d.nred, d.rel0, d.rel1, (int)d.nsweep, d.ctl, d.omega);
        }
        grid.sync();
    }
}

// ----------------------------------------------- batched (non-persistent) solve
// The same solve as k_ens_solve, one launch per phase over all members.
// Every decision lives on the device (each member's control block), so a
// batch of check intervals is a fixed launch sequence, replayed from a HIP
// graph; launches after a member's convergence return at once.
// In these separate launches the control blocks were written by earlier
// kernels, so plain loads are coherent (kernel boundaries order them).
__device__ __forceinline__ bool rebase_due(const EnsInst& d) {
    // the check that ends the current interval is number m/K + 1
    return rebase_due_at((d.ctl->m / d.K) + 1, d.K, d.R);
}

constexpr unsigned kAuxBlocks = 4096;   // grid of the fold / check phases

__global__ __launch_bounds__(kBlock) void k_ens_sweep(const EnsInst* __restrict__ I,
                                                      const unsigned char* __restrict__ owner_of,
                                                      const EnsOffsets* __restrict__ O, int colour,
                                                      int it) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = owner_of[L];
    const EnsInst& d = I[q];
    bool acc;
    if (!sweep_active(d.ctl, it, acc)) return;
    sweep_range(d, colour, acc, L - O->sweep[q], L - O->sweep[q] + 1);
}

// One fused red-black iteration of every member (all on the ensemble's
// fused variant <TX, 16 wavefronts, KT>): parity 0 reads pd and writes pa,
// 1 the reverse.
template <int TX, int KT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_ens_sweep_rb(
                                                       const EnsInst* __restrict__ I,
                                                       const unsigned char* __restrict__ owner_of,
                                                       const EnsOffsets* __restrict__ O, int parity,
                                                       int it) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    // the member is block-uniform: keep its descriptor in scalar registers
    const int q = __builtin_amdgcn_readfirstlane((int)owner_of[L]);
    const EnsInst& d = I[q];
    bool acc;
    const bool active = sweep_active(d.ctl, it, acc);
    if (!active && d.ctl->done) return;
    const float* a0 = parity ? d.P.pa[0] : d.P.pd[0];
    const float* a1 = parity ? d.P.pa[1] : d.P.pd[1];
    float* b0 = parity ? d.P.pd[0] : d.P.pa[0];
    float* b1 = parity ? d.P.pd[1] : d.P.pa[1];
    const unsigned lb = L - O->sweep[q];
    // the geometry by value, as a kernel argument would be: a reference into
    // global memory may alias the sweep's stores, and its fields are then
    // reloaded and its helpers kept in memory
    const Geo g = d.g;
    const float* r0 = d.P.r0[0];
    const float* r1 = d.P.r0[1];
    const float omega = d.omega;
    const int kt = fused_kt(g, TX, 16, KT);
    if (rb_lean_fits(g)) {   // members are uniform grids (stretched ones cannot join)
        if (!active)
            sor_rb_copy_u<TX, 16, KT>(g, a0, a1, b0, b1, lb, kt);
        else if (acc)
            sor_rb_body_u<TX, 16, KT, true>(g, a0, a1, r0, r1, b0, b1, omega, d.rel0, d.rel1, lb, kt);
        else
            sor_rb_body_u<TX, 16, KT, false>(g, a0, a1, r0, r1, b0, b1, omega, d.rel0, d.rel1, lb, kt);
        return;
    }
    sor_rb_body<TX, 16, KT>(g, a0, a1, r0, r1, b0, b1, omega, active && acc, !active, d.rel0, d.rel1, lb, kt);
}

// Two fused red-black iterations of every member (local iterations it and
// it + 1; the two-iteration variants, members all on the uniform-grid lean
// form): parity 0 reads pd and writes pa, parity 1 the reverse.  A member's
// blocks run k_sor_rb2's tiles on its own block range.
__global__ __launch_bounds__(1024) void k_ens_sweep_rb2(const EnsInst* __restrict__ I,
                                                        const unsigned char* __restrict__ owner_of,
                                                        const EnsOffsets* __restrict__ O, int parity, int it) {
    const unsigned L = xcd_block(blockIdx.x, gridDim.x);
    const int q = __builtin_amdgcn_readfirstlane((int)owner_of[L]);
    const EnsInst& d = I[q];
    bool acc1, acc2;
    const bool a1s = sweep_active(d.ctl, it, acc1);
    const bool a2s = sweep_active(d.ctl, it + 1, acc2);
    if (!a1s && d.ctl->done) return;
    // The member's control decisions and descriptor are block-uniform:
    // copied through scalar registers, so that the march's plane loop and
    // the sweep's buffer offsets stay scalar (read from memory the compiler
    // cannot prove unchanged, they would turn per-lane).
    const int flags = __builtin_amdgcn_readfirstlane((a1s ? 1 : 0) | (a2s ? 2 : 0) | (acc1 ? 4 : 0) | (acc2 ? 8 : 0));
    const bool act1 = flags & 1, act2 = flags & 2;
    const bool p1 = act1 && (flags & 4) && !act2, p2 = act1 && act2 && (flags & 8);
    struct Args {
        Geo g;
        const float* a0;
        const float* a1;
        float* b0;
        float* b1;
        const float* r0;
        const float* r1;
        double* rel0;
        double* rel1;
        float omega;
        int kt;
        unsigned lb;
        unsigned pad;
    } raw;
    raw.g = d.g;
    raw.a0 = parity ? d.P.pa[0] : d.P.pd[0];
    raw.a1 = parity ? d.P.pa[1] : d.P.pd[1];
    raw.b0 = parity ? d.P.pd[0] : d.P.pa[0];
    raw.b1 = parity ? d.P.pd[1] : d.P.pa[1];
    raw.r0 = d.P.r0[0];
    raw.r1 = d.P.r0[1];
    raw.rel0 = d.rel0;
    raw.rel1 = d.rel1;
    raw.omega = d.omega;
    raw.kt = d.kt_rb2;
    raw.lb = L - O->sweep[q];
    raw.pad = 0;
    const Args A = uniform_copy(raw);
    __shared__ Rb2Smem sm;
    if (!act1)
        sor_rb2_copy_u(A.g, A.a0, A.a1, A.b0, A.b1, A.lb, A.kt);
    else if (p1 || p2)
        sor_rb2_body_u<true>(sm, A.g, A.a0, A.a1, A.r0, A.r1, A.b0, A.b1, A.omega, act2, p1, p2, A.rel0, A.rel1,
                             A.lb, A.kt);
    else
        sor_rb2_body_u<false>(sm, A.g, A.a0, A.a1, A.r0, A.r1, A.b0, A.b1, A.omega, act2, false, false, A.rel0,
                              A.rel1, A.lb, A.kt);
}

// Launch of k_ens_sweep_rb for fused variant v over `grid` blocks.
void launch_ens_sweep_rb(int v, unsigned grid, hipStream_t s, const EnsInst* I,
                         const unsigned char* owner_of, const EnsOffsets* O, int parity, int it) {
    switch (v) {
        case 8: hipLaunchKernelGGL((k_ens_sweep_rb<32, 12>), dim3(grid), dim3(1024), 0, s, I, owner_of, O, parity, it); break;
        case 9: hipLaunchKernelGGL((k_ens_sweep_rb<64, 16>), dim3(grid), dim3(1024), 0, s, I, owner_of, O, parity, it); break;
        case 10: hipLaunchKernelGGL((k_ens_sweep_rb<32, 0>), dim3(grid), dim3(1024), 0, s, I, owner_of, O, parity, it); break;
        default: hipLaunchKernelGGL((k_ens_sweep_rb<64, 0>), dim3(grid), dim3(1024), 0, s, I, owner_of, O, parity, it); break;
    }
}

__global__ __launch_bounds__(kBlock) void k_ens_bound(const EnsInst* __restrict__ I) {
    const EnsInst& d = I[blockIdx.x];
    finalize_body<kBlock>(FIN_BOUND, nullptr, 0, d.rel0, d.rel1, (int)d.nsweep, d.ctl, d.omega);
}

// setup = 1: fold every unfinished member (start of the solve); else only
// those whose current interval ends with a rebase.
// Capped grids walking the item lists member by member (walk_items):
// members with nothing to do cost one test per block, not one block per item.
__global__ __launch_bounds__(kBlock) void k_ens_fold(const EnsInst* __restrict__ I, int n,
                                                     const EnsOffsets* __restrict__ O, int setup) {
    __shared__ unsigned s_off[kMaxEnsemble + 1];
    for (int q = threadIdx.x; q <= n; q += kBlock) s_off[q] = O->fold[q];
    __syncthreads();
    walk_items(s_off, n, [&](int q, unsigned a, unsigned b) {
        const EnsInst& d = I[q];
        if (d.ctl->done || !(setup || rebase_due(d))) return;
        for (unsigned L = a; L < b; ++L)
            fold_body(d.g.ctot, d.P.ph[0], d.P.pd[0], d.P.ph[1], d.P.pd[1],
                      (long long)L * kBlock + threadIdx.x);
    });
}

__global__ __launch_bounds__(kBlock) void k_ens_check(const EnsInst* __restrict__ I, int n,
                                                      const EnsOffsets* __restrict__ O, int setup) {
    __shared__ unsigned s_off[kMaxEnsemble + 1];
    for (int q = threadIdx.x; q <= n; q += kBlock) s_off[q] = O->red[q];
    __syncthreads();
    walk_items(s_off, n, [&](int q, unsigned a, unsigned b) {
        const EnsInst& d = I[q];
        if (d.ctl->done) return;
        if (setup || rebase_due(d)) {
            for (unsigned L = a; L < b; ++L) rebase_body(d.g, d.P, d.part, L, d.nred);
        } else if (!d.ctl->skip) {
            for (unsigned L = a; L < b; ++L) check_body(d.g, d.P, d.part, L, d.nred);
        }
    });
}

__global__ __launch_bounds__(kBlock) void k_ens_fin_check(const EnsInst* __restrict__ I, int setup) {
    const EnsInst& d = I[blockIdx.x];
    const int op = setup ? FIN_SETUP : (rebase_due(d) ? FIN_CHECK_FULL : FIN_CHECK);
    finalize_body<kBlock>(op, d.part, (int)d.nred, d.rel0, d.rel1, (int)d.nsweep, d.ctl, d.omega);
}

// Control block that lets every sweep run (autotuning only).
__global__ void k_ctl_probe_init(Ctl* ctl) { ctl_init_body(ctl, 1e-30, 1 << 30, 1 << 20); }

__global__ __launch_bounds__(kBlock) void k_zero(float* p, long long n) {
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) p[t] = 0.f;
}

// 1 when every member is done (read by the host one batch behind).
// flag: every member's solve has stopped; mask: bit q set when member q's has
__global__ void k_ens_all_done(const EnsInst* __restrict__ I, int n, int* flag,
                               unsigned long long* mask) {
    if (threadIdx.x != 0) return;
    int all = 1;
    unsigned long long m = 0;
    for (int q = 0; q < n; ++q) {
        const bool d = I[q].ctl->done != 0;
        all &= d ? 1 : 0;
        if (d) m |= 1ull << q;
    }
    *flag = all;
    *mask = m;
}

}  // namespace
}  // namespace les

using namespace les;

struct les_ensemble {
    int n = 0;
    std::vector<les_handle*> members;
    std::string err;
    hipStream_t stream = nullptr;
    EnsInst* d_inst = nullptr;
    EnsDyn* d_dyn = nullptr;
    EnsOffsets* d_off = nullptr;
    EnsOffsets h_off{};
    int* d_iters = nullptr;        // [capacity][n][iterations, status]
    int iters_cap = 0;             // steps the [step][member][2] buffers hold
    EnsDyn* h_dyn = nullptr;       // pinned
    int* h_iters = nullptr;        // pinned
    int K = 4;
    int max_checks = 0;
    int solve_grid = 0;
    int solve_per_cu = 0;
    int mode = LES_ENSEMBLE_BATCHED;
    unsigned char* d_owner = nullptr;   // sweep block -> member (batched mode)
    int* d_flag = nullptr;
    int* h_flag = nullptr;              // pinned, 2 slots
    unsigned long long* d_mask = nullptr;   // members whose solve has stopped, 2 slots
    unsigned long long* h_mask = nullptr;   // pinned
    // sweep work list over the members still iterating (batched mode):
    // device copies and two pinned staging copies used in turn
    unsigned char* d_owner_live = nullptr;
    EnsOffsets* d_off_live = nullptr;
    unsigned char* h_owner_live[2] = {nullptr, nullptr};
    EnsOffsets* h_off_live[2] = {nullptr, nullptr};
    unsigned owner_live_cap = 0;
    // two-iteration sweeps: planes per block and blocks of each member with
    // every member iterating (restored at the start of a solve after the
    // live work list changed them)
    std::vector<int> base_kt;
    std::vector<unsigned> base_nsweep;
    bool kt_changed = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipGraphExec_t chunk_graph = nullptr;
    int chunk_graph_checks = 0;
    unsigned owner_blocks = 0;
    int variant = -1;                   // -1: each member's own sweep variant
    double tune_us[kNumSorVariants] = {};
    bool descriptors_dirty = false;
    bool graphs_ready = false;
    hipGraphExec_t pre[2] = {nullptr, nullptr};
    hipGraphExec_t post[2] = {nullptr, nullptr};
    int64_t cells_total = 0;
    std::vector<EnsInst> h_inst;
};

namespace {

int ens_err(les_ensemble* e, int code, const char* what, hipError_t he = hipSuccess) {
    if (e) {
        e->err = what;
        if (he != hipSuccess) e->err += std::string(": ") + hipGetErrorString(he);
    }
    return code;
}

#define ECK(expr)                                                          \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) return ens_err(e, LES_EDEVICE, #expr, e_);   \
    } while (0)

unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Fused iterations run only when the ensemble itself chose one (every
// member then runs it: one launch shape), in the batched mode and with an
// even check interval; two iterations per launch need a check interval
// that is a multiple of 4 and every member on the lean uniform-grid form.
bool ens_fused(const les_ensemble* e) {
    if (e->variant < 0 || !sor_fused(e->variant) || e->mode != LES_ENSEMBLE_BATCHED) return false;
    if (!sor_fused2(e->variant)) return !(e->K & 1);
    if (e->K & 3) return false;
    for (int q = 0; q < e->n; ++q)
        if (e->members[q]->g.stretched || !rb_lean_fits(e->members[q]->g)) return false;
    return true;
}
bool ens_fused2(const les_ensemble* e) { return ens_fused(e) && sor_fused2(e->variant); }

// Planes per block of member h's two-iteration sweep (variant v) when n_live
// members share the chip: the plane count for its share of the resident
// blocks, never below the one for the grid alone (so its block count never
// exceeds the variant's, for which its partial sums are sized).
int ens_rb2_kt(const les_handle* h, int v, int n_live) {
    const int per_cu = kSorVariants[v].kt;
    const long long slots = std::max<long long>(1, 256LL * per_cu / std::max(1, n_live));
    return std::max(rb2_kt(h->g, per_cu), rb2_kt_slots(h->g, slots));
}

// The sweep variant a member runs in the ensemble: the ensemble's choice,
// else the member's own; a fused variant where the ensemble cannot run it
// becomes the grid's default half-sweep.
int ens_variant(const les_ensemble* e, const les_handle* h) {
    const int v = e->variant >= 0 ? e->variant : h->sor_variant;
    return (sor_fused(v) && !ens_fused(e)) ? sor_default_variant(h->g) : v;
}

// Host copies of the member descriptors and work-list offsets, from the
// members' current settings (inflow, sweep variant, parameters).
void build_descriptors(les_ensemble* e) {
    const int n = e->n;
    e->h_inst.assign(n, EnsInst{});
    EnsOffsets& o = e->h_off;
    std::memset(&o, 0, sizeof o);
    int max_iter_all = 0;
    e->cells_total = 0;
    for (int q = 0; q < n; ++q) {
        les_handle* h = e->members[q];
        EnsInst& d = e->h_inst[q];
        std::memset(&d, 0, sizeof d);
        d.g = h->g;
        for (int b = 0; b < 2; ++b) {
            d.u[b] = h->f.u[b];
            d.v[b] = h->f.v[b];
            d.w[b] = h->f.w[b];
        }
        d.nut = h->f.nut;
        d.fu = h->f.fu; d.fv = h->f.fv; d.fw = h->f.fw;
        d.su = h->f.su; d.sv = h->f.sv; d.sw = h->f.sw;
        d.flags = h->f.flags;
        d.prof = h->f.prof;
        d.prof1 = h->interp ? h->f.prof1 : h->f.prof;
        d.interp = h->interp ? 1 : 0;
        d.t0 = h->t0;
        d.t1 = h->t1;
        d.dt = h->dt;
        d.P = h->f.P;
        d.part = h->f.part[0];
        d.rel0 = h->f.part[1];
        d.rel1 = h->f.part[2];
        d.ctl = h->f.ctl;
        const double delta = std::cbrt((double)h->g.dx * h->g.dy * h->g.dz);
        d.c2 = (float)((h->prm.cs * delta) * (h->prm.cs * delta));
        d.nu = (float)h->prm.nu;
        d.alpha = (float)h->prm.alpha;
        d.beta = (float)h->prm.beta;
        d.omega = (float)h->prm.omega;
        d.amp = h->amp;
        d.seed = h->seed;
        d.tol = h->prm.tol;
        d.max_iter = h->prm.max_iter;
        d.K = h->prm.check_every;
        d.R = h->prm.rebase_every;
        d.variant = ens_variant(e, h);
        d.singular = h->g.outflow ? 0 : 1;
        d.inflow = h->g.inflow;
        d.nsweep = sor_sweep_blocks(h->g, d.variant);
        d.kt_rb2 = 0;
        if (sor_fused2(d.variant)) {   // the ensemble's choice: the chip shared by all members
            d.kt_rb2 = ens_rb2_kt(h, d.variant, n);
            d.nsweep = rb2_blocks(h->g, d.kt_rb2);
        }
        d.nred = red_blocks(h->g);
        max_iter_all = std::max(max_iter_all, h->prm.max_iter);
        d.kt_tile = tile_kt(h->g);
        o.tile[q + 1] = o.tile[q] + tile_blocks(h->g);
        o.cell[q + 1] = o.cell[q] + cell_blocks(h->g);
        o.half[q + 1] = o.half[q] + half_blocks(h->g);
        o.red[q + 1] = o.red[q] + d.nred;
        o.bc[q + 1] = o.bc[q] + bc_blocks(h->g);
        o.inflow[q + 1] = o.inflow[q] + nblk((long long)h->g.ny * h->g.nz);
        o.sweep[q + 1] = o.sweep[q] + d.nsweep;
        o.fold[q + 1] = o.fold[q] + nblk(2 * h->g.ctot);
        e->cells_total += (int64_t)h->g.nx * h->g.ny * h->g.nz;
    }
    e->max_checks = (max_iter_all + e->K - 1) / e->K;
    e->base_kt.resize(n);
    e->base_nsweep.resize(n);
    for (int q = 0; q < n; ++q) {
        e->base_kt[q] = e->h_inst[q].kt_rb2;
        e->base_nsweep[q] = e->h_inst[q].nsweep;
    }
    e->kt_changed = false;
}

// The stage sequence before the solve (nu_t .. rhs, mean removal) and the
// one after it (p mean, projection, boundary refresh, advance).
int enqueue_pre(les_ensemble* e, hipStream_t s) {
    const int n = e->n;
    const EnsOffsets& o = e->h_off;
    hipLaunchKernelGGL(k_ens_step_tile, dim3(o.tile[n]), dim3(kTileThreads), 0, s, e->d_inst, e->d_dyn, n,
                       e->d_off);
    hipLaunchKernelGGL(k_ens_inflow, dim3(o.inflow[n]), dim3(kBlock), 0, s, e->d_inst, e->d_dyn, n, e->d_off);
    hipLaunchKernelGGL(k_ens_ctl_init, dim3(n), dim3(kBlock), 0, s, e->d_inst);
    hipLaunchKernelGGL(k_ens_rhs, dim3(o.cell[n]), dim3(kBlock), 0, s, e->d_inst, e->d_dyn, n, e->d_off);
    hipLaunchKernelGGL(k_ens_fin_rhs, dim3(n), dim3(kBlock), 0, s, e->d_inst, e->d_off);
    hipLaunchKernelGGL(k_ens_rhs_mean, dim3(o.cell[n]), dim3(kBlock), 0, s, e->d_inst, n, e->d_off);
    hipLaunchKernelGGL(k_ens_fin_rhs_mean, dim3(n), dim3(kBlock), 0, s, e->d_inst, e->d_off);
    ECK(hipGetLastError());
    return LES_OK;
}

int enqueue_post(les_ensemble* e, hipStream_t s) {
    const int n = e->n;
    const EnsOffsets& o = e->h_off;
    hipLaunchKernelGGL(k_ens_p_sum, dim3(o.red[n]), dim3(kBlock), 0, s, e->d_inst, n, e->d_off);
    hipLaunchKernelGGL(k_ens_fin_p_sum, dim3(n), dim3(kBlock), 0, s, e->d_inst);
    hipLaunchKernelGGL(k_ens_p_sub, dim3(o.half[n]), dim3(kBlock), 0, s, e->d_inst, n, e->d_off);
    hipLaunchKernelGGL(k_ens_project, dim3(o.cell[n]), dim3(kBlock), 0, s, e->d_inst, e->d_dyn, n, e->d_off);
    hipLaunchKernelGGL(k_ens_bc, dim3(o.bc[n]), dim3(kBlock), 0, s, e->d_inst, e->d_dyn, n, e->d_off);
    hipLaunchKernelGGL(k_ens_advance, dim3((n + 63) / 64), dim3(64), 0, s, e->d_inst, e->d_dyn, n);
    ECK(hipGetLastError());
    return LES_OK;
}

// Sweep-block -> member map for the batched sweeps (rebuilt with the
// descriptors: the members' sweep variants may change).
int upload_owner_map(les_ensemble* e) {
    const EnsOffsets& o = e->h_off;
    const unsigned total = o.sweep[e->n];
    std::vector<unsigned char> map(total);
    for (int q = 0; q < e->n; ++q)
        for (unsigned L = o.sweep[q]; L < o.sweep[q + 1]; ++L) map[L] = (unsigned char)q;
    if (total > e->owner_blocks) {
        if (e->d_owner) ECK(hipFree(e->d_owner));
        e->d_owner = nullptr;
        ECK(hipMalloc(&e->d_owner, total));
        e->owner_blocks = total;
    }
    ECK(hipMemcpy(e->d_owner, map.data(), total, hipMemcpyHostToDevice));
    return LES_OK;
}

// One check interval of every member: 2K half-sweeps, the residual bound,
// the fold of members due for a rebase, the check (or rebase), the decision.
// The sweeps run over the work list (owner, off: sweep offsets, grid blocks).
int enqueue_chunk(les_ensemble* e, hipStream_t s, const unsigned char* owner, const EnsOffsets* off,
                  unsigned grid) {
    const int n = e->n;
    const EnsOffsets& o = e->h_off;
    if (grid > 0) {
        if (ens_fused2(e)) {   // K/2 launches, an even number: the interval ends on pd
            for (int it = 0; it < e->K; it += 2)
                hipLaunchKernelGGL(k_ens_sweep_rb2, dim3(grid), dim3(1024), 0, s, e->d_inst, owner, off,
                                   (it >> 1) & 1, it);
        } else if (ens_fused(e)) {
            for (int it = 0; it < e->K; ++it)
                launch_ens_sweep_rb(e->variant, grid, s, e->d_inst, owner, off, it & 1, it);
        } else {
            for (int it = 0; it < e->K; ++it)
                for (int c = 0; c < 2; ++c)
                    hipLaunchKernelGGL(k_ens_sweep, dim3(grid), dim3(kBlock), 0, s, e->d_inst, owner, off, c,
                                       it);
        }
    }
    hipLaunchKernelGGL(k_ens_bound, dim3(n), dim3(kBlock), 0, s, e->d_inst);
    hipLaunchKernelGGL(k_ens_fold, dim3(std::min(o.fold[n], kAuxBlocks)), dim3(kBlock), 0, s,
                       e->d_inst, n, e->d_off, 0);
    hipLaunchKernelGGL(k_ens_check, dim3(std::min(o.red[n], kAuxBlocks)), dim3(kBlock), 0, s,
                       e->d_inst, n, e->d_off, 0);
    hipLaunchKernelGGL(k_ens_fin_check, dim3(n), dim3(kBlock), 0, s, e->d_inst, 0);
    ECK(hipGetLastError());
    return LES_OK;
}

int run_batched_solve(les_ensemble* e, hipStream_t s) {
    const int n = e->n;
    const EnsOffsets& o = e->h_off;
    constexpr int kGraphChecks = 8;   // check intervals per graph replay
    hipLaunchKernelGGL(k_ens_fold, dim3(std::min(o.fold[n], kAuxBlocks)), dim3(kBlock), 0, s,
                       e->d_inst, n, e->d_off, 1);
    hipLaunchKernelGGL(k_ens_check, dim3(std::min(o.red[n], kAuxBlocks)), dim3(kBlock), 0, s,
                       e->d_inst, n, e->d_off, 1);
    hipLaunchKernelGGL(k_ens_fin_check, dim3(n), dim3(kBlock), 0, s, e->d_inst, 1);
    ECK(hipGetLastError());
    // kGraphChecks intervals captured over a sweep work list
    auto capture = [&](const unsigned char* owner, const EnsOffsets* off, unsigned grid,
                       hipGraphExec_t* ex) -> int {
        hipGraph_t gph = nullptr;
        ECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = LES_OK;
        for (int q = 0; q < kGraphChecks && rc == LES_OK; ++q) rc = enqueue_chunk(e, s, owner, off, grid);
        hipError_t ce = hipStreamEndCapture(s, &gph);
        if (rc != LES_OK) return rc;
        ECK(ce);
        const hipError_t ie = hipGraphInstantiate(ex, gph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gph);
        ECK(ie);
        return LES_OK;
    };
    if (!e->chunk_graph) {
        const int rc = capture(e->d_owner, e->d_off, o.sweep[n], &e->chunk_graph);
        if (rc != LES_OK) return rc;
        e->chunk_graph_checks = kGraphChecks;
    }
    // the live work list never holds more blocks than every member alone on
    // its variant (two-iteration plane counts only grow as members share)
    unsigned live_cap = o.sweep[n];
    if (ens_fused2(e)) {
        live_cap = 0;
        for (int q = 0; q < n; ++q) live_cap += sor_sweep_blocks(e->members[q]->g, e->variant);
        live_cap = std::max(live_cap, o.sweep[n]);
    }
    if (e->kt_changed) {   // the previous solve's live list changed plane counts
        for (int q = 0; q < n; ++q) {
            e->h_inst[q].kt_rb2 = e->base_kt[q];
            e->h_inst[q].nsweep = e->base_nsweep[q];
        }
        ECK(hipMemcpyAsync(e->d_inst, e->h_inst.data(), sizeof(EnsInst) * n, hipMemcpyHostToDevice, s));
        ECK(hipStreamSynchronize(s));   // the host copy is rewritten below
        e->kt_changed = false;
    }
    if (live_cap > e->owner_live_cap) {
        ECK(hipStreamSynchronize(s));
        if (e->d_owner_live) ECK(hipFree(e->d_owner_live));
        e->d_owner_live = nullptr;
        for (int k = 0; k < 2; ++k) {
            if (e->h_owner_live[k]) ECK(hipHostFree(e->h_owner_live[k]));
            e->h_owner_live[k] = nullptr;
        }
        ECK(hipMalloc(&e->d_owner_live, live_cap));
        for (int k = 0; k < 2; ++k) ECK(hipHostMalloc((void**)&e->h_owner_live[k], live_cap, hipHostMallocDefault));
        e->owner_live_cap = live_cap;
    }
    // Once members stop, the following batches sweep only the members still
    // iterating (the stopped ones' blocks would only return at once, but a
    // launch still dispatches them): the work list is rebuilt from the
    // done-mask one batch behind and a graph captured over it.  Staging copy
    // k % 2 is rewritten two rebuilds later, after an event recorded behind
    // its upload has been waited on; the device copy is rewritten behind the
    // launches that read it.
    std::vector<hipGraphExec_t> live_graphs;
    auto drop_live_graphs = [&]() {
        if (live_graphs.empty()) return;
        (void)hipStreamSynchronize(s);
        for (hipGraphExec_t g : live_graphs) (void)hipGraphExecDestroy(g);
        live_graphs.clear();
    };
    const unsigned long long all_members = n >= 64 ? ~0ull : ((1ull << n) - 1);
    unsigned long long listed = all_members;
    hipGraphExec_t cur = e->chunk_graph;
    int rebuilds = 0;
    const long long n_batches = (e->max_checks + kGraphChecks - 1) / kGraphChecks;
    int slot = 0;
    bool pending = false;
    int rc = LES_OK;
    for (long long b = 0; b < n_batches && rc == LES_OK; ++b) {
        hipError_t he = hipGraphLaunch(cur, s);
        if (he == hipSuccess) {
            hipLaunchKernelGGL(k_ens_all_done, dim3(1), dim3(64), 0, s, e->d_inst, n, e->d_flag + slot,
                               e->d_mask + slot);
            he = hipGetLastError();
        }
        if (he == hipSuccess)
            he = hipMemcpyAsync(&e->h_flag[slot], e->d_flag + slot, sizeof(int), hipMemcpyDeviceToHost, s);
        if (he == hipSuccess)
            he = hipMemcpyAsync(&e->h_mask[slot], e->d_mask + slot, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, s);
        if (he == hipSuccess) he = hipEventRecord(e->ev[slot], s);
        if (he == hipSuccess && pending) he = hipEventSynchronize(e->ev[1 - slot]);
        if (he != hipSuccess) {
            rc = ens_err(e, LES_EDEVICE, "batched solve launch", he);
            break;
        }
        if (pending) {
            if (e->h_flag[1 - slot]) break;
            const unsigned long long live = all_members & ~e->h_mask[1 - slot];
            if (live != listed) {
                // two-iteration sweeps: the live members' plane counts for
                // their larger share of the chip (the member descriptors are
                // rewritten behind the running batch; a blocking copy, so the
                // host copy may change afterwards)
                if (ens_fused2(e)) {
                    const int n_live = __builtin_popcountll(live);
                    bool upd = false;
                    for (int q = 0; q < n; ++q) {
                        if (!((live >> q) & 1)) continue;
                        const int kt = ens_rb2_kt(e->members[q], e->variant, n_live);
                        if (kt != e->h_inst[q].kt_rb2) {
                            e->h_inst[q].kt_rb2 = kt;
                            e->h_inst[q].nsweep = rb2_blocks(e->members[q]->g, kt);
                            upd = true;
                        }
                    }
                    if (upd) {
                        he = hipMemcpyAsync(e->d_inst, e->h_inst.data(), sizeof(EnsInst) * n, hipMemcpyHostToDevice, s);
                        if (he == hipSuccess) he = hipStreamSynchronize(s);
                        if (he != hipSuccess) {
                            rc = ens_err(e, LES_EDEVICE, "member descriptor upload", he);
                            break;
                        }
                        e->kt_changed = true;
                    }
                }
                const int k = rebuilds++ & 1;
                EnsOffsets& lo = *e->h_off_live[k];
                std::memset(&lo, 0, sizeof lo);
                for (int q = 0; q < n; ++q) {
                    const unsigned nb = ((live >> q) & 1) ? e->h_inst[q].nsweep : 0u;
                    lo.sweep[q + 1] = lo.sweep[q] + nb;
                    for (unsigned L = 0; L < nb; ++L) e->h_owner_live[k][lo.sweep[q] + L] = (unsigned char)q;
                }
                // offsets relative to the live list: a member's blocks keep
                // their indices within the member (L - sweep[q])
                he = hipMemcpyAsync(e->d_off_live, &lo, sizeof lo, hipMemcpyHostToDevice, s);
                if (he == hipSuccess && lo.sweep[n] > 0)
                    he = hipMemcpyAsync(e->d_owner_live, e->h_owner_live[k], lo.sweep[n], hipMemcpyHostToDevice, s);
                if (he != hipSuccess) {
                    rc = ens_err(e, LES_EDEVICE, "live work list upload", he);
                    break;
                }
                hipGraphExec_t ex = nullptr;
                rc = capture(e->d_owner_live, e->d_off_live, lo.sweep[n], &ex);
                if (rc != LES_OK) break;
                live_graphs.push_back(ex);
                cur = ex;
                listed = live;
            }
        }
        pending = true;
        slot = 1 - slot;
    }
    drop_live_graphs();
    return rc;
}

int launch_solve(les_ensemble* e, hipStream_t s) {
    if (e->mode == LES_ENSEMBLE_BATCHED) return run_batched_solve(e, s);
    const EnsInst* I = e->d_inst;
    int n = e->n;
    const EnsOffsets* O = e->d_off;
    int K = e->K, mc = e->max_checks;
    void* args[] = {(void*)&I, (void*)&n, (void*)&O, (void*)&K, (void*)&mc};
    ECK(hipLaunchCooperativeKernel((const void*)k_ens_solve, dim3(e->solve_grid), dim3(kBlock), args,
                                   0, s));
    return LES_OK;
}

}  // namespace

extern "C" {

int les_ensemble_create(int32_t n, les_handle* const* members, les_ensemble** out) {
    if (!out || !members || n < 1 || n > kMaxEnsemble) return LES_EINVAL;
    *out = nullptr;
    for (int q = 0; q < n; ++q) {
        if (!members[q]) return LES_EINVAL;
        for (int r = 0; r < q; ++r)
            if (members[r] == members[q]) return LES_EINVAL;
        if (members[q]->prm.check_every != members[0]->prm.check_every) return LES_EINVAL;
        if (members[q]->device != members[0]->device) return LES_EINVAL;
        if (members[q]->g.stretched) return LES_EINVAL;   // uniform members only
        if (members[q]->prm.zero_guess) return LES_EINVAL;
    }
    les_ensemble* e = new (std::nothrow) les_ensemble();
    if (!e) return LES_ENOMEM;
    e->n = n;
    e->members.assign(members, members + n);
    e->K = members[0]->prm.check_every;
    auto fail = [&](int code) {
        les_ensemble_destroy(e);
        return code;
    };
    if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) return fail(LES_EDEVICE);
    build_descriptors(e);
    if (hipMalloc(&e->d_inst, sizeof(EnsInst) * n) != hipSuccess) return fail(LES_ENOMEM);
    if (hipMalloc(&e->d_dyn, sizeof(EnsDyn) * n) != hipSuccess) return fail(LES_ENOMEM);
    if (hipMalloc(&e->d_off, sizeof(EnsOffsets)) != hipSuccess) return fail(LES_ENOMEM);
    if (hipHostMalloc((void**)&e->h_dyn, sizeof(EnsDyn) * n, hipHostMallocDefault) != hipSuccess)
        return fail(LES_ENOMEM);
    if (hipMemcpy(e->d_inst, e->h_inst.data(), sizeof(EnsInst) * n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(LES_EDEVICE);
    if (hipMemcpy(e->d_off, &e->h_off, sizeof(EnsOffsets), hipMemcpyHostToDevice) != hipSuccess)
        return fail(LES_EDEVICE);
    // cooperative grid: as many blocks as can be co-resident
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LES_EDEVICE);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(LES_EDEVICE);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_ens_solve, kBlock, 0) !=
            hipSuccess || per_cu < 1)
        return fail(LES_EDEVICE);
    e->solve_grid = cus * std::min(per_cu, 8);
    e->solve_per_cu = per_cu;
    if (hipMalloc(&e->d_flag, 2 * sizeof(int)) != hipSuccess) return fail(LES_ENOMEM);
    if (hipHostMalloc((void**)&e->h_flag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(LES_ENOMEM);
    if (hipMalloc(&e->d_mask, 2 * sizeof(unsigned long long)) != hipSuccess) return fail(LES_ENOMEM);
    if (hipHostMalloc((void**)&e->h_mask, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
        return fail(LES_ENOMEM);
    if (hipMalloc(&e->d_off_live, sizeof(EnsOffsets)) != hipSuccess) return fail(LES_ENOMEM);
    for (int k = 0; k < 2; ++k)
        if (hipHostMalloc((void**)&e->h_off_live[k], sizeof(EnsOffsets), hipHostMallocDefault) != hipSuccess)
            return fail(LES_ENOMEM);
    for (int q = 0; q < 2; ++q)
        if (hipEventCreateWithFlags(&e->ev[q], hipEventDisableTiming) != hipSuccess) return fail(LES_EDEVICE);
    if (upload_owner_map(e) != LES_OK) return fail(LES_EDEVICE);
    *out = e;
    return LES_OK;
}

void les_ensemble_destroy(les_ensemble* e) {
    if (!e) return;
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    for (int p = 0; p < 2; ++p) {
        if (e->pre[p]) (void)hipGraphExecDestroy(e->pre[p]);
        if (e->post[p]) (void)hipGraphExecDestroy(e->post[p]);
    }
    if (e->chunk_graph) (void)hipGraphExecDestroy(e->chunk_graph);
    if (e->d_owner) (void)hipFree(e->d_owner);
    if (e->d_flag) (void)hipFree(e->d_flag);
    if (e->h_flag) (void)hipHostFree(e->h_flag);
    if (e->d_mask) (void)hipFree(e->d_mask);
    if (e->h_mask) (void)hipHostFree(e->h_mask);
    if (e->d_owner_live) (void)hipFree(e->d_owner_live);
    if (e->d_off_live) (void)hipFree(e->d_off_live);
    for (int k = 0; k < 2; ++k) {
        if (e->h_owner_live[k]) (void)hipHostFree(e->h_owner_live[k]);
        if (e->h_off_live[k]) (void)hipHostFree(e->h_off_live[k]);
    }
    for (int q = 0; q < 2; ++q)
        if (e->ev[q]) (void)hipEventDestroy(e->ev[q]);
    if (e->d_inst) (void)hipFree(e->d_inst);
    if (e->d_dyn) (void)hipFree(e->d_dyn);
    if (e->d_off) (void)hipFree(e->d_off);
    if (e->d_iters) (void)hipFree(e->d_iters);
    if (e->h_dyn) (void)hipHostFree(e->h_dyn);
    if (e->h_iters) (void)hipHostFree(e->h_iters);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

const char* les_ensemble_last_error(const les_ensemble* e) { return e ? e->err.c_str() : ""; }

int les_ensemble_set_mode(les_ensemble* e, int32_t mode) {
    if (!e || (mode != LES_ENSEMBLE_BATCHED && mode != LES_ENSEMBLE_PERSISTENT)) return LES_EINVAL;
    e->mode = mode;
    return LES_OK;
}

int les_ensemble_set_variant(les_ensemble* e, int32_t variant) {
    if (!e || variant < -1 || variant >= kNumSorVariants) return LES_EINVAL;
    e->variant = variant;
    e->descriptors_dirty = true;
    return LES_OK;
}

int les_ensemble_autotune(les_ensemble* e, int32_t reps) {
    if (!e || reps < 1 || reps > 1000) return LES_EINVAL;
    const int n = e->n;
    // time the batched half-sweep of all members for each tile variant,
    // used by every member, on the members' scratch pressure systems (the
    // time-stepping state is not touched); keep the fastest
    for (int q = 0; q < n; ++q) {
        les_handle* h = e->members[q];
        if (!h->solve_arena) {
            les_solve_stats st{};
            (void)st;
            int rc = les_autotune(h, 1, nullptr, nullptr);   // allocates the scratch system
            if (rc != LES_OK) return ens_err(e, rc, "member scratch allocation");
        }
    }
    hipEvent_t a = nullptr, b = nullptr;
    ECK(hipEventCreate(&a));
    ECK(hipEventCreate(&b));
    double best = 1e300;
    int best_v = 0;
    const int saved = e->variant;
    for (int v = 0; v < kNumSorVariants; ++v) {
        e->variant = v;
        // persistent mode, an odd check interval (two iterations per
        // launch: not a multiple of 4, or a member off the lean form)
        if (sor_fused(v) && !ens_fused(e)) {
            e->tune_us[v] = 0.0;
            continue;
        }
        build_descriptors(e);
        for (int q = 0; q < n; ++q) e->h_inst[q].P = e->members[q]->S;
        ECK(hipMemcpy(e->d_inst, e->h_inst.data(), sizeof(EnsInst) * n, hipMemcpyHostToDevice));
        ECK(hipMemcpy(e->d_off, &e->h_off, sizeof(EnsOffsets), hipMemcpyHostToDevice));
        int rc = upload_owner_map(e);
        if (rc != LES_OK) return rc;
        for (int q = 0; q < n; ++q)
            hipLaunchKernelGGL(k_ctl_probe_init, dim3(1), dim3(64), 0, e->stream, e->h_inst[q].ctl);
        const unsigned grid = e->h_off.sweep[n];
        // two launches: two half-sweeps, two fused iterations or four (a
        // quarter of a two-iteration launch, half a fused iteration, is
        // charged per half-sweep below)
        auto pair = [&]() {
            for (int w = 0; w < 2; ++w) {
                if (sor_fused2(v))
                    hipLaunchKernelGGL(k_ens_sweep_rb2, dim3(grid), dim3(1024), 0, e->stream, e->d_inst,
                                       e->d_owner, e->d_off, w, 0);
                else if (sor_fused(v))
                    launch_ens_sweep_rb(v, grid, e->stream, e->d_inst, e->d_owner, e->d_off, w, 0);
                else
                    hipLaunchKernelGGL(k_ens_sweep, dim3(grid), dim3(kBlock), 0, e->stream, e->d_inst,
                                       e->d_owner, e->d_off, w, 0);
            }
        };
        pair();
        ECK(hipEventRecord(a, e->stream));
        for (int r = 0; r < reps; ++r) pair();
        ECK(hipEventRecord(b, e->stream));
        ECK(hipEventSynchronize(b));
        float ms = 0.f;
        ECK(hipEventElapsedTime(&ms, a, b));
        const double us = 1e3 * ms / ((sor_fused2(v) ? 8.0 : (sor_fused(v) ? 4.0 : 2.0)) * reps);
        e->tune_us[v] = us;
        if (us < best) {
            best = us;
            best_v = v;
        }
    }
    (void)saved;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    for (int q = 0; q < n; ++q)
        for (int c = 0; c < 2; ++c) {
            les_handle* h = e->members[q];
            hipLaunchKernelGGL(k_zero, dim3((unsigned)((h->g.ctot + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               e->stream, h->S.pd[c], h->g.ctot);
            hipLaunchKernelGGL(k_zero, dim3((unsigned)((h->g.ctot + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               e->stream, h->S.pa[c], h->g.ctot);
        }
    ECK(hipStreamSynchronize(e->stream));
    e->variant = best_v;
    e->descriptors_dirty = true;
    return LES_OK;
}

int les_ensemble_tuning(const les_ensemble* e, int32_t* variant, double* us_per_sweep) {
    if (!e) return LES_EINVAL;
    if (variant) *variant = e->variant;
    if (us_per_sweep)
        for (int v = 0; v < kNumSorVariants; ++v) us_per_sweep[v] = e->tune_us[v];
    return LES_OK;
}

int les_ensemble_step(les_ensemble* e, int32_t nsteps, les_ensemble_stats* st, int32_t* iters_out) {
    if (!e || nsteps < 0) return LES_EINVAL;
    const int n = e->n;
    for (int q = 0; q < n; ++q) {
        if (!e->members[q]->have_inflow) return ens_err(e, LES_ESTATE, "member without inflow");
        if (e->members[q]->warm_net || e->members[q]->cap_x)
            return ens_err(e, LES_ESTATE, "member with a warm start or capture set (single-handle only)");
    }
    auto t0 = std::chrono::steady_clock::now();
    // members' own streams finish first; the ensemble works on its stream
    for (int q = 0; q < n; ++q) ECK(hipStreamSynchronize(e->members[q]->stream));
    // current per-member state
    for (int q = 0; q < n; ++q) {
        les_handle* h = e->members[q];
        EnsDyn& s = e->h_dyn[q];
        std::memset(&s, 0, sizeof s);
        s.cur = h->cur;
        s.first = h->have_old ? 0 : 1;
        s.step = h->step;
    }
    ECK(hipMemcpyAsync(e->d_dyn, e->h_dyn, sizeof(EnsDyn) * n, hipMemcpyHostToDevice, e->stream));
    {
        const unsigned old_sweep = e->h_off.sweep[n];
        std::vector<int> old_var(n);
        for (int q = 0; q < n; ++q) old_var[q] = e->h_inst.empty() ? -1 : e->h_inst[q].variant;
        build_descriptors(e);
        bool changed = e->h_off.sweep[n] != old_sweep || e->descriptors_dirty;
        e->descriptors_dirty = false;
        for (int q = 0; q < n; ++q) changed = changed || old_var[q] != e->h_inst[q].variant;
        ECK(hipMemcpyAsync(e->d_inst, e->h_inst.data(), sizeof(EnsInst) * n, hipMemcpyHostToDevice, e->stream));
        ECK(hipMemcpyAsync(e->d_off, &e->h_off, sizeof(EnsOffsets), hipMemcpyHostToDevice, e->stream));
        if (changed) {
            ECK(hipStreamSynchronize(e->stream));
            int rc = upload_owner_map(e);
            if (rc != LES_OK) return rc;
            if (e->chunk_graph) ECK(hipGraphExecDestroy(e->chunk_graph));
            e->chunk_graph = nullptr;   // sweep grid size changed
        }
    }
    if (nsteps > e->iters_cap) {
        if (e->d_iters) ECK(hipFree(e->d_iters));
        if (e->h_iters) ECK(hipHostFree(e->h_iters));
        e->d_iters = nullptr;
        e->h_iters = nullptr;
        ECK(hipMalloc(&e->d_iters, 2 * sizeof(int) * (size_t)n * nsteps));
        ECK(hipHostMalloc((void**)&e->h_iters, 2 * sizeof(int) * (size_t)n * nsteps, hipHostMallocDefault));
        e->iters_cap = nsteps;
    }
    if (!e->graphs_ready && nsteps > 0) {
        for (int p = 0; p < 2; ++p) {
            for (int which = 0; which < 2; ++which) {
                hipGraph_t gph = nullptr;
                ECK(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
                int rc = which == 0 ? enqueue_pre(e, e->stream) : enqueue_post(e, e->stream);
                hipError_t ce = hipStreamEndCapture(e->stream, &gph);
                if (rc != LES_OK) return rc;
                ECK(ce);
                hipGraphExec_t& ex = which == 0 ? e->pre[p] : e->post[p];
                if (ex) ECK(hipGraphExecDestroy(ex));
                ex = nullptr;
                ECK(hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0));
                ECK(hipGraphDestroy(gph));
            }
        }
        e->graphs_ready = true;
    }
    for (int s = 0; s < nsteps; ++s) {
        ECK(hipGraphLaunch(e->pre[s & 1], e->stream));
        int rc = launch_solve(e, e->stream);
        if (rc != LES_OK) return rc;
        ECK(hipGraphLaunch(e->post[s & 1], e->stream));
        hipLaunchKernelGGL(k_ens_record, dim3((n + 63) / 64), dim3(64), 0, e->stream, e->d_dyn, n,
                           e->d_iters + 2 * (size_t)s * n);
        ECK(hipGetLastError());
    }
    ECK(hipMemcpyAsync(e->h_dyn, e->d_dyn, sizeof(EnsDyn) * n, hipMemcpyDeviceToHost, e->stream));
    if (nsteps > 0)
        ECK(hipMemcpyAsync(e->h_iters, e->d_iters, 2 * sizeof(int) * (size_t)n * nsteps,
                           hipMemcpyDeviceToHost, e->stream));
    ECK(hipStreamSynchronize(e->stream));
    int worst = LES_OK;
    les_ensemble_stats acc{};
    acc.members = n;
    acc.steps = nsteps;
    acc.cells_total = e->cells_total;
    // every member's buffer parity and step count first (the device advanced
    // all of them), then the check for non-finite members
    for (int q = 0; q < n; ++q) {
        les_handle* h = e->members[q];
        const EnsDyn& s = e->h_dyn[q];
        h->cur = s.cur;
        h->step = s.step;
        if (nsteps > 0) h->have_old = true;
    }
    for (int q = 0; q < n; ++q) {
        const EnsDyn& s = e->h_dyn[q];
        if (nsteps > 0 && (s.done == 3 || !std::isfinite(s.rhs2)))
            return ens_err(e, LES_ENONFINITE, "non-finite residual norm in a member");
    }
    for (int s = 0; s < nsteps; ++s)
        for (int q = 0; q < n; ++q) {
            const int it = e->h_iters[2 * ((size_t)s * n + q)];
            const int done = e->h_iters[2 * ((size_t)s * n + q) + 1];
            acc.sor_iters_total += it;
            if (iters_out) iters_out[(size_t)s * n + q] = it;
            if (done == 2) {
                acc.not_converged += 1;
                worst = LES_NOT_CONVERGED;
            }
        }
    acc.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = acc;
    return worst;
}

}  // extern "C"
