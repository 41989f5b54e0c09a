// Stencil kernels of one LES time step on gfx950 (all float32 fields,
// float64 norms).  One work-item per cell, x fastest, XCD-aware block
// numbering; every launch is sized from the geometry and every thread is
// guarded against the grid tail.
//
// Staggered (MAC) grid: u on x-faces, v on y-faces, w on z-faces, scalars
// at cell centres; see les_impl.h for the memory layouts.
#include "device_util.h"
#include "les_impl.h"

namespace les {
namespace {

inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Decompose a linear interior-cell index (0-based, x fastest) into 1-based
// cell coordinates.
__device__ __forceinline__ void cell_of(const Geo& g, long long t, int& i, int& j, int& k) {
    const unsigned tt = (unsigned)t;   // cells < 2^31 (checked at create)
    const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
    const unsigned kk = tt / nxy;
    const unsigned r = tt - kk * nxy;
    const unsigned jj = r / (unsigned)g.nx;
    i = (int)(r - jj * (unsigned)g.nx) + 1;
    j = (int)jj + 1;
    k = (int)kk + 1;
}

// ------------------------------------------------------------------ les
// Smagorinsky eddy viscosity nu_t = (Cs Delta)^2 |S|, |S| = sqrt(2 S_ij S_ij)
// (section 2.1, les).  S_ii from the two faces of the cell; S_ij (i != j)
// is the mean of the four edge values around the cell, each edge value
// being 1/2 (du_i/dx_j + du_j/dx_i) from the adjacent faces.  Launched over
// the whole ghosted box: a ghost cell takes the value of the nearest
// interior cell (mirrored ghost ring).
__global__ __launch_bounds__(kBlock) void k_nut(Geo g, const float* __restrict__ u,
                                                const float* __restrict__ v,
                                                const float* __restrict__ w,
                                                float* __restrict__ nut, float c2) {
    const long long nbox = (long long)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
    const long long t = (long long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (t >= nbox) return;
    const unsigned pxy = (unsigned)(g.nx + 2) * (unsigned)(g.ny + 2);
    const unsigned tt = (unsigned)t;
    const int k = (int)(tt / pxy);
    const unsigned r = tt - (unsigned)k * pxy;
    const int j = (int)(r / (unsigned)(g.nx + 2));
    const int i = (int)(r - (unsigned)j * (unsigned)(g.nx + 2));
    const int ic = min(max(i, 1), g.nx), jc = min(max(j, 1), g.ny), kc = min(max(k, 1), g.nz);
    auto U = [&](int a, int b, int c) { return u[g.nat(a, b, c)]; };
    auto V = [&](int a, int b, int c) { return v[g.nat(a, b, c)]; };
    auto W = [&](int a, int b, int c) { return w[g.nat(a, b, c)]; };
    const float s11 = (U(ic, jc, kc) - U(ic - 1, jc, kc)) * g.idx;
    const float s22 = (V(ic, jc, kc) - V(ic, jc - 1, kc)) * g.idy;
    const float s33 = (W(ic, jc, kc) - W(ic, jc, kc - 1)) * g.idz;
    float s12 = 0.f, s13 = 0.f, s23 = 0.f;
#pragma unroll
    for (int da = -1; da <= 0; ++da)
#pragma unroll
        for (int db = -1; db <= 0; ++db) {
            const int a = ic + da, b = jc + db;   // x-y edge (face a, face b)
            s12 += (U(a, b + 1, kc) - U(a, b, kc)) * g.idy + (V(a + 1, b, kc) - V(a, b, kc)) * g.idx;
            const int c = kc + db;                // x-z edge (face a, face c)
            s13 += (U(a, jc, c + 1) - U(a, jc, c)) * g.idz + (W(a + 1, jc, c) - W(a, jc, c)) * g.idx;
            const int b2 = jc + da;               // y-z edge (face b2, face c)
            s23 += (V(ic, b2, c + 1) - V(ic, b2, c)) * g.idz + (W(ic, b2 + 1, c) - W(ic, b2, c)) * g.idy;
        }
    s12 *= 0.125f;   // 1/4 (mean of 4 edges) * 1/2 (symmetric part)
    s13 *= 0.125f;
    s23 *= 0.125f;
    const float ss = 2.f * (s11 * s11 + s22 * s22 + s33 * s33) + 4.f * (s12 * s12 + s13 * s13 + s23 * s23);
    nut[g.nat(i, j, k)] = c2 * sqrtf(ss);
}

// ------------------------------------------- velfg + feedbf + adam (fused)
// Per cell (i,j,k) the tendencies of its east u-face, north v-face and top
// w-face:  F = -(covx + covy + covz) + nu lap + div(2 nu_t S).
// The cov pieces are the paper's velfg assembly (section 2.5.3): products
// of an averaged advecting velocity and a one-sided difference on the two
// half-points around the face, averaged onto the face; the diffusive part
// is the difference of the one-sided (diu) fluxes, i.e. the 7-point
// Laplacian.  The subgrid stress uses nu_t at centres for the normal
// component and the 4-cell edge mean for the shear components.
// Then building feedback forcing on solid faces (feedbf):
//   usum += dt u;  F += alpha usum + beta u
// and the Adams-Bashforth update (adam):
//   u* = u + dt (3/2 F - 1/2 F_old)  (F_old := F on the first step);  F_old <- F.
__global__ __launch_bounds__(kBlock) void k_tendency(
    Geo g, const float* __restrict__ u, const float* __restrict__ v, const float* __restrict__ w,
    const float* __restrict__ nut, float* __restrict__ fu, float* __restrict__ fv,
    float* __restrict__ fw, float* __restrict__ su, float* __restrict__ sv,
    float* __restrict__ sw, const uint8_t* __restrict__ flags, float* __restrict__ us,
    float* __restrict__ vs, float* __restrict__ ws, float nu, float alpha, float beta,
    int first) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    auto U = [&](int a, int b, int c) { return u[g.nat(a, b, c)]; };
    auto V = [&](int a, int b, int c) { return v[g.nat(a, b, c)]; };
    auto W = [&](int a, int b, int c) { return w[g.nat(a, b, c)]; };
    auto N = [&](int a, int b, int c) { return nut[g.nat(a, b, c)]; };
    // edge viscosities and strain rates
    auto n12 = [&](int a, int b, int c) { return 0.25f * (N(a, b, c) + N(a + 1, b, c) + N(a, b + 1, c) + N(a + 1, b + 1, c)); };
    auto n13 = [&](int a, int b, int c) { return 0.25f * (N(a, b, c) + N(a + 1, b, c) + N(a, b, c + 1) + N(a + 1, b, c + 1)); };
    auto n23 = [&](int a, int b, int c) { return 0.25f * (N(a, b, c) + N(a, b + 1, c) + N(a, b, c + 1) + N(a, b + 1, c + 1)); };
    auto e12 = [&](int a, int b, int c) { return 0.5f * ((U(a, b + 1, c) - U(a, b, c)) * g.idy + (V(a + 1, b, c) - V(a, b, c)) * g.idx); };
    auto e13 = [&](int a, int b, int c) { return 0.5f * ((U(a, b, c + 1) - U(a, b, c)) * g.idz + (W(a + 1, b, c) - W(a, b, c)) * g.idx); };
    auto e23 = [&](int a, int b, int c) { return 0.5f * ((V(a, b, c + 1) - V(a, b, c)) * g.idz + (W(a, b + 1, c) - W(a, b, c)) * g.idy); };

    const long long e = g.nat(i, j, k);
    const uint8_t fl = flags[e];
    const float dt = g.dt;

    if (i <= g.u_last) {
        const float uc = U(i, j, k);
        const float um = U(i - 1, j, k), up = U(i + 1, j, k);
        const float covx = 0.5f * (0.5f * (um + uc) * (uc - um) + 0.5f * (uc + up) * (up - uc)) * g.idx;
        const float covy = 0.5f * (0.5f * (V(i, j - 1, k) + V(i + 1, j - 1, k)) * (uc - U(i, j - 1, k)) +
                                   0.5f * (V(i, j, k) + V(i + 1, j, k)) * (U(i, j + 1, k) - uc)) * g.idy;
        const float covz = 0.5f * (0.5f * (W(i, j, k - 1) + W(i + 1, j, k - 1)) * (uc - U(i, j, k - 1)) +
                                   0.5f * (W(i, j, k) + W(i + 1, j, k)) * (U(i, j, k + 1) - uc)) * g.idz;
        const float lap = (up - 2.f * uc + um) * g.cx + (U(i, j + 1, k) - 2.f * uc + U(i, j - 1, k)) * g.cy +
                          (U(i, j, k + 1) - 2.f * uc + U(i, j, k - 1)) * g.cz;
        const float sgs = 2.f * (N(i + 1, j, k) * (up - uc) * g.idx - N(i, j, k) * (uc - um) * g.idx) * g.idx +
                          2.f * (n12(i, j, k) * e12(i, j, k) - n12(i, j - 1, k) * e12(i, j - 1, k)) * g.idy +
                          2.f * (n13(i, j, k) * e13(i, j, k) - n13(i, j, k - 1) * e13(i, j, k - 1)) * g.idz;
        float F = -(covx + covy + covz) + nu * lap + sgs;
        if (fl & F_USOLID) {
            const float s = su[e] + dt * uc;
            su[e] = s;
            F += alpha * s + beta * uc;
        }
        const float fo = first ? F : fu[e];
        us[e] = uc + dt * (1.5f * F - 0.5f * fo);
        fu[e] = F;
    }
    if (j <= g.ny - 1) {
        const float vc = V(i, j, k);
        const float vm = V(i, j - 1, k), vp = V(i, j + 1, k);
        const float covx = 0.5f * (0.5f * (U(i - 1, j, k) + U(i - 1, j + 1, k)) * (vc - V(i - 1, j, k)) +
                                   0.5f * (U(i, j, k) + U(i, j + 1, k)) * (V(i + 1, j, k) - vc)) * g.idx;
        const float covy = 0.5f * (0.5f * (vm + vc) * (vc - vm) + 0.5f * (vc + vp) * (vp - vc)) * g.idy;
        const float covz = 0.5f * (0.5f * (W(i, j, k - 1) + W(i, j + 1, k - 1)) * (vc - V(i, j, k - 1)) +
                                   0.5f * (W(i, j, k) + W(i, j + 1, k)) * (V(i, j, k + 1) - vc)) * g.idz;
        const float lap = (V(i + 1, j, k) - 2.f * vc + V(i - 1, j, k)) * g.cx + (vp - 2.f * vc + vm) * g.cy +
                          (V(i, j, k + 1) - 2.f * vc + V(i, j, k - 1)) * g.cz;
        const float sgs = 2.f * (n12(i, j, k) * e12(i, j, k) - n12(i - 1, j, k) * e12(i - 1, j, k)) * g.idx +
                          2.f * (N(i, j + 1, k) * (vp - vc) * g.idy - N(i, j, k) * (vc - vm) * g.idy) * g.idy +
                          2.f * (n23(i, j, k) * e23(i, j, k) - n23(i, j, k - 1) * e23(i, j, k - 1)) * g.idz;
        float F = -(covx + covy + covz) + nu * lap + sgs;
        if (fl & F_VSOLID) {
            const float s = sv[e] + dt * vc;
            sv[e] = s;
            F += alpha * s + beta * vc;
        }
        const float fo = first ? F : fv[e];
        vs[e] = vc + dt * (1.5f * F - 0.5f * fo);
        fv[e] = F;
    }
    if (k <= g.nz - 1) {
        const float wc = W(i, j, k);
        const float wm = W(i, j, k - 1), wp = W(i, j, k + 1);
        const float covx = 0.5f * (0.5f * (U(i - 1, j, k) + U(i - 1, j, k + 1)) * (wc - W(i - 1, j, k)) +
                                   0.5f * (U(i, j, k) + U(i, j, k + 1)) * (W(i + 1, j, k) - wc)) * g.idx;
        const float covy = 0.5f * (0.5f * (V(i, j - 1, k) + V(i, j - 1, k + 1)) * (wc - W(i, j - 1, k)) +
                                   0.5f * (V(i, j, k) + V(i, j, k + 1)) * (W(i, j + 1, k) - wc)) * g.idy;
        const float covz = 0.5f * (0.5f * (wm + wc) * (wc - wm) + 0.5f * (wc + wp) * (wp - wc)) * g.idz;
        const float lap = (W(i + 1, j, k) - 2.f * wc + W(i - 1, j, k)) * g.cx +
                          (W(i, j + 1, k) - 2.f * wc + W(i, j - 1, k)) * g.cy + (wp - 2.f * wc + wm) * g.cz;
        const float sgs = 2.f * (n13(i, j, k) * e13(i, j, k) - n13(i - 1, j, k) * e13(i - 1, j, k)) * g.idx +
                          2.f * (n23(i, j, k) * e23(i, j, k) - n23(i, j - 1, k) * e23(i, j - 1, k)) * g.idy +
                          2.f * (N(i, j, k + 1) * (wp - wc) * g.idz - N(i, j, k) * (wc - wm) * g.idz) * g.idz;
        float F = -(covx + covy + covz) + nu * lap + sgs;
        if (fl & F_WSOLID) {
            const float s = sw[e] + dt * wc;
            sw[e] = s;
            F += alpha * s + beta * wc;
        }
        const float fo = first ? F : fw[e];
        ws[e] = wc + dt * (1.5f * F - 0.5f * fo);
        fw[e] = F;
    }
}

// --------------------------------------------------------- bondv1: inflow
// splitmix64 (Steele, Lea & Flood 2014): output of the generator whose
// state is x.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// u*(0, j, k) = U(k) (1 + a (2 xi - 1)) on fluid inflow faces, 0 on solid
// ones; xi = top 24 bits of splitmix64(seed ^ (step 2^40 + k0 2^20 + j0)).
__global__ __launch_bounds__(kBlock) void k_inflow(Geo g, float* __restrict__ us,
                                                   const float* __restrict__ prof,
                                                   const uint8_t* __restrict__ flags, float amp,
                                                   uint64_t seed, long long step) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.ny * g.nz) return;
    const int k0 = t / g.ny, j0 = t - k0 * g.ny;
    const uint64_t ctr = ((uint64_t)step << 40) + ((uint64_t)k0 << 20) + (uint64_t)j0;
    const uint64_t r = splitmix64(seed ^ ctr);
    const float xi = (float)(r >> 40) * (1.0f / 16777216.0f);
    const bool solid = (flags[g.nat(1, j0 + 1, k0 + 1)] & F_CSOLID) != 0;
    us[g.nat(0, j0 + 1, k0 + 1)] = solid ? 0.f : prof[k0] * (1.f + amp * (2.f * xi - 1.f));
}

// ---------------------------------------------------------- control block
__global__ void k_ctl_init(Ctl* ctl, double tol, int max_iter, int K) {
    if (threadIdx.x == 0) {
        ctl->done = 0;
        ctl->m = 0;
        ctl->K = K;
        ctl->max_iter = max_iter;
        ctl->tol = tol;
        ctl->rhs2 = 0.0;
        ctl->rhs_sum = 0.0;
        ctl->resid = 0.0;
        ctl->reltmp2 = 0.0;
        ctl->skip = 0;
    }
}

// -------------------------------------------------------- press: the rhs
// rhs = div(u*) / dt at every cell, stored in the colour layout; float64
// sum of rhs^2 (or of rhs, when the operator is singular and the mean has
// to go first) reduced by the last block into the control block.
__global__ __launch_bounds__(kBlock) void k_rhs(Geo g, const float* __restrict__ us,
                                                const float* __restrict__ vs,
                                                const float* __restrict__ ws, float* rhs0,
                                                float* rhs1, double* __restrict__ part,
                                                int singular) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    double acc = 0.0;
    if (t < n) {
        int i, j, k;
        cell_of(g, t, i, j, k);
        const float div = (us[g.nat(i, j, k)] - us[g.nat(i - 1, j, k)]) * g.idx +
                          (vs[g.nat(i, j, k)] - vs[g.nat(i, j - 1, k)]) * g.idy +
                          (ws[g.nat(i, j, k)] - ws[g.nat(i, j, k - 1)]) * g.idz;
        const float r = div * g.idt;
        const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
        float* dst = ((i0 + j0 + k0) & 1) ? rhs1 : rhs0;
        dst[g.col(i0 >> 1, j0, k0)] = r;
        acc = singular ? (double)r : (double)r * (double)r;
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
}

// Singular operator: subtract the mean of rhs, then sum rhs^2.
__global__ __launch_bounds__(kBlock) void k_rhs_mean(Geo g, float* rhs0, float* rhs1,
                                                     double* __restrict__ part, Ctl* ctl) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    const float mean = (float)(ctl->rhs_sum / (double)n);
    double acc = 0.0;
    if (t < n) {
        int i, j, k;
        cell_of(g, t, i, j, k);
        const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
        float* dst = ((i0 + j0 + k0) & 1) ? rhs1 : rhs0;
        const long long e = g.col(i0 >> 1, j0, k0);
        const float r = dst[e] - mean;
        dst[e] = r;
        acc = (double)r * (double)r;
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
}

// ------------------------------------------------------- velnw: projection
// u = u* - dt grad p on faces between two cells and on the outflow face,
// where p = 0 on the face (ghost -p).  p is the pair base + correction of
// the pressure solve; differences are taken pairwise before the sum so
// the gradient keeps the correction's precision.
__global__ __launch_bounds__(kBlock) void k_project(Geo g, float* __restrict__ us,
                                                    float* __restrict__ vs, float* __restrict__ ws,
                                                    const float* __restrict__ ph0,
                                                    const float* __restrict__ ph1,
                                                    const float* __restrict__ pd0,
                                                    const float* __restrict__ pd1) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
    const int c = (i0 + j0 + k0) & 1;
    const float* phc = c ? ph1 : ph0;
    const float* pdc = c ? pd1 : pd0;
    const float* pho = c ? ph0 : ph1;   // neighbours have the other colour
    const float* pdo = c ? pd0 : pd1;
    const long long ec = g.col(i0 >> 1, j0, k0);
    const float hc = phc[ec], dc = pdc[ec];
    const float dt = g.dt;
    const long long e = g.nat(i, j, k);
    if (i0 + 1 < g.nx) {
        const long long en = g.col((i0 + 1) >> 1, j0, k0);
        us[e] -= dt * (((pho[en] - hc) + (pdo[en] - dc)) * g.idx);
    } else if (g.outflow) {
        us[e] -= dt * ((-2.f * hc - 2.f * dc) * g.idx);
    }
    if (j0 + 1 < g.ny) {
        const long long en = ec + g.S;
        vs[e] -= dt * (((pho[en] - hc) + (pdo[en] - dc)) * g.idy);
    }
    if (k0 + 1 < g.nz) {
        const long long en = ec + g.SP;
        ws[e] -= dt * (((pho[en] - hc) + (pdo[en] - dc)) * g.idz);
    }
}

// ------------------------------------------------ bondv1: ghost refresh
// One launch over the boundary range of section 2.4: (ny+2)(nz+2) items
// for the x faces, nx(nz+2) for the y faces and nx ny for the z faces,
// split by the item id; each item fills the low and the high ghost of its
// family for u, v and w.  Every ghost value is composed directly from an
// owned value (per axis: copy, negate or zero), so items never read what
// another item writes and edges/corners need no ordering.
struct AxisMap {
    int src;
    float sgn;
    bool ghost;
    bool zero;
};

__device__ __forceinline__ AxisMap map_x(const Geo& g, int comp, int i) {
    if (comp == 0) {   // u: owned faces 0..nx, ghost nx+1
        if (i == g.nx + 1) return {g.nx, 1.f, true, !g.outflow};
        return {i, 1.f, false, false};
    }
    if (i == 0) return {1, g.s_xm, true, false};
    if (i == g.nx + 1) return {g.nx, g.s_xp, true, false};
    return {i, 1.f, false, false};
}
__device__ __forceinline__ AxisMap map_y(const Geo& g, int comp, int j) {
    if (comp == 1) {   // v: owned faces 0..ny (0, ny walls), ny+1 unused
        if (j == g.ny + 1) return {j, 0.f, true, true};
        return {j, 1.f, false, false};
    }
    if (j == 0) return {1, g.s_ym, true, false};
    if (j == g.ny + 1) return {g.ny, g.s_yp, true, false};
    return {j, 1.f, false, false};
}
__device__ __forceinline__ AxisMap map_z(const Geo& g, int comp, int k) {
    if (comp == 2) {   // w: owned faces 0..nz (0, nz walls), nz+1 unused
        if (k == g.nz + 1) return {k, 0.f, true, true};
        return {k, 1.f, false, false};
    }
    if (k == 0) return {1, g.s_zm, true, false};
    if (k == g.nz + 1) return {g.nz, g.s_zp, true, false};
    return {k, 1.f, false, false};
}

__device__ __forceinline__ void fill_ghost(const Geo& g, float* f, int comp, int i, int j, int k) {
    const AxisMap ax = map_x(g, comp, i), ay = map_y(g, comp, j), az = map_z(g, comp, k);
    if (!(ax.ghost || ay.ghost || az.ghost)) return;   // owned value: untouched
    float val = 0.f;
    if (!(ax.zero || ay.zero || az.zero)) val = ax.sgn * ay.sgn * az.sgn * f[g.nat(ax.src, ay.src, az.src)];
    f[g.nat(i, j, k)] = val;
}

__global__ __launch_bounds__(kBlock) void k_bc(Geo g, float* u, float* v, float* w) {
    const long long id = (long long)blockIdx.x * kBlock + threadIdx.x;
    int fam, a, b;
    bc_item(g.nx, g.ny, g.nz, id, fam, a, b);
    if (fam < 0) return;   // guarded padding of the launch
    int p0[3], p1[3];
    if (fam == 0) {        // (j, k) = (a, b); i = 0 and nx+1
        p0[0] = 0; p0[1] = a; p0[2] = b;
        p1[0] = g.nx + 1; p1[1] = a; p1[2] = b;
    } else if (fam == 1) { // (i, k) = (a, b); j = 0 and ny+1
        p0[0] = a; p0[1] = 0; p0[2] = b;
        p1[0] = a; p1[1] = g.ny + 1; p1[2] = b;
    } else {               // (i, j) = (a, b); k = 0 and nz+1
        p0[0] = a; p0[1] = b; p0[2] = 0;
        p1[0] = a; p1[1] = b; p1[2] = g.nz + 1;
    }
    fill_ghost(g, u, 0, p0[0], p0[1], p0[2]);
    fill_ghost(g, v, 1, p0[0], p0[1], p0[2]);
    fill_ghost(g, w, 2, p0[0], p0[1], p0[2]);
    fill_ghost(g, u, 0, p1[0], p1[1], p1[2]);
    fill_ghost(g, v, 1, p1[0], p1[1], p1[2]);
    fill_ghost(g, w, 2, p1[0], p1[1], p1[2]);
}

// --------------------------------------------------- diagnostics (norms)
// sum div(u)^2 over the cells (float64) and max CFL = dt (|u|/dx + |v|/dy
// + |w|/dz) with cell-centred speeds.
__global__ __launch_bounds__(kBlock) void k_diag(Geo g, const float* __restrict__ u,
                                                 const float* __restrict__ v,
                                                 const float* __restrict__ w,
                                                 double* __restrict__ part) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    double d2 = 0.0, cf = 0.0;
    if (t < n) {
        int i, j, k;
        cell_of(g, t, i, j, k);
        const float u1 = u[g.nat(i, j, k)], u0 = u[g.nat(i - 1, j, k)];
        const float v1 = v[g.nat(i, j, k)], v0 = v[g.nat(i, j - 1, k)];
        const float w1 = w[g.nat(i, j, k)], w0 = w[g.nat(i, j, k - 1)];
        const double div = ((double)u1 - u0) / g.dx + ((double)v1 - v0) / g.dy + ((double)w1 - w0) / g.dz;
        d2 = div * div;
        cf = (double)g.dt * (0.5 * fabs((double)u1 + u0) / g.dx + 0.5 * fabs((double)v1 + v0) / g.dy +
                             0.5 * fabs((double)w1 + w0) / g.dz);
    }
    const double s = block_sum(d2);
    const double mx = block_max(cf);
    if (threadIdx.x == 0) {
        part[2 * lb] = s;
        part[2 * lb + 1] = mx;
    }
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

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t launch_nut(const Geo& g, hipStream_t st, const float* u, const float* v,
                      const float* w, float* nut, float c2) {
    const long long nbox = (long long)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
    hipLaunchKernelGGL(k_nut, dim3(nblocks(nbox)), dim3(kBlock), 0, st, g, u, v, w, nut, c2);
    return hipGetLastError();
}

hipError_t launch_tendency(const Geo& g, hipStream_t st, const float* u, const float* v,
                           const float* w, const float* nut, float* fu, float* fv, float* fw,
                           float* su, float* sv, float* sw, const uint8_t* flags, float* us,
                           float* vs, float* ws, float nu, float alpha, float beta, int first) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_tendency, dim3(nblocks(n)), dim3(kBlock), 0, st, g, u, v, w, nut, fu,
                       fv, fw, su, sv, sw, flags, us, vs, ws, nu, alpha, beta, first);
    return hipGetLastError();
}

hipError_t launch_inflow(const Geo& g, hipStream_t st, float* us, const float* prof,
                         const uint8_t* flags, float amp, uint64_t seed, int64_t step) {
    hipLaunchKernelGGL(k_inflow, dim3(nblocks((long long)g.ny * g.nz)), dim3(kBlock), 0, st, g,
                       us, prof, flags, amp, seed, (long long)step);
    return hipGetLastError();
}

hipError_t launch_ctl_init(hipStream_t st, Ctl* ctl, double tol, int max_iter, int K) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, ctl, tol, max_iter, K);
    return hipGetLastError();
}

hipError_t launch_rhs(const Geo& g, hipStream_t st, const float* us, const float* vs,
                      const float* ws, float* const rhs[2], double* part, Ctl* ctl,
                      int singular) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_rhs, dim3(nblocks(n)), dim3(kBlock), 0, st, g, us, vs, ws, rhs[0],
                       rhs[1], part, singular);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, singular ? FIN_RHS_SUM : FIN_RHS2, part, (int)nblocks(n), nullptr,
                           nullptr, 0, ctl);
}

hipError_t launch_remove_mean_rhs(const Geo& g, hipStream_t st, float* const rhs[2],
                                  double* part, Ctl* ctl) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_rhs_mean, dim3(nblocks(n)), dim3(kBlock), 0, st, g, rhs[0], rhs[1],
                       part, ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, FIN_RHS2, part, (int)nblocks(n), nullptr, nullptr, 0, ctl);
}

hipError_t launch_project(const Geo& g, hipStream_t st, float* us, float* vs, float* ws,
                          const PBufs& P) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_project, dim3(nblocks(n)), dim3(kBlock), 0, st, g, us, vs, ws, P.ph[0],
                       P.ph[1], P.pd[0], P.pd[1]);
    return hipGetLastError();
}

hipError_t launch_bc(const Geo& g, hipStream_t st, float* u, float* v, float* w) {
    const long long items = bc_items(g.nx, g.ny, g.nz);
    hipLaunchKernelGGL(k_bc, dim3(nblocks(items)), dim3(kBlock), 0, st, g, u, v, w);
    return hipGetLastError();
}

hipError_t launch_diag(const Geo& g, hipStream_t st, const float* u, const float* v,
                       const float* w, double* part, Ctl* ctl) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_diag, dim3(nblocks(n)), dim3(kBlock), 0, st, g, u, v, w, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(st, FIN_DIAG, part, (int)nblocks(n), nullptr, nullptr, 0, ctl);
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
