// Device bodies of every LES kernel, parameterized by the logical block
// index so that the same per-cell arithmetic runs in the single-instance
// launches (kernels_step.hip, kernels_sor.hip) and in the batched and
// persistent ensemble launches (ensemble.hip).
//
// Staggered (MAC) grid: u on x-faces, v on y-faces, w on z-faces, scalars
// at cell centres; layouts in les_impl.h.  All fields float32, all norms
// float64.
#pragma once

#include <type_traits>

#include "device_util.h"
#include "les_impl.h"

namespace les {

// Reductions over the H * ny * nz half-cells use at most kRedBlocks blocks;
// block L owns one contiguous chunk of half-cells, walked by its threads
// with unit stride, so finalizing sums few partials.
constexpr unsigned kRedBlocks = 2048;
// grid of the residual check, which mostly returns at once (skipped by the
// bound): fewer blocks to dispatch, still two per compute unit
constexpr unsigned kCheckBlocks = 512;
inline unsigned red_blocks(const Geo& g) {
    const long long n = (long long)g.H * g.ny * g.nz;
    const long long b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < (long long)kRedBlocks ? b : (long long)kRedBlocks);
}
inline unsigned check_blocks(const Geo& g) {
    const unsigned r = red_blocks(g);
    return r < kCheckBlocks ? r : kCheckBlocks;
}
inline unsigned cell_blocks(const Geo& g) {
    return (unsigned)(((long long)g.nx * g.ny * g.nz + kBlock - 1) / kBlock);
}
inline unsigned half_blocks(const Geo& g) {
    return (unsigned)(((long long)g.H * g.ny * g.nz + kBlock - 1) / kBlock);
}
inline unsigned box_blocks(const Geo& g) {   // one thread per cell of the ghosted box
    return (unsigned)(((long long)(g.nx + 2) * (g.ny + 2) * (g.nz + 2) + kBlock - 1) / kBlock);
}
inline unsigned bc_blocks(const Geo& g) {
    return (unsigned)((bc_items(g.nx, g.ny, g.nz) + kBlock - 1) / kBlock);
}

__device__ __forceinline__ void red_chunk(const Geo& g, unsigned lb, unsigned nb, long long& t0,
                                          long long& t1) {
    const long long n = (long long)g.H * g.ny * g.nz;
    const long long chunk = ((n + nb - 1) / nb + kBlock - 1) / kBlock * kBlock;
    t0 = (long long)lb * chunk;
    t1 = (t0 + chunk < n) ? t0 + chunk : n;
}

// Linear interior-cell index (0-based, x fastest) -> 1-based cell coordinates.
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

// Linear half-cell index -> colour-array coordinates (ii, j0, k0).
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

// Diagonal of A at 0-based cell (i0, j0, k0): 1/h^2 per interior neighbour,
// nothing across a wall or the inflow face (Neumann), 2/h^2 across the
// outflow face (p = 0 on the face); its x, y and z parts, summed in that
// order.
__device__ __forceinline__ float diag_x(const Geo& g, int i0) {
    return (i0 > 0 ? g.cx : 0.f) + (i0 < g.nx - 1 ? g.cx : (g.outflow ? 2.f * g.cx : 0.f));
}
__device__ __forceinline__ float diag_y(const Geo& g, int j0) {
    return (j0 > 0 ? g.cy : 0.f) + (j0 < g.ny - 1 ? g.cy : 0.f);
}
__device__ __forceinline__ float diag_z(const Geo& g, int k0) {
    return (k0 > 0 ? g.cz : 0.f) + (k0 < g.nz - 1 ? g.cz : 0.f);
}
__device__ __forceinline__ float diag_of(const Geo& g, int i0, int j0, int k0) {
    return diag_x(g, i0) + diag_y(g, j0) + diag_z(g, k0);
}

// Row `row` of an axis' metric table at 1-based index c (tables of n + 2
// entries per row; MetricRow in les_impl.h).
__device__ __forceinline__ float mrow(const float* __restrict__ m, int n, int row, int c) {
    return m[row * (n + 2) + c];
}

// ------------------------------------------------ les + velfg + feedbf + adam
// Smagorinsky eddy viscosity (section 2.1, les): nu_t = (Cs Delta)^2 |S|,
// |S| = sqrt(2 S_ij S_ij); S_ii from the two faces of the cell, S_ij (i != j)
// the mean of the four edge values around the cell, each edge value being
// 1/2 (du_i/dx_j + du_j/dx_i) from the adjacent faces; a ghost cell takes
// the value of the nearest interior cell (mirrored ghost ring).
//
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
struct TendArgs {
    const float* u; const float* v; const float* w; const float* nut;
    float* fu; float* fv; float* fw;
    float* su; float* sv; float* sw;
    const uint8_t* flags;
    float* us; float* vs; float* ws;
    float nu, alpha, beta;
    int first;
};

// ------------------------- les + velfg + feedbf + adam, fused, LDS-tiled
// One pass over the grid instead of two: a block owns a tile of kTileX x
// kTileY cells and marches up its chunk of planes.  Every velocity plane
// is read from HBM once into LDS with a two-cell ring (u, v, w; kTileVS
// planes in a ring buffer), nu_t is computed into LDS on the tile plus a
// one-cell ring (three planes), and the tendency, feedback forcing and AB2
// of the tile's cells read both from LDS.  nu_t of the tile's own cells is
// also stored (the les_get_aux diagnostic); the tendency never reads it
// back.  Per-cell arithmetic as described above; ghost-ring nu_t is the
// value of the nearest interior cell.
//
// March of a block over tendency planes [kb, ke): step p loads velocity
// plane p+1 into registers (issued a step ahead), publishes plane p, then
// after a barrier computes nu_t on plane p-1 and after a second barrier
// the tendency on plane p-2; a third barrier ends the step.  Four velocity
// slots then keep the slot written at step p (last read by the tendency of
// step p-1) clear of readers, and three nu_t slots likewise; the smaller
// ring (47 KB) lets three blocks share a compute unit instead of two.
constexpr int kTileX = 64, kTileY = 8;
constexpr int kTileThreads = kTileX * kTileY;   // one wavefront per tile row
constexpr int kTileLX = kTileX + 4, kTileLY = kTileY + 4;   // velocity: two-cell ring
constexpr int kTileNX = kTileX + 2, kTileNY = kTileY + 2;   // nu_t: one-cell ring
constexpr int kTileVS = 4;   // velocity plane slots
constexpr int kTileVel = kTileLX * kTileLY;     // entries of one velocity plane
constexpr int kTileNut = kTileNX * kTileNY;

// Planes per block on grid g: the most (32, 16 or 8) that still give at
// least two blocks per compute unit.
inline int tile_kt(const Geo& g) {
    const long long nxy = (long long)((g.nx + kTileX - 1) / kTileX) * ((g.ny + kTileY - 1) / kTileY);
    for (int kt = 32; kt > 8; kt /= 2)
        if (nxy * ((g.nz + kt - 1) / kt) >= 512) return kt;
    return 8;
}
inline unsigned tile_blocks(const Geo& g) {
    const int kt = tile_kt(g);
    return (unsigned)((g.nx + kTileX - 1) / kTileX) * (unsigned)((g.ny + kTileY - 1) / kTileY) *
           (unsigned)((g.nz + kt - 1) / kt);
}

struct TileShared {
    float vel[kTileVS][3][kTileLY][kTileLX];
    float nut[3][kTileNY][kTileNX];
};

__device__ __forceinline__ void step_tile_body(const Geo& g, const TendArgs& A, float* __restrict__ nut_out,
                                               float c2, int kt, unsigned lb, TileShared& sh) {
    const int ntx = (g.nx + kTileX - 1) / kTileX, nty = (g.ny + kTileY - 1) / kTileY;
    const int bx = (int)(lb % (unsigned)ntx);
    const unsigned rr = lb / (unsigned)ntx;
    const int by = (int)(rr % (unsigned)nty), bz = (int)(rr / (unsigned)nty);
    const int i0 = bx * kTileX + 1, j0 = by * kTileY + 1;   // first (1-based) cell of the tile
    const int kb = bz * kt + 1, ke = min(kb + kt, g.nz + 1);   // tendency planes [kb, ke)
    const int tid = threadIdx.x;
    const int lane = tid & 63, row = tid >> 6;
    const float* __restrict__ gu = A.u;
    const float* __restrict__ gv = A.v;
    const float* __restrict__ gw = A.w;

    // LDS views (global 1-based indices)
    auto vs = [](int k) { return (k + 2 * kTileVS) % kTileVS; };
    auto U = [&](int a, int b, int c) { return sh.vel[vs(c)][0][b - j0 + 2][a - i0 + 2]; };
    auto V = [&](int a, int b, int c) { return sh.vel[vs(c)][1][b - j0 + 2][a - i0 + 2]; };
    auto W = [&](int a, int b, int c) { return sh.vel[vs(c)][2][b - j0 + 2][a - i0 + 2]; };
    auto N = [&](int a, int b, int c) {
        const int cc = min(max(c, 1), g.nz);   // ghost planes: the nearest interior plane
        return sh.nut[cc % 3][b - j0 + 1][a - i0 + 1];
    };

    // one velocity plane: entries tid and tid + kTileThreads of the ring tile
    float reg[2][3];
    auto fetch = [&](int p) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = tid + r * kTileThreads;
            const int i = i0 - 2 + e % kTileLX, j = j0 - 2 + e / kTileLX;
            const bool ok = e < kTileVel && p >= 0 && p <= g.nz + 1 && i >= 0 && i <= g.nx + 1 &&
                            j >= 0 && j <= g.ny + 1;
            const long long x = ok ? g.nat(i, j, p) : 0;
            reg[r][0] = ok ? gu[x] : 0.f;
            reg[r][1] = ok ? gv[x] : 0.f;
            reg[r][2] = ok ? gw[x] : 0.f;
        }
    };
    auto publish = [&](int p) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = tid + r * kTileThreads;
            if (e < kTileVel) {
                const int ly = e / kTileLX, lx = e % kTileLX;
#pragma unroll
                for (int c = 0; c < 3; ++c) sh.vel[vs(p)][c][ly][lx] = reg[r][c];
            }
        }
    };

    fetch(kb - 2);
    for (int p = kb - 2; p <= ke + 1; ++p) {
        publish(p);
        if (p <= ke) fetch(p + 1);
        __syncthreads();
        // nu_t on plane c = p - 1 over the tile and its ring (interior planes only)
        const int c = p - 1;
        if (c >= kb - 1 && c <= ke && c >= 1 && c <= g.nz) {
            for (int e = tid; e < kTileNut; e += kTileThreads) {
                const int ny_ = e / kTileNX, nx_ = e % kTileNX;
                const int ia = i0 - 1 + nx_, jb = j0 - 1 + ny_;
                const int ic = min(max(ia, 1), g.nx), jc = min(max(jb, 1), g.ny), kc = c;
                const float s11 = (U(ic, jc, kc) - U(ic - 1, jc, kc)) * g.idx;
                const float s22 = (V(ic, jc, kc) - V(ic, jc - 1, kc)) * g.idy;
                const float s33 = (W(ic, jc, kc) - W(ic, jc, kc - 1)) * g.idz;
                float s12 = 0.f, s13 = 0.f, s23 = 0.f;
#pragma unroll
                for (int da = -1; da <= 0; ++da)
#pragma unroll
                    for (int db = -1; db <= 0; ++db) {
                        const int a = ic + da, b = jc + db;
                        s12 += (U(a, b + 1, kc) - U(a, b, kc)) * g.idy + (V(a + 1, b, kc) - V(a, b, kc)) * g.idx;
                        const int cz = kc + db;
                        s13 += (U(a, jc, cz + 1) - U(a, jc, cz)) * g.idz + (W(a + 1, jc, cz) - W(a, jc, cz)) * g.idx;
                        const int b2 = jc + da;
                        s23 += (V(ic, b2, cz + 1) - V(ic, b2, cz)) * g.idz + (W(ic, b2 + 1, cz) - W(ic, b2, cz)) * g.idy;
                    }
                s12 *= 0.125f;
                s13 *= 0.125f;
                s23 *= 0.125f;
                const float ss = 2.f * (s11 * s11 + s22 * s22 + s33 * s33) +
                                 4.f * (s12 * s12 + s13 * s13 + s23 * s23);
                const float nt = c2 * sqrtf(ss);
                sh.nut[c % 3][ny_][nx_] = nt;
                if (c >= kb && c < ke && nx_ >= 1 && nx_ <= kTileX && ny_ >= 1 && ny_ <= kTileY &&
                    ia <= g.nx && jb <= g.ny)
                    nut_out[g.nat(ia, jb, c)] = nt;
            }
        }
        __syncthreads();
        // tendency, feedback forcing and AB2 on plane k = p - 2
        const int k = p - 2, i = i0 + lane, j = j0 + row;
        if (k >= kb && k < ke && i <= g.nx && j <= g.ny) {
            auto n12 = [&](int a, int b, int cc) { return 0.25f * (N(a, b, cc) + N(a + 1, b, cc) + N(a, b + 1, cc) + N(a + 1, b + 1, cc)); };
            auto n13 = [&](int a, int b, int cc) { return 0.25f * (N(a, b, cc) + N(a + 1, b, cc) + N(a, b, cc + 1) + N(a + 1, b, cc + 1)); };
            auto n23 = [&](int a, int b, int cc) { return 0.25f * (N(a, b, cc) + N(a, b + 1, cc) + N(a, b, cc + 1) + N(a, b + 1, cc + 1)); };
            auto e12 = [&](int a, int b, int cc) { return 0.5f * ((U(a, b + 1, cc) - U(a, b, cc)) * g.idy + (V(a + 1, b, cc) - V(a, b, cc)) * g.idx); };
            auto e13 = [&](int a, int b, int cc) { return 0.5f * ((U(a, b, cc + 1) - U(a, b, cc)) * g.idz + (W(a + 1, b, cc) - W(a, b, cc)) * g.idx); };
            auto e23 = [&](int a, int b, int cc) { return 0.5f * ((V(a, b, cc + 1) - V(a, b, cc)) * g.idz + (W(a, b + 1, cc) - W(a, b, cc)) * g.idy); };
            const long long e = g.nat(i, j, k);
            const uint8_t fl = A.flags[e];
            const float dt = g.dt;
            const float nu = A.nu, alpha = A.alpha, beta = A.beta;
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
                    const float s = A.su[e] + dt * uc;
                    A.su[e] = s;
                    F += alpha * s + beta * uc;
                }
                const float fo = A.first ? F : A.fu[e];
                A.us[e] = uc + dt * (1.5f * F - 0.5f * fo);
                A.fu[e] = F;
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
                    const float s = A.sv[e] + dt * vc;
                    A.sv[e] = s;
                    F += alpha * s + beta * vc;
                }
                const float fo = A.first ? F : A.fv[e];
                A.vs[e] = vc + dt * (1.5f * F - 0.5f * fo);
                A.fv[e] = F;
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
                    const float s = A.sw[e] + dt * wc;
                    A.sw[e] = s;
                    F += alpha * s + beta * wc;
                }
                const float fo = A.first ? F : A.fw[e];
                A.ws[e] = wc + dt * (1.5f * F - 0.5f * fo);
                A.fw[e] = F;
            }
        }
        __syncthreads();   // the tendency's reads of this step end before the next publish
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
// U(k) = U0(k) + wt (U1(k) - U0(k)), the linear interpolation in time
// between two profile samples (wt = 0 gives U0 exactly).
__device__ __forceinline__ void inflow_body(const Geo& g, float* __restrict__ us,
                                            const float* __restrict__ prof,
                                            const float* __restrict__ prof1, float wt,
                                            const uint8_t* __restrict__ flags, float amp,
                                            uint64_t seed, long long step, unsigned lb) {
    const int t = (int)(lb * kBlock + threadIdx.x);
    if (t >= g.ny * g.nz) return;
    const int k0 = t / g.ny, j0 = t - k0 * g.ny;
    const uint64_t ctr = ((uint64_t)step << 40) + ((uint64_t)k0 << 20) + (uint64_t)j0;
    const uint64_t r = splitmix64(seed ^ ctr);
    const float xi = (float)(r >> 40) * (1.0f / 16777216.0f);
    const bool solid = (flags[g.nat(1, j0 + 1, k0 + 1)] & F_CSOLID) != 0;
    const float U = prof[k0] + wt * (prof1[k0] - prof[k0]);
    us[g.nat(0, j0 + 1, k0 + 1)] = solid ? 0.f : U * (1.f + amp * (2.f * xi - 1.f));
}

__device__ __forceinline__ void ctl_init_body(Ctl* ctl, double tol, int max_iter, int K) {
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
// rhs = div(u*) / dt at every cell, stored in the colour layout; one
// float64 partial per block of sum rhs^2 (or of rhs when the operator is
// singular and the mean has to go first).
__device__ __forceinline__ void rhs_body(const Geo& g, const float* __restrict__ us,
                                         const float* __restrict__ vs, const float* __restrict__ ws,
                                         float* rhs0, float* rhs1, double* __restrict__ part,
                                         int singular, unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
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

// Singular operator: subtract the mean of rhs (from ctl->rhs_sum), then
// leave partials of sum rhs^2.
__device__ __forceinline__ void rhs_mean_body(const Geo& g, float* rhs0, float* rhs1,
                                              double* __restrict__ part, const Ctl* ctl,
                                              unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
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
__device__ __forceinline__ void project_body(const Geo& g, float* __restrict__ us,
                                             float* __restrict__ vs, float* __restrict__ ws,
                                             const PBufs& P, unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)lb * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
    const int c = (i0 + j0 + k0) & 1;
    const float* __restrict__ phc = P.ph[c];
    const float* __restrict__ pdc = P.pd[c];
    const float* __restrict__ pho = P.ph[1 - c];   // neighbours have the other colour
    const float* __restrict__ pdo = P.pd[1 - c];
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
// One item of the boundary range of section 2.4: (ny+2)(nz+2) items for
// the x faces, nx(nz+2) for the y faces and nx ny for the z faces, split by
// the item id; each item fills the low and the high ghost of its family
// for u, v and w.  Every ghost value is composed directly from an owned
// value (per axis: copy, negate or zero), so items never read what another
// item writes and edges/corners need no ordering.
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

__device__ __forceinline__ void bc_body(const Geo& g, float* u, float* v, float* w, unsigned lb) {
    const long long id = (long long)lb * kBlock + threadIdx.x;
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

// ============================================== stretched grids (bodies)
// The same stages on a grid whose axes carry per-cell widths (the 1-D
// spacing arrays dx1 / dy1 / dzn of section 2.5.3).  Every difference is
// taken over the distance between the two values it spans: a cell width
// (M_IH) between the two faces of a cell, a centre distance (M_IG) across
// a face; a cell-centred quantity reaches a face of its own axis by the
// width-weighted linear interpolation (M_LO, M_HI: the paper's covx1
// weights), an edge by the plain mean of the two values around it (the
// edge is their midpoint).  Uniform grids keep the scalar-spacing bodies
// above; a uniform table reproduces them up to rounding.
struct StrAxis {
    const float* ih; const float* ig; const float* lo; const float* hi; const float* h23;
};
__device__ __forceinline__ StrAxis str_axis(const float* m, int n) {
    const int L = n + 2;
    return {m + M_IH * L, m + M_IG * L, m + M_LO * L, m + M_HI * L, m + M_H23 * L};
}

// Smagorinsky nu_t on a stretched grid: (Cs Delta)^2 |S| with the cell's
// own filter width Delta = (hx hy hz)^(1/3), i.e. Cs^2 hx^(2/3) hy^(2/3)
// hz^(2/3); strain components as in the uniform pass, each difference
// over its own distance.  Ghost ring: the nearest interior cell's value.
__device__ __forceinline__ void nut_body_str(const Geo& g, const float* __restrict__ u,
                                             const float* __restrict__ v, const float* __restrict__ w,
                                             float* __restrict__ nut, float cs2, unsigned lb) {
    const long long nbox = (long long)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
    const long long t = (long long)lb * kBlock + threadIdx.x;
    if (t >= nbox) return;
    const unsigned pxy = (unsigned)(g.nx + 2) * (unsigned)(g.ny + 2);
    const unsigned tt = (unsigned)t;
    const int k = (int)(tt / pxy);
    const unsigned r = tt - (unsigned)k * pxy;
    const int j = (int)(r / (unsigned)(g.nx + 2));
    const int i = (int)(r - (unsigned)j * (unsigned)(g.nx + 2));
    const int ic = min(max(i, 1), g.nx), jc = min(max(j, 1), g.ny), kc = min(max(k, 1), g.nz);
    const StrAxis X = str_axis(g.mx, g.nx), Y = str_axis(g.my, g.ny), Z = str_axis(g.mz, g.nz);
    auto U = [&](int a, int b, int c) { return u[g.nat(a, b, c)]; };
    auto V = [&](int a, int b, int c) { return v[g.nat(a, b, c)]; };
    auto W = [&](int a, int b, int c) { return w[g.nat(a, b, c)]; };
    const float s11 = (U(ic, jc, kc) - U(ic - 1, jc, kc)) * X.ih[ic];
    const float s22 = (V(ic, jc, kc) - V(ic, jc - 1, kc)) * Y.ih[jc];
    const float s33 = (W(ic, jc, kc) - W(ic, jc, kc - 1)) * Z.ih[kc];
    float s12 = 0.f, s13 = 0.f, s23 = 0.f;
#pragma unroll
    for (int da = -1; da <= 0; ++da)
#pragma unroll
        for (int db = -1; db <= 0; ++db) {
            const int a = ic + da, b = jc + db;   // x-y edge (face a, face b)
            s12 += (U(a, b + 1, kc) - U(a, b, kc)) * Y.ig[b] + (V(a + 1, b, kc) - V(a, b, kc)) * X.ig[a];
            const int c = kc + db;                // x-z edge (face a, face c)
            s13 += (U(a, jc, c + 1) - U(a, jc, c)) * Z.ig[c] + (W(a + 1, jc, c) - W(a, jc, c)) * X.ig[a];
            const int b2 = jc + da;               // y-z edge (face b2, face c)
            s23 += (V(ic, b2, c + 1) - V(ic, b2, c)) * Z.ig[c] + (W(ic, b2 + 1, c) - W(ic, b2, c)) * Y.ig[b2];
        }
    s12 *= 0.125f;
    s13 *= 0.125f;
    s23 *= 0.125f;
    const float ss = 2.f * (s11 * s11 + s22 * s22 + s33 * s33) + 4.f * (s12 * s12 + s13 * s13 + s23 * s23);
    const float c2 = cs2 * (X.h23[ic] * Y.h23[jc] * Z.h23[kc]);
    nut[g.nat(i, j, k)] = c2 * sqrtf(ss);
}

// velfg + feedbf + adam on a stretched grid: for each face value, the
// tendency is assembled on its own control volume (for u on face i: the
// centre distance g_i across x, the cell widths across y and z).  cov
// pieces along the component's own axis sit at the two neighbouring
// centres and reach the face by the width-weighted interpolation (covx1 of
// section 2.5.3); across it they sit on the two edges the face is the
// midpoint of (plain mean); an advecting velocity is interpolated onto an
// edge from its own two faces with the same width weights.  Diffusion and
// the subgrid stress are differences of one-sided fluxes over the control
// volume.  Feedback forcing and AB2 as in the uniform pass.
__device__ __forceinline__ void tendency_body_str(const Geo& g, const TendArgs& A, unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)lb * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    const float* __restrict__ u = A.u;
    const float* __restrict__ v = A.v;
    const float* __restrict__ w = A.w;
    const float* __restrict__ nut = A.nut;
    const StrAxis X = str_axis(g.mx, g.nx), Y = str_axis(g.my, g.ny), Z = str_axis(g.mz, g.nz);
    auto U = [&](int a, int b, int c) { return u[g.nat(a, b, c)]; };
    auto V = [&](int a, int b, int c) { return v[g.nat(a, b, c)]; };
    auto W = [&](int a, int b, int c) { return w[g.nat(a, b, c)]; };
    auto N = [&](int a, int b, int c) { return nut[g.nat(a, b, c)]; };
    auto n12 = [&](int a, int b, int c) { return 0.25f * (N(a, b, c) + N(a + 1, b, c) + N(a, b + 1, c) + N(a + 1, b + 1, c)); };
    auto n13 = [&](int a, int b, int c) { return 0.25f * (N(a, b, c) + N(a + 1, b, c) + N(a, b, c + 1) + N(a + 1, b, c + 1)); };
    auto n23 = [&](int a, int b, int c) { return 0.25f * (N(a, b, c) + N(a, b + 1, c) + N(a, b, c + 1) + N(a, b + 1, c + 1)); };
    auto e12 = [&](int a, int b, int c) { return 0.5f * ((U(a, b + 1, c) - U(a, b, c)) * Y.ig[b] + (V(a + 1, b, c) - V(a, b, c)) * X.ig[a]); };
    auto e13 = [&](int a, int b, int c) { return 0.5f * ((U(a, b, c + 1) - U(a, b, c)) * Z.ig[c] + (W(a + 1, b, c) - W(a, b, c)) * X.ig[a]); };
    auto e23 = [&](int a, int b, int c) { return 0.5f * ((V(a, b, c + 1) - V(a, b, c)) * Z.ig[c] + (W(a, b + 1, c) - W(a, b, c)) * Y.ig[b]); };

    const long long e = g.nat(i, j, k);
    const uint8_t fl = A.flags[e];
    const float dt = g.dt;
    const float nu = A.nu, alpha = A.alpha, beta = A.beta;

    if (i <= g.u_last) {
        const float lo = X.lo[i], hi = X.hi[i];
        auto c1 = [&](int c) { return 0.5f * (U(c - 1, j, k) + U(c, j, k)) * (U(c, j, k) - U(c - 1, j, k)) * X.ih[c]; };
        auto c2 = [&](int b) { return (lo * V(i, b, k) + hi * V(i + 1, b, k)) * (U(i, b + 1, k) - U(i, b, k)) * Y.ig[b]; };
        auto c3 = [&](int c) { return (lo * W(i, j, c) + hi * W(i + 1, j, c)) * (U(i, j, c + 1) - U(i, j, c)) * Z.ig[c]; };
        const float covx = lo * c1(i) + hi * c1(i + 1);
        const float covy = 0.5f * (c2(j - 1) + c2(j));
        const float covz = 0.5f * (c3(k - 1) + c3(k));
        auto fx = [&](int c) { return (U(c, j, k) - U(c - 1, j, k)) * X.ih[c]; };
        auto fy = [&](int b) { return (U(i, b + 1, k) - U(i, b, k)) * Y.ig[b]; };
        auto fz = [&](int c) { return (U(i, j, c + 1) - U(i, j, c)) * Z.ig[c]; };
        const float lap = (fx(i + 1) - fx(i)) * X.ig[i] + (fy(j) - fy(j - 1)) * Y.ih[j] + (fz(k) - fz(k - 1)) * Z.ih[k];
        const float sgs = (2.f * N(i + 1, j, k) * fx(i + 1) - 2.f * N(i, j, k) * fx(i)) * X.ig[i] +
                          (2.f * n12(i, j, k) * e12(i, j, k) - 2.f * n12(i, j - 1, k) * e12(i, j - 1, k)) * Y.ih[j] +
                          (2.f * n13(i, j, k) * e13(i, j, k) - 2.f * n13(i, j, k - 1) * e13(i, j, k - 1)) * Z.ih[k];
        const float uc = U(i, j, k);
        float F = -(covx + covy + covz) + nu * lap + sgs;
        if (fl & F_USOLID) {
            const float s = A.su[e] + dt * uc;
            A.su[e] = s;
            F += alpha * s + beta * uc;
        }
        const float fo = A.first ? F : A.fu[e];
        A.us[e] = uc + dt * (1.5f * F - 0.5f * fo);
        A.fu[e] = F;
    }
    if (j <= g.ny - 1) {
        const float lo = Y.lo[j], hi = Y.hi[j];
        auto c1 = [&](int a) { return (lo * U(a, j, k) + hi * U(a, j + 1, k)) * (V(a + 1, j, k) - V(a, j, k)) * X.ig[a]; };
        auto c2 = [&](int b) { return 0.5f * (V(i, b - 1, k) + V(i, b, k)) * (V(i, b, k) - V(i, b - 1, k)) * Y.ih[b]; };
        auto c3 = [&](int c) { return (lo * W(i, j, c) + hi * W(i, j + 1, c)) * (V(i, j, c + 1) - V(i, j, c)) * Z.ig[c]; };
        const float covx = 0.5f * (c1(i - 1) + c1(i));
        const float covy = lo * c2(j) + hi * c2(j + 1);
        const float covz = 0.5f * (c3(k - 1) + c3(k));
        auto fx = [&](int a) { return (V(a + 1, j, k) - V(a, j, k)) * X.ig[a]; };
        auto fy = [&](int b) { return (V(i, b, k) - V(i, b - 1, k)) * Y.ih[b]; };
        auto fz = [&](int c) { return (V(i, j, c + 1) - V(i, j, c)) * Z.ig[c]; };
        const float lap = (fx(i) - fx(i - 1)) * X.ih[i] + (fy(j + 1) - fy(j)) * Y.ig[j] + (fz(k) - fz(k - 1)) * Z.ih[k];
        const float sgs = (2.f * n12(i, j, k) * e12(i, j, k) - 2.f * n12(i - 1, j, k) * e12(i - 1, j, k)) * X.ih[i] +
                          (2.f * N(i, j + 1, k) * fy(j + 1) - 2.f * N(i, j, k) * fy(j)) * Y.ig[j] +
                          (2.f * n23(i, j, k) * e23(i, j, k) - 2.f * n23(i, j, k - 1) * e23(i, j, k - 1)) * Z.ih[k];
        const float vc = V(i, j, k);
        float F = -(covx + covy + covz) + nu * lap + sgs;
        if (fl & F_VSOLID) {
            const float s = A.sv[e] + dt * vc;
            A.sv[e] = s;
            F += alpha * s + beta * vc;
        }
        const float fo = A.first ? F : A.fv[e];
        A.vs[e] = vc + dt * (1.5f * F - 0.5f * fo);
        A.fv[e] = F;
    }
    if (k <= g.nz - 1) {
        const float lo = Z.lo[k], hi = Z.hi[k];
        auto c1 = [&](int a) { return (lo * U(a, j, k) + hi * U(a, j, k + 1)) * (W(a + 1, j, k) - W(a, j, k)) * X.ig[a]; };
        auto c2 = [&](int b) { return (lo * V(i, b, k) + hi * V(i, b, k + 1)) * (W(i, b + 1, k) - W(i, b, k)) * Y.ig[b]; };
        auto c3 = [&](int c) { return 0.5f * (W(i, j, c - 1) + W(i, j, c)) * (W(i, j, c) - W(i, j, c - 1)) * Z.ih[c]; };
        const float covx = 0.5f * (c1(i - 1) + c1(i));
        const float covy = 0.5f * (c2(j - 1) + c2(j));
        const float covz = lo * c3(k) + hi * c3(k + 1);
        auto fx = [&](int a) { return (W(a + 1, j, k) - W(a, j, k)) * X.ig[a]; };
        auto fy = [&](int b) { return (W(i, b + 1, k) - W(i, b, k)) * Y.ig[b]; };
        auto fz = [&](int c) { return (W(i, j, c) - W(i, j, c - 1)) * Z.ih[c]; };
        const float lap = (fx(i) - fx(i - 1)) * X.ih[i] + (fy(j) - fy(j - 1)) * Y.ih[j] + (fz(k + 1) - fz(k)) * Z.ig[k];
        const float sgs = (2.f * n13(i, j, k) * e13(i, j, k) - 2.f * n13(i - 1, j, k) * e13(i - 1, j, k)) * X.ih[i] +
                          (2.f * n23(i, j, k) * e23(i, j, k) - 2.f * n23(i, j - 1, k) * e23(i, j - 1, k)) * Y.ih[j] +
                          (2.f * N(i, j, k + 1) * fz(k + 1) - 2.f * N(i, j, k) * fz(k)) * Z.ig[k];
        const float wc = W(i, j, k);
        float F = -(covx + covy + covz) + nu * lap + sgs;
        if (fl & F_WSOLID) {
            const float s = A.sw[e] + dt * wc;
            A.sw[e] = s;
            F += alpha * s + beta * wc;
        }
        const float fo = A.first ? F : A.fw[e];
        A.ws[e] = wc + dt * (1.5f * F - 0.5f * fo);
        A.fw[e] = F;
    }
}

// rhs = div(u*) / dt on a stretched grid (face differences over the cell
// widths); float64 partials of sum rhs^2.
__device__ __forceinline__ void rhs_body_str(const Geo& g, const float* __restrict__ us,
                                             const float* __restrict__ vs, const float* __restrict__ ws,
                                             float* rhs0, float* rhs1, double* __restrict__ part,
                                             unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)lb * kBlock + threadIdx.x;
    double acc = 0.0;
    if (t < n) {
        int i, j, k;
        cell_of(g, t, i, j, k);
        const float div = (us[g.nat(i, j, k)] - us[g.nat(i - 1, j, k)]) * mrow(g.mx, g.nx, M_IH, i) +
                          (vs[g.nat(i, j, k)] - vs[g.nat(i, j - 1, k)]) * mrow(g.my, g.ny, M_IH, j) +
                          (ws[g.nat(i, j, k)] - ws[g.nat(i, j, k - 1)]) * mrow(g.mz, g.nz, M_IH, k);
        const float r = div * g.idt;
        const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
        float* dst = ((i0 + j0 + k0) & 1) ? rhs1 : rhs0;
        dst[g.col(i0 >> 1, j0, k0)] = r;
        acc = (double)r * (double)r;
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
}

// velnw on a stretched grid: u = u* - dt (p_{c+1} - p_c) / g_c across an
// interior face; on the outflow face p = 0 half a cell from the centre.
__device__ __forceinline__ void project_body_str(const Geo& g, float* __restrict__ us,
                                                 float* __restrict__ vs, float* __restrict__ ws,
                                                 const PBufs& P, unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)lb * kBlock + threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    cell_of(g, t, i, j, k);
    const int i0 = i - 1, j0 = j - 1, k0 = k - 1;
    const int c = (i0 + j0 + k0) & 1;
    const float* __restrict__ phc = P.ph[c];
    const float* __restrict__ pdc = P.pd[c];
    const float* __restrict__ pho = P.ph[1 - c];
    const float* __restrict__ pdo = P.pd[1 - c];
    const long long ec = g.col(i0 >> 1, j0, k0);
    const float hc = phc[ec], dc = pdc[ec];
    const float dt = g.dt;
    const long long e = g.nat(i, j, k);
    if (i0 + 1 < g.nx) {
        const long long en = g.col((i0 + 1) >> 1, j0, k0);
        us[e] -= dt * (((pho[en] - hc) + (pdo[en] - dc)) * mrow(g.mx, g.nx, M_IG, i));
    } else if (g.outflow) {
        us[e] -= dt * ((-2.f * hc - 2.f * dc) * mrow(g.mx, g.nx, M_IH, i));
    }
    if (j0 + 1 < g.ny) {
        const long long en = ec + g.S;
        vs[e] -= dt * (((pho[en] - hc) + (pdo[en] - dc)) * mrow(g.my, g.ny, M_IG, j));
    }
    if (k0 + 1 < g.nz) {
        const long long en = ec + g.SP;
        ws[e] -= dt * (((pho[en] - hc) + (pdo[en] - dc)) * mrow(g.mz, g.nz, M_IG, k));
    }
}

// --------------------------------------------------- diagnostics (norms)
// Partials [sum div(u)^2, max CFL]: CFL = dt (|u|/dx + |v|/dy + |w|/dz) with
// cell-centred speeds; float64.
__device__ __forceinline__ void diag_body(const Geo& g, const float* __restrict__ u,
                                          const float* __restrict__ v, const float* __restrict__ w,
                                          double* __restrict__ part, unsigned lb) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long t = (long long)lb * kBlock + threadIdx.x;
    double d2 = 0.0, cf = 0.0;
    if (t < n) {
        int i, j, k;
        cell_of(g, t, i, j, k);
        const float u1 = u[g.nat(i, j, k)], u0 = u[g.nat(i - 1, j, k)];
        const float v1 = v[g.nat(i, j, k)], v0 = v[g.nat(i, j - 1, k)];
        const float w1 = w[g.nat(i, j, k)], w0 = w[g.nat(i, j, k - 1)];
        // cell widths (the cell's own on a stretched grid)
        const double hx = g.stretched ? (double)mrow(g.mx, g.nx, M_H, i) : (double)g.dx;
        const double hy = g.stretched ? (double)mrow(g.my, g.ny, M_H, j) : (double)g.dy;
        const double hz = g.stretched ? (double)mrow(g.mz, g.nz, M_H, k) : (double)g.dz;
        const double div = ((double)u1 - u0) / hx + ((double)v1 - v0) / hy + ((double)w1 - w0) / hz;
        d2 = div * div;
        cf = (double)g.dt * (0.5 * fabs((double)u1 + u0) / hx + 0.5 * fabs((double)v1 + v0) / hy +
                             0.5 * fabs((double)w1 + w0) / hz);
    }
    const double s = block_sum(d2);
    const double mx = block_max(cf);
    if (threadIdx.x == 0) {
        part[2 * lb] = s;
        part[2 * lb + 1] = mx;
    }
}

}  // namespace les

// The red-black SOR bodies (section 2.6) live in their own header.
#include "sor_bodies.h"
