// Red-black SOR device bodies (section 2.6): point update, half-sweeps,
// fused and two-iteration sweeps (general and lean uniform-grid forms),
// fold, rebase, residual check and the single-block finalize.  Included
// at the end of les_bodies.h, whose helpers (diagonal shares, metric
// tables, reductions) these bodies use.
#pragma once

namespace les {

// ================================================================= SOR
// Red-black SOR for the pressure Poisson equation (section 2.6).
//
// The cells of one colour are stored contiguously (colour-split layout), so
// a half-sweep reads the other colour's array and its own arrays with unit
// stride and writes its own: 8 bytes per cell per half-sweep.  Within a
// colour every update only reads the other colour, so the parallel
// half-sweep equals the sequential one of the paper exactly.
//
// Precision.  p is held as a float32 base ph plus a float32 correction pd.
// The sweeps relax pd against r0 = rhs - A ph (evaluated in float64,
// stored in float32): SOR is affine, so the iterates ph + pd are those of
// plain SOR on p, but each update rounds relative to |pd| instead of |p|.
// Every few checks the correction is folded into the base (TwoSum, no
// loss) and r0 recomputed.  Residuals ||rhs - A p|| are float64.

// ------------------------------------------------------- point update
// One cell's update from its six neighbours of the other colour, its own
// correction p and its r0: returns p + reltmp, reltmp = omega (cn1
// (sum_nb cn_nb p_nb - r0) - p).  Contraction is pinned (explicit fmaf,
// no other fusion) so that every kernel that updates a cell rounds alike.
// The two halves are separate so that a kernel holding cn1 = 1/diag already
// (correctly rounded, as here) rounds exactly alike.
__device__ __forceinline__ float sor_nb(float west, float east, float ps, float pn, float pb, float pt,
                                        float cx, float cy, float cz) {
#pragma clang fp contract(off)
    return fmaf(cz, pb + pt, fmaf(cy, ps + pn, cx * (west + east)));
}
__device__ __forceinline__ float sor_relax(float nb, float inv, float r, float p, float omega,
                                           float& reltmp) {
#pragma clang fp contract(off)
    reltmp = omega * fmaf(inv, nb - r, -p);
    return p + reltmp;
}
__device__ __forceinline__ float sor_point(float west, float east, float ps, float pn, float pb,
                                           float pt, float cx, float cy, float cz, float diag,
                                           float r, float p, float omega, float& reltmp) {
    return sor_relax(sor_nb(west, east, ps, pn, pb, pt, cx, cy, cz), 1.0f / diag, r, p, omega, reltmp);
}

// The same update on a stretched grid: every neighbour has its own weight
// (the per-axis 1-D coefficients of section 2.6), the diagonal is the sum
// of the cell's per-axis shares.  Used by every sweep kernel of a
// stretched grid, so those round alike among themselves.
__device__ __forceinline__ float sor_point_w(float west, float east, float ps, float pn, float pb,
                                             float pt, float ww, float we, float ws, float wn,
                                             float wb, float wt, float diag, float r, float p,
                                             float omega, float& reltmp) {
#pragma clang fp contract(off)
    const float nb = fmaf(wt, pt, fmaf(wb, pb, fmaf(wn, pn, fmaf(ws, ps, fmaf(we, east, ww * west)))));
    const float inv = 1.0f / diag;
    reltmp = omega * fmaf(inv, nb - r, -p);
    return p + reltmp;
}

// ---------------------------------------------------------- half-sweep
// Colour c: for every cell of colour c,
//   reltmp = omega (cn1 (sum_nb cn_nb p_nb - rhs) - p);  p += reltmp
// with cn1 = 1/diag.  Outside the domain the other colour's array holds
// zeros, so the neighbour sum needs no boundary branches.  On the last
// iteration of a check interval (acc) the block also leaves the float64
// partials [sum reltmp^2, sum (diag reltmp)^2]: after the colour-1
// half-sweep, diag (omega-1)/omega reltmp is exactly the residual of a
// colour-1 cell, so the second sum bounds ||r|| from below.
//
// Tiling: a block is 4 wavefronts; a wavefront covers TX consecutive
// half-cells of 64/TX rows, and the block marches up KT planes (KT = 1:
// one cell per thread, the most memory-level parallelism).  The other
// colour's values at (ii, j0) stay in registers across k (the top
// neighbour of plane k is the in-row value of plane k+1 and the bottom one
// of plane k+2); east/west neighbours come from the adjacent lanes by
// cross-lane shuffles, north/south ones from the cache.  Within a row the
// cell parity is uniform.
template <int TX, int KT, bool STR = false>
__device__ __forceinline__ void sor_body(const Geo& g, int c, float* __restrict__ pself,
                                         const float* __restrict__ poth,
                                         const float* __restrict__ rself, float omega, bool acc,
                                         double* __restrict__ rel_part, unsigned lb) {
    constexpr int RPW = 64 / TX;            // rows per wavefront
    constexpr int TY = RPW * (kBlock / 64); // rows per block
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
    // stretched grid: the row's y weights and diagonal share (clamped row
    // index for lanes outside the grid, which update nothing)
    const int jm = min(j0, g.ny - 1);
    const float dyy = STR ? mrow(g.my, g.ny, M_DD, jm + 1) : diag_y(g, j0);
    const float wsy = STR ? mrow(g.my, g.ny, M_WM, jm + 1) : 0.f;
    const float wny = STR ? mrow(g.my, g.ny, M_WP, jm + 1) : 0.f;
    long long e = col_ok ? g.col(ii, j0, k_begin) : 0;
    float pb = col_ok ? poth[e - g.SP] : 0.f;
    float pc = col_ok ? poth[e] : 0.f;
    double r2 = 0.0, dr2 = 0.0;
    for (int k0 = k_begin; k0 < k_end; ++k0) {
        const float pt = col_ok ? poth[e + g.SP] : 0.f;
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
            float reltmp, diag;
            if constexpr (STR) {
                diag = mrow(g.mx, g.nx, M_DD, i0 + 1) + dyy + mrow(g.mz, g.nz, M_DD, k0 + 1);
                pself[e] = sor_point_w(west, east, ps, pn, pb, pt, mrow(g.mx, g.nx, M_WM, i0 + 1),
                                       mrow(g.mx, g.nx, M_WP, i0 + 1), wsy, wny,
                                       mrow(g.mz, g.nz, M_WM, k0 + 1), mrow(g.mz, g.nz, M_WP, k0 + 1),
                                       diag, rself[e], pself[e], omega, reltmp);
            } else {
                diag = diag_x(g, i0) + dyy + diag_z(g, k0);
                pself[e] = sor_point(west, east, ps, pn, pb, pt, cx, cy, cz, diag, rself[e], pself[e],
                                     omega, reltmp);
            }
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
        const double bs = block_sum(r2);
        const double bd = block_sum(dr2);
        if (threadIdx.x == 0) {
            rel_part[2 * lb] = bs;
            rel_part[2 * lb + 1] = bd;
        }
    }
}

// Whether the half-sweeps of local iteration it run, and whether they
// accumulate the reltmp partials (last iteration of the check interval).
__device__ __forceinline__ bool sweep_active(const Ctl* ctl, int it, bool& acc) {
    const int m = ctl->m, K = ctl->K, mx = ctl->max_iter;
    acc = (m + it + 1 == min(m + K, mx));
    return !(ctl->done || m + it >= mx);
}

// ------------------------------------------- fused red-black iteration
// One whole SOR iteration in one pass: colour 0 from the old colour-1
// values, then colour 1 from the new colour-0 values, with every read from
// the old arrays (a0, a1) and every write to the other pair (b0, b1), so
// blocks never see each other's results.  Each block owns a tile of TXO =
// TX-2 half-cells by TYO = TYB-2 rows by KT planes; it also updates colour
// 0 on a one-cell ring around the tile (halo lanes 0 and TX-1, halo rows 0
// and TYB-1, planes k_begin-1 and k_end), which colour 1 at the tile's edge
// needs, and writes only its own tile.  The per-cell arithmetic is that of
// the half-sweeps (sor_point), so the result equals two half-sweeps bit for
// bit, for 12 bytes per cell per iteration instead of 16.
//
// A block is NW wavefronts of 64/TX rows of TX lanes and marches up the
// planes: at step q it updates colour 0 on plane q, publishes the row in an
// LDS ring of three planes, and after one barrier updates colour 1 on plane
// q-1 from its own new colour-0 planes q-2..q (registers), its lanes' east
// and west values (cross-lane shuffles) and the rows above and below (LDS).
// Loads of plane q+1 are issued a step ahead.  With copy set (an
// iteration past max_iter inside the last check interval) the block copies
// a to b, so the result stays in the buffer the interval ends on.
template <int TX, int NW, int KT, bool STR = false>
__device__ __forceinline__ void sor_rb_body(const Geo& g, const float* __restrict__ a0,
                                            const float* __restrict__ a1,
                                            const float* __restrict__ r0c,
                                            const float* __restrict__ r1c, float* __restrict__ b0,
                                            float* __restrict__ b1, float omega, bool acc, bool copy,
                                            double* __restrict__ rel0, double* __restrict__ rel1,
                                            unsigned lb, int kt_run = 0) {
    constexpr int RPW = 64 / TX;
    constexpr int TYB = RPW * NW;
    constexpr int TXO = TX - 2, TYO = TYB - 2;
    const int kt = KT > 0 ? KT : kt_run;   // planes per block
    __shared__ float ring[3][TYB][TX];
    __shared__ double red3[3][NW];
    const unsigned nbx = (unsigned)(g.H + TXO - 1) / TXO;
    const unsigned nby = (unsigned)(g.ny + TYO - 1) / TYO;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int tx = lane % TX;
    const int row = (threadIdx.x >> 6) * RPW + lane / TX;
    const int ii = (int)bx * TXO - 1 + tx;
    const int j = (int)by * TYO - 1 + row;
    const int k_begin = (int)bk * kt;
    const int k_end = min(g.nz, k_begin + kt);
    const bool col_ok = ii >= 0 && ii < g.H && j >= 0 && j < g.ny;
    const bool inner = col_ok && tx >= 1 && tx <= TX - 2 && row >= 1 && row <= TYB - 2;
    const bool edge_lane = tx == 0 || tx == TX - 1;
    const int edge_off = tx == 0 ? -1 : 1;
    const float cx = g.cx, cy = g.cy, cz = g.cz;
    const int jm = min(max(j, 0), g.ny - 1);   // clamped for the stretched tables
    const float dyy = STR ? mrow(g.my, g.ny, M_DD, jm + 1) : diag_y(g, j);
    const float wsy = STR ? mrow(g.my, g.ny, M_WM, jm + 1) : 0.f;
    const float wny = STR ? mrow(g.my, g.ny, M_WP, jm + 1) : 0.f;
    const int qa = k_begin - 1;
    const long long e0 = col_ok ? g.col(ii, j, qa) : 0;
    // loads of step q: a1 one plane up, a1 in the rows below and above, the
    // edge lane's a1 east or west, a0 and r0 on plane q, r1 on plane q-1
    struct Step { float up, south, north, edge, p0, rr0, rr1; };
    auto fetch = [&](int q, Step& f) {
        const long long e = e0 + (long long)(q - qa) * g.SP;
        const bool pl = col_ok && q >= 0 && q < g.nz;
        f.up = (col_ok && q + 1 <= g.nz) ? a1[e + g.SP] : 0.f;
        f.south = pl ? a1[e - g.S] : 0.f;
        f.north = pl ? a1[e + g.S] : 0.f;
        f.edge = (pl && edge_lane) ? a1[e + edge_off] : 0.f;
        f.p0 = pl ? a0[e] : 0.f;
        f.rr0 = pl ? r0c[e] : 0.f;
        f.rr1 = (col_ok && q - 1 >= k_begin && q - 1 < k_end) ? r1c[e - g.SP] : 0.f;
    };
    // old colour 1 on planes q-1 (bm) and q (bc); new colour 0 on q-2, q-1
    float bm = (col_ok && qa - 1 >= -1) ? a1[e0 - g.SP] : 0.f;
    float bc = col_ok ? a1[e0] : 0.f;
    float rm2 = 0.f, rm1 = 0.f;
    double r2a = 0.0, r2b = 0.0, d2b = 0.0;
    Step cur, nxt;
    fetch(qa, cur);
    long long e = e0;
    for (int q = qa; q <= k_end; ++q) {
        if (q < k_end) fetch(q + 1, nxt);
        // colour 0 at (ii, j, q)
        float be = __shfl_down(bc, 1, TX);
        float bw = __shfl_up(bc, 1, TX);
        if (tx == TX - 1) be = cur.edge;
        if (tx == 0) bw = cur.edge;
        const int s = (j + q) & 1;
        const int i0 = 2 * ii + s;
        float rq = 0.f;
        if (col_ok && q >= 0 && q < g.nz && i0 < g.nx) {
            float rt = 0.f;
            if constexpr (STR) {
                const float diag = mrow(g.mx, g.nx, M_DD, i0 + 1) + dyy + mrow(g.mz, g.nz, M_DD, q + 1);
                rq = copy ? cur.p0
                          : sor_point_w(s ? bc : bw, s ? be : bc, cur.south, cur.north, bm, cur.up,
                                        mrow(g.mx, g.nx, M_WM, i0 + 1), mrow(g.mx, g.nx, M_WP, i0 + 1),
                                        wsy, wny, mrow(g.mz, g.nz, M_WM, q + 1),
                                        mrow(g.mz, g.nz, M_WP, q + 1), diag, cur.rr0, cur.p0, omega, rt);
            } else {
                const float diag = diag_x(g, i0) + dyy + diag_z(g, q);
                rq = copy ? cur.p0
                          : sor_point(s ? bc : bw, s ? be : bc, cur.south, cur.north, bm, cur.up, cx, cy,
                                      cz, diag, cur.rr0, cur.p0, omega, rt);
            }
            if (inner && q >= k_begin && q < k_end) {
                b0[e] = rq;
                if (acc) r2a += (double)rt * (double)rt;
            }
        }
        ring[(q - qa) % 3][row][tx] = rq;
        __syncthreads();
        // colour 1 at (ii, j, q-1)
        const int qb = q - 1;
        if (qb >= k_begin) {
            const int sl = (qb - qa) % 3;
            const float re = __shfl_down(rm1, 1, TX);
            const float rw = __shfl_up(rm1, 1, TX);
            const int sb = (1 + j + qb) & 1;
            const int i1 = 2 * ii + sb;
            if (inner && i1 < g.nx) {
                float rt = 0.f, diag, v;
                if constexpr (STR) {
                    diag = mrow(g.mx, g.nx, M_DD, i1 + 1) + dyy + mrow(g.mz, g.nz, M_DD, qb + 1);
                    v = copy ? bm
                             : sor_point_w(sb ? rm1 : rw, sb ? re : rm1, ring[sl][row - 1][tx],
                                           ring[sl][row + 1][tx], rm2, rq, mrow(g.mx, g.nx, M_WM, i1 + 1),
                                           mrow(g.mx, g.nx, M_WP, i1 + 1), wsy, wny,
                                           mrow(g.mz, g.nz, M_WM, qb + 1), mrow(g.mz, g.nz, M_WP, qb + 1),
                                           diag, cur.rr1, bm, omega, rt);
                } else {
                    diag = diag_x(g, i1) + dyy + diag_z(g, qb);
                    v = copy ? bm
                             : sor_point(sb ? rm1 : rw, sb ? re : rm1, ring[sl][row - 1][tx],
                                         ring[sl][row + 1][tx], rm2, rq, cx, cy, cz, diag,
                                         cur.rr1, bm, omega, rt);
                }
                b1[e - g.SP] = v;
                if (acc) {
                    const double rd = (double)rt;
                    r2b += rd * rd;
                    d2b += ((double)diag * rd) * ((double)diag * rd);
                }
            }
        }
        bm = bc;
        bc = cur.up;
        rm2 = rm1;
        rm1 = rq;
        cur = nxt;
        e += g.SP;
    }
    if (acc) {
        const double va = wave_sum(r2a), vb = wave_sum(r2b), vd = wave_sum(d2b);
        const int wid = threadIdx.x >> 6;
        if (lane == 0) {
            red3[0][wid] = va;
            red3[1][wid] = vb;
            red3[2][wid] = vd;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0, td = 0.0;
            for (int w = 0; w < NW; ++w) {
                ta += red3[0][w];
                tb += red3[1][w];
                td += red3[2][w];
            }
            rel0[2 * lb] = ta;
            rel0[2 * lb + 1] = 0.0;
            rel1[2 * lb] = tb;
            rel1[2 * lb + 1] = td;
        }
    }
}

// ------------------------- fused red-black iteration, uniform grids (lean)
// The iteration of sor_rb_body on a uniform grid, arranged for few vector
// instructions per cell (the k-march of sor_rb_body issues ~140 vector
// instructions per step and is bound by issue, not by memory).  Same lanes,
// same tiles, same per-cell arithmetic (sor_nb / sor_relax with cn1 = 1/diag
// correctly rounded), so the result equals sor_rb_body's bit for bit.
//  * Addressing: one block-uniform origin walks up the planes (scalar
//    registers); each lane holds constant 32-bit byte offsets from it for
//    its column and the column's neighbours.  Lanes outside the grid address
//    the zero padding column (half-index H, present in every row and plane),
//    so they read zeros everywhere and produce exact zeros: no per-lane
//    predicate on loads or values.
//  * x-neighbours: of a cell's two neighbours of the other colour one lies
//    in the lane's own column; the other (left or right, by plane parity) is
//    loaded for colour 0 and taken from the neighbouring lane's new value by
//    one ds_bpermute for colour 1.
//  * cn1: per lane and parity for the interior and the end planes; zero for
//    the missing cell at the end of an odd-length row, which then stays 0.
//  * The march is unrolled by four over an LDS ring of four planes (guard
//    rows above and below), so ring slots and parity are compile-time and
//    the loads of plane q+1 stay in flight across step q.
struct RbPar {
    unsigned lx;    // byte offset of the other x-neighbour (own padding element outside the grid)
    int src;        // ds_bpermute byte address of the lane holding that neighbour's new value
    float dxy;      // x and y shares of the diagonal
    float inv_mid;  // cn1 on planes with a neighbour above and below (0: no such cell)
    float inv_end;  // cn1 on the bottom and top planes
    bool store;     // the lane owns this cell of its tile
};
struct RbIn {
    float up, south, north, xn, p0, rr0, rr1;
};

// Buffer access to a colour array: the resource's base sits 2 SP elements
// before the array (so the block-uniform scalar offset of every plane from
// -1 to nz+1 is non-negative) and each lane adds a 32-bit byte offset.
// The whole array must lie within 4 GiB of that base (rb_lean_fits).
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc colour_rsrc(const Geo& g, const float* p) {
    const unsigned bytes = (unsigned)((g.ctot + 2 * g.SP) * 4);
    return __builtin_amdgcn_make_buffer_rsrc((void*)(p - 2 * g.SP), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bld(Rsrc r, unsigned voff, unsigned soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bst(Rsrc r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ float lane_perm(int byte_src, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_src, __float_as_int(v)));
}

template <int TX, int NW, int KT, bool ACC>
__device__ __forceinline__ void sor_rb_body_u(const Geo& g, const float* __restrict__ a0,
                                              const float* __restrict__ a1,
                                              const float* __restrict__ r0c,
                                              const float* __restrict__ r1c, float* __restrict__ b0,
                                              float* __restrict__ b1, float omega,
                                              double* __restrict__ rel0, double* __restrict__ rel1,
                                              unsigned lb, int kt_run) {
    constexpr int RPW = 64 / TX;
    constexpr int TYB = RPW * NW;
    constexpr int TXO = TX - 2, TYO = TYB - 2;
    const int kt = KT > 0 ? KT : kt_run;
    __shared__ float ring[4][TYB + 2][TX];   // row r of the tile at index r + 1
    __shared__ double red3[3][NW];
    const unsigned nbx = (unsigned)(g.H + TXO - 1) / TXO;
    const unsigned nby = (unsigned)(g.ny + TYO - 1) / TYO;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int tx = lane % TX;
    const int row = (threadIdx.x >> 6) * RPW + lane / TX;
    const int ii0 = (int)bx * TXO - 1, j0 = (int)by * TYO - 1;   // the tile's halo corner
    const int ii = ii0 + tx, j = j0 + row;
    const int k_begin = (int)bk * kt;
    const int k_end = min(g.nz, k_begin + kt);
    const int qa = k_begin - 1;
    const bool col_ok = ii >= 0 && ii < g.H && j >= 0 && j < g.ny;
    const bool inner = col_ok && tx >= 1 && tx <= TX - 2 && row >= 1 && row <= TYB - 2;
    // Byte offsets of the lane's column and its neighbours from the block's
    // moving origin, which for step q sits one plane, one row and one
    // element before the halo corner of plane q (so every offset is
    // non-negative): own plane q, south, north, up (q+1), below (q-1).
    // Lanes outside the grid take the padding column of a row inside it.
    const int iic = col_ok ? ii : g.H, jc = min(max(j, 0), g.ny - 1);
    const unsigned lc = (unsigned)(((jc - j0 + 1) * g.S + (iic - ii0) + 1) + g.SP) * 4u;
    const unsigned ls = lc - (unsigned)g.S * 4u, ln = lc + (unsigned)g.S * 4u;
    const unsigned lu = lc + (unsigned)g.SP * 4u, lbw = lc - (unsigned)g.SP * 4u;
    const float cx = g.cx, cy = g.cy, cz = g.cz;
    const float dyy = diag_y(g, j);
    const float dz_mid = g.cz + g.cz;      // diag_z of a plane with neighbours above and below
    const float dz_end = diag_z(g, 0);     // and of the bottom and top planes (equal)
    RbPar pe, po;                          // parity of the steps q - qa even / odd
    {
        const int se = (j + qa) & 1;
        auto make = [&](int s, RbPar& P) {
            const int i0 = 2 * ii + s;
            const bool ok = col_ok && i0 < g.nx;
            P.lx = col_ok ? (s ? lc + 4u : lc - 4u) : lc;
            P.src = ((s ? lane + 1 : lane - 1) & 63) * 4;
            P.dxy = diag_x(g, i0) + dyy;
            P.inv_mid = ok ? 1.0f / (P.dxy + dz_mid) : 0.f;
            P.inv_end = ok ? 1.0f / (P.dxy + dz_end) : 0.f;
            P.store = inner && ok;
        };
        make(se, pe);
        make(se ^ 1, po);
    }
    const Rsrc ra0 = colour_rsrc(g, a0), ra1 = colour_rsrc(g, a1), rr0c = colour_rsrc(g, r0c),
               rr1c = colour_rsrc(g, r1c), rb0 = colour_rsrc(g, b0), rb1 = colour_rsrc(g, b1);
    const unsigned sp4 = (unsigned)g.SP * 4u;
    // scalar byte offset (from the resources' base) of the origin of step qa
    const unsigned so0 =
        (unsigned)((long long)g.S + ((long long)qa * (g.ny + 2) + (j0 + 1)) * g.S + ii0 - 1 - g.S + 2 * g.SP) *
        4u;
    // Loads of step q (origin so).  Planes -1 and nz are ghost planes; where
    // a value is not needed (up above plane nz, rr1 below plane -1) the
    // origin is moved to a plane that exists, so every load is unconditional.
    auto fetch = [&](int q, unsigned so, RbIn& f, const RbPar& P) {
        f.up = bld(ra1, lu, q + 1 <= g.nz ? so : so - sp4);
        f.south = bld(ra1, ls, so);
        f.north = bld(ra1, ln, so);
        f.xn = bld(ra1, P.lx, so);
        f.p0 = bld(ra0, lc, so);
        f.rr0 = bld(rr0c, lc, so);
        f.rr1 = bld(rr1c, lbw, q - 1 >= -1 ? so : so + sp4);
    };
    // old colour 1 on planes q-1 (bm) and q (bc); new colour 0 on planes q-2
    // (rm2) and q-1 (rm1)
    float bm = qa - 1 >= -1 ? bld(ra1, lbw, so0) : 0.f;
    float bc = bld(ra1, lc, so0);
    float rm2 = 0.f, rm1 = 0.f;
    double r2a = 0.0, r2b = 0.0, d2b = 0.0;
    const int rw = row + 1;

    // one step of the march: colour 0 on plane q, colour 1 on plane q - 1;
    // P is this step's parity, PN the next one's (for the loads of q + 1)
    auto step = [&](auto slot_c, int q, unsigned so, const RbIn& cur, RbIn& nxt, const RbPar& P,
                    const RbPar& PN) {
        constexpr int SL = decltype(slot_c)::value;
        constexpr int SLP = (SL + 3) & 3;   // the slot of plane q - 1
        if (q < k_end) fetch(q + 1, so + sp4, nxt, PN);
        float rq = 0.f;
        if (q >= 0 && q < g.nz) {
            const float inv = (q == 0 || q == g.nz - 1) ? P.inv_end : P.inv_mid;
            float rt;
            const float v = sor_relax(sor_nb(bc, cur.xn, cur.south, cur.north, bm, cur.up, cx, cy, cz), inv,
                                      cur.rr0, cur.p0, omega, rt);
            rq = v;
            if (q >= k_begin && q < k_end && P.store) {
                bst(rb0, lc, so, v);
                if (ACC) r2a += (double)rt * (double)rt;
            }
        }
        ring[SL][rw][tx] = rq;
        __syncthreads();
        const int qb = q - 1;
        if (qb >= k_begin) {
            const float oth = lane_perm(P.src, rm1);
            const float ps = ring[SLP][rw - 1][tx], pn = ring[SLP][rw + 1][tx];
            const bool end_plane = qb == 0 || qb == g.nz - 1;
            const float inv = end_plane ? P.inv_end : P.inv_mid;
            float rt;
            const float v = sor_relax(sor_nb(rm1, oth, ps, pn, rm2, rq, cx, cy, cz), inv, cur.rr1, bm, omega,
                                      rt);
            if (P.store) {
                bst(rb1, lbw, so, v);
                if (ACC) {
                    const float diag = P.dxy + (end_plane ? dz_end : dz_mid);
                    const double rd = (double)rt;
                    r2b += rd * rd;
                    d2b += ((double)diag * rd) * ((double)diag * rd);
                }
            }
        }
        bm = bc;
        bc = cur.up;
        rm2 = rm1;
        rm1 = rq;
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    using S3 = std::integral_constant<int, 3>;
    RbIn A, B;
    fetch(qa, so0, A, pe);
    int q = qa;
    unsigned so = so0;
    for (; q + 3 <= k_end; q += 4, so += 4 * sp4) {
        step(S0{}, q, so, A, B, pe, po);
        step(S1{}, q + 1, so + sp4, B, A, po, pe);
        step(S2{}, q + 2, so + 2 * sp4, A, B, pe, po);
        step(S3{}, q + 3, so + 3 * sp4, B, A, po, pe);
    }
    if (q <= k_end) step(S0{}, q, so, A, B, pe, po);
    if (q + 1 <= k_end) step(S1{}, q + 1, so + sp4, B, A, po, pe);
    if (q + 2 <= k_end) step(S2{}, q + 2, so + 2 * sp4, A, B, pe, po);
    if (ACC) {
        const double va = wave_sum(r2a), vb = wave_sum(r2b), vd = wave_sum(d2b);
        const int wid = threadIdx.x >> 6;
        if (lane == 0) {
            red3[0][wid] = va;
            red3[1][wid] = vb;
            red3[2][wid] = vd;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0, td = 0.0;
            for (int w = 0; w < NW; ++w) {
                ta += red3[0][w];
                tb += red3[1][w];
                td += red3[2][w];
            }
            rel0[2 * lb] = ta;
            rel0[2 * lb + 1] = 0.0;
            rel1[2 * lb] = tb;
            rel1[2 * lb + 1] = td;
        }
    }
}

// An iteration past max_iter inside the last check interval, uniform grid:
// the block copies its tile of both colours from a to b, so the result
// stays in the buffer the interval ends on (the same cells sor_rb_body
// copies; a missing cell at the end of an odd-length row holds 0 in both).
template <int TX, int NW, int KT>
__device__ __forceinline__ void sor_rb_copy_u(const Geo& g, const float* __restrict__ a0,
                                              const float* __restrict__ a1, float* __restrict__ b0,
                                              float* __restrict__ b1, unsigned lb, int kt_run) {
    constexpr int RPW = 64 / TX;
    constexpr int TYB = RPW * NW;
    constexpr int TXO = TX - 2, TYO = TYB - 2;
    const int kt = KT > 0 ? KT : kt_run;
    const unsigned nbx = (unsigned)(g.H + TXO - 1) / TXO;
    const unsigned nby = (unsigned)(g.ny + TYO - 1) / TYO;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int tx = lane % TX;
    const int row = (threadIdx.x >> 6) * RPW + lane / TX;
    const int ii = (int)bx * TXO - 1 + tx, j = (int)by * TYO - 1 + row;
    const bool inner = ii >= 0 && ii < g.H && j >= 0 && j < g.ny && tx >= 1 && tx <= TX - 2 && row >= 1 &&
                       row <= TYB - 2;
    if (!inner) return;
    const int k_begin = (int)bk * kt;
    const int k_end = min(g.nz, k_begin + kt);
    for (int k = k_begin; k < k_end; ++k) {
        const long long e = g.col(ii, j, k);
        b0[e] = a0[e];
        b1[e] = a1[e];
    }
}

// ------------------------------------- two fused red-black iterations
// Two whole SOR iterations in one pass (temporal blocking): the four
// colour updates A (colour 0, iteration 1), B (colour 1, iteration 1),
// C (colour 0, iteration 2) and D (colour 1, iteration 2) run in one k-march,
// each one plane behind the previous: at step q, A on plane q, B on q-1,
// C on q-2, D on q-3.  Reads come from the old arrays (a0, a1, r0, r1),
// iteration 1 lives only in registers and LDS, and C and D go to the other
// buffer pair (b0, b1): 12 bytes per cell for two iterations instead of
// 24.  Each stage needs its predecessor on the cell's six neighbours, so a
// block recomputes a ring that shrinks by one cell per stage: of its 64
// lanes x 32 rows x (kt + 6) planes it writes the 58 x 26 x kt centre.
// The per-cell arithmetic is that of the half-sweeps (sor_point /
// sor_point_w), so the result equals four half-sweeps bit for bit.
//
// A block is 16 wavefronts of 64 lanes; each thread owns rows w and w + 16
// of its lane.  Own-column neighbours along k come from registers, east /
// west from cross-lane shuffles (edge lanes of stage A load theirs), north /
// south from LDS rows of the stage before (two planes per stage ring: the
// slot written at step q was last read at step q - 1, a barrier earlier).
// With `second` false (the interval's iteration budget ends after the first
// iteration) C and D copy the iteration-1 values; with `first` false too
// the block copies a to b.  acc1 / acc2: leave the float64 partials of the
// first / second iteration (the one that ends the check interval), as the
// single-iteration kernel does.
template <bool STR>
__device__ __forceinline__ float rb_relax(const Geo& g, int i0, int j, int k, float west, float east,
                                          float ps, float pn, float pb, float pt, float r, float p,
                                          float omega, float& rt) {
    if constexpr (STR) {
        const float diag = mrow(g.mx, g.nx, M_DD, i0 + 1) + mrow(g.my, g.ny, M_DD, j + 1) +
                           mrow(g.mz, g.nz, M_DD, k + 1);
        return sor_point_w(west, east, ps, pn, pb, pt, mrow(g.mx, g.nx, M_WM, i0 + 1),
                           mrow(g.mx, g.nx, M_WP, i0 + 1), mrow(g.my, g.ny, M_WM, j + 1),
                           mrow(g.my, g.ny, M_WP, j + 1), mrow(g.mz, g.nz, M_WM, k + 1),
                           mrow(g.mz, g.nz, M_WP, k + 1), diag, r, p, omega, rt);
    } else {
        const float diag = diag_x(g, i0) + diag_y(g, j) + diag_z(g, k);
        return sor_point(west, east, ps, pn, pb, pt, g.cx, g.cy, g.cz, diag, r, p, omega, rt);
    }
}
template <bool STR>
__device__ __forceinline__ float rb_diag(const Geo& g, int i0, int j, int k) {
    if constexpr (STR)
        return mrow(g.mx, g.nx, M_DD, i0 + 1) + mrow(g.my, g.ny, M_DD, j + 1) + mrow(g.mz, g.nz, M_DD, k + 1);
    else
        return diag_x(g, i0) + diag_y(g, j) + diag_z(g, k);
}

template <bool STR>
__device__ __forceinline__ void sor_rb2_body(const Geo& g, const float* __restrict__ a0,
                                             const float* __restrict__ a1,
                                             const float* __restrict__ r0c,
                                             const float* __restrict__ r1c, float* __restrict__ b0,
                                             float* __restrict__ b1, float omega, bool first,
                                             bool second, bool acc1, bool acc2,
                                             double* __restrict__ rel0, double* __restrict__ rel1,
                                             unsigned lb, int kt) {
    const bool acc = acc1 || acc2;   // partials of the iteration that ends the check interval
    constexpr int R = kRb2RowsPerThread;
    __shared__ float ringA[2][kRb2Rows][64];
    __shared__ float ringB[2][kRb2Rows][64];
    __shared__ float ringC[2][kRb2Rows][64];
    __shared__ double red3[3][16];
    const unsigned nbx = (unsigned)(g.H + kRb2TXO - 1) / kRb2TXO;
    const unsigned nby = (unsigned)(g.ny + kRb2TYO - 1) / kRb2TYO;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int ii = (int)bx * kRb2TXO - 3 + lane;
    const int k_begin = (int)bk * kt;
    const int k_end = min(g.nz, k_begin + kt);
    const bool lane_ok = ii >= 0 && ii < g.H;
    const bool out_lane = lane >= 3 && lane <= 60;
    const bool edge_lane = lane == 0 || lane == 63;
    const int edge_off = lane == 0 ? -1 : 1;
    int row[R], j[R];
    bool col_ok[R], out_ok[R];
    long long e0[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        row[t] = wv + 16 * t;
        j[t] = (int)by * kRb2TYO - 3 + row[t];
        col_ok[t] = lane_ok && j[t] >= 0 && j[t] < g.ny;
        out_ok[t] = col_ok[t] && out_lane && row[t] >= 3 && row[t] <= 28;
        e0[t] = col_ok[t] ? g.col(ii, j[t], k_begin - 3) : 0;
    }
    // per-row register pipelines (planes relative to the step q)
    float bm[R], bc[R];                       // old colour 1 at q-1, q
    float aQ[R], aM1[R], aM2[R];              // A at q, q-1, q-2
    float bQ1[R], bQ2[R], bQ3[R];             // B at q-1, q-2, q-3
    float cQ2[R], cQ3[R], cQ4[R];             // C at q-2, q-3, q-4
    float r0q[R], r0m1[R], r0m2[R];           // r0 colour 0 at q, q-1, q-2
    float r1m1[R], r1m2[R], r1m3[R];          // r0 colour 1 at q-1, q-2, q-3
    struct Ld { float up, south, north, edge, p0, rr0, rr1; };
    Ld cur[R], nxt[R], nxt2[R];   // loads of steps q, q+1, q+2 (issued two steps ahead)
    const int q0 = k_begin - 3;
    auto fetch = [&](int q, Ld* f) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const long long e = e0[t] + (long long)(q - q0) * g.SP;
            const bool pl = col_ok[t] && q >= 0 && q < g.nz;
            f[t].up = (col_ok[t] && q + 1 >= 0 && q + 1 <= g.nz) ? a1[e + g.SP] : 0.f;
            f[t].south = pl ? a1[e - g.S] : 0.f;
            f[t].north = pl ? a1[e + g.S] : 0.f;
            f[t].edge = (pl && edge_lane) ? a1[e + edge_off] : 0.f;
            f[t].p0 = pl ? a0[e] : 0.f;
            f[t].rr0 = pl ? r0c[e] : 0.f;
            f[t].rr1 = (col_ok[t] && q - 1 >= 0 && q - 1 < g.nz) ? r1c[e - g.SP] : 0.f;
        }
    };
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const bool okm = col_ok[t] && q0 - 1 >= -1;
        bm[t] = okm ? a1[e0[t] - g.SP] : 0.f;
        bc[t] = col_ok[t] && q0 >= -1 ? a1[e0[t]] : 0.f;
        aQ[t] = aM1[t] = aM2[t] = 0.f;
        bQ1[t] = bQ2[t] = bQ3[t] = 0.f;
        cQ2[t] = cQ3[t] = cQ4[t] = 0.f;
        r0q[t] = r0m1[t] = r0m2[t] = 0.f;
        r1m1[t] = r1m2[t] = r1m3[t] = 0.f;
    }
    double sC = 0.0, sD = 0.0, dD = 0.0;
    fetch(q0, cur);
    fetch(q0 + 1, nxt);
    for (int q = q0; q <= k_end + 2; ++q) {
        if (q + 2 <= k_end + 2) fetch(q + 2, nxt2);
        // ---- A: colour 0, iteration 1, plane q (old colour 1 around it)
#pragma unroll
        for (int t = 0; t < R; ++t) {
            float be = __shfl_down(bc[t], 1, 64);
            float bw = __shfl_up(bc[t], 1, 64);
            if (lane == 63) be = cur[t].edge;
            if (lane == 0) bw = cur[t].edge;
            const int s = (j[t] + q) & 1;
            const int i0 = 2 * ii + s;
            float v = 0.f;
            if (col_ok[t] && q >= 0 && q < g.nz && i0 < g.nx) {
                float rt = 0.f;
                v = first ? rb_relax<STR>(g, i0, j[t], q, s ? bc[t] : bw, s ? be : bc[t], cur[t].south,
                                          cur[t].north, bm[t], cur[t].up, cur[t].rr0, cur[t].p0, omega, rt)
                          : cur[t].p0;
                if (acc1 && out_ok[t] && q >= k_begin && q < k_end) sC += (double)rt * (double)rt;
            }
            aM2[t] = aM1[t];
            aM1[t] = aQ[t];
            aQ[t] = v;
            r0m2[t] = r0m1[t];
            r0m1[t] = r0q[t];
            r0q[t] = cur[t].rr0;
            ringA[q & 1][row[t]][lane] = v;
        }
        __syncthreads();
        // ---- B: colour 1, iteration 1, plane q-1 (A around it)
        const int qb = q - 1;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const float ae = __shfl_down(aM1[t], 1, 64);
            const float aw = __shfl_up(aM1[t], 1, 64);
            const int s = (1 + j[t] + qb) & 1;
            const int i1 = 2 * ii + s;
            float v = 0.f, rtb = 0.f;
            const float old1 = bm[t];   // old colour 1 at q-1
            if (col_ok[t] && qb >= 0 && qb < g.nz && i1 < g.nx) {
                const float sn = row[t] > 0 ? ringA[qb & 1][row[t] - 1][lane] : 0.f;
                const float nn = row[t] < kRb2Rows - 1 ? ringA[qb & 1][row[t] + 1][lane] : 0.f;
                v = first ? rb_relax<STR>(g, i1, j[t], qb, s ? aM1[t] : aw, s ? ae : aM1[t], sn, nn, aM2[t],
                                          aQ[t], cur[t].rr1, old1, omega, rtb)
                          : old1;
            }
            bQ3[t] = bQ2[t];
            bQ2[t] = bQ1[t];
            bQ1[t] = v;
            r1m3[t] = r1m2[t];
            r1m2[t] = r1m1[t];
            r1m1[t] = cur[t].rr1;
            if (acc1 && out_ok[t] && qb >= k_begin && qb < k_end && i1 < g.nx) {
                sD += (double)rtb * (double)rtb;
                const double dd = (double)rb_diag<STR>(g, i1, j[t], qb) * (double)rtb;
                dD += dd * dd;
            }
            ringB[qb & 1][row[t]][lane] = v;
        }
        __syncthreads();
        // ---- C: colour 0, iteration 2, plane q-2 (B around it)
        const int qc = q - 2;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const float be2 = __shfl_down(bQ2[t], 1, 64);
            const float bw2 = __shfl_up(bQ2[t], 1, 64);
            const int s = (j[t] + qc) & 1;
            const int i0 = 2 * ii + s;
            float v = 0.f;
            if (col_ok[t] && qc >= 0 && qc < g.nz && i0 < g.nx) {
                const float sn = row[t] > 0 ? ringB[qc & 1][row[t] - 1][lane] : 0.f;
                const float nn = row[t] < kRb2Rows - 1 ? ringB[qc & 1][row[t] + 1][lane] : 0.f;
                float rt = 0.f;
                v = second ? rb_relax<STR>(g, i0, j[t], qc, s ? bQ2[t] : bw2, s ? be2 : bQ2[t], sn, nn,
                                           bQ3[t], bQ1[t], r0m2[t], aM2[t], omega, rt)
                           : aM2[t];
                if (out_ok[t] && qc >= k_begin && qc < k_end) {
                    b0[e0[t] + (long long)(qc - q0) * g.SP] = v;
                    if (acc2) sC += (double)rt * (double)rt;
                }
            }
            cQ4[t] = cQ3[t];
            cQ3[t] = cQ2[t];
            cQ2[t] = v;
            ringC[qc & 1][row[t]][lane] = v;
        }
        __syncthreads();
        // ---- D: colour 1, iteration 2, plane q-3 (C around it)
        const int qd = q - 3;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const float ce = __shfl_down(cQ3[t], 1, 64);
            const float cw = __shfl_up(cQ3[t], 1, 64);
            const int s = (1 + j[t] + qd) & 1;
            const int i1 = 2 * ii + s;
            if (out_ok[t] && qd >= k_begin && qd < k_end && i1 < g.nx) {
                const float sn = ringC[qd & 1][row[t] - 1][lane];
                const float nn = ringC[qd & 1][row[t] + 1][lane];
                float rt = 0.f;
                const float v = second ? rb_relax<STR>(g, i1, j[t], qd, s ? cQ3[t] : cw, s ? ce : cQ3[t], sn, nn,
                                                       cQ4[t], cQ2[t], r1m3[t], bQ3[t], omega, rt)
                                       : bQ3[t];
                b1[e0[t] + (long long)(qd - q0) * g.SP] = v;
                if (acc2) {
                    const double rd = (double)rt;
                    sD += rd * rd;
                    const double dd = (double)rb_diag<STR>(g, i1, j[t], qd) * rd;
                    dD += dd * dd;
                }
            }
        }
        // advance the old colour 1 and the loads
#pragma unroll
        for (int t = 0; t < R; ++t) {
            bm[t] = bc[t];
            bc[t] = cur[t].up;
            cur[t] = nxt[t];
            nxt[t] = nxt2[t];
        }
    }
    if (acc) {
        const double va = wave_sum(sC), vb = wave_sum(sD), vd = wave_sum(dD);
        if (lane == 0) {
            red3[0][wv] = va;
            red3[1][wv] = vb;
            red3[2][wv] = vd;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0, td = 0.0;
            for (int w = 0; w < 16; ++w) {
                ta += red3[0][w];
                tb += red3[1][w];
                td += red3[2][w];
            }
            rel0[2 * lb] = ta;
            rel0[2 * lb + 1] = 0.0;
            rel1[2 * lb] = tb;
            rel1[2 * lb + 1] = td;
        }
    }
}

// ------------------------------ two fused iterations, uniform grids (lean)
// The two iterations of sor_rb2_body on a uniform grid with the lean
// sweep's arrangement: buffer loads at a block-uniform scalar offset plus a
// per-lane byte offset, lanes outside the grid on the zero padding column
// (cn1 = 0 there and at the missing cell of an odd-length row, so every
// stage leaves them exactly 0), rows outside the grid skipped as a whole
// (a row is one wavefront), one parity per step for all four stages and
// both rows of a thread.  Load planes are clamped into the ghost planes -1
// and nz, which hold zeros: exactly the values the stages take outside the
// grid.  Register pipelines are indexed by plane modulo 3 and the march is
// unrolled by six, so no value is moved between registers; one barrier per
// step suffices (every stage reads the LDS rows of planes written in the
// previous step, and the two-slot rings are rewritten only after that
// step's barrier).  Same per-cell arithmetic as sor_rb2_body: bit for bit.
// LDS of one block (declared once per kernel, shared by both instantiations)
struct Rb2Smem {
    float ringA[2][kRb2Rows + 2][64];   // tile row r at index r + 1 (guard rows 0 and kRb2Rows + 1)
    float ringB[2][kRb2Rows + 2][64];
    float ringC[2][kRb2Rows + 2][64];
    double red3[3][16];
};

// plane modes of a two-iteration step (below): general, interior
constexpr int kQGen = -1000, kQInt = -2000;

template <bool ACC>
__device__ __forceinline__ void sor_rb2_body_u(Rb2Smem& sm, const Geo& g, const float* __restrict__ a0,
                                               const float* __restrict__ a1,
                                               const float* __restrict__ r0c,
                                               const float* __restrict__ r1c, float* __restrict__ b0,
                                               float* __restrict__ b1, float omega, bool second,
                                               bool acc1, bool acc2, double* __restrict__ rel0,
                                               double* __restrict__ rel1, unsigned lb, int kt) {
    constexpr int R = kRb2RowsPerThread;
    constexpr int NR = kRb2Rows;
    static_assert(R == 2 && NR == 32, "one thread: rows w and w + 16 of a 32-row tile");
    auto& ringA = sm.ringA;
    auto& ringB = sm.ringB;
    auto& ringC = sm.ringC;
    auto& red3 = sm.red3;
    const unsigned nbx = (unsigned)(g.H + kRb2TXO - 1) / kRb2TXO;
    const unsigned nby = (unsigned)(g.ny + kRb2TYO - 1) / kRb2TYO;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ii0 = (int)bx * kRb2TXO - 3, j0 = (int)by * kRb2TYO - 3;
    const int ii = ii0 + lane;
    const int k_begin = (int)bk * kt;
    const int k_end = min(g.nz, k_begin + kt);
    const int qs = k_begin - 3;
    const bool lane_ok = ii >= 0 && ii < g.H;
    const bool out_lane = lane >= 3 && lane <= 60;
    // rows of this wavefront (uniform): wv and wv + 16
    int jr[R];
    bool row_ok[R], out_row[R];
    float dyy[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int row = wv + 16 * t;
        jr[t] = j0 + row;
        row_ok[t] = jr[t] >= 0 && jr[t] < g.ny;
        out_row[t] = row_ok[t] && row >= 3 && row <= NR - 4;
        dyy[t] = diag_y(g, jr[t]);
    }
    // guard rows of the rings read as 0
    if (threadIdx.x < 64) {
        for (int s = 0; s < 2; ++s) {
            ringA[s][0][lane] = ringA[s][NR + 1][lane] = 0.f;
            ringB[s][0][lane] = ringB[s][NR + 1][lane] = 0.f;
            ringC[s][0][lane] = ringC[s][NR + 1][lane] = 0.f;
        }
    }
    // lane byte offsets from the row's origin on a plane (one plane, one row
    // and one element before the lane-0 column of the row)
    const int iic = lane_ok ? ii : g.H;
    const unsigned lc = (unsigned)((iic - ii0) + 1 + g.S + g.SP) * 4u;
    const unsigned ls = lc - (unsigned)g.S * 4u, ln = lc + (unsigned)g.S * 4u;
    const float dz_mid = g.cz + g.cz, dz_end = diag_z(g, 0);
    // per-parity lane constants (parity of the steps q - qs even / odd;
    // all four stages of a step and both rows share it)
    struct Par {
        unsigned lx;         // stage A's x-neighbour of the other colour
        int src;             // ds_bpermute source of stages B, C, D's x-neighbour
        float dx;            // diag_x of the cell
        float im[R], ie[R];  // cn1, interior and end planes, per row (0: no cell)
        bool own;            // the lane owns its cell in the tile's output columns
    } pe, po;
    {
        const int se = (j0 + wv + qs) & 1;
        auto make = [&](int s, Par& P) {
            const int i0 = 2 * ii + s;
            const bool ok = lane_ok && i0 < g.nx;
            P.lx = lane_ok ? (s ? lc + 4u : lc - 4u) : lc;
            P.src = ((s ? lane + 1 : lane - 1) & 63) * 4;
            P.dx = diag_x(g, i0);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const float dxy = P.dx + dyy[t];
                P.im[t] = ok && row_ok[t] ? 1.0f / (dxy + dz_mid) : 0.f;
                P.ie[t] = ok && row_ok[t] ? 1.0f / (dxy + dz_end) : 0.f;
            }
            P.own = ok && out_lane;
        };
        make(se, pe);
        make(se ^ 1, po);
    }
    const Rsrc ra0 = colour_rsrc(g, a0), ra1 = colour_rsrc(g, a1), rr0c = colour_rsrc(g, r0c),
               rr1c = colour_rsrc(g, r1c), rb0 = colour_rsrc(g, b0), rb1 = colour_rsrc(g, b1);
    const unsigned sp4 = (unsigned)g.SP * 4u;
    // scalar byte offset of row t's origin on plane p, p clamped into the
    // planes -1 .. nz (those outside read the ghost planes' zeros)
    // (rows outside the grid address the ghost row -1, which holds zeros in
    // every array; with cn1 = 0 their updates are exactly 0)
    unsigned so_row[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int jc = row_ok[t] ? jr[t] : -1;
        so_row[t] = (unsigned)(((long long)g.S + ((long long)jc + 1) * g.S + ii0 - 1 - g.S - g.SP + 2 * g.SP) * 4);
    }
    auto so_at = [&](int t, int p) -> unsigned {
        const int pc = min(max(p, -1), g.nz);
        return so_row[t] + (unsigned)(pc + 1) * sp4;
    };
    const float cx = g.cx, cy = g.cy, cz = g.cz;
    // pipelines, indexed by plane modulo 3 (plane p at (p - qs) % 3)
    float oc[3][R];   // old colour 1
    float av[3][R];   // A: colour 0, iteration 1
    float bv[3][R];   // B: colour 1, iteration 1
    float cv[3][R];   // C: colour 0, iteration 2
    float r0v[3][R];  // r0 of colour 0
    float r1v[3][R];  // r0 of colour 1
    // loads two steps ahead: step T reads buffer T & 1, then refills it with
    // the loads of step T + 2
    struct Ld { float up, south, north, xn, p0, rr0, rr1; } ld[2][R];
    auto fetch = [&](int q, const Par& P, Ld* L) {   // loads of step q (plane q; rr1 of plane q - 1)
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const unsigned so = so_at(t, q);
            L[t].up = bld(ra1, lc, so_at(t, q + 1));
            L[t].south = bld(ra1, ls, so);
            L[t].north = bld(ra1, ln, so);
            L[t].xn = bld(ra1, P.lx, so);
            L[t].p0 = bld(ra0, lc, so);
            L[t].rr0 = bld(rr0c, lc, so);
            L[t].rr1 = bld(rr1c, lc, so_at(t, q - 1));
        }
    };
    double sC = 0.0, sD = 0.0, dD = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
        // old colour 1 on planes qs - 1 and qs (ghost zeros below the grid)
        oc[2][t] = bld(ra1, lc, so_at(t, qs - 1));
        oc[0][t] = bld(ra1, lc, so_at(t, qs));
#pragma unroll
        for (int m = 0; m < 3; ++m) av[m][t] = bv[m][t] = cv[m][t] = r0v[m][t] = r1v[m][t] = 0.f;
    }
    fetch(qs, pe, ld[0]);
    fetch(qs + 1, po, ld[1]);
    __syncthreads();   // guard rows written

    // step q = qs + T: A on q, B on q-1, C on q-2, D on q-3.  Every stage
    // runs on every row and plane (rows outside the grid and planes outside
    // it come out as exact zeros through cn1 = 0), so no stage branches.
    // The plane mode QM: kQInt when all four planes lie in 1 .. nz-2 (cn1 is
    // the interior one), a plane number when q is known at compile time (the
    // bottom of the column, with nz >= 10 so that no plane there is nz-1),
    // kQGen otherwise; the first two imply a live second iteration.
    auto step = [&](auto tc, auto qm, int q, const Par& P) {
        constexpr int T = decltype(tc)::value;
        constexpr int QM = decltype(qm)::value;
        constexpr bool INT = QM == kQInt;
        constexpr bool KNOWN = QM > kQGen;
        constexpr bool LIVE2 = INT || KNOWN;
        // cn1 of row t on plane pl = q - S: 0 outside the grid's planes, where
        // the update then returns p = 0 exactly (the ghost planes hold zeros)
        auto inv_at = [&](auto sc, int t, int pl) -> float {
            constexpr int S = decltype(sc)::value;
            if constexpr (INT) {
                return P.im[t];
            } else if constexpr (KNOWN) {
                constexpr int pk = QM - S;
                if constexpr (pk < 0) return 0.f;
                else if constexpr (pk == 0) return P.ie[t];
                else return P.im[t];
            } else {
                const float c = (pl == 0 || pl == g.nz - 1) ? P.ie[t] : P.im[t];
                return (pl >= 0 && pl < g.nz) ? c : 0.f;
            }
        };
        auto end_plane = [&](auto sc, int pl) -> bool {
            constexpr int S = decltype(sc)::value;
            if constexpr (INT) return false;
            else if constexpr (KNOWN) return QM - S == 0;
            else return pl == 0 || pl == g.nz - 1;
        };
        using S0c = std::integral_constant<int, 0>;
        using S1c = std::integral_constant<int, 1>;
        using S2c = std::integral_constant<int, 2>;
        using S3c = std::integral_constant<int, 3>;
        constexpr int M0 = T % 3, M1 = (T + 2) % 3, M2 = (T + 1) % 3;   // planes q, q-1, q-2 (q-3: M0)
        constexpr int S0 = T & 1, S1 = (T + 1) & 1;                     // ring slots of q, q-1 (q-2: S0, q-3: S1)
        const int qb = q - 1, qc = q - 2, qd = q - 3;
        Ld* ldc = ld[S0];
        // ---- A: colour 0, iteration 1, plane q
#pragma unroll
        for (int t = 0; t < R; ++t) {
            float rt;
            const float v = sor_relax(sor_nb(oc[M0][t], ldc[t].xn, ldc[t].south, ldc[t].north, oc[M1][t],
                                             ldc[t].up, cx, cy, cz),
                                      inv_at(S0c{}, t, q), ldc[t].rr0, ldc[t].p0, omega, rt);
            if (ACC && acc1 && out_row[t] && q >= k_begin && q < k_end && P.own) sC += (double)rt * (double)rt;
            av[M0][t] = v;
            r0v[M0][t] = ldc[t].rr0;
            r1v[M1][t] = ldc[t].rr1;
            oc[M2][t] = ldc[t].up;   // old colour 1 on plane q + 1 (slot of q - 2, no longer needed)
            ringA[S0][wv + 16 * t + 1][lane] = v;
        }
        if (q + 1 < qs + 5 + (k_end - k_begin)) fetch(q + 2, P, ldc);   // loads of step q + 2 (same parity)
        // ---- B: colour 1, iteration 1, plane q-1
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const float oth = lane_perm(P.src, av[M1][t]);
            const int rw = wv + 16 * t + 1;
            const float ps = ringA[S1][rw - 1][lane], pn = ringA[S1][rw + 1][lane];
            float rt;
            const float v = sor_relax(sor_nb(av[M1][t], oth, ps, pn, av[M2][t], av[M0][t], cx, cy, cz),
                                      inv_at(S1c{}, t, qb), r1v[M1][t], oc[M1][t], omega, rt);
            if (ACC && acc1 && out_row[t] && qb >= k_begin && qb < k_end && P.own) {
                const double rd = (double)rt;
                sD += rd * rd;
                const bool endp = end_plane(S1c{}, qb);
                const double dd = (double)((P.dx + dyy[t]) + (endp ? dz_end : dz_mid)) * rd;
                dD += dd * dd;
            }
            bv[M1][t] = v;
            ringB[S1][rw][lane] = v;
        }
        // ---- C: colour 0, iteration 2, plane q-2
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const float oth = lane_perm(P.src, bv[M2][t]);
            const int rw = wv + 16 * t + 1;
            const float ps = ringB[S0][rw - 1][lane], pn = ringB[S0][rw + 1][lane];
            float rt;
            const float w = sor_relax(sor_nb(bv[M2][t], oth, ps, pn, bv[M0][t], bv[M1][t], cx, cy, cz),
                                      inv_at(S2c{}, t, qc), r0v[M2][t], av[M2][t], omega, rt);
            const float v = (LIVE2 || second) ? w : av[M2][t];
            if (out_row[t] && qc >= k_begin && qc < k_end && P.own) {
                bst(rb0, lc, so_at(t, qc), v);
                if (ACC && acc2) sC += (double)rt * (double)rt;
            }
            cv[M2][t] = v;
            ringC[S0][rw][lane] = v;
        }
        // ---- D: colour 1, iteration 2, plane q-3
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (out_row[t] && qd >= k_begin && qd < k_end) {
                const float oth = lane_perm(P.src, cv[M0][t]);
                const int rw = wv + 16 * t + 1;
                const float ps = ringC[S1][rw - 1][lane], pn = ringC[S1][rw + 1][lane];
                const bool endp = end_plane(S3c{}, qd);
                const float inv = inv_at(S3c{}, t, qd);
                float rt = 0.f;
                const float w = sor_relax(sor_nb(cv[M0][t], oth, ps, pn, cv[M1][t], cv[M2][t], cx, cy, cz), inv,
                                          r1v[M0][t], bv[M0][t], omega, rt);
                const float v = (LIVE2 || second) ? w : bv[M0][t];
                if (P.own) {
                    bst(rb1, lc, so_at(t, qd), v);
                    if (ACC && acc2) {
                        const double rd = (double)rt;
                        sD += rd * rd;
                        const double dd = (double)((P.dx + dyy[t]) + (endp ? dz_end : dz_mid)) * rd;
                        dD += dd * dd;
                    }
                }
            }
        }
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using Gen = std::integral_constant<int, kQGen>;
    using Int = std::integral_constant<int, kQInt>;
    auto gen6 = [&](int q) {
        step(I0{}, Gen{}, q, pe);
        step(I1{}, Gen{}, q + 1, po);
        step(I2{}, Gen{}, q + 2, pe);
        step(I3{}, Gen{}, q + 3, po);
        step(I4{}, Gen{}, q + 4, pe);
        step(I5{}, Gen{}, q + 5, po);
    };
    auto int6 = [&](int q) {
        step(I0{}, Int{}, q, pe);
        step(I1{}, Int{}, q + 1, po);
        step(I2{}, Int{}, q + 2, pe);
        step(I3{}, Int{}, q + 3, po);
        step(I4{}, Int{}, q + 4, pe);
        step(I5{}, Int{}, q + 5, po);
    };
    auto pl = [](auto c) { return std::integral_constant<int, decltype(c)::value>{}; };
    const int q_last = k_end + 2;
    int q = qs;
    // the bottom column (qs = -3): its first twelve steps, planes -6 .. 8,
    // with every plane known at compile time
    if (k_begin == 0 && second && q_last >= qs + 11 && g.nz >= 10) {
        step(I0{}, pl(std::integral_constant<int, -3>{}), -3, pe);
        step(I1{}, pl(std::integral_constant<int, -2>{}), -2, po);
        step(I2{}, pl(std::integral_constant<int, -1>{}), -1, pe);
        step(I3{}, pl(std::integral_constant<int, 0>{}), 0, po);
        step(I4{}, pl(std::integral_constant<int, 1>{}), 1, pe);
        step(I5{}, pl(std::integral_constant<int, 2>{}), 2, po);
        step(I0{}, pl(std::integral_constant<int, 3>{}), 3, pe);
        step(I1{}, pl(std::integral_constant<int, 4>{}), 4, po);
        step(I2{}, pl(std::integral_constant<int, 5>{}), 5, pe);
        step(I3{}, pl(std::integral_constant<int, 6>{}), 6, po);
        step(I4{}, pl(std::integral_constant<int, 7>{}), 7, pe);
        step(I5{}, pl(std::integral_constant<int, 8>{}), 8, po);
        q = qs + 12;
    }
    // groups of six steps: those whose planes q-3 .. q+5 all lie in 1 .. nz-2
    // form one run in the middle of the march (uniform bounds)
    for (; q + 5 <= q_last && q - 3 < 1; q += 6) gen6(q);
    for (; second && q + 5 <= q_last && q + 5 <= g.nz - 2; q += 6) int6(q);
    for (; q + 5 <= q_last; q += 6) gen6(q);
    if (q <= q_last) {
        if (second && q - 3 >= 1 && q <= g.nz - 2) step(I0{}, Int{}, q, pe);
        else step(I0{}, Gen{}, q, pe);
    }
    if (q + 1 <= q_last) step(I1{}, Gen{}, q + 1, po);
    if (q + 2 <= q_last) step(I2{}, Gen{}, q + 2, pe);
    if (q + 3 <= q_last) step(I3{}, Gen{}, q + 3, po);
    if (q + 4 <= q_last) step(I4{}, Gen{}, q + 4, pe);
    if (ACC) {
        const double va = wave_sum(sC), vb = wave_sum(sD), vd = wave_sum(dD);
        if (lane == 0) {
            red3[0][wv] = va;
            red3[1][wv] = vb;
            red3[2][wv] = vd;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0, td = 0.0;
            for (int w = 0; w < 16; ++w) {
                ta += red3[0][w];
                tb += red3[1][w];
                td += red3[2][w];
            }
            rel0[2 * lb] = ta;
            rel0[2 * lb + 1] = 0.0;
            rel1[2 * lb] = tb;
            rel1[2 * lb + 1] = td;
        }
    }
}

// Both iterations past max_iter (the first one already): the block copies
// its output tile of both colours from a to b (rb2 tiling).
__device__ __forceinline__ void sor_rb2_copy_u(const Geo& g, const float* __restrict__ a0,
                                               const float* __restrict__ a1, float* __restrict__ b0,
                                               float* __restrict__ b1, unsigned lb, int kt) {
    const unsigned nbx = (unsigned)(g.H + kRb2TXO - 1) / kRb2TXO;
    const unsigned nby = (unsigned)(g.ny + kRb2TYO - 1) / kRb2TYO;
    const unsigned bx = lb % nbx;
    const unsigned rr = lb / nbx;
    const unsigned by = rr % nby;
    const unsigned bk = rr / nby;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int ii = (int)bx * kRb2TXO - 3 + lane;
    if (!(ii >= 0 && ii < g.H && lane >= 3 && lane <= 60)) return;
    const int k_begin = (int)bk * kt;
    const int k_end = min(g.nz, k_begin + kt);
    for (int t = 0; t < kRb2RowsPerThread; ++t) {
        const int row = wv + 16 * t;
        const int j = (int)by * kRb2TYO - 3 + row;
        if (j < 0 || j >= g.ny || row < 3 || row > kRb2Rows - 4) continue;
        for (int k = k_begin; k < k_end; ++k) {
            const long long e = g.col(ii, j, k);
            b0[e] = a0[e];
            b1[e] = a1[e];
        }
    }
}

// ------------------------------------------------------------- fold
// ph <- fl(ph + pd), pd <- exact remainder (Knuth's TwoSum), pointwise over
// the whole colour arrays (padding stays 0 + 0 = 0).
__device__ __forceinline__ void fold_body(long long n, float* __restrict__ ph0,
                                          float* __restrict__ pd0, float* __restrict__ ph1,
                                          float* __restrict__ pd1, long long t) {
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

// The float64 operator of the residual, rebase and check: the diagonal
// at 0-based cell (i0, j0, k0), and (A x) there from the float32 colour
// arrays x_own / x_oth.  Uniform grids: 1/h^2 in float64; stretched grids:
// the float64 weight tables.  (The sweeps use the float32 weights; with
// the residual in float64 the fold-and-rebase cycle refines towards the
// float64 operator's solution, so rounding of the weights -- exact for
// power-of-two spacings, not otherwise -- does not bias the result.)
__device__ __forceinline__ double wrow(const double* __restrict__ m, int n, int row, int c) {
    return m[row * (n + 2) + c];
}
template <bool STR = false>
__device__ __forceinline__ double diag64(const Geo& g, int i0, int j0, int k0) {
    if constexpr (STR) {
        return wrow(g.wx, g.nx, 2, i0 + 1) + wrow(g.wy, g.ny, 2, j0 + 1) + wrow(g.wz, g.nz, 2, k0 + 1);
    } else {
        const double dx = (i0 > 0 ? g.cxd : 0.0) + (i0 < g.nx - 1 ? g.cxd : (g.outflow ? 2.0 * g.cxd : 0.0));
        const double dy = (j0 > 0 ? g.cyd : 0.0) + (j0 < g.ny - 1 ? g.cyd : 0.0);
        const double dz = (k0 > 0 ? g.czd : 0.0) + (k0 < g.nz - 1 ? g.czd : 0.0);
        return dx + dy + dz;
    }
}
template <bool STR = false>
__device__ __forceinline__ double apply_A64(const Geo& g, const float* xo, const float* xn,
                                            long long e, int s, double d, int i0 = 0, int j0 = 0,
                                            int k0 = 0) {
    if constexpr (STR) {
        const double nb = wrow(g.wx, g.nx, 0, i0 + 1) * (double)xn[e - 1 + s] +
                          wrow(g.wx, g.nx, 1, i0 + 1) * (double)xn[e + s] +
                          wrow(g.wy, g.ny, 0, j0 + 1) * (double)xn[e - g.S] +
                          wrow(g.wy, g.ny, 1, j0 + 1) * (double)xn[e + g.S] +
                          wrow(g.wz, g.nz, 0, k0 + 1) * (double)xn[e - g.SP] +
                          wrow(g.wz, g.nz, 1, k0 + 1) * (double)xn[e + g.SP];
        return nb - d * (double)xo[e];
    } else {
        const double nb = g.cxd * ((double)xn[e - 1 + s] + (double)xn[e + s]) +
                          g.cyd * ((double)xn[e - g.S] + (double)xn[e + g.S]) +
                          g.czd * ((double)xn[e - g.SP] + (double)xn[e + g.SP]);
        return nb - d * (double)xo[e];
    }
}

// ------------------------------------------------------------ rebase
// After a fold: r0 = rhs - A ph in float64, stored in float32, and partials
// of the float64 residual of the iterate, rhs - A (ph + pd).  Each thread
// handles the two cells (one per colour) of its half-cells.
template <bool STR = false>
__device__ __forceinline__ void rebase_body(const Geo& g, const PBufs& P, double* __restrict__ part,
                                            unsigned lb, unsigned nb) {
    long long t0, t1;
    red_chunk(g, lb, nb, t0, t1);
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
                const double d = diag64<STR>(g, i0, j0, k0);
                const double rb =
                    (double)P.rhs[c][e] - apply_A64<STR>(g, P.ph[c], P.ph[1 - c], e, s, d, i0, j0, k0);
                P.r0[c][e] = (float)rb;
                const double rt = rb - apply_A64<STR>(g, P.pd[c], P.pd[1 - c], e, s, d, i0, j0, k0);
                acc += rt * rt;
            }
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
}

// ------------------------------------------------------------- check
// Partials of the residual of the iterate from the correction:
// r = r0 - A pd (float64).
template <bool STR = false>
__device__ __forceinline__ void check_body(const Geo& g, const PBufs& P, double* __restrict__ part,
                                           unsigned lb, unsigned nb) {
    long long t0, t1;
    red_chunk(g, lb, nb, t0, t1);
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
                const double d = diag64<STR>(g, i0, j0, k0);
                const double rt =
                    (double)P.r0[c][e] - apply_A64<STR>(g, P.pd[c], P.pd[1 - c], e, s, d, i0, j0, k0);
                acc += rt * rt;
            }
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
}

// Partials over the cells of a colour-array pair (or the pair a + b when
// b0 is given): mode 0 sum x^2, mode 1 sum x.
__device__ __forceinline__ void colour_sum_body(const Geo& g, const float* a0, const float* a1,
                                                const float* b0, const float* b1, int mode,
                                                double* __restrict__ part, unsigned lb,
                                                unsigned nb) {
    long long t0, t1;
    red_chunk(g, lb, nb, t0, t1);
    double acc = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
        const long long e = g.col(ii, j0, k0);
        for (int c = 0; c < 2; ++c) {
            const int i0 = 2 * ii + ((c + j0 + k0) & 1);
            if (i0 < g.nx) {
                double x = (double)(c ? a1 : a0)[e];
                if (b0) x += (double)(c ? b1 : b0)[e];
                acc += mode ? x : x * x;
            }
        }
    }
    const double bs = block_sum(acc);
    if (threadIdx.x == 0) part[lb] = bs;
}

// Subtract the mean (ctl->rhs_sum / cells) from the (base + correction)
// pair, keeping the correction's precision: the float32-rounded mean goes
// out of the base, its rounding error out of the correction.
__device__ __forceinline__ void p_sub_body(const Geo& g, const PBufs& P, const Ctl* ctl,
                                           unsigned lb) {
    const long long t = (long long)lb * kBlock + threadIdx.x;
    int ii, j0, k0;
    if (!half_cell(g, t, ii, j0, k0)) return;
    const double mean = ctl->rhs_sum / ((double)g.nx * g.ny * g.nz);
    const long long e = g.col(ii, j0, k0);
    const float mh = (float)mean;
    const float ml = (float)(mean - (double)mh);
    for (int c = 0; c < 2; ++c) {
        const int i0 = 2 * ii + ((c + j0 + k0) & 1);
        if (i0 < g.nx) {
            P.ph[c][e] = P.ph[c][e] - mh;
            P.pd[c][e] = P.pd[c][e] - ml;
        }
    }
}

// ------------------------------------------------------------ finalize
// Block-wide fixed-order reductions for a block of NT threads.
template <int NT>
__device__ __forceinline__ double nt_sum(const double* part, int n, int stride = 1) {
    __shared__ double red[NT / 64];
    // four independent accumulators: four loads in flight per thread
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * NT < n; i += 4 * NT) {
        v0 += part[(long long)i * stride];
        v1 += part[(long long)(i + NT) * stride];
        v2 += part[(long long)(i + 2 * NT) * stride];
        v3 += part[(long long)(i + 3 * NT) * stride];
    }
    for (; i < n; i += NT) v0 += part[(long long)i * stride];
    double v = (v0 + v1) + (v2 + v3);
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t += red[i];
    __syncthreads();
    return t;   // valid in every thread
}

// The three sums of the residual bound in one pass: a = sum rel0[2i],
// b = sum rel1[2i], d = sum rel1[2i+1] (fixed order, every thread gets them).
template <int NT>
__device__ __forceinline__ void nt_sum3(const double* rel0, const double* rel1, int n, double& a, double& b,
                                        double& d) {
    __shared__ double red3[3][NT / 64];
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, d0 = 0.0, d1 = 0.0;
    int i = threadIdx.x;
    for (; i + NT < n; i += 2 * NT) {
        a0 += rel0[2LL * i];
        b0 += rel1[2LL * i];
        d0 += rel1[2LL * i + 1];
        a1 += rel0[2LL * (i + NT)];
        b1 += rel1[2LL * (i + NT)];
        d1 += rel1[2LL * (i + NT) + 1];
    }
    if (i < n) {
        a0 += rel0[2LL * i];
        b0 += rel1[2LL * i];
        d0 += rel1[2LL * i + 1];
    }
    const double va = wave_sum(a0 + a1), vb = wave_sum(b0 + b1), vd = wave_sum(d0 + d1);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red3[0][wid] = va;
        red3[1][wid] = vb;
        red3[2][wid] = vd;
    }
    __syncthreads();
    a = b = d = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
        a += red3[0][w];
        b += red3[1][w];
        d += red3[2][w];
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ double nt_max(const double* part, int n, int stride = 1) {
    __shared__ double redm[NT / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) v = fmax(v, part[(long long)i * stride]);
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) redm[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t = fmax(t, redm[i]);
    __syncthreads();
    return t;
}

// Decision after a residual check.
__device__ __forceinline__ void decide(Ctl* ctl, double sum_r2) {
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

// Fixed-order sums of the partials of a preceding reduction, then the
// bookkeeping of op (one block of NT threads):
//   FIN_BOUND  after the sweeps of a check interval: sum reltmp^2 for the
//              report, and the colour-1 residual lower bound
//              |omega-1|/omega sqrt(sum (diag reltmp)^2) <= ||r||; if it
//              exceeds 1.5 tol the coming check cannot succeed and is
//              skipped (never the last check before max_iter)
//   FIN_CHECK  decide on the residual (or just count a skipped check)
//   FIN_CHECK_FULL  decide on the residual (rebase checks never skip)
template <int NT>
__device__ __forceinline__ void finalize_body(int op, const double* __restrict__ part, int n,
                                              const double* __restrict__ rel0,
                                              const double* __restrict__ rel1, int nrel, Ctl* ctl,
                                              double omega) {
    const bool sor_op = op == FIN_CHECK || op == FIN_CHECK_FULL || op == FIN_SETUP || op == FIN_BOUND;
    if (sor_op && ctl->done) return;
    if (op == FIN_DIAG) {
        const double a = nt_sum<NT>(part, n, 2);
        const double b = nt_max<NT>(part + 1, n, 2);
        if (threadIdx.x == 0) {
            ctl->div2 = a;
            ctl->cfl = b;
        }
        return;
    }
    if (op == FIN_BOUND) {
        double r0s, r1s, d1s;
        nt_sum3<NT>(rel0, rel1, nrel, r0s, r1s, d1s);
        if (threadIdx.x == 0) {
            ctl->reltmp2 = r0s + r1s;
            const double lbd = fabs(omega - 1.0) / omega * sqrt(d1s) / sqrt(ctl->rhs2);
            const int m_next = min(ctl->m + ctl->K, ctl->max_iter);
            ctl->skip = (m_next < ctl->max_iter && lbd > 1.5 * ctl->tol) ? 1 : 0;
        }
        return;
    }
    if (op == FIN_CHECK) {
        const bool skip = ctl->skip != 0;
        __syncthreads();   // every thread has read the flag before thread 0 clears it
        if (skip) {
            if (threadIdx.x == 0) {
                ctl->m = min(ctl->m + ctl->K, ctl->max_iter);
                ctl->skip = 0;
            }
            return;
        }
    }
    const double s = nt_sum<NT>(part, n);
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

}  // namespace les
