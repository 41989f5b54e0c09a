// Warm-start network for the SOR solve: a small 3-D U-Net (3 levels,
// 16/32/64 channels, two 3x3x3 convolutions per level, 2x2x2 max pooling,
// 2x2x2 stride-2 transposed convolutions, skip concatenation, ReLU, a
// 1x1x1 head), trained on pairs the LES itself produces.  BF16 activations
// and weights, FP32 accumulation on the matrix cores, FP32 master weights
// updated by Adam (Kingma & Ba 2015).
//
// Forward and backward are implicit GEMMs (M = voxels, N = output channels):
//   conv forward     gather 27 neighbours,            W[co][(t, ci)]           k_conv_brick
//   conv dgrad       gather 27 neighbours of dY*relu', W flipped in t, [ci][(t, co)]  k_conv_brick
//   up forward       same voxel, output scattered to child s (grid y), U_s[co][ci]    k_gemm
//   up dgrad         gather the 8 children of dY,     U[ci][(s, co)]           k_gemm
// and weight gradients (K = voxels) on k_wgrad with a fixed-order split over
// voxels (deterministic).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device_util.h"
#include "les_impl.h"
#include "lesnet_kernels.h"

namespace les {
namespace net {
namespace {

__device__ __forceinline__ void vox_of(long long v, int D, int H, int W, int& b, int& z, int& y,
                                       int& x) {
    x = (int)(v % W);
    long long r = v / W;
    y = (int)(r % H);
    r /= H;
    z = (int)(r % D);
    b = (int)(r / D);
}

__device__ __forceinline__ long long vox_id(int b, int z, int y, int x, int D, int H, int W) {
    return (((long long)b * D + z) * H + y) * W + x;
}

// ------------------------------------------------------ implicit GEMM
// A wavefront computes MW tiles of 16 voxels x NT tiles of 16 channels;
// the weight fragment of each K step is loaded once and used for the MW
// voxel tiles.  Voxel counts < 2^31 (checked on the host).
template <int NT, int MW>
__global__ __launch_bounds__(kNetBlock) void k_gemm(GemmArgs a) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const unsigned M = (unsigned)a.B * a.D * a.H * a.W;
    const unsigned m0 = (blockIdx.x * 4u + wave) * 16u * MW;
    if (m0 >= M) return;   // whole wavefront past the end (no block-wide sync below)
    const int slice = a.scatter_child ? (int)blockIdx.y : 0;
    const bf16* wt = a.wt + (size_t)slice * a.cout * a.kp;
    const unsigned D = a.D, H = a.H, W = a.W;
    int vb[MW], vz[MW], vy[MW], vx[MW];
    bool vok[MW];
#pragma unroll
    for (int mw = 0; mw < MW; ++mw) {
        const unsigned mv = m0 + 16u * mw + (l & 15);
        vok[mw] = mv < M;
        const unsigned vv = vok[mw] ? mv : 0u;
        vx[mw] = (int)(vv % W);
        const unsigned r = vv / W;
        vy[mw] = (int)(r % H);
        const unsigned r2 = r / H;
        vz[mw] = (int)(r2 % D);
        vb[mw] = (int)(r2 / D);
    }
    const int ntaps = a.gather == G_TAP27 ? 27 : (a.gather == G_CHILD8 ? 8 : 1);
    const int K = ntaps * a.cin_p;
    const int kgrp = (l >> 4) * 8;
    f32x4 acc[MW][NT];
#pragma unroll
    for (int mw = 0; mw < MW; ++mw)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mw][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < a.kp; k0 += 32) {
        const int k = k0 + kgrp;
        bf16x8 bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            bv[nt] = *reinterpret_cast<const bf16x8*>(wt + (size_t)(16 * nt + (l & 15)) * a.kp + k);
        const int t = k >> a.cin_shift;
        const int ci = k - (t << a.cin_shift);
#pragma unroll
        for (int mw = 0; mw < MW; ++mw) {
            bf16x8 av;
#pragma unroll
            for (int i = 0; i < 8; ++i) av[i] = (bf16)0.f;
            if (vok[mw] && k < K) {
                const int b = vb[mw], z = vz[mw], y = vy[mw], x = vx[mw];
                long long iv = -1;
                if (a.gather == G_TAP27) {
                    const int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
                    if (zz >= 0 && zz < (int)D && yy >= 0 && yy < (int)H && xx >= 0 && xx < (int)W)
                        iv = (((long long)b * D + zz) * H + yy) * W + xx;
                } else if (a.gather == G_CHILD8) {
                    iv = (((long long)b * 2 * D + 2 * z + (t >> 2)) * 2 * H + 2 * y + ((t >> 1) & 1)) * 2 * W +
                         2 * x + (t & 1);
                } else {
                    iv = m0 + 16u * mw + (l & 15);
                }
                if (iv >= 0) {
                    av = *reinterpret_cast<const bf16x8*>(a.in + iv * a.in_cs + ci);
                    if (a.mask) {
                        const bf16x8 mk = *reinterpret_cast<const bf16x8*>(a.mask + iv * a.mask_cs + ci);
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (!((float)mk[i] > 0.f)) av[i] = (bf16)0.f;
                    }
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mw][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[mw][nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mw = 0; mw < MW; ++mw)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int ch = 16 * nt + (l & 15);
            const float bias = a.bias ? a.bias[ch] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned ov = m0 + 16u * mw + 4 * (l >> 4) + i;
                if (ov >= M) continue;
                float val = acc[mw][nt][i] + bias;
                if (a.relu) val = fmaxf(val, 0.f);
                size_t dst = ov;
                if (a.scatter_child) {
                    const unsigned ox = ov % W, r = ov / W, oy = r % H, r2 = r / H, oz = r2 % D, ob = r2 / D;
                    dst = (((size_t)ob * 2 * D + 2 * oz + (slice >> 2)) * 2 * H + 2 * oy + ((slice >> 1) & 1)) *
                              2 * W + 2 * ox + (slice & 1);
                }
                if (a.out_f32) a.out_f32[dst * a.out_cs + a.out_coff + ch] = val;
                else a.out[dst * a.out_cs + a.out_coff + ch] = (bf16)val;
            }
        }
}

// ------------------------------------------------------ convolution, LDS brick
// The 27-tap gather (convolution forward, and its input gradient from the
// masked output gradient) with the input staged in LDS.  A block owns
// BZ x BY x 16 output voxels (z, y, x) of one sample and loads the
// (BZ+2) x (BY+2) x 18 input voxels around them once (16-byte chunks of 8
// channels, zero outside the grid, the optional mask applied on load);
// every A operand is then a 16-byte LDS read.  A tile (the MFMA's 16 M
// rows) is one x-row of 16 voxels; wavefront w takes tiles w, w+4, ...;
// each weight fragment is loaded once per K step for all of them.
template <int NT, int CINP, int BZ, int BY>
__global__ __launch_bounds__(kNetBlock) void k_conv_brick(GemmArgs a) {
    constexpr int BX = 16;
    constexpr int HZ = BZ + 2, HY = BY + 2, HX = BX + 2;
    constexpr int CH = CINP / 8;       // 16-byte chunks per voxel
    constexpr int TPW = BZ * BY / 4;   // tiles per wavefront
    __shared__ bf16x8 brick[HZ * HY * HX * CH];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int D = a.D, H = a.H, W = a.W;
    const int nbx = (W + BX - 1) / BX, nby = (H + BY - 1) / BY, nbz = (D + BZ - 1) / BZ;
    int bid = blockIdx.x;
    const int bx = bid % nbx;
    bid /= nbx;
    const int by = bid % nby;
    bid /= nby;
    const int bz = bid % nbz;
    const int b = bid / nbz;
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
    bf16x8 zero;
#pragma unroll
    for (int i = 0; i < 8; ++i) zero[i] = (bf16)0.f;
    for (int q = threadIdx.x; q < HZ * HY * HX * CH; q += kNetBlock) {
        const int ch = q % CH;
        const int v = q / CH;
        const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
        const int gz = z0 - 1 + hz, gy = y0 - 1 + hy, gx = x0 - 1 + hx;
        bf16x8 val = zero;
        if (gz >= 0 && gz < D && gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const size_t iv = (((size_t)b * D + gz) * H + gy) * W + gx;
            val = *reinterpret_cast<const bf16x8*>(a.in + iv * a.in_cs + ch * 8);
            if (a.mask) {
                const bf16x8 mk = *reinterpret_cast<const bf16x8*>(a.mask + iv * a.mask_cs + ch * 8);
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (!((float)mk[i] > 0.f)) val[i] = (bf16)0.f;
            }
        }
        brick[q] = val;
    }
    __syncthreads();
    const int kgrp = (l >> 4) * 8;
    const int m = l & 15;
    f32x4 acc[TPW][NT];
#pragma unroll
    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[tw][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The K loop, fully unrolled (K = 27 taps x CINP channels, padded to a
    // multiple of 32): lane group l >> 4 holds K values kgrp .. kgrp + 7 of
    // each step, so its tap and channel chunk are compile-time per step up to
    // the lane group, and the brick offset of a tap is a constant.  K values
    // past 27 CINP (the padding of the last step) read tap 26 of the brick
    // against weights that are zero there (the weight layouts pad with
    // zeros), so no operand is masked.
    constexpr int KP = (27 * CINP + 31) / 32 * 32;
    auto tap_off = [](int t) {   // brick offset (16-byte chunks) of tap t, window shifted by one
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        return ((dz * HY + dy) * HX + dx) * CH;
    };
    const int lg = l >> 4;
    int tb[TPW];   // brick chunk of each tile's lane voxel at tap 0, channel chunk 0
#pragma unroll
    for (int tw = 0; tw < TPW; ++tw) {
        const int tile = wave + 4 * tw;
        tb[tw] = (((tile / BY) * HY + (tile % BY)) * HX + m) * CH;
    }
    // weight fragments one K step ahead: the next step's loads are in
    // flight while this step's matrix operations run
    bf16x8 bnext[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
        bnext[nt] = *reinterpret_cast<const bf16x8*>(a.wt + (size_t)(16 * nt + (l & 15)) * KP + kgrp);
    auto kstep = [&](int st) {
        bf16x8 bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bv[nt] = bnext[nt];
        if (st + 1 < KP / 32) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                bnext[nt] = *reinterpret_cast<const bf16x8*>(a.wt + (size_t)(16 * nt + (l & 15)) * KP +
                                                             32 * (st + 1) + kgrp);
        }
        // this lane group's tap and channel chunk: k = 32 st + 8 lg
        int off;
        if constexpr (CINP >= 32) {   // one tap per step for every lane: a block-uniform offset
            const int t = min(32 * st / CINP, 26);
            off = tap_off(t) + ((32 * st) % CINP) / 8 + lg;
        } else if constexpr (CINP == 16) {
            const int t0 = min(2 * st, 26), t1 = min(2 * st + 1, 26);
            off = (lg >= 2 ? tap_off(t1) : tap_off(t0)) + (lg & 1);
        } else {   // CINP == 8: four taps per step
            const int t0 = min(4 * st, 26), t1 = min(4 * st + 1, 26), t2 = min(4 * st + 2, 26),
                      t3 = min(4 * st + 3, 26);
            off = lg == 0 ? tap_off(t0) : (lg == 1 ? tap_off(t1) : (lg == 2 ? tap_off(t2) : tap_off(t3)));
        }
#pragma unroll
        for (int tw = 0; tw < TPW; ++tw) {
            const bf16x8 av = brick[tb[tw] + off];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[tw][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[tw][nt], 0, 0, 0);
        }
    };
    if constexpr (CINP >= 32) {
#pragma unroll 1
        for (int st = 0; st < KP / 32; ++st) kstep(st);   // uniform tap: scalar offsets
    } else {
#pragma unroll
        for (int st = 0; st < KP / 32; ++st) kstep(st);   // per-lane-group taps: constants once unrolled
    }
#pragma unroll
    for (int tw = 0; tw < TPW; ++tw) {
        const int tile = wave + 4 * tw;
        const int z = z0 + tile / BY, y = y0 + tile % BY;
        if (z >= D || y >= H) continue;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int chn = 16 * nt + (l & 15);
            const float bias = a.bias ? a.bias[chn] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + 4 * (l >> 4) + i;
                if (x >= W) continue;
                float val = acc[tw][nt][i] + bias;
                if (a.relu) val = fmaxf(val, 0.f);
                const size_t dst = (((size_t)b * D + z) * H + y) * W + x;
                if (a.out_f32) a.out_f32[dst * a.out_cs + a.out_coff + chn] = val;
                else a.out[dst * a.out_cs + a.out_coff + chn] = (bf16)val;
            }
        }
    }
}

// ------------------------------------------------------ weight gradients
// Block = 4 wavefronts over one chunk of voxels and TPB consecutive taps
// (tap group = grid y).  Each wavefront walks 32-voxel steps (the MFMA K);
// the operand that does not depend on the tap (the output gradient of a
// convolution, the input of an up layer) is loaded once per step and
// reused for the TPB taps.  The block sums its four wavefronts in LDS in
// a fixed order and stores one partial per chunk and tap.
template <int MT, int NT, int TPB, bool ROW8>
__global__ __launch_bounds__(kNetBlock) void k_wgrad(WgradArgs a) {
    __shared__ float red[TPB][MT * 16][NT * 16];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int taps = a.up ? 8 : 27;
    const int tb = blockIdx.y * TPB;
    // voxel counts < 2^31 (checked on the host): 32-bit index arithmetic
    const unsigned M = (unsigned)a.B * a.D * a.H * a.W;
    const unsigned c0 = blockIdx.x * (unsigned)a.chunk;
    const unsigned c1 = c0 + (unsigned)a.chunk < M ? c0 + (unsigned)a.chunk : M;
    const unsigned D = a.D, H = a.H, W = a.W;
    f32x4 acc[TPB][MT][NT];
#pragma unroll
    for (int tt = 0; tt < TPB; ++tt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[tt][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const unsigned kgrp = (l >> 4) * 8;
    for (unsigned v0 = c0 + wave * 32; v0 < c1; v0 += 4 * 32) {
        // coordinates of the lane's 8 voxels v0 + kgrp + i; with ROW8 (W a
        // multiple of 8) they are one aligned run along x
        int vb[ROW8 ? 1 : 8], vz[ROW8 ? 1 : 8], vy[ROW8 ? 1 : 8], vx[ROW8 ? 1 : 8];
        bool ok[8];
#pragma unroll
        for (int i = 0; i < (ROW8 ? 1 : 8); ++i) {
            const unsigned v = v0 + kgrp + i;
            const unsigned vv = v < c1 ? v : c0;
            vx[i] = (int)(vv % W);
            const unsigned r = vv / W;
            vy[i] = (int)(r % H);
            const unsigned r2 = r / H;
            vz[i] = (int)(r2 % D);
            vb[i] = (int)(r2 / D);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) ok[i] = v0 + kgrp + i < c1;
        auto coord = [&](int i, int& b, int& z, int& y, int& x) {
            if (ROW8) {
                b = vb[0]; z = vz[0]; y = vy[0]; x = vx[0] + i;
            } else {
                b = vb[i]; z = vz[i]; y = vy[i]; x = vx[i];
            }
        };
        auto vid = [&](int b, int z, int y, int x, unsigned d, unsigned h, unsigned w) {
            return (((unsigned)b * d + (unsigned)z) * h + (unsigned)y) * w + (unsigned)x;
        };
        // the tap-independent operand
        bf16x8 sh_a[MT], sh_b[NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 8; ++i) sh_a[mt][i] = (bf16)0.f;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 8; ++i) sh_b[nt][i] = (bf16)0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (!ok[i]) continue;
            const size_t v = v0 + kgrp + i;
            if (!a.up) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int co = 16 * nt + (l & 15);
                    bf16 g = a.dout[v * a.dout_cs + co];
                    if (a.mask && !((float)a.mask[v * a.mask_cs + co] > 0.f)) g = (bf16)0.f;
                    sh_b[nt][i] = g;
                }
            } else {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int ci = 16 * mt + (l & 15);
                    if (ci < a.cin) sh_a[mt][i] = a.in[v * a.in_cs + ci];
                }
            }
        }
#pragma unroll
        for (int tt = 0; tt < TPB; ++tt) {
            const int t = tb + tt;
            if (t >= taps) break;   // uniform over the block
            bf16x8 av[MT], bv[NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) av[mt] = sh_a[mt];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bv[nt] = sh_b[nt];
            const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int b, z, y, x;
                coord(i, b, z, y, x);
                if (!a.up) {
                    const int zz = z + dz, yy = y + dy, xx = x + dx;
                    const bool in_grid = ok[i] && zz >= 0 && zz < (int)D && yy >= 0 && yy < (int)H && xx >= 0 &&
                                         xx < (int)W;
                    const size_t ia = in_grid ? vid(b, zz, yy, xx, D, H, W) : 0;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const int ci = 16 * mt + (l & 15);
                        av[mt][i] = (in_grid && ci < a.cin) ? a.in[ia * a.in_cs + ci] : (bf16)0.f;
                    }
                } else {
                    const size_t ib = vid(b, 2 * z + (t >> 2), 2 * y + ((t >> 1) & 1), 2 * x + (t & 1), 2 * D,
                                          2 * H, 2 * W);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const int co = 16 * nt + (l & 15);
                        bv[nt][i] = ok[i] ? a.dout[ib * a.dout_cs + co] : (bf16)0.f;
                    }
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[tt][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv[nt], acc[tt][mt][nt], 0, 0, 0);
        }
    }
    // wavefronts add their tiles in turn (fixed order 0, 1, 2, 3)
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int tt = 0; tt < TPB; ++tt)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float& r = red[tt][16 * mt + 4 * (l >> 4) + i][16 * nt + (l & 15)];
                            r = (w == 0 ? 0.f : r) + acc[tt][mt][nt][i];
                        }
        }
        __syncthreads();
    }
    constexpr int tile = MT * 16 * NT * 16;
    for (int tt = 0; tt < TPB; ++tt) {
        const int t = tb + tt;
        if (t >= taps) break;
        float* dst = a.part + ((size_t)blockIdx.x * taps + t) * tile;
        for (int e = threadIdx.x; e < tile; e += kNetBlock) dst[e] = red[tt][e / (NT * 16)][e % (NT * 16)];
    }
}

// Convolution weight gradients with both operands staged in LDS.  The
// output grid is cut into bricks of BZ x BY x 16 voxels; a block takes the
// bricks of one chunk and TPB consecutive taps (tap group = grid y).  Per
// brick it loads the (BZ+2) x (BY+2) x 18 input voxels around it and the
// masked output gradient of the brick (zero outside the grid).  4 x 4 x 16
// bricks store both channel-major, x fastest: a thread loads eight voxels'
// 16-byte channel octets of one x-row, transposes them in registers and
// writes one 8-voxel run per channel; K = 32 voxels (two x-rows of the
// brick) and a lane's 8 K values are 8 consecutive voxels of one channel,
// so each MFMA operand is one 16-byte LDS read: B[voxel][co] aligned,
// A[ci][voxel] (the input shifted by the tap) at a 2-byte offset, which the
// LDS serves as an unaligned access.  2 x 2 x 16 bricks store channels last
// (one octet per store) and gather each operand element by element.  Wavefront w takes the K steps w, w+4, ... of each
// brick; the four wavefronts' tiles are summed in a fixed order at the end
// and one partial per chunk and tap is stored.  Dynamic LDS: max of the
// operands ((BZ+2)(BY+2) 18 cinp + BZ BY 16 cout bf16) and the reduction
// tiles (TPB x MT 16 x NT 16 float), which reuse the operands' space at the
// end.
template <int MT, int NT, int TPB, int BZ, int BY>
__global__ __launch_bounds__(kNetBlock) void k_wgrad_brick(WgradArgs a, int cinp, int bricks_per_chunk,
                                                           float* bias_part) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int BX = 16, HZ = BZ + 2, HY = BY + 2, HX = BX + 2;
    constexpr int NV = BZ * BY * BX;   // voxels per brick
    constexpr int KS = NV / 32;        // K steps per brick
    // channel-major operands for the 4 x 4 x 16 bricks; the 2 x 2 x 16
    // bricks (wide channel counts) keep channels last, where the transposing
    // fill costs more than the single-read operands save
    constexpr bool CM = BZ == 4;
    bf16* s_in = reinterpret_cast<bf16*>(smem);
    bf16* s_g = s_in + HZ * HY * HX * cinp;
    float(*red)[MT * 16][NT * 16] = reinterpret_cast<float(*)[MT * 16][NT * 16]>(smem);
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int D = a.D, H = a.H, W = a.W, cout = a.cout;
    const int nbx = (W + BX - 1) / BX, nby = (H + BY - 1) / BY, nbz = (D + BZ - 1) / BZ;
    const int nbricks = a.B * nbz * nby * nbx;
    const int tb = blockIdx.y * TPB;
    const int br0 = blockIdx.x * bricks_per_chunk;
    const int br1 = min(nbricks, br0 + bricks_per_chunk);
    bf16x8 zero;
#pragma unroll
    for (int i = 0; i < 8; ++i) zero[i] = (bf16)0.f;
    f32x4 acc[TPB][MT][NT];
#pragma unroll
    for (int tt = 0; tt < TPB; ++tt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[tt][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int gi = l >> 4;   // lane group: voxels 8 gi .. 8 gi + 7 of a K step
    // bias gradient (tap group 0 only): this thread sums channel tid % cout
    // over the voxels tid / cout, + 256 / cout, ... of every brick
    const bool do_bias = bias_part != nullptr && blockIdx.y == 0;
    float bsum = 0.f;
    for (int br = br0; br < br1; ++br) {
        int bid = br;
        const int bx = bid % nbx;
        bid /= nbx;
        const int by = bid % nby;
        bid /= nby;
        const int bz = bid % nbz;
        const int b = bid / nbz;
        const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
        __syncthreads();   // the previous brick's operands are no longer read
        if constexpr (CM) {
            // input halo: units (channel octet, row hz hy, x run of 8, 8, 2)
            const int cchi = cinp / 8;
            for (int q = threadIdx.x; q < cchi * HZ * HY * 3; q += kNetBlock) {
                const int xc = q % 3;
                const int r = (q / 3) % (HZ * HY);
                const int c8 = q / (3 * HZ * HY);
                const int hy = r % HY, hz = r / HY;
                const int gz = z0 - 1 + hz, gy = y0 - 1 + hy;
                const bool row_ok = gz >= 0 && gz < D && gy >= 0 && gy < H;
                const int nv = xc < 2 ? 8 : HX - 16;
                bf16x8 vox[8];
    #pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int gx = x0 - 1 + 8 * xc + i;
                    vox[i] = zero;
                    if (i < nv && row_ok && gx >= 0 && gx < W) {
                        const size_t iv = (((size_t)b * D + gz) * H + gy) * W + gx;
                        vox[i] = *reinterpret_cast<const bf16x8*>(a.in + iv * a.in_cs + c8 * 8);
                    }
                }
    #pragma unroll
                for (int c = 0; c < 8; ++c) {
                    bf16* dst = s_in + ((size_t)((8 * c8 + c) * HZ + hz) * HY + hy) * HX + 8 * xc;
                    if (xc < 2) {
                        bf16x8 run;
    #pragma unroll
                        for (int i = 0; i < 8; ++i) run[i] = vox[i][c];
                        __builtin_memcpy(dst, &run, sizeof run);   // 4-byte aligned
                    } else {
                        dst[0] = vox[0][c];
                        dst[1] = vox[1][c];
                    }
                }
            }
            // masked output gradient: units (channel octet, row lz ly, x run of 8)
            const int ccho = cout / 8;
            for (int q = threadIdx.x; q < ccho * BZ * BY * 2; q += kNetBlock) {
                const int xc = q % 2;
                const int r = (q / 2) % (BZ * BY);
                const int c8 = q / (2 * BZ * BY);
                const int ly = r % BY, lz = r / BY;
                const int gz = z0 + lz, gy = y0 + ly;
                bf16x8 vox[8];
    #pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int gx = x0 + 8 * xc + i;
                    vox[i] = zero;
                    if (gz < D && gy < H && gx < W) {
                        const size_t iv = (((size_t)b * D + gz) * H + gy) * W + gx;
                        bf16x8 val = *reinterpret_cast<const bf16x8*>(a.dout + iv * a.dout_cs + c8 * 8);
                        if (a.mask) {
                            const bf16x8 mk = *reinterpret_cast<const bf16x8*>(a.mask + iv * a.mask_cs + c8 * 8);
    #pragma unroll
                            for (int k = 0; k < 8; ++k)
                                if (!((float)mk[k] > 0.f)) val[k] = (bf16)0.f;
                        }
                        vox[i] = val;
                    }
                }
    #pragma unroll
                for (int c = 0; c < 8; ++c) {
                    bf16x8 run;
    #pragma unroll
                    for (int i = 0; i < 8; ++i) run[i] = vox[i][c];
                    *reinterpret_cast<bf16x8*>(s_g + (size_t)(8 * c8 + c) * NV + r * BX + 8 * xc) = run;
                }
            }
        } else {   // channels last, one 16-byte octet per store
            const int cchi = cinp / 8;
            for (int q = threadIdx.x; q < HZ * HY * HX * cchi; q += kNetBlock) {
                const int ch = q % cchi;
                const int v = q / cchi;
                const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
                const int gz = z0 - 1 + hz, gy = y0 - 1 + hy, gx = x0 - 1 + hx;
                bf16x8 val = zero;
                if (gz >= 0 && gz < D && gy >= 0 && gy < H && gx >= 0 && gx < W) {
                    const size_t iv = (((size_t)b * D + gz) * H + gy) * W + gx;
                    val = *reinterpret_cast<const bf16x8*>(a.in + iv * a.in_cs + ch * 8);
                }
                *reinterpret_cast<bf16x8*>(s_in + (size_t)q * 8) = val;
            }
            const int ccho = cout / 8;
            for (int q = threadIdx.x; q < NV * ccho; q += kNetBlock) {
                const int ch = q % ccho;
                const int v = q / ccho;
                const int lx = v % BX, ly = (v / BX) % BY, lz = v / (BX * BY);
                const int gz = z0 + lz, gy = y0 + ly, gx = x0 + lx;
                bf16x8 val = zero;
                if (gz < D && gy < H && gx < W) {
                    const size_t iv = (((size_t)b * D + gz) * H + gy) * W + gx;
                    val = *reinterpret_cast<const bf16x8*>(a.dout + iv * a.dout_cs + ch * 8);
                    if (a.mask) {
                        const bf16x8 mk = *reinterpret_cast<const bf16x8*>(a.mask + iv * a.mask_cs + ch * 8);
    #pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (!((float)mk[i] > 0.f)) val[i] = (bf16)0.f;
                    }
                }
                *reinterpret_cast<bf16x8*>(s_g + (size_t)q * 8) = val;
            }
        }
        __syncthreads();
        if (do_bias)
            for (int v = threadIdx.x / cout; v < NV; v += kNetBlock / cout)
                bsum += (float)(CM ? s_g[(size_t)(threadIdx.x % cout) * NV + v] : s_g[v * cout + threadIdx.x % cout]);
        for (int ks = wave; ks < KS; ks += 4) {
            // the lane's 8 voxels: brick row ks * 2 + gi / 2, x = 8 (gi % 2) + i
            const int row = ks * 2 + (gi >> 1);
            const int lz = row / BY, ly = row % BY, xb = 8 * (gi & 1);
            bf16x8 bv[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = 16 * nt + (l & 15);
                if constexpr (CM) {
                    bv[nt] = *reinterpret_cast<const bf16x8*>(s_g + (size_t)co * NV + row * BX + xb);
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i) bv[nt][i] = s_g[((row * BX) + xb + i) * cout + co];
                }
            }
#pragma unroll
            for (int tt = 0; tt < TPB; ++tt) {
                const int t = tb + tt;
                if (t >= 27) break;   // uniform over the block
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;   // window offsets 0..2
                const int hbase = ((lz + dz) * HY + (ly + dy)) * HX + xb + dx;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int ci = 16 * mt + (l & 15);
                    bf16x8 av;
                    if constexpr (CM) {
                        // 8 consecutive voxels of channel ci (2-byte aligned)
                        av = zero;
                        if (ci < cinp) __builtin_memcpy(&av, s_in + ci * (HZ * HY * HX) + hbase, sizeof av);
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) av[i] = ci < cinp ? s_in[(hbase + i) * cinp + ci] : (bf16)0.f;
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[tt][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[tt][mt][nt], 0, 0, 0);
                }
            }
        }
    }
    if (do_bias) {   // fixed-order sum of the threads of each channel
        __shared__ float bred[kNetBlock];
        bred[threadIdx.x] = bsum;
        __syncthreads();
        if (threadIdx.x < cout) {
            float t = 0.f;
            for (int r = 0; r < kNetBlock / cout; ++r) t += bred[r * cout + threadIdx.x];
            bias_part[(size_t)blockIdx.x * cout + threadIdx.x] = t;
        }
    }
    __syncthreads();   // operands done: the reduction tiles reuse their space
    // wavefronts add their tiles in turn (fixed order 0, 1, 2, 3)
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int tt = 0; tt < TPB; ++tt)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float& r = red[tt][16 * mt + 4 * (l >> 4) + i][16 * nt + (l & 15)];
                            r = (w == 0 ? 0.f : r) + acc[tt][mt][nt][i];
                        }
        }
        __syncthreads();
    }
    constexpr int tile = MT * 16 * NT * 16;
    for (int tt = 0; tt < TPB; ++tt) {
        const int t = tb + tt;
        if (t >= 27) break;
        float* dst = a.part + ((size_t)blockIdx.x * 27 + t) * tile;
        for (int e = threadIdx.x; e < tile; e += kNetBlock) dst[e] = red[tt][e / (NT * 16)][e % (NT * 16)];
    }
}

// dW[t][ci][co] (the oracle layout, ci < cin) = sum over chunks in a fixed
// order.  A block of 1024 threads takes 64 consecutive output elements
// (lanes: consecutive elements, so the partial loads are coalesced); its 16
// wavefronts sum the chunks g, g+16, ... (wavefront g) in turn, and the 16
// sums are added in wavefront order.
constexpr int kReduceBlock = 1024;
__global__ __launch_bounds__(kReduceBlock) void k_wgrad_reduce(const float* part, int chunks, int taps, int cin,
                                                               int cin_t, int cout, float* dw) {
    __shared__ float red[kReduceBlock / 64][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const long long e = (long long)blockIdx.x * 64 + lane;
    const long long n = (long long)taps * cin * cout;
    const bool live = e < n;
    const long long ee = live ? e : 0;
    const int co = (int)(ee % cout);
    const long long r = ee / cout;
    const int ci = (int)(r % cin);
    const int t = (int)(r / cin);
    const size_t stride = (size_t)taps * cin_t * cout;
    const size_t off = ((size_t)t * cin_t + ci) * cout + co;
    float s = 0.f;
    if (live)
        for (int c = g; c < chunks; c += kReduceBlock / 64) s += part[c * stride + off];
    red[g][lane] = s;
    __syncthreads();
    if (g == 0 && live) {
        float tot = 0.f;
        for (int w = 0; w < kReduceBlock / 64; ++w) tot += red[w][lane];
        dw[e] = tot;
    }
}

// Per-block channel sums of dout * relu'(mask): bias gradients (partials).
__global__ __launch_bounds__(kNetBlock) void k_bias_part(const bf16* dout, int dout_cs, const bf16* mask,
                                                         int mask_cs, int C, long long M, long long chunk,
                                                         float* part) {
    __shared__ float red[kNetBlock];
    const long long c0 = (long long)blockIdx.x * chunk;
    const long long c1 = c0 + chunk < M ? c0 + chunk : M;
    const int lanes_per_c = kNetBlock / C;   // C divides 256
    const int c = threadIdx.x % C, q = threadIdx.x / C;
    float s = 0.f;
    for (long long v = c0 + q; v < c1; v += lanes_per_c) {
        float g = (float)dout[v * dout_cs + c];
        if (mask && !((float)mask[v * mask_cs + c] > 0.f)) g = 0.f;
        s += g;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.f;
        for (int r = 0; r < lanes_per_c; ++r) t += red[r * C + threadIdx.x];
        part[(size_t)blockIdx.x * C + threadIdx.x] = t;
    }
}

// out[c] = sum over rows of part[row][c] (one block per column, fixed order)
__global__ __launch_bounds__(kNetBlock) void k_col_sum(const float* part, int rows, int cols, float* out) {
    const int c = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += kNetBlock) s += (double)part[(size_t)r * cols + c];
    s = block_sum(s);
    if (threadIdx.x == 0) out[c] = (float)s;
}

// ------------------------------------------------------ pooling
// 2x2x2 max over the children of coarse voxel v; idx = child of the max
// (first in child order on ties).
__global__ __launch_bounds__(kNetBlock) void k_pool(const bf16* in, int in_cs, bf16* out, int out_cs,
                                                    uint8_t* idx, int C, int B, int D, int H, int W) {
    const long long e = (long long)blockIdx.x * kNetBlock + threadIdx.x;
    const long long Mc = (long long)B * D * H * W;
    if (e >= Mc * C) return;
    const int c = (int)(e % C);
    const long long v = e / C;
    int b, z, y, x;
    vox_of(v, D, H, W, b, z, y, x);
    float best = -INFINITY;
    int bi = 0;
    for (int s = 0; s < 8; ++s) {
        const long long f = vox_id(b, 2 * z + (s >> 2), 2 * y + ((s >> 1) & 1), 2 * x + (s & 1), 2 * D, 2 * H, 2 * W);
        const float val = (float)in[f * in_cs + c];
        if (val > best) {
            best = val;
            bi = s;
        }
    }
    out[v * out_cs + c] = (bf16)best;
    idx[e] = (uint8_t)bi;
}

// dfine[child s of v][c] = (idx == s ? dcoarse[v][c] : 0) + skip[child][c].
__global__ __launch_bounds__(kNetBlock) void k_unpool_add(const bf16* dcoarse, int dc_cs, const uint8_t* idx,
                                                          const bf16* skip, int skip_cs, bf16* dfine, int df_cs,
                                                          int C, int B, int D, int H, int W) {
    const long long e = (long long)blockIdx.x * kNetBlock + threadIdx.x;
    const long long Mf = (long long)B * D * H * W * 8;
    if (e >= Mf * C) return;
    const int c = (int)(e % C);
    const long long f = e / C;
    int b, z, y, x;
    vox_of(f, 2 * D, 2 * H, 2 * W, b, z, y, x);
    const int s = ((z & 1) << 2) | ((y & 1) << 1) | (x & 1);
    const long long v = vox_id(b, z >> 1, y >> 1, x >> 1, D, H, W);
    float g = (idx[v * C + c] == s) ? (float)dcoarse[v * dc_cs + c] : 0.f;
    g += (float)skip[f * skip_cs + c];
    dfine[f * df_cs + c] = (bf16)g;
}

// ------------------------------------------------------ head, loss
__global__ __launch_bounds__(kNetBlock) void k_head(const bf16* in, int cs, int C, const float* w,
                                                    const float* bias, long long M, float* y) {
    const long long v = (long long)blockIdx.x * kNetBlock + threadIdx.x;
    if (v >= M) return;
    float s = bias[0];
    for (int c = 0; c < C; ++c) s += (float)in[v * cs + c] * w[c];
    y[v] = s;
}

// dy = 2 (y - t) / n; partial float64 sums of (y - t)^2 per block.
__global__ __launch_bounds__(kNetBlock) void k_mse(const float* y, const float* t, long long n, float* dy,
                                                   double* part) {
    const long long v = (long long)blockIdx.x * kNetBlock + threadIdx.x;
    double r2 = 0.0;
    if (v < n) {
        const float r = y[v] - t[v];
        dy[v] = 2.f * r / (float)n;
        r2 = (double)r * (double)r;
    }
    const double s = block_sum(r2);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Head backward: dd[v][c] = dy[v] w[c] (bf16); partial dW/db per block.
__global__ __launch_bounds__(kNetBlock) void k_head_back(const bf16* in, int cs, int C, const float* w,
                                                         const float* dy, long long M, bf16* dd, int dd_cs,
                                                         float* part) {
    __shared__ float red[kNetBlock][33];   // C <= 32
    const long long v = (long long)blockIdx.x * kNetBlock + threadIdx.x;
    float g = 0.f;
    for (int c = 0; c <= C; ++c) red[threadIdx.x][c] = 0.f;
    if (v < M) {
        g = dy[v];
        for (int c = 0; c < C; ++c) {
            dd[v * dd_cs + c] = (bf16)(g * w[c]);
            red[threadIdx.x][c] = (float)in[v * cs + c] * g;
        }
        red[threadIdx.x][C] = g;
    }
    __syncthreads();
    if (threadIdx.x <= C) {
        float s = 0.f;
        for (int r = 0; r < kNetBlock; ++r) s += red[r][threadIdx.x];
        part[(size_t)blockIdx.x * (C + 1) + threadIdx.x] = s;
    }
}

__global__ void k_sum_f64(const double* part, int n, double* out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kNetBlock) s += part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------ weights, Adam
// Forward layout of a conv3 (taps 27) or up (taps 8, per-child slices):
//   conv: wt[co][t cin_p + ci] = W[t][ci][co]
//   up:   wt[s][co][ci]         = U[s][ci][co]
// Dgrad layout:
//   conv: wd[ci][t' cout + co] = W[26 - t'][ci][co]
//   up:   wd[ci][s cout + co]  = U[s][ci][co]
// Zero where ci >= cin or k >= the filled K.
__global__ void k_layout_fwd(const float* W, int taps, int cin, int cout, int cin_p, int kp, int up,
                             bf16* wt) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int slices = up ? taps : 1;
    const long long n = (long long)slices * cout * kp;
    if (e >= n) return;
    const int k = (int)(e % kp);
    const long long r = e / kp;
    const int co = (int)(r % cout);
    const int sl = (int)(r / cout);
    float val = 0.f;
    if (up) {
        if (k < cin) val = W[((size_t)sl * cin + k) * cout + co];
    } else {
        const int t = k / cin_p, ci = k % cin_p;
        if (t < taps && ci < cin) val = W[((size_t)t * cin + ci) * cout + co];
    }
    wt[e] = (bf16)val;
}

__global__ void k_layout_dgrad(const float* W, int taps, int cin, int cout, int kp, int up, bf16* wd) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)cin * kp;
    if (e >= n) return;
    const int k = (int)(e % kp);
    const int ci = (int)(e / kp);
    const int t = k / cout, co = k % cout;
    float val = 0.f;
    if (t < taps) {
        const int src = up ? t : (taps - 1 - t);
        val = W[((size_t)src * cin + ci) * cout + co];
    }
    wd[e] = (bf16)val;
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// float [v][3] -> bf16 [v][8] (channels 3..7 zero)
__global__ void k_pack_input(const float* x, long long M, bf16* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * 8) return;
    const int c = (int)(e & 7);
    const long long v = e >> 3;
    out[e] = (bf16)(c < 3 ? x[v * 3 + c] : 0.f);
}

// float [v][c] -> bf16 [v][cp] (channels c..cp-1 zero)
__global__ void k_to_bf16(const float* x, long long M, int c, int cp, bf16* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * cp) return;
    const int q = (int)(e % cp);
    const long long v = e / cp;
    out[e] = (bf16)(q < c ? x[v * c + q] : 0.f);
}

// bf16-round a float array in place of a copy (weights of single ops)
__global__ void k_round_bf16(const float* x, long long n, float* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = (float)(bf16)x[e];
}

inline unsigned nb(long long n, int b = kNetBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace
}  // namespace net
}  // namespace les

using namespace les;
using namespace les::net;

// ============================================================ host side
namespace {

struct Layer {
    const char* name;
    int up;          // 0: conv3 (27 taps), 1: up (8 children)
    int cin, cout;
    int cin_p;       // input channel padding (conv) / K padding base (up)
    long long w_off, b_off;   // offsets in the flat float parameter array
    long long wt_off, wd_off; // offsets in the bf16 layout arena
    int kp_f, kp_d;           // padded K of the forward / dgrad layouts
};

int rup(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

struct lesnet {
    std::string err;
    int c1 = 16, c2 = 32, c3 = 64;
    uint64_t seed = 0;
    double lr = 1e-3, beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
    int64_t t = 0;
    std::vector<Layer> L;
    long long nparam = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // device, fp32
    bf16* lay = nullptr;                                           // device, bf16 layouts
    long long nlay = 0;
    bool layout_fresh = false;
    // activation workspace for (B, D, H, W)
    int B = 0, D = 0, H = 0, W = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    struct Act {
        bf16 *x, *e1a, *C1, *p1, *e2a, *C2, *p2, *b1, *b2, *d2a, *d2b, *d1a, *d1b;
        uint8_t *i1, *i2;
        float *y, *dy;
        bf16 *g_d1b, *g_d1a, *gC1, *g_d2b, *g_d2a, *gC2, *g_b2, *g_b1, *g_p2, *g_e2b, *g_e2a, *g_p1, *g_e1b, *g_e1a;
        float* part;
        double* dpart;
        double* dsum;
        long long part_n;
    } a{};
    double target_scale = 1.0;
};

namespace {

int net_err(lesnet* n, int code, const char* what, hipError_t he = hipSuccess) {
    if (n) {
        n->err = what;
        if (he != hipSuccess) n->err += std::string(": ") + hipGetErrorString(he);
    }
    return code;
}

#define NCK(expr)                                                        \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) return net_err(n, LES_EDEVICE, #expr, e_); \
    } while (0)

void build_layers(lesnet* n) {
    const int c1 = n->c1, c2 = n->c2, c3 = n->c3;
    struct Spec { const char* nm; int up, cin, cout; };
    const Spec spec[] = {{"e1a", 0, 3, c1},      {"e1b", 0, c1, c1},      {"e2a", 0, c1, c2},
                         {"e2b", 0, c2, c2},     {"b1", 0, c2, c3},       {"b2", 0, c3, c3},
                         {"u2", 1, c3, c2},      {"d2a", 0, 2 * c2, c2},  {"d2b", 0, c2, c2},
                         {"u1", 1, c2, c1},      {"d1a", 0, 2 * c1, c1},  {"d1b", 0, c1, c1}};
    n->L.clear();
    long long off = 0, loff = 0;
    for (const Spec& s : spec) {
        Layer l{};
        l.name = s.nm;
        l.up = s.up;
        l.cin = s.cin;
        l.cout = s.cout;
        l.cin_p = s.cin < 8 ? 8 : s.cin;
        const int taps = s.up ? 8 : 27;
        l.w_off = off;
        off += (long long)taps * s.cin * s.cout;
        l.b_off = off;
        off += s.cout;
        l.kp_f = s.up ? rup(s.cin, 32) : rup(27 * l.cin_p, 32);
        l.kp_d = rup(taps * s.cout, 32);
        l.wt_off = loff;
        loff += (long long)(s.up ? 8 : 1) * s.cout * l.kp_f;
        l.wd_off = loff;
        loff += (long long)s.cin * l.kp_d;
        n->L.push_back(l);
    }
    // head: W [c1][1], b [1]
    Layer h{};
    h.name = "head";
    h.up = -1;
    h.cin = c1;
    h.cout = 1;
    h.w_off = off;
    off += c1;
    h.b_off = off;
    off += 1;
    n->L.push_back(h);
    n->nparam = off;
    n->nlay = loff;
}

Layer& layer(lesnet* n, const char* nm) {
    for (Layer& l : n->L)
        if (std::strcmp(l.name, nm) == 0) return l;
    return n->L.back();
}

int refresh_layouts(lesnet* n, hipStream_t s) {
    if (n->layout_fresh) return LES_OK;
    for (const Layer& l : n->L) {
        if (l.up < 0) continue;
        const int taps = l.up ? 8 : 27;
        const long long nf = (long long)(l.up ? 8 : 1) * l.cout * l.kp_f;
        hipLaunchKernelGGL(k_layout_fwd, dim3(nb(nf)), dim3(kNetBlock), 0, s, n->w + l.w_off, taps, l.cin,
                           l.cout, l.cin_p, l.kp_f, l.up, n->lay + l.wt_off);
        const long long nd = (long long)l.cin * l.kp_d;
        hipLaunchKernelGGL(k_layout_dgrad, dim3(nb(nd)), dim3(kNetBlock), 0, s, n->w + l.w_off, taps, l.cin,
                           l.cout, l.kp_d, l.up, n->lay + l.wd_off);
    }
    NCK(hipGetLastError());
    n->layout_fresh = true;
    return LES_OK;
}

int layer_wgrad_chunks(int up, int cin, int cout, int B, int D, int H, int W, long long* chunk, int* bpc);

int ensure_ws(lesnet* n, int B, int D, int H, int W) {
    if (n->ws && n->B == B && n->D == D && n->H == H && n->W == W) return LES_OK;
    if (n->ws) NCK(hipFree(n->ws));
    n->ws = nullptr;
    const long long V1 = (long long)B * D * H * W, V2 = V1 / 8, V3 = V2 / 8;
    const int c1 = n->c1, c2 = n->c2, c3 = n->c3;
    std::vector<std::pair<void**, size_t>> req;
    auto bf = [&](bf16** p, long long elems) { req.push_back({(void**)p, (size_t)elems * sizeof(bf16)}); };
    lesnet::Act& a = n->a;
    bf(&a.x, V1 * 8);
    bf(&a.e1a, V1 * c1);
    bf(&a.C1, V1 * 2 * c1);
    bf(&a.p1, V2 * c1);
    bf(&a.e2a, V2 * c2);
    bf(&a.C2, V2 * 2 * c2);
    bf(&a.p2, V3 * c2);
    bf(&a.b1, V3 * c3);
    bf(&a.b2, V3 * c3);
    bf(&a.d2a, V2 * c2);
    bf(&a.d2b, V2 * c2);
    bf(&a.d1a, V1 * c1);
    bf(&a.d1b, V1 * c1);
    req.push_back({(void**)&a.i1, (size_t)V2 * c1});
    req.push_back({(void**)&a.i2, (size_t)V3 * c2});
    req.push_back({(void**)&a.y, (size_t)V1 * 4});
    req.push_back({(void**)&a.dy, (size_t)V1 * 4});
    bf(&a.g_d1b, V1 * c1);
    bf(&a.g_d1a, V1 * c1);
    bf(&a.gC1, V1 * 2 * c1);
    bf(&a.g_d2b, V2 * c2);
    bf(&a.g_d2a, V2 * c2);
    bf(&a.gC2, V2 * 2 * c2);
    bf(&a.g_b2, V3 * c3);
    bf(&a.g_b1, V3 * c3);
    bf(&a.g_p2, V3 * c2);
    bf(&a.g_e2b, V2 * c2);
    bf(&a.g_e2a, V2 * c2);
    bf(&a.g_p1, V2 * c1);
    bf(&a.g_e1b, V1 * c1);
    bf(&a.g_e1a, V1 * c1);
    // partials: the largest weight-gradient need over the layers plus the
    // bias partials (at most 1024 chunks x 64), or the head's (blocks x 33)
    long long need = 0;
    for (const Layer& l : n->L) {
        if (l.up < 0) continue;
        const bool lvl1 = !strcmp(l.name, "e1a") || !strcmp(l.name, "e1b") || !strcmp(l.name, "d1a") ||
                          !strcmp(l.name, "d1b");
        const bool lvl3 = !strcmp(l.name, "b1") || !strcmp(l.name, "b2") || !strcmp(l.name, "u2");
        const int f = lvl1 ? 1 : (lvl3 ? 4 : 2);   // grid of the weight-gradient sum (u1: level 2, u2: level 3)
        long long chunk;
        int bpc;
        const int chunks = layer_wgrad_chunks(l.up, l.cin, l.cout, B, D / f, H / f, W / f, &chunk, &bpc);
        need = std::max(need, (long long)chunks * (l.up ? 8 : 27) * rup(l.cin, 16) * l.cout);
    }
    a.part_n = std::max(need + 1024LL * 64, (V1 / kNetBlock + 1) * 33);
    req.push_back({(void**)&a.part, (size_t)a.part_n * 4});
    req.push_back({(void**)&a.dpart, (size_t)(V1 / kNetBlock + 16) * 8});
    req.push_back({(void**)&a.dsum, 64});
    size_t total = 0;
    for (auto& r : req) total += (r.second + 255) & ~(size_t)255;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) return net_err(n, LES_ENOMEM, "hipMalloc(network workspace)", e);
    n->ws = p;
    n->ws_bytes = total;
    char* c = (char*)p;
    for (auto& r : req) {
        *r.first = c;
        c += (r.second + 255) & ~(size_t)255;
    }
    NCK(hipMemset(p, 0, total));
    n->B = B;
    n->D = D;
    n->H = H;
    n->W = W;
    return LES_OK;
}

// Voxel chunking of the weight-gradient reduction: at most 512 chunks of
// at least 512 voxels (multiples of 128: four wavefronts x 32).
void wgrad_chunking(long long M, long long* chunk, int* chunks) {
    long long c = std::max<long long>(512, (M + 511) / 512);
    c = (c + 127) / 128 * 128;
    *chunk = c;
    *chunks = (int)((M + c - 1) / c);
}

// Taps per block of k_wgrad: as many as the accumulators allow.
int wgrad_tpb(int MT, int NT, int up) {
    const int t = MT * NT;
    if (!up) return t <= 2 ? 9 : (t <= 8 ? 3 : 1);
    return t <= 2 ? 8 : (t <= 4 ? 4 : (t <= 8 ? 2 : 1));
}
// taps per block of the brick kernel: one or two 16 x 16 tiles take all 27
// taps, so their (transposing) operand fill is paid once per brick
int wgrad_brick_tpb(int MT, int NT) { return MT * NT <= 2 ? 27 : wgrad_tpb(MT, NT, 0); }

template <bool ROW8>
hipError_t launch_wgrad_t(hipStream_t s, const WgradArgs& a, int chunks) {
    const int MT = rup(a.cin, 16) / 16, NT = a.cout / 16;
    const int taps = a.up ? 8 : 27;
    const int tpb = wgrad_tpb(MT, NT, a.up);
    const dim3 grid(chunks, (taps + tpb - 1) / tpb);
#define WG(mt, nt, tp)                                                                                  \
    if (MT == mt && NT == nt && tpb == tp)                                                              \
    hipLaunchKernelGGL((k_wgrad<mt, nt, tp, ROW8>), grid, dim3(kNetBlock), 0, s, a)
    WG(1, 1, 9); else WG(1, 1, 8); else WG(1, 2, 9); else WG(1, 2, 8); else WG(2, 1, 9); else WG(2, 1, 8);
    else WG(1, 4, 3); else WG(1, 4, 4); else WG(2, 2, 3); else WG(2, 2, 4); else WG(4, 1, 3); else WG(4, 1, 4);
    else WG(2, 4, 3); else WG(2, 4, 2); else WG(4, 2, 3); else WG(4, 2, 2);
    else WG(4, 4, 1);
    else return hipErrorInvalidValue;
#undef WG
    return hipGetLastError();
}

hipError_t launch_wgrad(hipStream_t s, const WgradArgs& a, int chunks) {
    return a.W % 8 == 0 ? launch_wgrad_t<true>(s, a, chunks) : launch_wgrad_t<false>(s, a, chunks);
}

// Convolution weight gradients on the LDS-brick kernel: chunks of whole
// bricks, at most 512 chunks.  Returns the chunk count
// (partials [chunks][27][cin_t][cout]) or -1 for an unsupported shape.
// Dynamic LDS of a weight-gradient block with bricks of bz x bz x 16
// voxels, and the brick (4 x 4 x 16 voxels, else 2 x 2 x 16) that keeps the
// block within 64 KB.
size_t wgrad_brick_lds(const WgradArgs& a, int bz) {
    const int cinp = a.cin <= 8 ? 8 : a.cin;
    const int MT = rup(a.cin, 16) / 16, NT = a.cout / 16;
    const size_t red = (size_t)wgrad_brick_tpb(MT, NT) * MT * 16 * NT * 16 * sizeof(float);
    const size_t ops = ((size_t)(bz + 2) * (bz + 2) * 18 * cinp + (size_t)bz * bz * 16 * a.cout) * sizeof(bf16);
    return std::max(red, ops);
}

int wgrad_brick_bz(const WgradArgs& a) { return wgrad_brick_lds(a, 4) <= 63 * 1024 ? 4 : 2; }   // + 1 KB static

int wgrad_brick_chunks(const WgradArgs& a, int* bpc_out) {
    const int bz = wgrad_brick_bz(a), by = bz;
    const long long nbricks = (long long)a.B * ((a.D + bz - 1) / bz) * ((a.H + by - 1) / by) * ((a.W + 15) / 16);
    const int bpc = (int)std::max<long long>(1, (nbricks + 511) / 512);
    *bpc_out = bpc;
    return (int)((nbricks + bpc - 1) / bpc);
}

hipError_t launch_wgrad_brick(hipStream_t s, const WgradArgs& a, int chunks, int bpc, float* bias_part) {
    const int cinp = a.cin <= 8 ? 8 : a.cin;
    const int MT = rup(a.cin, 16) / 16, NT = a.cout / 16;
    const int bz = wgrad_brick_bz(a);
    const size_t lds = wgrad_brick_lds(a, bz);
    const int tpb = wgrad_brick_tpb(MT, NT);
    const dim3 grid(chunks, (27 + tpb - 1) / tpb);
#define WB(mt, nt, tp, z, y)                                                                          \
    if (MT == mt && NT == nt && tpb == tp && bz == z)                                                 \
    hipLaunchKernelGGL((k_wgrad_brick<mt, nt, tp, z, y>), grid, dim3(kNetBlock), lds, s, a, cinp, bpc, bias_part)
    WB(1, 1, 27, 4, 4); else WB(1, 2, 27, 4, 4); else WB(2, 1, 27, 4, 4); else WB(2, 2, 3, 4, 4);
    else WB(1, 4, 3, 4, 4); else WB(4, 1, 3, 4, 4); else WB(2, 4, 3, 4, 4); else WB(4, 2, 3, 4, 4);
    else WB(4, 4, 1, 4, 4);
    else WB(1, 1, 27, 2, 2); else WB(1, 2, 27, 2, 2); else WB(2, 1, 27, 2, 2); else WB(2, 2, 3, 2, 2);
    else WB(1, 4, 3, 2, 2); else WB(4, 1, 3, 2, 2); else WB(2, 4, 3, 2, 2); else WB(4, 2, 3, 2, 2);
    else WB(4, 4, 1, 2, 2);
    else return hipErrorInvalidValue;
#undef WB
    return hipGetLastError();
}

// Chunks of the weight-gradient sum of a layer (and its chunk size in
// voxels / bricks per chunk): the brick kernel for convolutions, the
// voxel-chunked one for up layers.
int layer_wgrad_chunks(int up, int cin, int cout, int B, int D, int H, int W, long long* chunk, int* bpc) {
    const long long M = (long long)B * D * H * W;
    int chunks;
    wgrad_chunking(M, chunk, &chunks);
    *bpc = 0;
    if (up) return chunks;
    WgradArgs a{};
    a.cin = cin;
    a.cout = cout;
    a.B = B; a.D = D; a.H = H; a.W = W;
    return wgrad_brick_chunks(a, bpc);
}

// Convolutions (27-tap gathers) on the LDS-brick kernel: bricks of
// 4 x 4 x 16 outputs (2 x 4 x 16 for 64 input channels).  Taller bricks
// (8 x 8 x 16 for 16 output channels, 4 x 8 x 16 for 32) feed more matrix
// operations per K step but were slower over the whole forward pass at
// 64 x 128 x 128 (0.676 against 0.565 ms): fewer resident blocks per
// compute unit to hide the staging of the next brick.
hipError_t conv_brick(hipStream_t s, const GemmArgs& a) {
    const int NT = a.cout / 16, C = a.cin_p;
    const int bz = C == 64 ? 2 : 4, by = 4;
    const long long blocks =
        (long long)a.B * ((a.D + bz - 1) / bz) * ((a.H + by - 1) / by) * ((a.W + 15) / 16);
    const dim3 grid((unsigned)blocks);
#define CB(nt, c, z) \
    if (NT == nt && C == c) hipLaunchKernelGGL((k_conv_brick<nt, c, z, 4>), grid, dim3(kNetBlock), 0, s, a)
    CB(1, 8, 4); else CB(1, 16, 4); else CB(1, 32, 4); else CB(1, 64, 2);
    else CB(2, 8, 4); else CB(2, 16, 4); else CB(2, 32, 4); else CB(2, 64, 2);
    else CB(4, 8, 4); else CB(4, 16, 4); else CB(4, 32, 4); else CB(4, 64, 2);
    else return hipErrorInvalidValue;
#undef CB
    return hipGetLastError();
}

// One GEMM launch: 27-tap gathers on the LDS-brick kernel; the others on
// k_gemm with NT = cout / 16 in {1, 2, 4} and MW = 4 / NT voxel tiles per
// wavefront while the grid keeps at least 1024 blocks, else 1.
hipError_t gemm(hipStream_t s, const GemmArgs& a) {
    if (a.gather == G_TAP27 && !a.scatter_child &&
        (a.cin_p == 8 || a.cin_p == 16 || a.cin_p == 32 || a.cin_p == 64) && a.kp == (27 * a.cin_p + 31) / 32 * 32)
        return conv_brick(s, a);
    const long long M = (long long)a.B * a.D * a.H * a.W;
    const int NT = a.cout / 16;
    int MW = NT == 1 ? 4 : (NT == 2 ? 2 : 1);
    if (nb(M, 64 * MW) < 1024) MW = 1;
    const dim3 grid(nb(M, 64 * MW), a.scatter_child ? 8 : 1);
#define GM(nt, mw) \
    if (NT == nt && MW == mw) hipLaunchKernelGGL((k_gemm<nt, mw>), grid, dim3(kNetBlock), 0, s, a)
    GM(1, 4); else GM(1, 1); else GM(2, 2); else GM(2, 1); else GM(4, 1);
    else return hipErrorInvalidValue;
#undef GM
    return hipGetLastError();
}

int log2i(int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

// conv3 / up forward of layer l: in (cs) -> out (cs, coff)
int fwd_layer(lesnet* n, hipStream_t s, const Layer& l, const bf16* in, int in_cs, bf16* out, int out_cs,
              int out_coff, int B, int D, int H, int W) {
    GemmArgs a{};
    a.in = in;
    a.in_cs = in_cs;
    a.cin_p = l.up ? l.cin : l.cin_p;   // up: K = cin, padded to kp_f by zero weights
    a.cin_shift = log2i(a.cin_p);
    a.wt = n->lay + l.wt_off;
    a.kp = l.kp_f;
    a.bias = n->w + l.b_off;
    a.out = out;
    a.out_cs = out_cs;
    a.out_coff = out_coff;
    a.cout = l.cout;
    a.relu = l.up ? 0 : 1;
    a.gather = l.up ? G_TAP1 : G_TAP27;
    a.scatter_child = l.up ? 1 : 0;
    a.B = B; a.D = D; a.H = H; a.W = W;   // grid of the GEMM rows (coarse grid for up)
    NCK(gemm(s, a));
    return LES_OK;
}

// input gradient of layer l: dout (cs) masked by the layer output (mask, cs)
// -> din (cs, coff); the GEMM rows are the layer's input grid
int dgrad_layer(lesnet* n, hipStream_t s, const Layer& l, const bf16* dout, int dout_cs, const bf16* mask,
                int mask_cs, bf16* din, int din_cs, int B, int D, int H, int W) {
    GemmArgs a{};
    a.in = dout;
    a.in_cs = dout_cs;
    a.cin_p = l.cout;
    a.cin_shift = log2i(l.cout);
    a.mask = mask;
    a.mask_cs = mask_cs;
    a.wt = n->lay + l.wd_off;
    a.kp = l.kp_d;
    a.out = din;
    a.out_cs = din_cs;
    a.out_coff = 0;
    a.cout = l.cin;
    a.gather = l.up ? G_CHILD8 : G_TAP27;
    a.B = B; a.D = D; a.H = H; a.W = W;
    NCK(gemm(s, a));
    return LES_OK;
}

// weight and bias gradients of layer l into n->g
int wgrad_layer(lesnet* n, hipStream_t s, const Layer& l, const bf16* in, int in_cs, const bf16* dout,
                int dout_cs, const bf16* mask, int mask_cs, int B, int D, int H, int W) {
    const long long M = (long long)B * D * H * W;
    const int taps = l.up ? 8 : 27;
    const int cin_t = rup(l.cin, 16);
    long long chunk;
    int bpc;
    const int chunks = layer_wgrad_chunks(l.up, l.cin, l.cout, B, D, H, W, &chunk, &bpc);
    const long long Mo = l.up ? M * 8 : M;   // the layer's output grid
    const long long bchunk = std::max<long long>(1024, (Mo + 1023) / 1024);
    const int bchunks = (int)((Mo + bchunk - 1) / bchunk);
    const long long wparts = (long long)chunks * taps * cin_t * l.cout;
    if (wparts + (long long)std::max(bchunks, chunks) * l.cout > n->a.part_n)
        return net_err(n, LES_ENOMEM, "wgrad partials");
    WgradArgs a{};
    a.in = in; a.in_cs = in_cs; a.cin = l.cin;
    a.dout = dout; a.dout_cs = dout_cs; a.cout = l.cout;
    a.mask = mask; a.mask_cs = mask_cs;
    a.up = l.up;
    a.B = B; a.D = D; a.H = H; a.W = W;
    a.chunk = chunk;
    a.part = n->a.part;
    // bias: sum of dout * relu' over the layer's output grid (convolutions:
    // per chunk inside the weight-gradient kernel)
    float* bpart = n->a.part + wparts;
    if (!l.up) NCK(launch_wgrad_brick(s, a, chunks, bpc, bpart));
    else NCK(launch_wgrad(s, a, chunks));
    const long long nw = (long long)taps * l.cin * l.cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(nw, 64)), dim3(kReduceBlock), 0, s, n->a.part, chunks, taps,
                       l.cin, cin_t, l.cout, n->g + l.w_off);
    int brows = chunks;
    if (l.up) {
        hipLaunchKernelGGL(k_bias_part, dim3(bchunks), dim3(kNetBlock), 0, s, dout, dout_cs, mask, mask_cs, l.cout,
                           Mo, bchunk, bpart);
        brows = bchunks;
    }
    hipLaunchKernelGGL(k_col_sum, dim3(l.cout), dim3(kNetBlock), 0, s, bpart, brows, l.cout, n->g + l.b_off);
    NCK(hipGetLastError());
    return LES_OK;
}

int forward(lesnet* n, hipStream_t s, int B, int D, int H, int W) {
    lesnet::Act& a = n->a;
    const int c1 = n->c1, c2 = n->c2, c3 = n->c3;
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4;
    int rc;
    if ((rc = refresh_layouts(n, s)) != LES_OK) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "e1a"), a.x, 8, a.e1a, c1, 0, B, D, H, W))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "e1b"), a.e1a, c1, a.C1, 2 * c1, c1, B, D, H, W))) return rc;
    hipLaunchKernelGGL(k_pool, dim3(nb((long long)B * D2 * H2 * W2 * c1)), dim3(kNetBlock), 0, s, a.C1 + c1,
                       2 * c1, a.p1, c1, a.i1, c1, B, D2, H2, W2);
    if ((rc = fwd_layer(n, s, layer(n, "e2a"), a.p1, c1, a.e2a, c2, 0, B, D2, H2, W2))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "e2b"), a.e2a, c2, a.C2, 2 * c2, c2, B, D2, H2, W2))) return rc;
    hipLaunchKernelGGL(k_pool, dim3(nb((long long)B * D3 * H3 * W3 * c2)), dim3(kNetBlock), 0, s, a.C2 + c2,
                       2 * c2, a.p2, c2, a.i2, c2, B, D3, H3, W3);
    if ((rc = fwd_layer(n, s, layer(n, "b1"), a.p2, c2, a.b1, c3, 0, B, D3, H3, W3))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "b2"), a.b1, c3, a.b2, c3, 0, B, D3, H3, W3))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "u2"), a.b2, c3, a.C2, 2 * c2, 0, B, D3, H3, W3))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "d2a"), a.C2, 2 * c2, a.d2a, c2, 0, B, D2, H2, W2))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "d2b"), a.d2a, c2, a.d2b, c2, 0, B, D2, H2, W2))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "u1"), a.d2b, c2, a.C1, 2 * c1, 0, B, D2, H2, W2))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "d1a"), a.C1, 2 * c1, a.d1a, c1, 0, B, D, H, W))) return rc;
    if ((rc = fwd_layer(n, s, layer(n, "d1b"), a.d1a, c1, a.d1b, c1, 0, B, D, H, W))) return rc;
    const Layer& hd = layer(n, "head");
    const long long V1 = (long long)B * D * H * W;
    hipLaunchKernelGGL(k_head, dim3(nb(V1)), dim3(kNetBlock), 0, s, a.d1b, c1, c1, n->w + hd.w_off,
                       n->w + hd.b_off, V1, a.y);
    NCK(hipGetLastError());
    return LES_OK;
}

// Backward from a.dy: every gradient into n->g.
int backward(lesnet* n, hipStream_t s, int B, int D, int H, int W) {
    lesnet::Act& a = n->a;
    const int c1 = n->c1, c2 = n->c2, c3 = n->c3;
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4;
    const long long V1 = (long long)B * D * H * W;
    int rc;
    // head
    const Layer& hd = layer(n, "head");
    const unsigned hb = nb(V1);
    hipLaunchKernelGGL(k_head_back, dim3(hb), dim3(kNetBlock), 0, s, a.d1b, c1, c1, n->w + hd.w_off, a.dy, V1,
                       a.g_d1b, c1, a.part);
    hipLaunchKernelGGL(k_col_sum, dim3(c1 + 1), dim3(kNetBlock), 0, s, a.part, (int)hb, c1 + 1, n->g + hd.w_off);
    NCK(hipGetLastError());
    // d1b (output d1b, input d1a)
    const Layer &d1b = layer(n, "d1b"), &d1a = layer(n, "d1a"), &u1 = layer(n, "u1");
    const Layer &d2b = layer(n, "d2b"), &d2a = layer(n, "d2a"), &u2 = layer(n, "u2");
    const Layer &b2 = layer(n, "b2"), &b1 = layer(n, "b1"), &e2b = layer(n, "e2b"), &e2a = layer(n, "e2a");
    const Layer &e1b = layer(n, "e1b"), &e1a = layer(n, "e1a");
    if ((rc = wgrad_layer(n, s, d1b, a.d1a, c1, a.g_d1b, c1, a.d1b, c1, B, D, H, W))) return rc;
    if ((rc = dgrad_layer(n, s, d1b, a.g_d1b, c1, a.d1b, c1, a.g_d1a, c1, B, D, H, W))) return rc;
    if ((rc = wgrad_layer(n, s, d1a, a.C1, 2 * c1, a.g_d1a, c1, a.d1a, c1, B, D, H, W))) return rc;
    if ((rc = dgrad_layer(n, s, d1a, a.g_d1a, c1, a.d1a, c1, a.gC1, 2 * c1, B, D, H, W))) return rc;
    // u1: output = gC1[..., 0:c1] (no relu), input d2b on the coarse grid
    if ((rc = wgrad_layer(n, s, u1, a.d2b, c2, a.gC1, 2 * c1, nullptr, 0, B, D2, H2, W2))) return rc;
    if ((rc = dgrad_layer(n, s, u1, a.gC1, 2 * c1, nullptr, 0, a.g_d2b, c2, B, D2, H2, W2))) return rc;
    if ((rc = wgrad_layer(n, s, d2b, a.d2a, c2, a.g_d2b, c2, a.d2b, c2, B, D2, H2, W2))) return rc;
    if ((rc = dgrad_layer(n, s, d2b, a.g_d2b, c2, a.d2b, c2, a.g_d2a, c2, B, D2, H2, W2))) return rc;
    if ((rc = wgrad_layer(n, s, d2a, a.C2, 2 * c2, a.g_d2a, c2, a.d2a, c2, B, D2, H2, W2))) return rc;
    if ((rc = dgrad_layer(n, s, d2a, a.g_d2a, c2, a.d2a, c2, a.gC2, 2 * c2, B, D2, H2, W2))) return rc;
    if ((rc = wgrad_layer(n, s, u2, a.b2, c3, a.gC2, 2 * c2, nullptr, 0, B, D3, H3, W3))) return rc;
    if ((rc = dgrad_layer(n, s, u2, a.gC2, 2 * c2, nullptr, 0, a.g_b2, c3, B, D3, H3, W3))) return rc;
    if ((rc = wgrad_layer(n, s, b2, a.b1, c3, a.g_b2, c3, a.b2, c3, B, D3, H3, W3))) return rc;
    if ((rc = dgrad_layer(n, s, b2, a.g_b2, c3, a.b2, c3, a.g_b1, c3, B, D3, H3, W3))) return rc;
    if ((rc = wgrad_layer(n, s, b1, a.p2, c2, a.g_b1, c3, a.b1, c3, B, D3, H3, W3))) return rc;
    if ((rc = dgrad_layer(n, s, b1, a.g_b1, c3, a.b1, c3, a.g_p2, c2, B, D3, H3, W3))) return rc;
    hipLaunchKernelGGL(k_unpool_add, dim3(nb((long long)B * D2 * H2 * W2 * c2)), dim3(kNetBlock), 0, s, a.g_p2,
                       c2, a.i2, a.gC2 + c2, 2 * c2, a.g_e2b, c2, c2, B, D3, H3, W3);
    NCK(hipGetLastError());
    if ((rc = wgrad_layer(n, s, e2b, a.e2a, c2, a.g_e2b, c2, a.C2 + c2, 2 * c2, B, D2, H2, W2))) return rc;
    if ((rc = dgrad_layer(n, s, e2b, a.g_e2b, c2, a.C2 + c2, 2 * c2, a.g_e2a, c2, B, D2, H2, W2))) return rc;
    if ((rc = wgrad_layer(n, s, e2a, a.p1, c1, a.g_e2a, c2, a.e2a, c2, B, D2, H2, W2))) return rc;
    if ((rc = dgrad_layer(n, s, e2a, a.g_e2a, c2, a.e2a, c2, a.g_p1, c1, B, D2, H2, W2))) return rc;
    hipLaunchKernelGGL(k_unpool_add, dim3(nb(V1 * c1)), dim3(kNetBlock), 0, s, a.g_p1, c1, a.i1, a.gC1 + c1,
                       2 * c1, a.g_e1b, c1, c1, B, D2, H2, W2);
    NCK(hipGetLastError());
    if ((rc = wgrad_layer(n, s, e1b, a.e1a, c1, a.g_e1b, c1, a.C1 + c1, 2 * c1, B, D, H, W))) return rc;
    if ((rc = dgrad_layer(n, s, e1b, a.g_e1b, c1, a.C1 + c1, 2 * c1, a.g_e1a, c1, B, D, H, W))) return rc;
    if ((rc = wgrad_layer(n, s, e1a, a.x, 8, a.g_e1a, c1, a.e1a, c1, B, D, H, W))) return rc;
    return LES_OK;
}

bool dims_ok(int B, int D, int H, int W) {
    return B >= 1 && D >= 4 && H >= 4 && W >= 4 && D % 4 == 0 && H % 4 == 0 && W % 4 == 0 &&
           (long long)B * D * H * W < (1LL << 31);
}

}  // namespace

namespace les {
namespace net {
int ws_prepare(lesnet* n, int B, int D, int H, int W) {
    if (!dims_ok(B, D, H, W)) return net_err(n, LES_EINVAL, "network grid");
    return ensure_ws(n, B, D, H, W);
}
bf16* ws_input(lesnet* n) { return n->a.x; }
const float* ws_output(const lesnet* n) { return n->a.y; }
int ws_forward(lesnet* n, hipStream_t s, int B, int D, int H, int W) { return forward(n, s, B, D, H, W); }
}  // namespace net
}  // namespace les

extern "C" {

int lesnet_default_config(lesnet_config* cfg) {
    if (!cfg) return LES_EINVAL;
    *cfg = lesnet_config{};
    cfg->c1 = 16;
    cfg->c2 = 32;
    cfg->c3 = 64;
    cfg->seed = 0;
    cfg->lr = 1e-3;
    cfg->beta1 = 0.9;
    cfg->beta2 = 0.999;
    cfg->eps = 1e-8;
    return LES_OK;
}

int lesnet_create(const lesnet_config* cfg, lesnet** out) {
    if (!out) return LES_EINVAL;
    *out = nullptr;
    lesnet* n = new (std::nothrow) lesnet();
    if (!n) return LES_ENOMEM;
    if (cfg) {
        // tile limits: channel counts are MFMA tiles of 16; the concatenated
        // inputs (2 c1, 2 c2) and c3 are at most 64; the head reads <= 32
        auto tile = [](int c, int hi) { return c == 16 || c == 32 || (c == 64 && hi >= 64); };
        if (!tile(cfg->c1, 32) || !tile(cfg->c2, 32) || !tile(cfg->c3, 64) || !(cfg->lr > 0) ||
            !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0)) {
            delete n;
            return LES_EINVAL;
        }
        n->c1 = cfg->c1; n->c2 = cfg->c2; n->c3 = cfg->c3;
        n->seed = cfg->seed;
        n->lr = cfg->lr; n->beta1 = cfg->beta1; n->beta2 = cfg->beta2; n->eps = cfg->eps;
    }
    build_layers(n);
    const size_t pb = (size_t)n->nparam * 4;
    if (hipMalloc(&n->w, pb) != hipSuccess || hipMalloc(&n->g, pb) != hipSuccess ||
        hipMalloc(&n->m, pb) != hipSuccess || hipMalloc(&n->v, pb) != hipSuccess ||
        hipMalloc(&n->lay, (size_t)n->nlay * sizeof(bf16)) != hipSuccess) {
        lesnet_destroy(n);
        return LES_ENOMEM;
    }
    (void)hipMemset(n->g, 0, pb);
    (void)hipMemset(n->m, 0, pb);
    (void)hipMemset(n->v, 0, pb);
    (void)hipMemset(n->lay, 0, (size_t)n->nlay * sizeof(bf16));
    // He-normal initial weights (Box-Muller on splitmix64 counters), zero biases
    std::vector<float> w((size_t)n->nparam, 0.f);
    uint64_t ctr = n->seed * 0x9E3779B97F4A7C15ULL;
    auto u01 = [&]() {
        uint64_t z = (ctr += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    for (const Layer& l : n->L) {
        const long long nw = l.up < 0 ? l.cin : (long long)(l.up ? 8 : 27) * l.cin * l.cout;
        const double fan = l.up < 0 ? l.cin : (double)(l.up ? 8 : 27) * l.cin;
        const double sd = std::sqrt(2.0 / fan);
        for (long long q = 0; q < nw; ++q) {
            const double r = std::sqrt(-2.0 * std::log(u01())) * std::cos(6.283185307179586 * u01());
            w[(size_t)(l.w_off + q)] = (float)(sd * r);
        }
    }
    if (hipMemcpy(n->w, w.data(), pb, hipMemcpyHostToDevice) != hipSuccess) {
        lesnet_destroy(n);
        return LES_EDEVICE;
    }
    *out = n;
    return LES_OK;
}

void lesnet_destroy(lesnet* n) {
    if (!n) return;
    (void)hipDeviceSynchronize();
    if (n->w) (void)hipFree(n->w);
    if (n->g) (void)hipFree(n->g);
    if (n->m) (void)hipFree(n->m);
    if (n->v) (void)hipFree(n->v);
    if (n->lay) (void)hipFree(n->lay);
    if (n->ws) (void)hipFree(n->ws);
    delete n;
}

const char* lesnet_last_error(const lesnet* n) { return n ? n->err.c_str() : ""; }

int lesnet_num_params(const lesnet* n, int64_t* count) {
    if (!n || !count) return LES_EINVAL;
    *count = n->nparam;
    return LES_OK;
}

int lesnet_get_params(lesnet* n, float* host, int64_t count) {
    if (!n || !host || count != n->nparam) return LES_EINVAL;
    NCK(hipMemcpy(host, n->w, (size_t)count * 4, hipMemcpyDeviceToHost));
    return LES_OK;
}

int lesnet_set_params(lesnet* n, const float* host, int64_t count) {
    if (!n || !host || count != n->nparam) return LES_EINVAL;
    NCK(hipMemcpy(n->w, host, (size_t)count * 4, hipMemcpyHostToDevice));
    n->layout_fresh = false;
    return LES_OK;
}

int lesnet_get_grads(lesnet* n, float* host, int64_t count) {
    if (!n || !host || count != n->nparam) return LES_EINVAL;
    NCK(hipMemcpy(host, n->g, (size_t)count * 4, hipMemcpyDeviceToHost));
    return LES_OK;
}

int lesnet_forward(lesnet* n, int32_t B, int32_t D, int32_t H, int32_t W, const float* d_x, float* d_y,
                   void* stream) {
    if (!n || !d_x || !d_y || !dims_ok(B, D, H, W)) return LES_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_ws(n, B, D, H, W);
    if (rc != LES_OK) return rc;
    const long long V1 = (long long)B * D * H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(nb(V1 * 8)), dim3(kNetBlock), 0, s, d_x, V1, n->a.x);
    NCK(hipGetLastError());
    if ((rc = forward(n, s, B, D, H, W)) != LES_OK) return rc;
    NCK(hipMemcpyAsync(d_y, n->a.y, (size_t)V1 * 4, hipMemcpyDeviceToDevice, s));
    return LES_OK;
}

int lesnet_gradients(lesnet* n, int32_t B, int32_t D, int32_t H, int32_t W, const float* d_x,
                     const float* d_dy, void* stream) {
    if (!n || !d_x || !d_dy || !dims_ok(B, D, H, W)) return LES_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_ws(n, B, D, H, W);
    if (rc != LES_OK) return rc;
    const long long V1 = (long long)B * D * H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(nb(V1 * 8)), dim3(kNetBlock), 0, s, d_x, V1, n->a.x);
    NCK(hipGetLastError());
    if ((rc = forward(n, s, B, D, H, W)) != LES_OK) return rc;
    NCK(hipMemcpyAsync(n->a.dy, d_dy, (size_t)V1 * 4, hipMemcpyDeviceToDevice, s));
    return backward(n, s, B, D, H, W);
}

// One layer operation on its own (see lesnet.h).  Allocates its own
// workspace and synchronises the stream before returning.
int lesnet_op(int32_t op, int32_t B, int32_t D, int32_t H, int32_t W, int32_t cin, int32_t cout,
              const float* d_a, const float* d_b, const float* d_c, float* d_out, void* stream) {
    const bool up = op == LESNET_OP_UP || op == LESNET_OP_UP_DGRAD || op == LESNET_OP_UP_WGRAD;
    if (op < LESNET_OP_CONV3 || op > LESNET_OP_UP_WGRAD || !d_a || !d_b || !d_out) return LES_EINVAL;
    if (B < 1 || D < 1 || H < 1 || W < 1 || (long long)B * D * H * W * 8 >= (1LL << 31)) return LES_EINVAL;
    auto t16 = [](int c) { return c == 16 || c == 32 || c == 64; };
    if (!t16(cout)) return LES_EINVAL;
    const bool dgrad = op == LESNET_OP_CONV3_DGRAD || op == LESNET_OP_UP_DGRAD;
    const bool wgrad = op == LESNET_OP_CONV3_WGRAD || op == LESNET_OP_UP_WGRAD;
    if (dgrad ? !t16(cin) : !(t16(cin) || (cin >= 1 && cin <= 8))) return LES_EINVAL;
    if (wgrad && !d_b) return LES_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int taps = up ? 8 : 27;
    const long long M = (long long)B * D * H * W;          // GEMM grid (coarse grid for up)
    const long long Mf = up ? M * 8 : M;                    // output grid of the layer
    const int cin_p = cin <= 8 ? 8 : cin;
    // workspace: bf16 copies of the activations, weight layouts, partials
    const long long na = (dgrad ? Mf * cout : M * cin_p), nbw = Mf * cout;
    const int kp_f = up ? rup(cin, 32) : rup(27 * cin_p, 32), kp_d = rup(taps * cout, 32);
    const long long nlay = (long long)(up ? 8 : 1) * cout * kp_f + (long long)cin * kp_d;
    long long chunk;
    int bpc;
    const int chunks = layer_wgrad_chunks(up ? 1 : 0, cin, cout, B, D, H, W, &chunk, &bpc);
    const int cin_t = rup(cin, 16);
    const long long npart = (long long)chunks * taps * cin_t * cout;
    const size_t bytes = ((size_t)na * 2 + 255) / 256 * 256 + ((size_t)nbw * 2 + 255) / 256 * 256 +
                         ((size_t)nlay * 2 + 255) / 256 * 256 + (size_t)npart * 4 + 256;
    void* ws = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess) return LES_ENOMEM;
    char* c = (char*)ws;
    bf16* abuf = (bf16*)c;
    c += ((size_t)na * 2 + 255) / 256 * 256;
    bf16* bbuf = (bf16*)c;
    c += ((size_t)nbw * 2 + 255) / 256 * 256;
    bf16* lay = (bf16*)c;
    c += ((size_t)nlay * 2 + 255) / 256 * 256;
    float* part = (float*)c;
    hipError_t e = hipSuccess;
    GemmArgs g{};
    g.B = B; g.D = D; g.H = H; g.W = W;
    if (op == LESNET_OP_CONV3 || op == LESNET_OP_UP) {
        hipLaunchKernelGGL(k_to_bf16, dim3(nb(M * cin_p)), dim3(kNetBlock), 0, s, d_a, M, cin, cin_p, abuf);
        hipLaunchKernelGGL(k_layout_fwd, dim3(nb((long long)(up ? 8 : 1) * cout * kp_f)), dim3(kNetBlock), 0, s,
                           d_b, taps, cin, cout, cin_p, kp_f, up ? 1 : 0, lay);
        g.in = abuf; g.in_cs = cin_p;
        g.cin_p = cin_p;
        g.cin_shift = log2i(g.cin_p);
        g.wt = lay; g.kp = kp_f; g.bias = d_c;
        g.out_f32 = d_out; g.out_cs = cout; g.cout = cout;
        g.gather = up ? G_TAP1 : G_TAP27;
        g.scatter_child = up ? 1 : 0;
        e = gemm(s, g);
    } else if (dgrad) {
        hipLaunchKernelGGL(k_to_bf16, dim3(nb(Mf * cout)), dim3(kNetBlock), 0, s, d_a, Mf, cout, cout, abuf);
        hipLaunchKernelGGL(k_layout_dgrad, dim3(nb((long long)cin * kp_d)), dim3(kNetBlock), 0, s, d_b, taps, cin,
                           cout, kp_d, up ? 1 : 0, lay);
        g.in = abuf; g.in_cs = cout; g.cin_p = cout; g.cin_shift = log2i(cout);
        g.wt = lay; g.kp = kp_d;
        g.out_f32 = d_out; g.out_cs = cin; g.cout = cin;
        g.gather = up ? G_CHILD8 : G_TAP27;
        e = gemm(s, g);
    } else {
        hipLaunchKernelGGL(k_to_bf16, dim3(nb(M * cin_p)), dim3(kNetBlock), 0, s, d_a, M, cin, cin_p, abuf);
        hipLaunchKernelGGL(k_to_bf16, dim3(nb(Mf * cout)), dim3(kNetBlock), 0, s, d_b, Mf, cout, cout, bbuf);
        WgradArgs w{};
        w.in = abuf; w.in_cs = cin_p; w.cin = cin;
        w.dout = bbuf; w.dout_cs = cout; w.cout = cout;
        w.up = up ? 1 : 0;
        w.B = B; w.D = D; w.H = H; w.W = W;
        w.chunk = chunk; w.part = part;
        e = up ? launch_wgrad(s, w, chunks) : launch_wgrad_brick(s, w, chunks, bpc, nullptr);
        if (e == hipSuccess)
            hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb((long long)taps * cin * cout, 64)),
                               dim3(kReduceBlock), 0, s, part, chunks, taps, cin, cin_t, cout, d_out);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    return e == hipSuccess ? LES_OK : LES_EDEVICE;
}

int lesnet_set_lr(lesnet* n, double lr) {
    if (!n || !(std::isfinite(lr) && lr > 0.0)) return LES_EINVAL;
    n->lr = lr;
    return LES_OK;
}

int lesnet_train_step(lesnet* n, int32_t B, int32_t D, int32_t H, int32_t W, const float* d_x,
                      const float* d_t, double* loss, void* stream) {
    if (!n || !d_x || !d_t || !dims_ok(B, D, H, W)) return LES_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_ws(n, B, D, H, W);
    if (rc != LES_OK) return rc;
    const long long V1 = (long long)B * D * H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(nb(V1 * 8)), dim3(kNetBlock), 0, s, d_x, V1, n->a.x);
    NCK(hipGetLastError());
    if ((rc = forward(n, s, B, D, H, W)) != LES_OK) return rc;
    const unsigned mb = nb(V1);
    hipLaunchKernelGGL(k_mse, dim3(mb), dim3(kNetBlock), 0, s, n->a.y, d_t, V1, n->a.dy, n->a.dpart);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kNetBlock), 0, s, n->a.dpart, (int)mb, n->a.dsum);
    NCK(hipGetLastError());
    if ((rc = backward(n, s, B, D, H, W)) != LES_OK) return rc;
    n->t += 1;
    const double c1 = 1.0 - std::pow(n->beta1, (double)n->t), c2 = 1.0 - std::pow(n->beta2, (double)n->t);
    hipLaunchKernelGGL(k_adam, dim3(nb(n->nparam)), dim3(kNetBlock), 0, s, n->w, n->g, n->m, n->v, n->nparam,
                       (float)n->lr, (float)n->beta1, (float)n->beta2, (float)n->eps, (float)c1, (float)c2);
    NCK(hipGetLastError());
    n->layout_fresh = false;
    if (loss) {
        double h = 0.0;
        NCK(hipMemcpyAsync(&h, n->a.dsum, 8, hipMemcpyDeviceToHost, s));
        NCK(hipStreamSynchronize(s));
        *loss = h / (double)V1;
    }
    return LES_OK;
}

}  // extern "C"
