// Kernels of the warm-start network (3-D U-Net, BF16 activations and
// weights, FP32 accumulation on the gfx950 matrix cores).
//
// Tensors are channels-last: voxel v = ((b D + z) H + y) W + x, channel c at
// v * cs + c with a channel stride cs >= C (concatenated tensors are one
// buffer whose two halves are written by two producers).
//
// Matrix-core use: __builtin_amdgcn_mfma_f32_16x16x32_bf16.  Operand lane
// layout (verified on the device): lane l holds A[m = l % 16][k = 8 (l/16)
// + i] and B[k = 8 (l/16) + i][n = l % 16], i = 0..7; the accumulator holds
// D[m = 4 (l/16) + i][n = l % 16], i = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct lesnet;

namespace les {
namespace net {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetBlock = 256;   // 4 wavefronts

enum Gather { G_TAP27 = 0, G_CHILD8 = 1, G_TAP1 = 2 };

// Implicit GEMM: out[v][co] = act(bias[co] + sum_k A[v][k] W[co][k]) where
// k = (tap, ci) and A[v][(t, ci)] = in[gather(v, t)][ci] (zero outside the
// grid), optionally masked by mask[gather(v, t)][ci] > 0 (the ReLU
// derivative of the layer that produced `in` in the backward pass).
struct GemmArgs {
    const bf16* in; int in_cs; int cin_p; int cin_shift;   // cin_p = 1 << cin_shift, multiple of 8
    const bf16* mask; int mask_cs;
    const bf16* wt; int kp;                                // [slices][cout][kp]
    const float* bias;
    bf16* out; int out_cs; int out_coff;
    float* out_f32;       // non-null: float32 output here instead of out (same indexing)
    int cout;
    int relu;
    int gather;
    int scatter_child;    // 1: output voxel = child blockIdx.y of v on the 2x grid, weight slice blockIdx.y
    int B, D, H, W;       // grid of v (the GEMM's M)
};

// Weight gradient of one tap t (grid y): dW_t[ci][co] = sum_v A[ci][v] B[v][co],
// A[ci][v] = in[gA(v, t)][ci], B[v][co] = dout[gB(v, t)][co] * (mask > 0).
// Conv layers: gA = neighbour t, gB = v.  Up layers: gA = v, gB = child t.
struct WgradArgs {
    const bf16* in; int in_cs; int cin;
    const bf16* dout; int dout_cs; int cout;
    const bf16* mask; int mask_cs;     // null: no ReLU on this layer's output
    int up;                            // 0 conv (27 taps), 1 up (8 children)
    int B, D, H, W;                    // grid of v
    long long chunk;                   // voxels per block (multiple of 32 * 4)
    float* part;                       // [chunks][taps][cin_t][cout] (cin_t = cin rounded up to 16)
};

// Host-side hooks of the LES coupling (defined with the network): size the
// activation workspace, the packed bf16 input [V][8] it reads, its float32
// output [V], and a forward pass over that input.
int ws_prepare(struct ::lesnet* n, int B, int D, int H, int W);
bf16* ws_input(struct ::lesnet* n);
const float* ws_output(const struct ::lesnet* n);
int ws_forward(struct ::lesnet* n, hipStream_t s, int B, int D, int H, int W);

}  // namespace net
}  // namespace les
