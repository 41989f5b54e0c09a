/*
 * lesnet.h -- C ABI of the learned warm start of the pressure solve.
 *
 * Not part of the paper's method: the paper starts each SOR solve from the
 * previous step's pressure (section 2.6, press).  This library adds a small
 * 3-D U-Net that predicts the change of pressure over a step from the
 * residual of that start, and hands SOR whichever start has the smaller
 * residual, so the solve still stops at the same tolerance and the result
 * keeps the paper's accuracy.
 *
 * Network (channels c1, c2, c3; default 16, 32, 64):
 *   e1 = relu(conv3(relu(conv3(x))))                  c1, full grid (skip)
 *   e2 = relu(conv3(relu(conv3(pool(e1)))))           c2, 1/2 grid (skip)
 *   b  = relu(conv3(relu(conv3(pool(e2)))))           c3, 1/4 grid
 *   d2 = relu(conv3(relu(conv3(cat(up(b), e2)))))     c2
 *   d1 = relu(conv3(relu(conv3(cat(up(d2), e1)))))    c1
 *   y  = head(d1)                                     1 channel, float32
 * conv3: 3x3x3, zero padding; pool: 2x2x2 max; up: 2x2x2 stride-2
 * transposed convolution; head: 1x1x1.  Activations and weights are
 * bfloat16 on the matrix cores with float32 accumulation; the master
 * weights, their gradients and the Adam moments are float32.
 *
 * Tensors: x [B][D][H][W][3] float32 (channels last), y and targets
 * [B][D][H][W] float32, all device pointers.  D, H, W are multiples of 4
 * (two poolings), >= 4.  Calls are ordered on `stream` (NULL: the default
 * stream) and do not synchronise unless stated.
 *
 * Flat parameter vector (float32), layer by layer in the order e1a, e1b,
 * e2a, e2b, b1, b2, u2, d2a, d2b, u1, d1a, d1b, head; per layer the weight
 * then the bias.  Weight layouts (C order): conv3 [27][Cin][Cout] with tap
 * t = 9 (dz+1) + 3 (dy+1) + (dx+1) reading x[z+dz][y+dy][x+dx];
 * up [8][Cin][Cout] with child s = 4 dz + 2 dy + dx written at
 * (2z+dz, 2y+dy, 2x+dx); head [c1][1].  Cin of e1a is 3, of d2a 2 c2,
 * of d1a 2 c1 (upsampled channels first, then the skip).
 *
 * Statuses are the LES_* codes of les.h.
 */
#ifndef LESNET_H_
#define LESNET_H_

#include <stdint.h>

#include "les.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lesnet lesnet;

typedef struct {
    int32_t c1, c2, c3;   /* channels per level: c1, c2 in {16, 32}; c3 in {16, 32, 64} */
    int32_t pad_;
    uint64_t seed;        /* initial weights: He-normal, zero biases */
    double lr;            /* Adam step size (default 1e-3) */
    double beta1, beta2;  /* Adam moment decays (0.9, 0.999) */
    double eps;           /* Adam denominator guard (1e-8) */
} lesnet_config;

int lesnet_default_config(lesnet_config* cfg);
/* cfg NULL: defaults.  LES_EINVAL on channel counts outside the sets above
 * or non-positive lr/eps, LES_ENOMEM if the parameter buffers fail. */
int lesnet_create(const lesnet_config* cfg, lesnet** out);
void lesnet_destroy(lesnet* n);
const char* lesnet_last_error(const lesnet* n);

/* Parameter access: host float32 arrays of exactly lesnet_num_params
 * entries (else LES_EINVAL); synchronous.  lesnet_set_params leaves the
 * Adam moments and step count as they are.  lesnet_get_grads returns the
 * gradients of the last lesnet_gradients / lesnet_train_step call.  One
 * handle per host thread; handles do not share state. */
int lesnet_num_params(const lesnet* n, int64_t* count);
int lesnet_get_params(lesnet* n, float* host, int64_t count);
int lesnet_set_params(lesnet* n, const float* host, int64_t count);
int lesnet_get_grads(lesnet* n, float* host, int64_t count);

/* y = net(x).  Activations live in a workspace sized for the last (B, D,
 * H, W) seen and kept by the handle. */
int lesnet_forward(lesnet* n, int32_t B, int32_t D, int32_t H, int32_t W, const float* d_x,
                   float* d_y, void* stream);
/* Gradients of sum(y * dy) with respect to every parameter for the given
 * output gradient dy (a forward pass runs first); read them with
 * lesnet_get_grads. */
int lesnet_gradients(lesnet* n, int32_t B, int32_t D, int32_t H, int32_t W, const float* d_x,
                     const float* d_dy, void* stream);
/* One Adam step on the mean squared error between net(x) and t over all
 * B D H W voxels.  *loss (optional) receives the loss before the step;
 * asking for it synchronises the stream. */
int lesnet_train_step(lesnet* n, int32_t B, int32_t D, int32_t H, int32_t W, const float* d_x,
                      const float* d_t, double* loss, void* stream);
/* Adam step size of the following train steps (a schedule); LES_EINVAL
 * unless positive and finite. */
int lesnet_set_lr(lesnet* n, double lr);

/*
 * One layer operation on the matrix cores, on its own (no handle): the
 * float32 operands are rounded to bfloat16 on the device, products are
 * accumulated in float32 and the result is returned in float32, so a
 * caller can check each kernel of the network in isolation.  Grids as for
 * the network (B, D, H, W; channels last); for the up operations (B, D, H,
 * W) is the coarse grid and the fine grid is twice it per axis.
 *   LESNET_OP_CONV3        a = x [B][D][H][W][cin], b = W [27][cin][cout],
 *                          c = bias [cout] or NULL; out = y [..][cout] (no ReLU)
 *   LESNET_OP_CONV3_DGRAD  a = dy [..][cout], b = W; out = dx [..][cin]
 *   LESNET_OP_CONV3_WGRAD  a = x [..][cin], b = dy [..][cout]; out = dW [27][cin][cout]
 *   LESNET_OP_UP           a = x coarse [..][cin], b = U [8][cin][cout], c = bias
 *                          or NULL; out = y fine [B][2D][2H][2W][cout]
 *   LESNET_OP_UP_DGRAD     a = dy fine [..][cout], b = U; out = dx coarse [..][cin]
 *   LESNET_OP_UP_WGRAD     a = x coarse, b = dy fine; out = dU [8][cin][cout]
 * cout in {16, 32, 64}; cin in {16, 32, 64}, or 1..8 for the forward and
 * weight-gradient operations.  Device pointers; allocates its own
 * workspace and synchronises `stream` before returning.  LES_EINVAL for
 * other sizes or NULL operands, LES_ENOMEM, LES_EDEVICE.
 */
enum {
    LESNET_OP_CONV3 = 0,
    LESNET_OP_CONV3_DGRAD = 1,
    LESNET_OP_CONV3_WGRAD = 2,
    LESNET_OP_UP = 3,
    LESNET_OP_UP_DGRAD = 4,
    LESNET_OP_UP_WGRAD = 5
};
int lesnet_op(int32_t op, int32_t B, int32_t D, int32_t H, int32_t W, int32_t cin, int32_t cout,
              const float* d_a, const float* d_b, const float* d_c, float* d_out, void* stream);

/* ---- training-set preparation on the device ----
 * The learned part's data path: windows of captured pairs, their mirror
 * images in y, mini-batch gathers and the target scaling, as library
 * kernels.  All device pointers, ordered on `stream` (NULL: the default
 * stream), no synchronisation, no allocation.  LES_EINVAL on NULL pointers
 * or out-of-range sizes, LES_EDEVICE if a launch fails.
 *
 * lesnet_crop: copy the window [z, z+cd) x [y, y+ch) x [x, x+cw) of a
 * [D][H][W][C] float32 array into d_dst [cd][ch][cw][C]; with mirror_y the
 * window is reflected in y (row c of d_dst is source row y + ch - 1 - c).
 * The y walls carry the same boundary condition on both sides, so the
 * pressure operator commutes with that reflection and a reflected pair is
 * a valid training pair.  d_src and d_dst must not overlap. */
int lesnet_crop(const float* d_src, int32_t D, int32_t H, int32_t W, int32_t C, int32_t z, int32_t y,
                int32_t x, int32_t cd, int32_t ch, int32_t cw, int32_t mirror_y, float* d_dst, void* stream);
/* lesnet_gather: d_dst[b] = d_src[idx[b]] for b < n (1 <= n <= 64), items
 * of `item` floats, d_src holding `count` items; idx is a host array. */
int lesnet_gather(const float* d_src, int64_t item, int64_t count, const int32_t* idx, int32_t n,
                  float* d_dst, void* stream);
/* lesnet_sum_squares: *d_out (device float64) = sum of x^2 over n floats,
 * accumulated in float64 in a fixed order (deterministic); d_x may be NULL
 * when n is 0 (the sum is 0). */
int lesnet_sum_squares(const float* d_x, int64_t n, double* d_out, void* stream);
/* lesnet_scale_div: d_y = d_x / s elementwise (float32 division; d_y may be
 * d_x); s finite and > 0; nothing to do (pointers unused) when n is 0. */
int lesnet_scale_div(const float* d_x, int64_t n, float s, float* d_y, void* stream);

/*
 * Coupling to an LES handle.  The network grid of a handle is (D, H, W) =
 * (nz, ny, nx) each rounded up to a multiple of 4; voxel (z, y, x) is cell
 * (i, j, k) = (x+1, y+1, z+1), the padding voxels are zero.  With
 * r = rhs - A p_prev the residual of the previous pressure and N the cell
 * count, the three input channels are
 *   r / RMS(r),  1 for a building cell else 0,  p_prev / RMS(p_prev)
 * (a channel whose RMS is 0 is zero), and the network's output y gives the
 * candidate start
 *   p0 = p_prev + y * RMS(r) / dbar * target_scale,  dbar = 2 (1/dx^2 + 1/dy^2 + 1/dz^2).
 * The training target of a step is (p* - p_prev) dbar / RMS(r), p* the
 * converged pressure.
 */
int les_warm_grid(const les_handle* h, int32_t* D, int32_t* H, int32_t* W);
/* Choice between the two starts (les_set_warm_start).  Whichever start is
 * taken, the solve itself runs to the handle's tolerance, and when p_prev
 * is kept the step is bit for bit the plain one. */
enum {
    LES_WARM_RESIDUAL = 0,   /* p0 if its float64 residual norm is strictly smaller */
    LES_WARM_TRIAL = 1,      /* SOR runs `param` iterations (whole check intervals)
                                from each start in a scratch copy; p0 if its residual
                                is then strictly smaller.  The trial iterations are
                                extra work, not counted in sor_iters */
    LES_WARM_SMOOTH = 2,     /* both residuals are smoothed by `param` passes (rounded
                                up to even) of the 7-point mean over the cells, p0
                                if the smoothed norm is strictly smaller: the rule
                                weighs the smooth error that SOR removes slowly */
    LES_WARM_ALWAYS = 3      /* always p0 (for measurements) */
};
/* Use n (NULL: switch off) in every following les_step: after the
 * right-hand side is built the network proposes p0 and `rule` picks the
 * start; param is the trial iterations or smoothing passes (1..100000,
 * unused by the other rules).  `smooth` passes of the 7-point mean over
 * the cells (0..100000) are applied to the network's output before it
 * forms p0: a network trained on targets captured with the same
 * smoothing proposes only the smooth part of the change, the part SOR is
 * slow to find.  All rules but LES_WARM_TRIAL decide on the device
 * without a host round trip.  The handle borrows n; keep it alive while
 * set.  les_step_stats reports the choice and the two norms compared
 * (relative to ||rhs||).  LES_EINVAL for target_scale not positive and
 * finite, an unknown rule, param or smooth out of range. */
int les_set_warm_start(les_handle* h, lesnet* n, double target_scale, int32_t rule, int32_t param,
                       int32_t smooth);
/* Training-pair capture (NULL, NULL: off): every following les_step writes
 * the network input of the step to d_x [D][H][W][3] and, after the solve,
 * its training target to d_t [D][H][W] (device buffers owned by the
 * caller, overwritten by each step), the target smoothed by `smooth`
 * passes (rounded up to even) of the mean described above. */
int les_set_capture(les_handle* h, float* d_x, float* d_t, int32_t smooth);

#ifdef __cplusplus
}
#endif

#endif /* LESNET_H_ */
