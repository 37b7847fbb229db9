/*
 * lbm_nn.h -- C ABI of the layers of the warm-start network in liblbm.so.
 *
 * The learned warm start is not part of the paper's method: a 3D U-Net maps a voxel
 * geometry (pore mask, pore-diameter map) to initial fields of the flow and Knudsen
 * solves (u, rho - 1, C), which the solvers take as u_init / c_init.  The solvers still
 * iterate to their own convergence criterion, so the network only changes the number
 * of steps, and a solve from rest remains the reference for its error.
 *
 * Conventions (as in lbm.h: status codes, device pointers unless named *_h, `stream`
 * a hipStream_t passed as void*, gfx950 only):
 *  - A tensor is channels-last bfloat16 (uint16_t bit patterns): element (voxel v,
 *    channel c) at v * cs + c, voxel v = x + nx (y + ny z).  A view is a pointer to its
 *    first channel and the channel stride cs; pointers must be 8-byte aligned and the
 *    channel strides multiples of 4 where a call says so.
 *  - Convolution weights are bf16 [27][cout][cin], tap t = 9 (dz + 1) + 3 (dy + 1) +
 *    (dx + 1); gradients and biases are binary32.
 *  - Products accumulate in binary32 (matrix cores); results are rounded to bf16 to
 *    nearest even.  Reductions that form weight gradients and losses run in a fixed
 *    order: results are bitwise reproducible for equal inputs.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_NN_RELU 1 /* apply max(0, .) to the convolution output */
#define LBM_NN_FLIP 2 /* use tap offsets -d_t (the input-gradient convolution) */

/* 3x3x3 zero-padded cross-correlation on the grid n = (nx, ny, nz):
 *   y[v][c] = act(bias[c] + sum_t sum_k x[v + d_t][k] w[t][c][k]),  d_t negated with
 *   LBM_NN_FLIP, neighbours beyond the box reading 0.
 * With LBM_NN_FLIP and weights from lbm_nn_transpose_weights this is the gradient with
 * respect to the input of a convolution (given the gradient of its pre-activation).
 * x: view with cin channels (cin a multiple of 16, <= x_cs, x_cs a multiple of 4);
 * w: [27][cout][cin]; bias: float[cout], nullable; y: view with cout channels (cout in
 * {16, 32, 48, 64, 96, 128, 192}, <= y_cs).  nx ny nz must be a multiple of 16.
 * Errors: LBM_E_INVAL (shapes, strides, alignment, flags), LBM_E_DEVICE. */
lbm_status lbm_nn_conv3d(const int32_t n[3], const uint16_t *x, int32_t x_cs, int32_t cin,
                         const uint16_t *w, const float *bias, uint16_t *y, int32_t y_cs,
                         int32_t cout, int32_t flags, void *stream);

/* Workspace bytes of lbm_nn_conv3d_wgrad for this grid and channel counts. */
size_t lbm_nn_wgrad_workspace(const int32_t n[3], int32_t cin, int32_t cout);

/* Weight and bias gradients of a convolution given its input x and the gradient g of
 * its pre-activation output:
 *   dw[t][co][ci] = sum_v g[v][co] x[v + d_t][ci],   db[co] = sum_v g[v][co]
 * (written, or added to the existing values with accumulate = 1).  cin and cout
 * multiples of 16 (cin in {16, 32, 48, 64, 96, 128, 192}); db nullable.
 * Errors: LBM_E_INVAL, LBM_E_NOMEM (workspace), LBM_E_DEVICE. */
lbm_status lbm_nn_conv3d_wgrad(const int32_t n[3], const uint16_t *x, int32_t x_cs, int32_t cin,
                               const uint16_t *g, int32_t g_cs, int32_t cout, float *dw, float *db,
                               int32_t accumulate, void *workspace, size_t ws_bytes, void *stream);

/* wt[t][ci][co] = w[t][co][ci]: the weights of the input-gradient convolution. */
lbm_status lbm_nn_transpose_weights(const uint16_t *w, int32_t cout, int32_t cin, uint16_t *wt,
                                    void *stream);

/* 2x2x2 mean pooling of c channels from the fine grid n_fine (even sizes) to the coarse
 * grid, and its adjoint (each fine voxel receives 1/8 of its parent's gradient); with
 * accumulate = 1 the result is added to the output view. */
lbm_status lbm_nn_pool2(const int32_t n_fine[3], int32_t c, const uint16_t *x, int32_t x_cs,
                        uint16_t *y, int32_t y_cs, int32_t accumulate, void *stream);
lbm_status lbm_nn_pool2_bwd(const int32_t n_fine[3], int32_t c, const uint16_t *gy, int32_t gy_cs,
                            uint16_t *gx, int32_t gx_cs, int32_t accumulate, void *stream);

/* Nearest upsampling of c channels from the coarse grid to the fine grid n_fine (each
 * fine voxel copies its parent), and its adjoint (each parent sums its 8 children). */
lbm_status lbm_nn_up2(const int32_t n_fine[3], int32_t c, const uint16_t *x, int32_t x_cs,
                      uint16_t *y, int32_t y_cs, void *stream);
lbm_status lbm_nn_up2_bwd(const int32_t n_fine[3], int32_t c, const uint16_t *gy, int32_t gy_cs,
                          uint16_t *gx, int32_t gx_cs, void *stream);

/* g = gy where the layer output y is positive, 0 elsewhere (the ReLU gradient). */
lbm_status lbm_nn_relu_bwd(int64_t nvox, int32_t c, const uint16_t *y, int32_t y_cs,
                           const uint16_t *gy, int32_t gy_cs, uint16_t *g, int32_t g_cs,
                           void *stream);

/* Workspace bytes of lbm_nn_head with a target. */
size_t lbm_nn_head_workspace(int64_t nvox, int32_t no);

/* The 1x1x1 output head on 16 input channels: out[o][v] = bh[o] + sum_c wh[o][c] x[v][c]
 * (float, planar [no][nvox], nullable; 1 <= no <= 8; wh float[no][16], bh float[no]).
 * With a target (float planar [no][nvox]): loss_h = sum_v mask[v] sum_o wt[o]
 * (out - target)^2 / n_mask, gwh / gbh its gradients (written), and gx (bf16 view with
 * 16 channels, nullable) the gradient with respect to x.  mask: uint8[nvox], wt:
 * float[no] (device).  Synchronises the stream when a target is given.
 * Errors: LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_nn_head(int64_t nvox, const uint16_t *x, int32_t x_cs, int32_t no, const float *wh,
                       const float *bh, float *out, const float *target, const uint8_t *mask,
                       const float *wt, double n_mask, uint16_t *gx, int32_t gx_cs, float *gwh,
                       float *gbh, double *loss_h, void *workspace, size_t ws_bytes,
                       void *stream);

/* One Adam step (bias-corrected with beta^step) on n binary32 weights; refreshes their
 * bf16 copy w_bf16 (nullable). */
lbm_status lbm_nn_adam(int64_t n, float *w, const float *g, float *m, float *v, uint16_t *w_bf16,
                       float lr, float beta1, float beta2, float eps, int64_t step, void *stream);

/* dst = bf16(src), n values. */
lbm_status lbm_nn_to_bf16(int64_t n, const float *src, uint16_t *dst, void *stream);

/* The network input: channel 0 the pore mask (0/1), channel 1 diam / d_scale, the other
 * channels up to x_cs zero.  mask uint8[nvox], diam double[nvox]. */
lbm_status lbm_nn_make_input(int64_t nvox, const uint8_t *mask, const double *diam, double d_scale,
                             uint16_t *x, int32_t x_cs, void *stream);

/* Warm-start fields from the head output: fields[k][v] = mask[v] ? out[k][v] * scale[k]
 * : 0 for k < nk (scale: device float[nk]). */
lbm_status lbm_nn_to_fields(int64_t nvox, int32_t nk, const float *out, const uint8_t *mask,
                            const float *scale, float *fields, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_NN_H */
