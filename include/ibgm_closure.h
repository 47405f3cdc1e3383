/*
 * ibgm_closure.h -- C ABI of the learned-closure kernels in libibgm.so.
 *
 * A coarse IB-GM solve (mesh 2h, time step 2 dt) is corrected toward the
 * restriction of the fine solve (mesh h, time step dt) by a three-layer 3-D
 * convolutional network: 3x3x3 taps, 32 hidden channels, ReLU after layers 1
 * and 2, BF16 weights and activations, FP32 accumulation on the matrix cores.
 * The closure is not part of the paper's method; the method itself generates
 * its training pairs (fine and coarse runs of the IB-GM step), and the plain
 * fine solve judges its error.
 *
 * Conventions (in addition to those of ibgm.h)
 *   Activations  BF16 (raw 16-bit storage, uint16_t here), [B][D2][D1][D0][C]:
 *                a batch of bricks, x fastest, channels last.  C (the padded
 *                channel count) is 16 or 32 for inputs of a convolution and 32
 *                for hidden outputs; padding channels hold zeros.
 *   Weights      FP32 masters [27][ci][co] with tap t = 9 tz + 3 ty + tx
 *                (tz, ty, tx in {0, 1, 2}).  Convolutions read them packed
 *                (ib_conv3d_pack) into BF16 matrix-core operand tiles of
 *                IB_CONV_PACKED_BYTES(ci_pad) bytes.
 *   Modes        Output voxel p reads input voxel p + (tz, ty, tx) + off:
 *                IB_CONV_PERIODIC: off = -1, indices wrap, output size = input
 *                IB_CONV_VALID:    off = 0, output = input - 2 per axis
 *                IB_CONV_FULL:     off = -2, voxels outside read 0, output =
 *                                  input + 2 (the adjoint of VALID)
 *   Streams, errors and ownership as in ibgm.h: every pointer is a device
 *   pointer unless marked host, the caller owns all memory, work is enqueued
 *   on `hip_stream`, IB_E_INVALID means nothing was enqueued.
 */
#ifndef IBGM_CLOSURE_H
#define IBGM_CLOSURE_H

#include <stddef.h>
#include <stdint.h>

#include "ibgm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IB_CONV_PERIODIC 0
#define IB_CONV_VALID 1
#define IB_CONV_FULL 2

#define IB_CONV_RELU 1    /* ReLU on the output */
#define IB_CONV_OUT_F32 2 /* FP32 output (default BF16) */
#define IB_CONV_NARROW 4  /* weights in the narrow packing (co <= 16, ci_pad 32) */

#define IB_CONV_PACK_FORWARD 0
#define IB_CONV_PACK_ADJOINT 1
#define IB_CONV_PACK_NARROW 2
#define IB_CONV_PACKED_NARROW_BYTES ((size_t)27 * 64 * 16)

#define IB_CONV_OUT_CHANNELS 32 /* output channels of every convolution (padded) */
#define IB_CONV_PACKED_BYTES(ci_pad) ((size_t)27 * ((ci_pad) / 16) * 64 * 16)
/* workspace of ib_conv3d_bwd_weight: per-workgroup partial sums */
#define IB_CONV_WGRAD_BLOCKS 256
#define IB_CONV_WGRAD_WORKSPACE_BYTES \
  ((size_t)IB_CONV_WGRAD_BLOCKS * (27 * 32 * 32 + 32) * sizeof(float))

/* Pack FP32 weights W[27][ci][co] (ci <= ci_pad, co <= 32, ci_pad 16 or 32)
 * into the operand layout of ib_conv3d_fwd (transpose = IB_CONV_PACK_FORWARD,
 * IB_CONV_PACKED_BYTES(ci_pad) bytes).  IB_CONV_PACK_ADJOINT packs the
 * weights of the adjoint convolution instead: taps reversed (t -> 26 - t) and
 * channel roles swapped, W'[t][co][ci] = W[26 - t][ci][co], for a convolution
 * with input channels co (ci_pad must then be 32) and output channels ci;
 * ib_conv3d_bwd_data takes this packing.  IB_CONV_PACK_NARROW (co <= 16,
 * ci_pad 32, IB_CONV_PACKED_NARROW_BYTES) is the operand layout of the
 * 16-wide forward kernel, selected by IB_CONV_NARROW. */
ib_status ib_conv3d_pack(const float *W, int32_t ci, int32_t co, int32_t ci_pad,
                         int32_t transpose, void *packed, void *hip_stream);

/* y = act(conv(x, W) + bias) for a batch of `batch` bricks of in_dims (x, y,
 * z sizes) with ci_pad input channels; output dims follow from `mode`.
 * flags: IB_CONV_RELU, IB_CONV_OUT_F32, IB_CONV_NARROW (weights in the
 * narrow packing: ci_pad 32, co_store <= 16).  Channels co < co_store of each
 * output voxel are written at y + voxel * y_stride + co (y_stride >= co_store;
 * 32 for a hidden activation).  bias: FP32 [co_store] or NULL. */
ib_status ib_conv3d_fwd(const uint16_t *x, int32_t batch, const int32_t in_dims[3],
                        int32_t ci_pad, const void *packed, const float *bias,
                        int32_t mode, int32_t flags, void *y, int32_t co_store,
                        int32_t y_stride, void *hip_stream);

/* Gradient with respect to a layer's input: gx = conv^T(gy, W), where gy
 * (BF16, 32 channels) has the layer's output dims out_dims and the layer ran
 * in `mode` (PERIODIC or VALID); `packed` is ib_conv3d_pack(..., transpose=1).
 * If act_below is not NULL (the BF16 post-ReLU activation that fed the layer,
 * 32 channels), gx is multiplied by [act_below > 0] (the ReLU derivative).
 * gx: BF16, 32 channels per voxel (the first ci_out of them meaningful). */
ib_status ib_conv3d_bwd_data(const uint16_t *gy, int32_t batch, const int32_t out_dims[3],
                             const void *packed, int32_t mode, const uint16_t *act_below,
                             uint16_t *gx, void *hip_stream);

/* Gradients of the weights and bias of a layer that ran in `mode` on input x
 * (BF16, ci_pad channels, in_dims) and produced an output whose gradient is gy
 * (BF16, 32 channels): dW[t][ci][co] = sum_p x[p + t + off][ci] gy[p][co] and
 * db[co] = sum_p gy[p][co], written (not accumulated) as FP32 [27][ci][co] and
 * [co] for the first ci <= ci_pad, co <= 32 channels.  workspace: device,
 * IB_CONV_WGRAD_WORKSPACE_BYTES, 256-byte aligned. */
ib_status ib_conv3d_bwd_weight(const uint16_t *x, const uint16_t *gy, int32_t batch,
                               const int32_t in_dims[3], int32_t ci_pad, int32_t mode,
                               int32_t ci, int32_t co, float *dW, float *db,
                               void *workspace, void *hip_stream);

/* Mean-squared error of pred against target (FP32, n_vox x nch, nch <= 32):
 * *loss = mean((pred - target)^2) (device FP32 scalar) and
 * grad[v][c] = 2 (pred - target) / (n_vox nch) as BF16 with 32 channels per
 * voxel (zeros beyond nch).  workspace: device, 4 * 1024 bytes. */
ib_status ib_mse_grad(const float *pred, const float *target, int64_t n_vox, int32_t nch,
                      float *loss, uint16_t *grad, void *workspace, void *hip_stream);

/* One Adam update (Kingma & Ba 2015, Algorithm 1) of n FP32 parameters
 * theta with gradient g and moments m, v at step t >= 1. */
ib_status ib_adam_step(float *theta, const float *g, float *m, float *v, int64_t n,
                       float lr, float beta1, float beta2, float eps, int32_t t,
                       void *hip_stream);

/* Restriction of a 3-D MAC field on the fine grid nf (each even) to the grid
 * nf/2: kind 0, 1, 2 = the velocity component normal to that axis (the coarse
 * face coincides with fine face 2I and averages the 2 x 2 fine faces around
 * it); kind 3 = cell-centred (average of 2 x 2 x 2 cells).  dtype: ib_dtype
 * of both arrays. */
ib_status ib_restrict(const void *fine, int32_t dtype, const int32_t nf[3], int32_t kind,
                      void *coarse, void *hip_stream);

/* Gather network inputs or targets from nsrc (<= IB_GATHER_MAX_SOURCES) FP32
 * fields on the periodic grid n: for brick b with origin origins[b] =
 * (x0, y0, z0) (device int32 [batch][3]) and voxel (i, j, k) of dims, output
 * channel c is the sum of scales[s] src[s][(z0 + k) mod n2][(y0 + j) mod n1]
 * [(x0 + i) mod n0] over the sources s with chan[s] = c (src: host array of
 * device pointers; scales, chan: host arrays of nsrc; channels no source
 * names are 0).  out_f32 = 0: BF16 output with out_ch = 16 channels per voxel;
 * out_f32 = 1: FP32 output with out_ch (1..16) channels per voxel. */
#define IB_GATHER_MAX_SOURCES 12
ib_status ib_closure_gather(const float *const *src, const float *scales, const int32_t *chan,
                            int32_t nsrc, const int32_t n[3], const int32_t *origins,
                            int32_t batch, const int32_t dims[3], int32_t out_f32,
                            int32_t out_ch, void *out, void *hip_stream);

/* Apply a predicted correction on the periodic grid n: u[c][v] += scale *
 * y[v * 3 + c] for c < 3 (u: FP32 component arrays, y: FP32 [n_vox][3]). */
ib_status ib_closure_apply(float *const u[3], const int32_t n[3], const float *y, float scale,
                           void *hip_stream);

/* The network's last layer and the correction in one pass: for the periodic
 * 3x3x3 convolution of x (BF16, 32 channels, [n2][n1][n0][32]) with weights
 * in the narrow packing (IB_CONV_PACK_NARROW, co = 3) and bias (FP32 [3] or
 * NULL), u[c][v] = fma(scale, y[v][c], u[c][v]) for c < 3, where y is what
 * ib_conv3d_fwd(x, 1, n, 32, packed, bias, IB_CONV_PERIODIC,
 * IB_CONV_OUT_F32 | IB_CONV_NARROW, y, 3, 3) would write -- the same
 * arithmetic as that call followed by ib_closure_apply, bit for bit, without
 * the intermediate output.  u: three distinct FP32 arrays of n[0] n[1] n[2]
 * values, updated in place; scale must be finite. */
ib_status ib_closure_conv_apply(const uint16_t *x, const int32_t n[3], const void *packed,
                                const float *bias, float scale, float *const u[3],
                                void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
