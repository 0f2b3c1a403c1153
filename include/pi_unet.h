/*
 * pi_unet.h -- layer operations of the learned warm start for libpi.
 *
 * The warm start is a small convolutional U-Net that maps a (coarsened)
 * pressure-gradient field to an initial pressure guess {P^0} for Algorithm 1
 * (which the paper starts from {P^0} = 0; Section "Effect of Pressure
 * Magnitude at the Boundaries" shows that the iteration count grows with the
 * distance of the boundary pressures from the initial guess, and Section
 * "Wall-clock Time Convergence" that a good starting field shortens the
 * solve).  The solver always finishes from the guess, so the guess only
 * changes the iteration count, never the answer.
 *
 * These entry points are the network's arithmetic: BF16 matrix-core (MFMA)
 * convolutions with FP32 accumulation, their data and weight gradients,
 * pooling, the output head, the loss, the optimizer step, and the transfers
 * between the solver's grids and the network's.  A driver (the Python
 * package) strings them together.
 *
 * Tensors are channels-last BF16 (or FP32 where stated) arrays
 * [n][d][h][w][ld], of which channels [off, off + c) are used, so a tensor can
 * be a channel slice of a wider buffer (skip concatenation).  All pointers
 * are device pointers owned by the caller; every call is asynchronous on
 * `stream` (a hipStream_t as void*) and returns PI_ERR_INVALID_ARG for
 * inconsistent shapes, else PI_OK (or PI_ERR_DEVICE if a launch fails).
 */
#ifndef PI_UNET_H
#define PI_UNET_H

#include <stddef.h>
#include <stdint.h>

#include "pi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pu_tensor {
  void *ptr;
  int32_t n, d, h, w;   /* batch and grid */
  int32_t c;            /* channels used */
  int32_t ld;           /* channel stride of the buffer (>= off + c) */
  int32_t off;          /* first channel */
} pu_tensor;

/*
 * pu_conv -- y[o(p), co] = act(sum_t sum_ci x[g_t(p), ci] w[t][co][ci] + b[co])
 * over the positions p of an (md, mh, mw) grid per sample, with
 * g_t(p) = p * sin + offs[t] (zero outside x) and o(p) = p * sout + oo.
 *   3x3x3 convolution:           taps 27, offsets {-1,0,1}^3, sin = sout = 1,
 *                                weights [t][cout][cin] (per-tap transposed
 *                                from the layer's [t][cin][cout])
 *   its data gradient:           the layer's [t][cin][cout] weights as
 *                                [t][N = cin][K = cout], negated offsets
 *   2x2x2 stride-2 transposed conv (one output parity oo): taps 1, sout = 2
 *   its data gradient:           taps 8, offsets {0,1}^3, sin = 2
 * offs: host array of 3 * taps int8 offsets (dz, dy, dx) per tap, copied
 * into the launch.  w: BF16 [taps][cout][cin] device array (K = cin
 * contiguous), 16-byte aligned; bias: FP32 [cout] or NULL; relu: 0/1;
 * y_fp32: 1 stores FP32 (y->ptr is float*), else BF16.  accumulate: 1 adds
 * into y instead of overwriting it.
 */
pi_status pu_conv(const pu_tensor *x, const void *w, int32_t taps, const int8_t *offs, const float *bias,
                  const pu_tensor *y, int32_t md, int32_t mh, int32_t mw, int32_t sin, int32_t sout,
                  const int32_t oo[3], int32_t relu, int32_t y_fp32, int32_t accumulate, void *stream);

/*
 * pu_conv_wgrad -- dw[t][ci][cout] = sum_p x[g_t(p), ci] gy[o(p), co] with the
 * maps of pu_conv, FP32 output [taps][cin][cout] (overwritten), and
 * db[co] = sum_p gy[o(p), co] when db != NULL.  `work` is an FP32 scratch of
 * at least pu_wgrad_work_floats(...) floats.
 */
size_t pu_wgrad_work_floats(int32_t taps, int32_t cin, int32_t cout, int64_t positions);
pi_status pu_conv_wgrad(const pu_tensor *x, const pu_tensor *gy, int32_t taps, const int8_t *offs, float *dw,
                        float *db, int32_t md, int32_t mh, int32_t mw, int32_t sin, int32_t sout,
                        const int32_t oo[3], float *work, void *stream);

/* Per-tap transpose of BF16 weights: wt[t][co][ci] = w[t][ci][co]. */
pi_status pu_transpose_taps(const void *w, void *wt, int32_t taps, int32_t cin, int32_t cout, void *stream);

/* g <- g * (y > 0) elementwise over matching tensors (ReLU backward). */
pi_status pu_relu_backward(const pu_tensor *y, const pu_tensor *g, void *stream);

/* 2x2x2 average pooling and its backward (accumulate: add into gx). */
pi_status pu_pool(const pu_tensor *x, const pu_tensor *y, void *stream);
pi_status pu_pool_backward(const pu_tensor *gy, const pu_tensor *gx, int32_t accumulate, void *stream);

/*
 * Head: y[p] = sum_c x[p, c] w[c] + b[0] (FP32 y [n][d][h][w], w and b FP32
 * device arrays); backward gives
 * gx (BF16 tensor), gw[c] (FP32) and gb (FP32 scalar) from gy (FP32); the
 * backward's work is an FP32 scratch of at least 1025 * (x->c + 1) floats.
 */
pi_status pu_head(const pu_tensor *x, const float *w, const float *b, float *y, void *stream);
pi_status pu_head_backward(const pu_tensor *x, const float *w, const float *gy, const pu_tensor *gx, float *gw,
                           float *gb, float *work, void *stream);

/*
 * Masked mean squared error over count = n*d*h*w cells: loss (FP32 scalar,
 * device) and grad = 2 m (pred - target) / sum(m) (NULL to skip).  mask: uint8
 * or NULL.  work: FP32 scratch of at least 2049 floats.
 */
pi_status pu_mse(const float *pred, const float *target, const uint8_t *mask, int64_t count, float *loss,
                 float *grad, float *work, void *stream);

/*
 * Adam step on FP32 master weights w (count elements) with gradient g,
 * moments m, v; writes the BF16 copy wb (NULL to skip).  step >= 1.
 */
pi_status pu_adam(float *w, const float *g, float *m, float *v, void *wb, int64_t count, float lr, float beta1,
                  float beta2, float eps, int32_t step, void *stream);

/*
 * Solver grid -> network input: average the gradient components over
 * factor^ndim blocks of data cells, scale them, and write a channels-last
 * BF16 tensor [1][d/f][h/f][w/f][4] = (gx, gy, gz, data fraction); 2-D grids
 * use d = 1 and gz = NULL.  gx, gy, gz are FP32 in the solver's layout; mask
 * is uint8 or NULL.  Grid sizes must be multiples of factor.
 */
pi_status pu_prepare_input(const float *gx, const float *gy, const float *gz, const uint8_t *mask,
                           const int64_t dims[3], int32_t factor, float scale, const pu_tensor *out,
                           void *stream);

/*
 * Coarse-grid view of a gradient field for the coarse solve of the warm
 * start: per block of factor^3 cells (factor^2 in 2-D, gz NULL), the FP32
 * mean of each component over the block's data cells (0 where none), written
 * to ox, oy, oz (oz ignored in 2-D) in the solver's layout of the coarse grid
 * (nx/f, ny/f[, nz/f]).  dims must be divisible by factor.
 */
pi_status pu_block_mean(const float *gx, const float *gy, const float *gz, const uint8_t *mask,
                        const int64_t dims[3], int32_t factor, float *ox, float *oy, float *oz, void *stream);

/*
 * Network output -> solver grid: trilinear interpolation of the cell-centred
 * coarse field (FP32 [d/f][h/f][w/f]) onto the fine cells, times scale,
 * written as float, or as double with PU_OUT_FP64, in the solver's layout;
 * with PU_OUT_ADD added to what P holds instead of replacing it.  factor 1
 * copies (scaled).
 */
#define PU_OUT_FP64 0x1
#define PU_OUT_ADD 0x2
pi_status pu_upsample_output(const float *coarse, const int64_t dims[3], int32_t factor, float scale, void *P,
                             int32_t flags, void *stream);

/*
 * Normalisation of the network input: rms = sqrt(sum |g|^2 / valid cells) over
 * the `count` cells of the solver's layout (gz NULL in 2-D), as an FP32 scalar
 * in device memory.  work: FP32 scratch of at least 1025 floats.
 */
pi_status pu_grad_rms(const float *gx, const float *gy, const float *gz, const uint8_t *mask, int64_t count,
                      float *rms, float *work, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PI_UNET_H */
