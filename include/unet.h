/* unet.h - C ABI of the U-Net surrogate kernels (BF16 MFMA, gfx950).
 *
 * A small U-Net predicts the steady non-wetting saturation of a drainage
 * problem (solid mask, contact-angle plane and pressure-step plane in;
 * per-node saturation out) and warm-starts the lattice Boltzmann solver of
 * lbm.h.  The network is not part of the paper's method: it only supplies an
 * initial density field, and the solver's own steady state decides the
 * answer.  These entry points are the network's layer operations (forward and
 * backward) and its optimiser; a host driver strings them together.
 *
 * Conventions:
 *  - Every pointer is a device pointer owned by the caller; nothing is
 *    allocated.  Work is enqueued on the HIP stream `s` (void*, NULL = the
 *    null stream) and runs asynchronously; results are valid once the stream
 *    has reached them.
 *  - Activations are BF16 (uint16_t bit patterns), NHWC: element (n, y, x, c)
 *    of a tensor with channel stride cs sits at n*H*W*cs + (y*W + x)*cs + c.
 *    A channel offset `co` selects a channel slice of a wider tensor (the
 *    skip concatenations write into slices).  Reduction channel counts and
 *    the strides/offsets of MFMA operands are multiples of 8 (16-byte
 *    vector loads); tensors start 16-byte aligned.
 *  - 3x3 weights are [Cout][3][3][Cin] BF16; 2x2 transposed-convolution
 *    weights are [Cout][2][2][Cin] BF16; biases, gradients, master weights
 *    and optimiser moments are FP32.
 *  - Products run on the matrix cores (v_mfma_f32_32x32x16_bf16) and
 *    accumulate in FP32; outputs are rounded to BF16 (round to nearest even).
 *  - Sums (weight, bias and head gradients, the loss) are taken in a fixed
 *    order: results are bitwise reproducible.
 *  - Return 0 on success; -1 on invalid arguments (checked before any
 *    launch: null pointers, non-positive sizes, misaligned channel counts);
 *    -100 if a launch failed.
 */
#ifndef UNET_H
#define UNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One MFMA for checking the operand layout: C = A B with A 32x16, B 16x32
 * (BF16, row-major) and C 32x32 (FP32, row-major).  One wave. */
int unet_mfma_probe(const uint16_t *A, const uint16_t *B, float *C, void *s);

/* y = act(conv3x3(x, w) + b) over an n x h x w grid with zero padding
 * (cross-correlation: y[p][co] = b[co] + sum_{ky,kx,ci} w[co][ky][kx][ci]
 * x[p + (ky-1, kx-1)][ci]); act = ReLU if relu != 0.  bias may be NULL. */
int unet_conv3x3_fwd(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co,
                     const uint16_t *wgt, const float *bias, int cout,
                     uint16_t *y, int y_cs, int y_co, int relu, void *s);

/* Weights of the data gradient: wt[ci][ky][kx][co] = w[co][2-ky][2-kx][ci],
 * so that dx = conv3x3(dy, wt) (no bias, no ReLU) with the forward entry. */
int unet_conv3x3_flip(const uint16_t *wgt, int cout, int cin, uint16_t *wt, void *s);

/* Weight gradient of the 3x3 convolution:
 *   dw[co][ky][kx][ci] (+)= sum_p dy[p][co] x[p + (ky-1, kx-1)][ci]
 *   db[co]             (+)= sum_p dy[p][co]        (if db != NULL)
 * accumulate = 0 overwrites.  partial: FP32 scratch of at least
 * unet_wgrad_scratch_floats(n, h, w, cin, cout, 9) floats. */
int64_t unet_wgrad_scratch_floats(int n, int h, int w, int cin, int cout, int taps);
int unet_conv3x3_wgrad(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co,
                       const uint16_t *dy, int cout, int dy_cs, int dy_co,
                       float *dw, float *db, float *partial, int accumulate, void *s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the weight
 * gradient of unet_conv3x3_wgrad with the same arguments except `partial`.
 * Its split-K partial sums live in a library-held device array of
 * 4 Mi floats (16 MiB) per GPU, held until the process ends; problems with
 * unet_wgrad_scratch_floats(n, h, w, cin, cout, 9) above that return -2
 * before any device work.  The array's address is looked up once per device
 * (hipGetSymbolAddress, with that device current).  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race on it.  Nothing in it needs to start at zero.  Returns
 * 0, -1 (invalid arguments, as unet_conv3x3_wgrad), -2 (too large) or -100
 * (the lookup or a launch failed). */
int unet_conv3x3_wgrad_noalloc(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co,
                               const uint16_t *dy, int cout, int dy_cs, int dy_co,
                               float *dw, float *db, int accumulate, void *s);

/* dy[p][c] = 0 where y[p][c] <= 0 (ReLU backward, in place on a slice). */
int unet_relu_bwd(const uint16_t *y, int n_pix, int c, int y_cs, int y_co,
                  uint16_t *dy, int dy_cs, int dy_co, void *s);

/* 2x2 max pooling with stride 2 (h, w even): y is n x h/2 x w/2.  Backward
 * recomputes the argmax from x (ties: first in (dy, dx) raster order) and
 * routes dy there; accumulate = 0 writes every element of the 2x2 window
 * (the others get 0), accumulate != 0 adds to the argmax element only. */
int unet_maxpool_fwd(const uint16_t *x, int n, int h, int w, int c, int x_cs, int x_co,
                     uint16_t *y, int y_cs, int y_co, void *s);
int unet_maxpool_bwd(const uint16_t *x, int n, int h, int w, int c, int x_cs, int x_co,
                     const uint16_t *dy, int dy_cs, int dy_co, uint16_t *dx, int dx_cs, int dx_co,
                     int accumulate, void *s);

/* 2x2 stride-2 transposed convolution from an n x h x w grid to 2h x 2w:
 *   y[2i+a][2j+b][co] = b[co] + sum_ci w[co][a][b][ci] x[i][j][ci]. */
int unet_upconv_fwd(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co,
                    const uint16_t *wgt, const float *bias, int cout,
                    uint16_t *y, int y_cs, int y_co, void *s);
/* Its data gradient dx[i][j][ci] = sum_{a,b,co} w[co][a][b][ci] dy[2i+a][2j+b][co]
 * (h, w: the input grid); wt: scratch of 4*cin*cout BF16 (rearranged weights). */
int unet_upconv_bwd_data(const uint16_t *dy, int n, int h, int w, int cout, int dy_cs, int dy_co,
                         const uint16_t *wgt, int cin, uint16_t *wt,
                         uint16_t *dx, int dx_cs, int dx_co, void *s);
/* Its weight gradient dw[co][a][b][ci] = sum_{i,j} dy[2i+a][2j+b][co] x[i][j][ci]
 * and db[co] = sum dy[.][co] (if db != NULL), both overwritten; partial:
 * unet_wgrad_scratch_floats(n, h, w, cin, cout, 4) floats. */
int unet_upconv_wgrad(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co,
                      const uint16_t *dy, int cout, int dy_cs, int dy_co,
                      float *dw, float *db, float *partial, void *s);

/* 1x1 head: z = b[0] + sum_c w[c] x[p][c], sat[p] = sigmoid(z) (FP32 out).
 * c divides 256. */
int unet_head_fwd(const uint16_t *x, int n_pix, int c, int x_cs, const float *w, const float *b,
                  float *sat, void *s);
/* Masked binary cross-entropy on the logits and its gradients:
 *   loss[0] = scale * sum_{mask[p] != 0} (softplus(z_p) - t_p z_p)
 *   g_p     = scale * (sigmoid(z_p) - t_p) on masked pixels, else 0
 *   dx[p][c] = g_p w[c] (BF16, [n_pix][c] contiguous; skipped if dx == NULL),
 *   dw[c] = sum_p g_p x[p][c], db[0] = sum_p g_p (each skipped if NULL).
 * scale is normally 1 / (number of masked pixels).  partial: FP32 scratch of
 * unet_head_scratch_floats(n_pix, c) floats. */
int64_t unet_head_scratch_floats(int n_pix, int c);
int unet_head_loss_bwd(const uint16_t *x, int n_pix, int c, int x_cs, const float *w, const float *b,
                       const float *target, const uint8_t *mask, float scale, float *loss,
                       uint16_t *dx, float *dw, float *db, float *partial, void *s);

/* Adam (Kingma & Ba 2015) on FP32 master weights p with moments m, v; step
 * counts from 1 (bias correction).  If p_bf16 != NULL it receives the
 * rounded weights for the kernels. */
int unet_adam(float *p, const float *g, float *m, float *v, uint16_t *p_bf16, int64_t count,
              float lr, float beta1, float beta2, float eps, int step, void *s);

/* float -> bf16 (round to nearest even) and bf16 -> float. */
int unet_to_bf16(const float *x, uint16_t *y, int64_t count, void *s);
int unet_to_f32(const uint16_t *x, float *y, int64_t count, void *s);

#ifdef __cplusplus
}
#endif
#endif /* UNET_H */
