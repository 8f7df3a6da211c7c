/*
 * psl_nn.h -- kernels of the start-vector network (libpsl, gfx950).
 *
 * A small 3D encoder/decoder network maps the permeability field and the right-hand side
 * of the pressure equation to a start vector for psl_solve (use_x0 = 1). The network is
 * a project addition: the paper has no learned component. Its start vector matters only
 * through P2 x0 (x = Z E^-1 Z^T b + P2 xhat does not depend on the deflated part of the
 * start, Section 3.1), which is what its training loss measures.
 *
 * Conventions shared by every entry point:
 *  - Activations are channels-last on the cell grid: element (c, ch) at c * C + ch with
 *    c = ix + nx (iy + ny iz). Stored as bfloat16 (uint16 bit patterns) when they are
 *    operands of a matrix product, as float32 otherwise (gradients between layers).
 *  - 3x3x3 weights are bfloat16 rows of kp = round_up(27 * Cin, 32) entries: entry
 *    k = t * Cin + ci of row co, tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), zero padded.
 *    Products run on the bf16 matrix cores with float32 accumulation.
 *  - All pointers are device pointers owned by the caller; `stream` is a hipStream_t.
 *  - Every call returns PSL_OK or PSL_EINVAL (sizes or alignment outside what the kernel
 *    supports: Cin multiple of 8, Cout multiple of 16, buffers 16-byte aligned, nx a
 *    multiple of 8 for the weight gradient, even extents for pooling) and enqueues work
 *    only when the arguments are valid.
 */
#ifndef PSL_NN_H
#define PSL_NN_H

#include <stdint.h>

#include "psl.h"

#ifdef __cplusplus
extern "C" {
#endif

/* kp for a given Cin (row length of a packed 3x3x3 weight matrix). */
int32_t psl_nn_kp(int32_t cin);

/*
 * y = act(conv3x3x3(x, w) + bias): out(c, co) = bias[co] + sum_t sum_ci
 * w[co][t*cin+ci] x(c + tap_t, ci), zero outside the grid; act = ReLU if relu != 0.
 *   x     bf16 [n][cin] (cin multiple of 8),  w bf16 [cout][kp] (cout multiple of 16, <= 128)
 *   bias  float [cout] or NULL (zero)
 *   y     bf16 [n][cout] or NULL;  yf float [n][cout] or NULL (at least one given)
 * The gradient with respect to x is this same product applied to the output gradient
 * with the weights from psl_nn_adam_conv's flipped copy (and no bias or ReLU).
 */
int psl_nn_conv3(const psl_grid* g, const uint16_t* x, int32_t cin, const uint16_t* w,
                 int32_t cout, const float* bias, int32_t relu, uint16_t* y, float* yf,
                 void* stream);

/* Floats of workspace psl_nn_conv3_wgrad needs for this grid and layer. */
int64_t psl_nn_wgrad_work(const psl_grid* g, int32_t cin, int32_t cout);

/*
 * dw[co][k] = sum_c gy(c, co) x(c + tap_t, ci) for k = t*cin + ci < 27 cin, and
 * dw[co][kp] = sum_c gy(c, co) (the bias gradient); other columns 0.
 *   gy    bf16 [n][cout] (the output gradient after the ReLU mask),  x bf16 [n][cin]
 *   dw    float [cout][kp + 16] (out),  work float[psl_nn_wgrad_work(...)]
 * Sums run over fixed voxel chunks and are added in chunk order (deterministic).
 */
int psl_nn_conv3_wgrad(const psl_grid* g, const uint16_t* gy, int32_t cout, const uint16_t* x,
                       int32_t cin, float* dw, float* work, void* stream);

/* gq(c, ch) = bf16(gy(c, ch) if y(c, ch) > 0 else 0); relu = 0 skips the mask.
 * gy float [n*C], y bf16 [n*C], gq bf16 [n*C]. */
int psl_nn_relu_grad(int64_t count, const float* gy, const uint16_t* y, int32_t relu,
                     uint16_t* gq, void* stream);

/* y(coarse cell, ch) = bf16(mean of the 8 children x(child, ch)); grid g is the fine one
 * (even extents). x bf16 [n][C], y bf16 [n/8][C]. */
int psl_nn_pool2(const psl_grid* g, const uint16_t* x, int32_t c, uint16_t* y, void* stream);

/* gx(fine cell, ch) += gy(parent, ch) / 8 (adjoint of psl_nn_pool2); g is the fine grid.
 * gy float [n/8][C], gx float [n][C]. */
int psl_nn_pool2_grad_add(const psl_grid* g, const float* gy, int32_t c, float* gx,
                          void* stream);

/* Decoder input: y(c, 0:ca) = h(parent(c), :), y(c, ca:ca+cb) = s(c, :) on the fine grid
 * g (even extents). h bf16 [n/8][ca], s bf16 [n][cb], y bf16 [n][ca+cb]. */
int psl_nn_upcat(const psl_grid* g, const uint16_t* h, int32_t ca, const uint16_t* s,
                 int32_t cb, uint16_t* y, void* stream);

/* Adjoint of psl_nn_upcat: gh(p, ch) = sum over the 8 children of gy(child, ch) for
 * ch < ca; gs(c, ch) = gy(c, ca + ch). gy float [n][ca+cb], gh float [n/8][ca],
 * gs float [n][cb]. */
int psl_nn_upcat_grad(const psl_grid* g, const float* gy, int32_t ca, int32_t cb, float* gh,
                      float* gs, void* stream);

/*
 * 1x1x1 output layer, cin -> 1: y(c) = bias[0] + sum_ci w[ci] h(c, ci) (float32 sums of
 * bf16 operands). h bf16 [n][cin], w bf16 [cin], bias float [1] (device), y float [n].
 */
int psl_nn_conv1(int64_t n, const uint16_t* h, int32_t cin, const uint16_t* w,
                 const float* bias, float* y, void* stream);

/* Floats of workspace psl_nn_conv1_grad needs. */
int64_t psl_nn_conv1_work(int64_t n, int32_t cin);

/*
 * Its gradients for the output gradient gy (rounded to bf16 first, like every product
 * operand): gh(c, ci) = gq(c) w[ci] (float), dw[ci] = sum_c gq(c) h(c, ci), dw[cin] =
 * sum_c gq(c). gy float [n], gh float [n][cin], dw float [cin + 1], work as sized above.
 */
int psl_nn_conv1_grad(int64_t n, const float* gy, const uint16_t* h, int32_t cin,
                      const uint16_t* w, float* gh, float* dw, float* work, void* stream);

/* Floats of workspace psl_nn_make_input needs. */
int64_t psl_nn_input_work(int64_t n);

/*
 * Network input, 8 channels (2 used): x(c, 0) = bf16((log10 K(c) - mean) / std) over the
 * grid (population std), x(c, 1) = bf16(b(c) / max |b|) (0 if b = 0), x(c, 2..7) = 0.
 * K, b float64 [n] (K > 0), x bf16 [n][8].
 */
int psl_nn_make_input(int64_t n, const double* K, const double* b, uint16_t* x, double* work,
                      void* stream);

/* Doubles of workspace psl_nn_energy needs. */
int64_t psl_nn_energy_work(int64_t n);

/*
 * Energy-norm loss of the network output y, relative to ||P2 x*||_A^2 = c = (x*, P1 b)
 * (||P2 e||_A^2 = (e, P1 A e); A x* = b gives P1 A x* = P1 b). With u = (y, P1 b) and
 * v = (y, P1 A y):
 *   sigma > 0 (training): regression on t = x* / sigma,
 *     L = (sigma^2 v - 2 sigma u + c) / c,  gy = 2 (sigma^2 P1 A y - sigma P1 b) / c;
 *   sigma = 0: the error of the best multiple alpha y,
 *     L = 1 - u^2 / (v c),  gy = (2u / (v c)) ((u / v) P1 A y - P1 b);
 *   x0 = alpha y with alpha = u / v (0 when v <= 0: the zero start), never worse than
 *   x0 = 0 in this norm (float64, written when x0 != NULL).
 * y float [n], P1b and P1Ay float64 [n] (from psl_deflate / psl_apply_A), out double[4]
 * = {L, alpha, u, v} on the device, gy float [n] or NULL. c = 0 (unknown) skips L and gy.
 */
int psl_nn_energy(int64_t n, const float* y, const double* P1b, const double* P1Ay, double c,
                  double sigma, double* out, float* gy, double* x0, double* work,
                  void* stream);

/* Doubles of workspace psl_nn_wl2 needs. */
int64_t psl_nn_wl2_work(int64_t n);

/*
 * Training regression of the output y on a target t with cell weights d > 0:
 * L = sum d (y - t)^2 / sum d t^2 -> out[0] (device), gy = 2 d (y - t) / sum d t^2.
 * y, t, d float [n]; gy float [n] or NULL.
 */
int psl_nn_wl2(int64_t n, const float* y, const float* t, const float* d, double* out,
               float* gy, double* work, void* stream);

/* d(c) = sum of the six face transmissibilities of cell c (= diag(A)), float32, from the
 * float64 face arrays of psl_assemble_tpfa. */
int psl_nn_cell_diag(const psl_grid* g, const double* Tx, const double* Ty, const double* Tz,
                     float* d, void* stream);

/* y64 = (double) y32 (n entries). */
int psl_nn_widen(int64_t n, const float* y, double* y64, void* stream);

/*
 * Adam step t (Kingma and Ba, bias-corrected) on a 3x3x3 layer's float32 master
 * weights p[cout][27 cin] and bias pb[cout] with moments m, v (same shapes; mb, vb for
 * the bias), from dw [cout][kp + 16] of psl_nn_conv3_wgrad (column kp is the bias
 * gradient); then repacks the bf16 operands: w[cout][kp] for the forward product and
 * wt[cin][kpt] (kpt = kp of cout) with wt[ci][(26 - t) cout + co] = w[co][t cin + ci]
 * for the input gradient (wt may be NULL). t = 0 only repacks (initialisation).
 */
int psl_nn_adam_conv(int32_t cout, int32_t cin, float* p, float* m, float* v, float* pb,
                     float* mb, float* vb, const float* dw, int32_t t, float lr, float b1,
                     float b2, float eps, uint16_t* w, uint16_t* wt, void* stream);

/* The same for the 1x1x1 layer: p, m, v [cin + 1] (bias last), dw [cin + 1]; w bf16
 * [cin] is repacked. */
int psl_nn_adam_vec(int32_t count, float* p, float* m, float* v, const float* dw, int32_t t,
                    float lr, float b1, float b2, float eps, uint16_t* w, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PSL_NN_H */
