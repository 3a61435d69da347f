/*
 * ghostmg_cnn.h -- C ABI of the learned initial guess for the ghost-cell multigrid solver.
 *
 * A small convolutional network maps (phi, f, g, boundary-condition mask), sampled on one
 * coarse level of a solver hierarchy, to a prediction of the solution there; the
 * prediction, scaled back and interpolated to the finest grid, is the initial iterate of
 * mg_solve, which still iterates to its tolerance (the zero guess remains the fallback).
 * The network and its use as an initial guess are not part of the paper; they follow the
 * solver's own definition of the discrete problem (Eq. (discr)).
 *
 * Tensors are NHWC: [batch][height][width][channels], BF16 activations (channel counts
 * padded to 8 or a multiple of 16), FP32 accumulation in the matrix cores (gfx950
 * v_mfma_f32_16x16x32_bf16), FP32 master weights, losses and optimiser state.  Weight
 * layout of a layer: FP32 [cout][3][3][cin] (tap-major within an output channel).  All
 * pointers are device memory unless stated; work is ordered on `stream` (hipStream_t, NULL
 * = null stream).  Calls return MG_OK or a negative mg_status from ghostmg.h.
 */
#ifndef GHOSTMG_CNN_H
#define GHOSTMG_CNN_H

#include <stdint.h>

#include "ghostmg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Padded channel count used for activations of c channels (8 for c <= 8, else a multiple
 * of 16), and the padded reduction length 9 * cin_pad rounded up to 32. */
int cnn_cpad(int c);
int cnn_kpad(int cin_pad);

/* Pack FP32 master weights [cout][3][3][cin] into BF16 operands: wt_fwd [cout_pad16][kpad(cin_pad)]
 * for the forward convolution and wt_bwd [cin_pad16][kpad(cout_pad)] (taps flipped, channels
 * transposed) for the input gradient.  cout_pad16 = max(16, round up cout to 16). */
int cnn_pack(const float* w, int cin, int cout, void* wt_fwd, void* wt_bwd, void* stream);

/* y = act(conv3x3_dil(x) + bias) with zero padding; x: BF16 [B][H][W][cin_pad];
 * wt: packed BF16 operand; bias: FP32 [cout] or NULL; act 1 = ReLU, 0 = none;
 * relu_of: if not NULL (BF16, same shape as y, channel pad cout_pad) the output is multiplied
 * by (relu_of > 0) (the ReLU derivative in the backward pass).  y: BF16 [B][H][W][cout_pad],
 * or FP32 [B][H][W] of channel 0 when y_f32 != 0. */
int cnn_conv(const void* x, int B, int H, int W, int cin_pad, const void* wt, const float* bias,
             int cout, int cout_pad, int dil, int act, const void* relu_of, void* y, int y_f32,
             void* stream);

/* Weight and bias gradients of y = conv3x3_dil(x): dw FP32 [cout][3][3][cin],
 * db FP32 [cout] (both overwritten).  x: BF16 [B][H][W][cin_pad]; dy: BF16
 * [B][H][W][cout_pad].  work: FP32 scratch of cnn_wgrad_work(...) floats.  Shapes: cout <= 32
 * and cin <= 48 (cin <= 32 when cout > 16), else MG_EINVAL.  The sums are taken in a fixed
 * order: repeated calls give identical results. */
int64_t cnn_wgrad_work(int B, int H, int W, int cin, int cout);
int cnn_wgrad(const void* x, const void* dy, int B, int H, int W, int cin, int cin_pad,
              int cout, int cout_pad, int dil, float* work, float* dw, float* db, void* stream);

/* cnn_wgrad without a workspace argument and without any device allocation, for callers that
 * cannot allocate (code under stream capture, tight loops, harnesses that forbid hipMalloc).
 * The per-block partial sums live in a 16 MiB array of device memory that the library holds
 * for the life of the process on every GPU it runs on: cnn_wgrad_work(B, H, W, cin, cout) must
 * not exceed 4,194,304 floats (for cin = cout = 32: B*H*W <= 464,896 pixels), else MG_EINVAL.
 * Every call on one GPU shares that array, so calls that overlap on one GPU (two streams, two
 * threads) race; calls ordered on one stream do not.  Same results as cnn_wgrad. */
int cnn_wgrad_noalloc(const void* x, const void* dy, int B, int H, int W, int cin, int cin_pad,
                      int cout, int cout_pad, int dil, float* dw, float* db, void* stream);

/* Masked mean squared error of pred against target over mask != 0 (FP32 [n] each):
 * *loss (device FP32) and dy = d loss / d pred as BF16 [n][8] (channel 0, others zero). */
int cnn_loss(const float* pred, const float* target, const float* mask, int64_t n, float* loss,
             void* dy, void* stream);

/* One Adam step on n FP32 parameters (bias-corrected, step t >= 1). */
int cnn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
             float beta2, float eps, int t, void* stream);

/* Network inputs on level `level` of the handle's hierarchy for every problem:
 * x BF16 [batch][n_l+1][n_l+1][8] with channels (clip(phi / h_l, -4, 4), f / s, g / s,
 * +1 at Dirichlet ghosts and -1 at Neumann ghosts, 0...); s = max(|f|, |g|) per problem over the
 * finest unknowns (FP32 scale[batch], device).  f, g: the finest-grid arrays of mg_solve.
 * 2D hierarchies only. */
int mg_cnn_features(mg_handle_t h, int level, const double* f, const double* g, void* x,
                    float* scale);

/* Training target on level `level`: target[b][i] = u_finest(node i) / scale[b] and
 * mask = 1 at the level's unknowns whose finest node is an unknown too, else 0 (FP32
 * [batch][(n_l+1)^2] each). */
int mg_cnn_target(mg_handle_t h, int level, const double* u, const float* scale, float* target,
                  float* mask);

/* Initial guess: u0 on the finest grid = scale * multilinear interpolation of pred (FP32
 * [batch][(n_l+1)^2]) over the level's unknowns whose finest node is an unknown (weights
 * renormalised), at the finest unknowns; 0 elsewhere and where no such node is near. */
int mg_cnn_apply(mg_handle_t h, int level, const float* pred, const float* scale, double* u0);

#ifdef __cplusplus
}
#endif

#endif /* GHOSTMG_CNN_H */
