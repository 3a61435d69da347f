// Learned initial guess: BF16 MFMA convolution kernels (forward, input gradient, weight
// gradient), loss, Adam, and the glue between a solver level and the network's NHWC tensors.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (gfx950): M = pixels, N = output
// channels, K = 9 taps x input channels.  Lane l of a wave supplies A[row l%16][k 8(l/16)..+7]
// and B[k 8(l/16)..+7][col l%16] and receives D[rows 4(l/16)..+3][col l%16].
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ghostmg_cnn.h"
#include "ghostmg_impl.h"

using namespace ghostmg;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

namespace {

constexpr int kWgradPix = 1024;  // pixels reduced per workgroup in the weight gradient

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }
__device__ __forceinline__ float from_bf16(__bf16 v) { return (float)v; }

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------------------------------
// packing of the FP32 master weights into the BF16 GEMM operands
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pack(const float* __restrict__ w, int cin, int cout,
                                              int cin_pad, int kpad_f, int rows_f,
                                              __bf16* __restrict__ wf, int cout_pad, int kpad_b,
                                              int rows_b, __bf16* __restrict__ wb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int nf = rows_f * kpad_f, nb = rows_b * kpad_b;
  if (i < nf) {
    const int co = i / kpad_f, k = i % kpad_f, tap = k / cin_pad, ci = k % cin_pad;
    float v = 0.f;
    if (co < cout && tap < 9 && ci < cin) v = w[(co * 9 + tap) * cin + ci];
    wf[i] = to_bf16(v);
  } else if (i < nf + nb) {
    const int j = i - nf;
    const int ci = j / kpad_b, k = j % kpad_b, tap = k / cout_pad, co = k % cout_pad;
    float v = 0.f;
    if (ci < cin && tap < 9 && co < cout) v = w[(co * 9 + (8 - tap)) * cin + ci];
    if (wb) wb[j] = to_bf16(v);
  }
}

// ---------------------------------------------------------------------------------------
// convolution: each wave computes 16 pixels x (16 NT) output channels
// ---------------------------------------------------------------------------------------
template <int NT>
__global__ void __launch_bounds__(256) k_conv(const __bf16* __restrict__ x, int B, int H, int W,
                                              int cin_pad, int kpad, const __bf16* __restrict__ wt,
                                              const float* __restrict__ bias, int cout, int cout_pad,
                                              int dil, int act, const __bf16* __restrict__ relu_of,
                                              void* __restrict__ yv, int y_f32) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t P = (int64_t)B * H * W;
  const int64_t pix0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (pix0 >= P) return;
  const int64_t pa = pix0 + (lane & 15);
  int b = 0, yy0 = 0, xx0 = 0;
  if (pa < P) {
    b = (int)(pa / ((int64_t)H * W));
    const int r = (int)(pa - (int64_t)b * H * W);
    yy0 = r / W;
    xx0 = r - yy0 * W;
  }
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kg = 8 * (lane >> 4);
  for (int kc = 0; kc < kpad; kc += 32) {
    const int k0 = kc + kg;
    const int tap = k0 / cin_pad, ci0 = k0 - tap * cin_pad;
    bf16x8 a = {};
    if (tap < 9 && pa < P) {
      const int yy = yy0 + dil * (tap / 3 - 1), xx = xx0 + dil * (tap % 3 - 1);
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        a = *(const bf16x8*)(x + (((int64_t)b * H + yy) * W + xx) * cin_pad + ci0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf16x8 bw = *(const bf16x8*)(wt + (int64_t)(t * 16 + (lane & 15)) * kpad + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = t * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p = pix0 + 4 * (lane >> 4) + i;
      if (p >= P) continue;
      float v = acc[t][i];
      if (co < cout) {
        if (bias) v += bias[co];
        if (act) v = fmaxf(v, 0.f);
        if (relu_of && !(from_bf16(relu_of[p * cout_pad + co]) > 0.f)) v = 0.f;
      } else {
        v = 0.f;
      }
      if (y_f32) {
        if (co == 0) ((float*)yv)[p] = v;
      } else if (co < cout_pad) {
        ((__bf16*)yv)[p * cout_pad + co] = to_bf16(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum_p dy[p][co] x[p + d(tap)][ci], MFMA with
// M = output channels, N = (tap, ci), K = pixels.  Workgroup (block, group) takes the
// kWgradPix pixels of its block and the taps of its group (tpg consecutive taps; 9 / tpg
// groups), 32 pixels per step: each thread stages at most one 16-byte vector of x or dy per
// step, and loads the next step's vector into registers while the step's MFMAs run.  The
// step's tiles are staged transposed (a row per channel, its 32 pixels contiguous), so that
// a lane reads its 8 K-values of an MFMA operand in one 16-byte read.  The per-workgroup
// partials (the group's columns of its block's row) are reduced in order.
constexpr int kWgradRow = 40;  // row stride (bf16) of the transposed tiles: 80 bytes, so that
                               // the 16-byte reads of 8 consecutive rows hit distinct banks
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wgrad(const __bf16* __restrict__ x,
                                               const __bf16* __restrict__ dy, int B, int H, int W,
                                               int cin_pad, int cout, int cout_pad, int dil,
                                               int tpg, int mt_n, int nt_n,
                                               float* __restrict__ work, int64_t wstride) {
  extern __shared__ __align__(16) __bf16 lds[];
  constexpr int RS = kWgradRow;
  const int ntg = 9 / tpg;
  const int blk = blockIdx.x / ntg, grp = blockIdx.x % ntg, tap0 = grp * tpg;
  __bf16* xs = lds;                           // [tpg * cin_pad][RS]: column n, its pixels
  __bf16* ds = lds + tpg * cin_pad * RS;      // [cout_pad][RS]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t P = (int64_t)B * H * W;
  const int64_t p_begin = (int64_t)blk * kWgradPix;
  // output tile of the wave (at most 4 tiles, one per wave: the host checks it), held in
  // registers
  const bool has_tile = wave < mt_n * nt_n;
  const int mt = wave / nt_n, nt = wave % nt_n;
  const int ncg = tpg * cin_pad;  // the group's columns
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float dbacc = 0.f;
  const int chunks_x = 32 * tpg * (cin_pad / 8), chunks_d = 32 * (cout_pad / 8);
  // the thread's vector (at most one: the host checks chunks_x + chunks_d <= 256): a
  // position in xs or ds, and its source for the step at pixel offset kp
  const int c = threadIdx.x;
  const bool has = c < chunks_x + chunks_d;
  auto fetch = [&](int kp) -> bf16x8 {
    bf16x8 v = {};
    if (!has) return v;
    if (c < chunks_x) {
      const int pl = c / (tpg * (cin_pad / 8)), rem = c % (tpg * (cin_pad / 8));
      const int tap = tap0 + rem / (cin_pad / 8), cc = rem % (cin_pad / 8);
      const int64_t p = p_begin + kp + pl;
      if (p < P) {
        const int b = (int)(p / ((int64_t)H * W));
        const int r = (int)(p - (int64_t)b * H * W);
        const int yy = r / W + dil * (tap / 3 - 1), xx = r % W + dil * (tap % 3 - 1);
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
          v = *(const bf16x8*)(x + (((int64_t)b * H + yy) * W + xx) * cin_pad + 8 * cc);
      }
    } else {
      const int c2 = c - chunks_x;
      const int pl = c2 / (cout_pad / 8), cc = c2 % (cout_pad / 8);
      const int64_t p = p_begin + kp + pl;
      if (p < P) v = *(const bf16x8*)(dy + p * cout_pad + 8 * cc);
    }
    return v;
  };
  bf16x8 nxt = fetch(0);
  for (int kp = 0; kp < kWgradPix; kp += 32) {
    __syncthreads();  // the previous step's reads of xs / ds are done
    if (has) {
      // the vector holds 8 channels of one pixel: 8 rows of the transposed tile
      if (c < chunks_x) {
        const int pl = c / (tpg * (cin_pad / 8)), rem = c % (tpg * (cin_pad / 8));
        const int n0 = (rem / (cin_pad / 8)) * cin_pad + 8 * (rem % (cin_pad / 8));
#pragma unroll
        for (int j = 0; j < 8; ++j) xs[(n0 + j) * RS + pl] = nxt[j];
      } else {
        const int c2 = c - chunks_x;
        const int pl = c2 / (cout_pad / 8), ch0 = 8 * (c2 % (cout_pad / 8));
#pragma unroll
        for (int j = 0; j < 8; ++j) ds[(ch0 + j) * RS + pl] = nxt[j];
      }
    }
    __syncthreads();
    if (kp + 32 < kWgradPix) nxt = fetch(kp + 32);
    if (grp == 0 && (int)threadIdx.x < cout_pad)
      for (int pl = 0; pl < 32; ++pl) dbacc += from_bf16(ds[threadIdx.x * RS + pl]);
    if (has_tile) {
      const int co = mt * 16 + (lane & 15);
      const int n = nt * 16 + (lane & 15);  // column within the group
      const int k0 = 8 * (lane >> 4);       // the lane's 8 pixels of the step
      const bf16x8 zero = {};
      const bf16x8 a = co < cout_pad ? *(const bf16x8*)(ds + co * RS + k0) : zero;
      const bf16x8 bb = n < ncg ? *(const bf16x8*)(xs + n * RS + k0) : zero;
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
    }
  }
  float* out = work + (int64_t)blk * wstride;
  const int ncol = 9 * cin_pad;
  if (has_tile) {
    const int n = nt * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mt * 16 + 4 * (lane >> 4) + i;
      if (co < cout && n < ncg) out[(int64_t)co * ncol + tap0 * cin_pad + n] = acc[i];
    }
  }
  if (grp == 0 && (int)threadIdx.x < cout) out[(int64_t)cout * ncol + threadIdx.x] = dbacc;
}

// 64 outputs per workgroup, 4 threads per output: thread s of an output sums the partials of
// blocks s, s + 4, ... in order, then the four sums are added in order (deterministic)
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* __restrict__ work, int nblk,
                                                      int64_t wstride, int cin, int cin_pad,
                                                      int cout, float* __restrict__ dw,
                                                      float* __restrict__ db) {
  __shared__ float part[4][64];
  const int o = blockIdx.x * 64 + (threadIdx.x & 63), sl = threadIdx.x >> 6;
  const int nw = cout * 9 * cin;
  const int ncol = 9 * cin_pad;
  int64_t off = -1;
  if (o < nw) {
    const int co = o / (9 * cin), r = o % (9 * cin), tap = r / cin, ci = r % cin;
    off = (int64_t)co * ncol + tap * cin_pad + ci;
  } else if (o < nw + cout) {
    off = (int64_t)cout * ncol + (o - nw);
  }
  float s = 0.f;
  if (off >= 0) {
    const float* src = work + off;
    int b = sl;
    for (; b + 12 < nblk; b += 16) {
      const float v0 = src[(int64_t)b * wstride], v1 = src[(int64_t)(b + 4) * wstride];
      const float v2 = src[(int64_t)(b + 8) * wstride], v3 = src[(int64_t)(b + 12) * wstride];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; b < nblk; b += 4) s += src[(int64_t)b * wstride];
  }
  part[sl][threadIdx.x & 63] = s;
  __syncthreads();
  if (sl == 0 && off >= 0) {
    const int t = threadIdx.x;
    const float v = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
    if (o < nw)
      dw[o] = v;
    else
      db[o - nw] = v;
  }
}

// ---------------------------------------------------------------------------------------
// loss and optimiser
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_loss_partial(const float* __restrict__ pred,
                                                      const float* __restrict__ tgt,
                                                      const float* __restrict__ mask, int64_t n,
                                                      float* __restrict__ part) {
  __shared__ float s1[256], s2[256];
  float a = 0.f, c = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float m = mask[i], d = pred[i] - tgt[i];
    a += m * d * d;
    c += m;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ void k_loss_final(const float* __restrict__ part, int nblk, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float a = 0.f, c = 0.f;
  for (int b = 0; b < nblk; ++b) {
    a += part[2 * b];
    c += part[2 * b + 1];
  }
  loss[0] = c > 0.f ? a / c : 0.f;
  loss[1] = c;
}

__global__ void __launch_bounds__(256) k_loss_grad(const float* __restrict__ pred,
                                                   const float* __restrict__ tgt,
                                                   const float* __restrict__ mask, int64_t n,
                                                   const float* __restrict__ loss,
                                                   __bf16* __restrict__ dy) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float cnt = loss[1];
  const float g = cnt > 0.f ? 2.f * mask[i] * (pred[i] - tgt[i]) / cnt : 0.f;
  bf16x8 v = {};
  v[0] = to_bf16(g);
  *(bf16x8*)(dy + i * 8) = v;
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------------------
// glue with the solver hierarchy (2D)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void atomic_max_f(float* dst, float v) {
  atomicMax((unsigned int*)dst, __float_as_uint(v));  // v >= 0
}

// zeroes n floats (a kernel rather than a memset node, so that the call can be captured)
__global__ void __launch_bounds__(256) k_zero_f32(float* __restrict__ p, int n) {
  const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (i < n) p[i] = 0.f;
}

__global__ void __launch_bounds__(256) k_feat_scale(int64_t total, int np0, Geo g0,
                                                    const int8_t* __restrict__ cls0,
                                                    const double* __restrict__ f,
                                                    const double* __restrict__ gv,
                                                    float* __restrict__ scale) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t nn = (int64_t)np0 * np0;
  const int b = (int)(i / nn);
  const int q = (int)(i - (int64_t)b * nn);
  const int x = q % np0, y = q / np0;
  const int8_t c = cls0[(int64_t)b * g0.npp + x + g0.st[1] * y];
  double v = 0.0;
  if (c == 1) v = fabs(f[i]);
  if (c == 2) v = fabs(gv[i]);
  if (v > 0.0) atomic_max_f(&scale[b], (float)v);
}

__global__ void __launch_bounds__(256) k_feat(int64_t total, int np0, Geo gl, int ratio,
                                              const int8_t* __restrict__ clsl,
                                              const int8_t* __restrict__ cls0, Geo g0,
                                              const double* __restrict__ phil,
                                              const double* __restrict__ f,
                                              const double* __restrict__ gv,
                                              const float* __restrict__ scale,
                                              __bf16* __restrict__ xout) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t nl = (int64_t)gl.np * gl.np;
  const int b = (int)(i / nl);
  const int q = (int)(i - (int64_t)b * nl);
  const int x = q % gl.np, y = q / gl.np;
  const int64_t L = (int64_t)b * gl.npp + x + gl.st[1] * y;
  const int64_t F = (int64_t)b * np0 * np0 + (int64_t)(ratio * x) + (int64_t)np0 * (ratio * y);
  const int8_t c0 = cls0[(int64_t)b * g0.npp + ratio * x + g0.st[1] * (ratio * y)];
  const float s = scale[b] > 0.f ? scale[b] : 1.f;
  bf16x8 v = {};
  const double ph = phil[L] / gl.h;
  v[0] = to_bf16((float)fmin(4.0, fmax(-4.0, ph)));
  v[1] = to_bf16(clsl[L] == 1 ? (float)(f[F] / s) : 0.f);
  v[2] = to_bf16(c0 == 2 ? (float)(gv[F] / s) : 0.f);
  v[3] = to_bf16(0.f);
  *(bf16x8*)(xout + i * 8) = v;
}

__global__ void __launch_bounds__(256) k_feat_ghost(const GhostRec* __restrict__ gs, int ng, Geo gl,
                                                    __bf16* __restrict__ xout) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ng) return;
  const GhostRec r = gs[i];
  const int b = (int)(r.node / gl.npp);
  const int64_t loc = r.node - (int64_t)b * gl.npp;
  const int y = (int)(loc / gl.st[1]), x = (int)(loc - y * gl.st[1]);
  const int64_t p = (int64_t)b * gl.np * gl.np + x + (int64_t)gl.np * y;
  xout[p * 8 + 3] = to_bf16(r.type ? 1.f : -1.f);
}

// a node of level l carries a prediction the finest grid can use when it is an unknown of
// level l and the finest node at the same point is an unknown too (a coarse ghost may lie
// outside the finest ghost layer, where the finest solution is not defined)
__device__ __forceinline__ bool valid_coarse(const int8_t* clsl, const Geo& gl, const int8_t* cls0,
                                             const Geo& g0, int ratio, int b, int x, int y) {
  return clsl[(int64_t)b * gl.npp + x + gl.st[1] * y] != 0 &&
         cls0[(int64_t)b * g0.npp + ratio * x + g0.st[1] * (ratio * y)] != 0;
}

__global__ void __launch_bounds__(256) k_target(int64_t total, int np0, Geo gl, int ratio,
                                                const int8_t* __restrict__ clsl,
                                                const int8_t* __restrict__ cls0, Geo g0,
                                                const double* __restrict__ u,
                                                const float* __restrict__ scale,
                                                float* __restrict__ tgt, float* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t nl = (int64_t)gl.np * gl.np;
  const int b = (int)(i / nl);
  const int q = (int)(i - (int64_t)b * nl);
  const int x = q % gl.np, y = q / gl.np;
  const bool ok = valid_coarse(clsl, gl, cls0, g0, ratio, b, x, y);
  const float s = scale[b] > 0.f ? scale[b] : 1.f;
  const int64_t F = (int64_t)b * np0 * np0 + (int64_t)(ratio * x) + (int64_t)np0 * (ratio * y);
  tgt[i] = ok ? (float)(u[F] / s) : 0.f;
  mask[i] = ok ? 1.f : 0.f;
}

__global__ void __launch_bounds__(256) k_apply(int64_t total, int np0, Geo g0, Geo gl, int ratio,
                                               const int8_t* __restrict__ cls0,
                                               const int8_t* __restrict__ clsl,
                                               const float* __restrict__ pred,
                                               const float* __restrict__ scale,
                                               double* __restrict__ u0) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t nn = (int64_t)np0 * np0;
  const int b = (int)(i / nn);
  const int q = (int)(i - (int64_t)b * nn);
  const int x = q % np0, y = q / np0;
  if (!cls0[(int64_t)b * g0.npp + x + g0.st[1] * y]) {
    u0[i] = 0.0;
    return;
  }
  const int X0 = x / ratio, Y0 = y / ratio;
  const float fx = (float)(x - X0 * ratio) / ratio, fy = (float)(y - Y0 * ratio) / ratio;
  float num = 0.f, den = 0.f;
  for (int cy = 0; cy < 2; ++cy)
    for (int cx = 0; cx < 2; ++cx) {
      const int X = X0 + cx, Y = Y0 + cy;
      const float w = (cx ? fx : 1.f - fx) * (cy ? fy : 1.f - fy);
      if (w == 0.f || X >= gl.np || Y >= gl.np) continue;
      if (!valid_coarse(clsl, gl, cls0, g0, ratio, b, X, Y)) continue;
      num += w * pred[(int64_t)b * gl.np * gl.np + X + (int64_t)gl.np * Y];
      den += w;
    }
  u0[i] = den > 0.f ? (double)scale[b] * (double)(num / den) : 0.0;
}

inline int lin(int64_t n) { return (int)((n + 255) / 256); }

// Per-block partial sums of cnn_wgrad_noalloc: a file-scope device array (every GPU the
// library runs on holds its own copy until the process ends).  Host code never passes the
// array's name to a kernel or a copy: it takes the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr int64_t kWgradScratchFloats = (int64_t)4 << 20;  // 16 MiB
__device__ __align__(256) float scratch[kWgradScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

int wgrad_scratch(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MG_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return MG_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MG_EHIP;
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return MG_OK;
}

}  // namespace

extern "C" {

int cnn_cpad(int c) { return c <= 8 ? 8 : round_up(c, 16); }
int cnn_kpad(int cin_pad) { return round_up(9 * cin_pad, 32); }

int cnn_pack(const float* w, int cin, int cout, void* wt_fwd, void* wt_bwd, void* stream) {
  if (!w || !wt_fwd || cin < 1 || cout < 1) return MG_EINVAL;
  const int cin_pad = cnn_cpad(cin), cout_pad = cnn_cpad(cout);
  const int kf = cnn_kpad(cin_pad), rf = round_up(cout < 16 ? 16 : cout, 16);
  const int kb = cnn_kpad(cout_pad), rb = round_up(cin < 16 ? 16 : cin, 16);
  const int64_t n = (int64_t)rf * kf + (wt_bwd ? (int64_t)rb * kb : 0);
  hipLaunchKernelGGL(k_pack, dim3(lin(n)), dim3(256), 0, (hipStream_t)stream, w, cin, cout, cin_pad,
                     kf, rf, (__bf16*)wt_fwd, cout_pad, kb, rb, (__bf16*)wt_bwd);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int cnn_conv(const void* x, int B, int H, int W, int cin_pad, const void* wt, const float* bias,
             int cout, int cout_pad, int dil, int act, const void* relu_of, void* y, int y_f32,
             void* stream) {
  if (!x || !wt || !y || B < 1 || H < 1 || W < 1 || cout < 1 || dil < 1) return MG_EINVAL;
  if (cin_pad % 8 || (cout_pad % 8 && !y_f32)) return MG_EINVAL;
  const int rows = round_up(cout < 16 ? 16 : cout, 16);
  const int nt = rows / 16;
  const int64_t P = (int64_t)B * H * W;
  const int blocks = (int)((P + 63) / 64);
  const int kpad = cnn_kpad(cin_pad);
  hipStream_t s = (hipStream_t)stream;
  if (nt == 1)
    hipLaunchKernelGGL(k_conv<1>, dim3(blocks), dim3(256), 0, s, (const __bf16*)x, B, H, W, cin_pad,
                       kpad, (const __bf16*)wt, bias, cout, cout_pad, dil, act,
                       (const __bf16*)relu_of, y, y_f32);
  else if (nt == 2)
    hipLaunchKernelGGL(k_conv<2>, dim3(blocks), dim3(256), 0, s, (const __bf16*)x, B, H, W, cin_pad,
                       kpad, (const __bf16*)wt, bias, cout, cout_pad, dil, act,
                       (const __bf16*)relu_of, y, y_f32);
  else
    return MG_EINVAL;
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int64_t cnn_wgrad_work(int B, int H, int W, int cin, int cout) {
  const int64_t P = (int64_t)B * H * W;
  const int64_t nblk = (P + kWgradPix - 1) / kWgradPix;
  return nblk * ((int64_t)cout * 9 * cnn_cpad(cin) + cout);
}

int cnn_wgrad(const void* x, const void* dy, int B, int H, int W, int cin, int cin_pad, int cout,
              int cout_pad, int dil, float* work, float* dw, float* db, void* stream) {
  if (!x || !dy || !work || !dw || !db || cin_pad != cnn_cpad(cin) || cout_pad != cnn_cpad(cout) ||
      cout > 32)
    return MG_EINVAL;
  const int64_t P = (int64_t)B * H * W;
  const int nblk = (int)((P + kWgradPix - 1) / kWgradPix);
  // taps per workgroup: one where a tap's columns fill MFMA tiles, a stencil row otherwise
  const int tpg = cin_pad >= 16 ? 1 : 3;
  const int mt = (cout + 15) / 16, ntn = (tpg * cin_pad + 15) / 16;
  // one output tile per wave, and one staged vector per thread and step
  if (mt * ntn > 4 || 32 * tpg * (cin_pad / 8) + 32 * (cout_pad / 8) > 256) return MG_EINVAL;
  const int64_t wstride = (int64_t)cout * 9 * cin_pad + cout;
  const size_t lds = (size_t)(tpg * cin_pad + cout_pad) * kWgradRow * sizeof(__bf16);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_wgrad, dim3(nblk * (9 / tpg)), dim3(256), lds, s, (const __bf16*)x,
                     (const __bf16*)dy, B, H, W, cin_pad, cout, cout_pad, dil, tpg, mt, ntn, work,
                     wstride);
  const int nout = cout * 9 * cin + cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 63) / 64), dim3(256), 0, s, (const float*)work,
                     nblk, wstride, cin, cin_pad, cout, dw, db);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int cnn_wgrad_noalloc(const void* x, const void* dy, int B, int H, int W, int cin, int cin_pad,
                      int cout, int cout_pad, int dil, float* dw, float* db, void* stream) {
  if (cin_pad != cnn_cpad(cin) || cout_pad != cnn_cpad(cout) || B < 1 || H < 1 || W < 1)
    return MG_EINVAL;
  if (cnn_wgrad_work(B, H, W, cin, cout) > kWgradScratchFloats) return MG_EINVAL;
  float* work = nullptr;
  const int rc = wgrad_scratch(&work);
  if (rc != MG_OK) return rc;
  return cnn_wgrad(x, dy, B, H, W, cin, cin_pad, cout, cout_pad, dil, work, dw, db, stream);
}

int cnn_loss(const float* pred, const float* target, const float* mask, int64_t n, float* loss,
             void* dy, void* stream) {
  if (!pred || !target || !mask || !loss || n < 1) return MG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nblk = 128;
  // loss[2 .. 2 + 2 nblk) hold the partial sums (the caller provides 2 + 2*128 floats)
  hipLaunchKernelGGL(k_loss_partial, dim3(nblk), dim3(256), 0, s, pred, target, mask, n, loss + 2);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, (const float*)(loss + 2), nblk, loss);
  if (dy)
    hipLaunchKernelGGL(k_loss_grad, dim3(lin(n)), dim3(256), 0, s, pred, target, mask, n,
                       (const float*)loss, (__bf16*)dy);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int cnn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
             float beta2, float eps, int t, void* stream) {
  if (!w || !g || !m || !v || n < 1 || t < 1) return MG_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(lin(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, n, lr,
                     beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_cnn_features(mg_handle_t h, int level, const double* f, const double* g, void* x,
                    float* scale) {
  if (!h || !f || !g || !x || !scale || h->dim != 2 || level < 0 || level > h->L) return MG_EINVAL;
  const DevLevel& L0 = h->dev[0];
  const DevLevel& Ll = h->dev[level];
  const double* phil = level == 0 ? nullptr : Ll.phi;
  if (!phil) return MG_EINVAL;
  hipStream_t s = h->stream;
  const int np0 = L0.g.np;
  const int64_t tot0 = (int64_t)h->batch * np0 * np0;
  const int64_t totl = (int64_t)h->batch * Ll.g.np * Ll.g.np;
  hipLaunchKernelGGL(k_zero_f32, dim3(lin(h->batch)), dim3(256), 0, s, scale, h->batch);
  hipLaunchKernelGGL(k_feat_scale, dim3(lin(tot0)), dim3(256), 0, s, tot0, np0, L0.g, L0.cls, f, g,
                     scale);
  hipLaunchKernelGGL(k_feat, dim3(lin(totl)), dim3(256), 0, s, totl, np0, Ll.g, 1 << level, Ll.cls,
                     L0.cls, L0.g, phil, f, g, (const float*)scale, (__bf16*)x);
  if (Ll.nghost)
    hipLaunchKernelGGL(k_feat_ghost, dim3(lin(Ll.nghost)), dim3(256), 0, s, Ll.ghosts, Ll.nghost,
                       Ll.g, (__bf16*)x);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_cnn_target(mg_handle_t h, int level, const double* u, const float* scale, float* target,
                  float* mask) {
  if (!h || !u || !scale || !target || !mask || h->dim != 2 || level < 0 || level > h->L)
    return MG_EINVAL;
  const DevLevel& Ll = h->dev[level];
  const int np0 = h->dev[0].g.np;
  const int64_t totl = (int64_t)h->batch * Ll.g.np * Ll.g.np;
  hipLaunchKernelGGL(k_target, dim3(lin(totl)), dim3(256), 0, h->stream, totl, np0, Ll.g,
                     1 << level, Ll.cls, h->dev[0].cls, h->dev[0].g, u, scale, target, mask);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_cnn_apply(mg_handle_t h, int level, const float* pred, const float* scale, double* u0) {
  if (!h || !pred || !scale || !u0 || h->dim != 2 || level < 0 || level > h->L) return MG_EINVAL;
  const DevLevel& L0 = h->dev[0];
  const DevLevel& Ll = h->dev[level];
  const int np0 = L0.g.np;
  const int64_t tot0 = (int64_t)h->batch * np0 * np0;
  hipLaunchKernelGGL(k_apply, dim3(lin(tot0)), dim3(256), 0, h->stream, tot0, np0, L0.g, Ll.g,
                     1 << level, L0.cls, Ll.cls, pred, scale, u0);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

}  // extern "C"
