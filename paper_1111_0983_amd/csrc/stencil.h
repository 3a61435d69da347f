// Boundary-operator weights of the ghost-cell discretisation, shared by the host setup
// (coarsest-grid matrix assembly) and the device relaxation / defect kernels.
//
// A ghost G with closest boundary point B (Sec. 2.3, Eq. (clpt)) owns an upwind stencil
// of nodes G + sum_a s_a k_a h e_a, k in {0,1,2}^D (Eq. (St_G)).  Its row of the discrete
// boundary operator L_h (Eq. (discrBC)) is the value (Dirichlet) or the normal derivative
// along n_B (Neumann) of an interpolant on that stencil, evaluated at B:
//   rung 1  tensor-quadratic on the 3^D stencil
//   rung 2  tensor-linear on the 2^D corner (the 2x2 reduced stencil of Remark 3)
//   rung 3  linear through G and G + s_a e_a, a = 0..D-1
//   rung 4  linear through G and G + s_ax e_ax (two points along one axis)
// xi_a = s_a (B_a - G_a) / h are the local coordinates of B.  Template position t encodes
// k with k_x the slowest base-3 digit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ghostmg {

struct GhostRec {     // 64 bytes, one per ghost point
  int32_t node;       // node index (problem offset included)
  int8_t type;        // 1 Dirichlet, 0 Neumann
  int8_t rung;        // 1..4
  int8_t axis;        // axis of rung 4
  int8_t pad0;
  int8_t s[3];        // upwind signs
  int8_t pad1;
  int32_t pad2;
  double xi[3];       // local coordinates of B
  double nb[3];       // unit normal at B from the interpolant of phi (Neumann rows)
};
static_assert(sizeof(GhostRec) == 64, "GhostRec layout");

template <int D>
struct Pow3 {
  static constexpr int value = 3 * Pow3<D - 1>::value;
};
template <>
struct Pow3<0> {
  static constexpr int value = 1;
};

// One-dimensional Lagrange bases on the stencil nodes 0, 1, 2 at local coordinate x:
// quadratic for rung 1, linear (nodes 0, 1) for rung 2.
__host__ __device__ inline void basis_1d(int rung, double x, double* b, double* db) {
  if (rung == 1) {
    b[0] = 0.5 * (x - 1.0) * (x - 2.0);
    b[1] = x * (2.0 - x);
    b[2] = 0.5 * x * (x - 1.0);
    db[0] = x - 1.5;
    db[1] = 2.0 - 2.0 * x;
    db[2] = x - 0.5;
  } else {
    b[0] = 1.0 - x;
    b[1] = x;
    b[2] = 0.0;
    db[0] = -1.0;
    db[1] = 1.0;
    db[2] = 0.0;
  }
}

// Weights of the interpolant of a row: for dir != 0 the value at B, otherwise the
// derivative along dvec (e.g. n_B) at B.  w[t] is zero where unused; returns the used mask.
template <int D>
__host__ __device__ inline uint32_t stencil_weights(int rung, int axis, const int8_t* s,
                                                    const double* xi, double inv_h, int dir,
                                                    const double* dvec, double* w) {
  constexpr int K = Pow3<D>::value;
  uint32_t used = 0;
  for (int t = 0; t < K; ++t) w[t] = 0.0;
  if (rung <= 2) {
    double b[D][3], db[D][3];
    for (int a = 0; a < D; ++a) basis_1d(rung, xi[a], b[a], db[a]);
    for (int t = 0; t < K; ++t) {
      int k[D];
      int tt = t;
      bool ok = true;
      for (int a = D - 1; a >= 0; --a) {
        k[a] = tt % 3;
        tt /= 3;
        if (rung == 2 && k[a] == 2) ok = false;
      }
      if (!ok) continue;
      used |= 1u << t;
      if (dir) {
        double v = 1.0;
        for (int a = 0; a < D; ++a) v *= b[a][k[a]];
        w[t] = v;
      } else {
        double acc = 0.0;
        for (int a = 0; a < D; ++a) {
          double g = dvec[a] * (double)s[a] * inv_h * db[a][k[a]];
          for (int c = 0; c < D; ++c)
            if (c != a) g *= b[c][k[c]];
          acc += g;
        }
        w[t] = acc;
      }
    }
  } else {
    // linear interpolant through G (t = 0) and G + s_a e_a (t = 3^(D-1-a))
    double sx = 0.0, g0 = 0.0;
    used |= 1u;
    for (int a = 0; a < D; ++a) {
      if (rung == 4 && a != axis) continue;
      int ta = 1;
      for (int c = D - 1; c > a; --c) ta *= 3;
      used |= 1u << ta;
      if (dir) {
        w[ta] = xi[a];
        sx += xi[a];
      } else {
        double g = dvec[a] * (double)s[a] * inv_h;
        w[ta] = g;
        g0 -= g;
      }
    }
    w[0] = dir ? 1.0 - sx : g0;
  }
  return used;
}

// Row of L_h of one ghost (Eq. (discrBC)): value weights (Dirichlet) or weights of the
// derivative along n_B (Neumann).
template <int D>
__host__ __device__ inline uint32_t ghost_row(const GhostRec& g, double inv_h, double* w) {
  return stencil_weights<D>(g.rung, g.axis, g.s, g.xi, inv_h, g.type, g.nb, w);
}

// node offset of template position t for signs s and strides st
template <int D>
__host__ __device__ inline int64_t template_offset(int t, const int8_t* s, const int64_t* st) {
  int64_t off = 0;
  for (int a = D - 1; a >= 0; --a) {
    off += (int64_t)s[a] * (t % 3) * st[a];
    t /= 3;
  }
  return off;
}

// Restriction code of a coarse node: bits 2a (box starts at -1 on axis a) and 2a+1 (box ends
// at +1 on axis a); kNoUnknown marks coarse nodes that carry no unknown.
constexpr uint8_t kNoUnknown = 0xFF;

// 1D factors of the partial full-weighting transfer (Sec. 1.3.1 and Sec. 2.5): the full
// box [-1,1] weighs (1,2,1)/4, a one-sided box (2,2)/4, a single node 1.
__host__ __device__ inline double restrict_w1d(int lo_m1, int hi_p1, int k) {
  if (lo_m1 && hi_p1) return k == 0 ? 0.5 : 0.25;
  if (!lo_m1 && !hi_p1) return 1.0;
  return 0.5;
}

}  // namespace ghostmg
