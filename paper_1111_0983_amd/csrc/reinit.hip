// Level-set reinitialisation, Eq. (sdf) of Sec. 2.2: d phi / d t = sgn(phi0) (1 - |grad phi|)
// in pseudo-time from phi = phi0, so that phi becomes a signed distance function near the
// boundary (the closest points of Eq. (clpt) assume one).  Forward Euler with dt = h / 2;
// away from the boundary |grad phi| is the upwind (Godunov) value for the sign of phi0;
// nodes next to the boundary relax towards the distance D = phi0 / |grad phi0| estimated
// from phi0 alone (the subcell fix), with bounded differences where phi0 has a kink.  One
// launch per step, one thread per node; x is the fastest index, so every row of a wave reads
// contiguous memory and the axis neighbours come from the same or adjacent cache lines.
#include <hip/hip_runtime.h>

#include "../../include/ghostmg.h"

namespace {

struct ReinitGeo {
  int dim, np;
  int64_t st[3], per, total;
  double h, inv_h, dt;
};

template <int D>
__global__ void __launch_bounds__(256) k_reinit_step(ReinitGeo g, const double* __restrict__ phi0,
                                                     const double* __restrict__ phi,
                                                     double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= g.total) return;
  const int64_t loc = i % g.per;
  int j[3];
  j[0] = (int)(loc % g.np);
  j[1] = (int)((loc / g.np) % g.np);
  j[2] = D == 3 ? (int)(loc / ((int64_t)g.np * g.np)) : 0;
  const double p0 = phi0[i], p = phi[i];
  // axis neighbours (a face of the box counts as the node itself)
  double a0m[3], a0p[3], am[3], ap[3];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int64_t lo = j[a] > 0 ? i - g.st[a] : i;
    const int64_t hi = j[a] < g.np - 1 ? i + g.st[a] : i;
    a0m[a] = phi0[lo];
    a0p[a] = phi0[hi];
    am[a] = phi[lo];
    ap[a] = phi[hi];
  }
  bool near = p0 == 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) near = near || p0 * a0m[a] <= 0.0 || p0 * a0p[a] <= 0.0;
  const double sgn = p0 > 0.0 ? 1.0 : (p0 < 0.0 ? -1.0 : 0.0);
  double v;
  if (near) {
    double g2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double ga = fabs(a0p[a] - a0m[a]) / 2.0;
      ga = fmax(ga, fabs(a0p[a] - p0));
      ga = fmax(ga, fabs(p0 - a0m[a]));
      ga = fmax(ga, 1e-12 * g.h);
      const double q = ga / g.h;
      g2 += q * q;
    }
    const double dist = p0 / sqrt(g2);
    v = p - (g.dt / g.h) * (sgn * fabs(p) - dist);
  } else {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double dm = (p - am[a]) / g.h, dp = (ap[a] - p) / g.h;
      double t;
      if (p0 > 0.0) {
        const double x = fmax(dm, 0.0), y = fmin(dp, 0.0);
        t = fmax(x * x, y * y);
      } else {
        const double x = fmin(dm, 0.0), y = fmax(dp, 0.0);
        t = fmax(x * x, y * y);
      }
      s += t;
    }
    v = p - g.dt * sgn * (sqrt(s) - 1.0);
  }
  out[i] = v;
}

}  // namespace

extern "C" int mg_reinit(int dim, int n, int batch, double lo, double hi, const double* phi0,
                         int iters, double* phi, double* tmp, void* stream) {
  if ((dim != 2 && dim != 3) || n < 2 || batch < 1 || !(hi > lo) || iters < 0 || !phi0 ||
      !phi || !tmp || phi == phi0 || tmp == phi0 || tmp == phi)
    return MG_EINVAL;
  ReinitGeo g;
  g.dim = dim;
  g.np = n + 1;
  g.st[0] = 1;
  g.st[1] = g.np;
  g.st[2] = (int64_t)g.np * g.np;
  g.per = dim == 3 ? g.st[2] * g.np : g.st[2];
  g.total = g.per * batch;
  g.h = (hi - lo) / n;
  g.inv_h = 1.0 / g.h;
  g.dt = 0.5 * g.h;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(phi, phi0, g.total * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return MG_EHIP;
  const int blocks = (int)((g.total + 255) / 256);
  // steps alternate between phi and tmp; an odd count ends with a copy back into phi
  for (int k = 0; k < iters; ++k) {
    const double* src = (k & 1) ? tmp : phi;
    double* dst = (k & 1) ? phi : tmp;
    if (dim == 2)
      hipLaunchKernelGGL(k_reinit_step<2>, dim3(blocks), dim3(256), 0, s, g, phi0, src, dst);
    else
      hipLaunchKernelGGL(k_reinit_step<3>, dim3(blocks), dim3(256), 0, s, g, phi0, src, dst);
  }
  if (iters & 1)
    if (hipMemcpyAsync(phi, tmp, g.total * sizeof(double), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return MG_EHIP;
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}
