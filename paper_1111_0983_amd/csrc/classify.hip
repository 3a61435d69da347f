// Classification of one level of one problem on the GPU (Sec. 2.2-2.3): interior nodes
// (phi < 0), ghost nodes (outside nodes with an interior axis neighbour), and every ghost's
// record: its closest boundary point B (Eq. (clpt), from the central-difference gradient of
// phi), its boundary-condition type, the upwind signs of its stencil (Eq. (St_G)), the rung of
// the reduced-stencil ladder (Remark 3 of Sec. 2.3), the local coordinates of B and, for
// Neumann ghosts, the unit normal at B from the same interpolant of phi (Eq. (neu2d)).
//
// Node pass: one thread per node of the level (read from the level-0 phi at stride 2^l).
// Ghost list: per-block counts, one scan, then every block writes its ghosts in node order,
// so the list is ordered as a sequential scan would order it.  Ghost pass: one thread per
// ghost.  This file is compiled without floating-point contraction, so every geometric
// decision (tie tests, rule sides) and every stored value is the exact result of the
// expression as written, independent of the device.
#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.h"

namespace ghostmg {
namespace {

enum { kOut = 0, kIn = 1, kGhost = 2 };
constexpr int kFlagNonFinite = 1, kFlagGeom = 2;
constexpr int kScanThreads = 1024;

struct LevelGeo {
  int D, n, np;
  int64_t nn;         // nodes of the level (np^D)
  int64_t st[3];      // unpadded strides of the level
  int64_t st0[3];     // level-0 strides times 2^l
  int64_t base0;      // the problem's first level-0 node
  double lo, h, inv_h;
};

__device__ __forceinline__ void node_coords(const LevelGeo& g, int64_t i, int j[3]) {
  j[0] = j[1] = j[2] = 0;
  for (int a = 0; a < g.D; ++a) {
    j[a] = (int)(i % g.np);
    i /= g.np;
  }
}

__device__ __forceinline__ bool inside_box(const LevelGeo& g, const int j[3]) {
  for (int a = 0; a < g.D; ++a)
    if (j[a] < 0 || j[a] > g.n) return false;
  return true;
}

__device__ __forceinline__ int64_t level0_index(const LevelGeo& g, const int j[3]) {
  int64_t q = g.base0;
  for (int a = 0; a < g.D; ++a) q += (int64_t)j[a] * g.st0[a];
  return q;
}

// classes and the level's phi; per block the number of ghosts
__global__ void __launch_bounds__(256) k_classify_nodes(LevelGeo g, const double* __restrict__ phi0,
                                                        double* __restrict__ phi, int8_t* __restrict__ cls,
                                                        int* __restrict__ counts, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int8_t c = kOut;
  if (i < g.nn) {
    int j[3];
    node_coords(g, i, j);
    const double v = phi0[level0_index(g, j)];
    phi[i] = v;
    if (!isfinite(v)) atomicOr(flags, kFlagNonFinite);
    if (v < 0.0) {
      c = kIn;
      for (int a = 0; a < g.D; ++a)
        if (j[a] == 0 || j[a] == g.n) atomicOr(flags, kFlagGeom);  // the domain touches the box
    } else {
      for (int a = 0; a < g.D && c != kGhost; ++a)
        for (int dir = -1; dir <= 1; dir += 2) {
          int q[3] = {j[0], j[1], j[2]};
          q[a] += dir;
          if (inside_box(g, q) && phi0[level0_index(g, q)] < 0.0) c = kGhost;
        }
    }
    cls[i] = c;
  }
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const unsigned long long m = __ballot(c == kGhost);
  if ((threadIdx.x & 63) == 0) atomicAdd(&cnt, __popcll(m));
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = cnt;
}

// exclusive scan of the block counts (one workgroup); total[0] receives their sum and
// total[1] the number of interior nodes seen as flagged below
__global__ void __launch_bounds__(kScanThreads) k_scan_counts(const int* __restrict__ counts, int nb,
                                                              int* __restrict__ offsets,
                                                              int* __restrict__ total) {
  __shared__ int part[kScanThreads];
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += counts[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < kScanThreads; ++t) {
      const int v = part[t];
      part[t] = acc;
      acc += v;
    }
    total[0] = acc;
  }
  __syncthreads();
  int acc = part[threadIdx.x];
  for (int b = b0; b < b1; ++b) {
    offsets[b] = acc;
    acc += counts[b];
  }
}

// ghost node indices in node order
__global__ void __launch_bounds__(256) k_list_ghosts(int64_t nn, const int8_t* __restrict__ cls,
                                                     const int* __restrict__ offsets,
                                                     int32_t* __restrict__ list) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool gh = i < nn && cls[i] == kGhost;
  __shared__ int wave_count[4];
  const unsigned long long m = __ballot(gh);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) wave_count[w] = __popcll(m);
  __syncthreads();
  int before = 0;
  for (int v = 0; v < w; ++v) before += wave_count[v];
  const unsigned long long lower = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
  if (gh) list[offsets[blockIdx.x] + before + __popcll(lower)] = (int32_t)i;
}

// the nodes of the rung's stencil (signs s) are inside the box and carry unknowns
__device__ bool stencil_contained(const LevelGeo& g, const int8_t* __restrict__ cls, const int jG[3],
                                  const int8_t* s, int rung) {
  int K = 1;
  for (int a = 0; a < g.D; ++a) K *= 3;
  for (int t = 0; t < K; ++t) {
    int k[3] = {0, 0, 0}, tt = t;
    for (int a = g.D - 1; a >= 0; --a) {
      k[a] = tt % 3;
      tt /= 3;
    }
    bool need;
    if (rung == 1) {
      need = true;
    } else if (rung == 2) {
      need = true;
      for (int a = 0; a < g.D; ++a)
        if (k[a] == 2) need = false;
    } else {
      // rung 3: the ghost and one step along each axis
      int nonzero = 0, far = 0;
      for (int a = 0; a < g.D; ++a) {
        nonzero += k[a] != 0;
        far += k[a] > 1;
      }
      need = nonzero <= 1 && far == 0;
    }
    if (!need) continue;
    int j[3] = {jG[0], jG[1], jG[2]};
    for (int a = 0; a < g.D; ++a) j[a] += s[a] * k[a];
    if (!inside_box(g, j)) return false;
    int64_t q = 0;
    for (int a = g.D - 1; a >= 0; --a) q = q * g.np + j[a];
    const int8_t c = cls[q];
    if (c != kIn && c != kGhost) return false;
  }
  return true;
}

template <int D>
__global__ void __launch_bounds__(256) k_ghost_records(LevelGeo g, int ng, const int32_t* __restrict__ list,
                                                       const double* __restrict__ phi,
                                                       const int8_t* __restrict__ cls, mg_bc_rule rule,
                                                       int have_rule, GhostRec* __restrict__ recs,
                                                       double* __restrict__ Bout, int* __restrict__ flags) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= ng) return;
  const int64_t Gi = list[q];
  int jG[3];
  node_coords(g, Gi, jG);
  // gradient of phi: central differences, one-sided second order on the box faces
  double gr[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D; ++a) {
    const int64_t s = g.st[a];
    if (jG[a] > 0 && jG[a] < g.n)
      gr[a] = (phi[Gi + s] - phi[Gi - s]) / (2.0 * g.h);
    else if (jG[a] == 0)
      gr[a] = (-3.0 * phi[Gi] + 4.0 * phi[Gi + s] - phi[Gi + 2 * s]) / (2.0 * g.h);
    else
      gr[a] = (3.0 * phi[Gi] - 4.0 * phi[Gi - s] + phi[Gi - 2 * s]) / (2.0 * g.h);
  }
  double n2 = 0.0;
  for (int a = 0; a < D; ++a) n2 += gr[a] * gr[a];
  const double nrm = sqrt(n2);
  GhostRec r;
  r.node = (int32_t)Gi;
  r.type = 0;
  r.rung = 0;
  r.axis = 0;
  r.pad0 = 0;
  r.s[0] = r.s[1] = r.s[2] = 0;
  r.pad1 = 0;
  r.pad2 = 0;
  for (int a = 0; a < 3; ++a) r.xi[a] = r.nb[a] = 0.0;
  double B[3] = {0.0, 0.0, 0.0}, xG[3] = {0.0, 0.0, 0.0};
  if (!(nrm > 0.0)) {
    atomicOr(flags, kFlagGeom);
    recs[q] = r;
    for (int a = 0; a < 3; ++a) Bout[3 * q + a] = 0.0;
    return;
  }
  for (int a = 0; a < D; ++a) {
    const double na = gr[a] / nrm;
    xG[a] = g.lo + g.h * (double)jG[a];
    B[a] = xG[a] - na * phi[Gi];  // closest boundary point, Eq. (clpt)
  }
  if (have_rule) {
    double v = rule.c;
    for (int a = 0; a < D; ++a) v += rule.a[a] * B[a];
    r.type = (rule.strict ? (v > 0.0) : (v >= 0.0)) ? 1 : 0;
  }
  // upwind signs of Eq. (St_G); where B is level with the ghost along an axis (a tie), the
  // side of the smaller-phi neighbour
  int8_t pref[3] = {1, 1, 1};
  int tiedax[3] = {0, 0, 0}, ntied = 0;
  for (int a = 0; a < D; ++a) {
    const double df = B[a] - xG[a];
    if (fabs(df) > 1e-12 * g.h) {
      pref[a] = df > 0.0 ? 1 : -1;
    } else {
      tiedax[ntied++] = a;
      const double pm = jG[a] > 0 ? phi[Gi - g.st[a]] : INFINITY;
      const double pp = jG[a] < g.n ? phi[Gi + g.st[a]] : INFINITY;
      pref[a] = pm < pp ? -1 : 1;
    }
  }
  // the ladder: the first rung (and, for tied axes, the first choice of sides) whose
  // stencil stays on unknowns
  int rung = 0, axis = 0;
  int8_t s[3] = {1, 1, 1};
  for (int rg = 1; rg <= 3 && !rung; ++rg)
    for (int m = 0; m < (1 << ntied) && !rung; ++m) {
      for (int a = 0; a < 3; ++a) s[a] = pref[a];
      for (int b = 0; b < ntied; ++b)
        if (m & (1 << b)) s[tiedax[b]] = (int8_t)-pref[tiedax[b]];
      if (stencil_contained(g, cls, jG, s, rg)) rung = rg;
    }
  if (!rung) {
    // two points along the axis of the interior neighbour with the smallest phi
    double best = INFINITY;
    int ba = -1, bs = 0;
    for (int a = 0; a < D; ++a)
      for (int dir = -1; dir <= 1; dir += 2) {
        int qj[3] = {jG[0], jG[1], jG[2]};
        qj[a] += dir;
        if (!inside_box(g, qj)) continue;
        const int64_t Q = Gi + dir * g.st[a];
        if (cls[Q] != kIn) continue;
        if (phi[Q] < best) {
          best = phi[Q];
          ba = a;
          bs = dir;
        }
      }
    if (ba < 0) {
      // no stencil at all: the setup fails; nothing below is evaluated for this ghost
      atomicOr(flags, kFlagGeom);
      recs[q] = r;
      for (int a = 0; a < 3; ++a) Bout[3 * q + a] = a < D ? B[a] : 0.0;
      return;
    }
    for (int a = 0; a < 3; ++a) s[a] = pref[a];
    s[ba] = (int8_t)bs;
    axis = ba;
    rung = 4;
  }
  r.rung = (int8_t)rung;
  r.axis = (int8_t)axis;
  for (int a = 0; a < 3; ++a) r.s[a] = a < D ? s[a] : 0;
  for (int a = 0; a < D; ++a) r.xi[a] = (double)s[a] * (B[a] - xG[a]) / g.h;
  if (!r.type) {
    // unit normal at B from the same interpolant of phi (Neumann rows); with a caller's
    // partition the type is not known here: the normal is computed for every ghost, and a
    // ghost without one is marked (pad0) for the host to reject if it is a Neumann ghost
    double gp[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) {
      double e[3] = {0.0, 0.0, 0.0};
      e[a] = 1.0;
      double w[Pow3<D>::value];
      const uint32_t used = stencil_weights<D>(rung, axis, s, r.xi, g.inv_h, 0, e, w);
      for (int t = 0; t < Pow3<D>::value; ++t) {
        if (!(used >> t & 1u)) continue;
        gp[a] += w[t] * phi[Gi + template_offset<D>(t, s, g.st)];
      }
    }
    double g2 = 0.0;
    for (int a = 0; a < D; ++a) g2 += gp[a] * gp[a];
    const double gn = sqrt(g2);
    if (gn > 0.0) {
      for (int a = 0; a < D; ++a) r.nb[a] = gp[a] / gn;
    } else if (have_rule) {
      atomicOr(flags, kFlagGeom);
    } else {
      r.pad0 = 1;
    }
  }
  recs[q] = r;
  for (int a = 0; a < 3; ++a) Bout[3 * q + a] = a < D ? B[a] : 0.0;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
  int alloc(size_t bytes) {
    return hipMalloc(&p, bytes ? bytes : 1) == hipSuccess ? MG_OK : MG_ENOMEM;
  }
};

}  // namespace

int classify_level_gpu(const double* phi0, int D, int n0, int l, int problem, double lo, double h,
                       const mg_bc_rule* rule, LevelClass& out) {
  LevelGeo g;
  g.D = D;
  g.n = n0 >> l;
  g.np = g.n + 1;
  g.nn = 1;
  const int64_t np0 = (int64_t)n0 + 1;
  int64_t s0 = 1;
  for (int a = 0; a < 3; ++a) {
    g.st[a] = a < D ? g.nn : 0;
    g.st0[a] = a < D ? s0 * ((int64_t)1 << l) : 0;
    if (a < D) {
      g.nn *= g.np;
      s0 *= np0;
    }
  }
  g.base0 = (int64_t)problem * s0;
  g.lo = lo;
  g.h = h;
  g.inv_h = 1.0 / h;
  const int nb = (int)((g.nn + 255) / 256);
  DevBuf dphi, dcls, dcnt, doff, dtot, dflags;
  int rc;
  if ((rc = dphi.alloc(g.nn * sizeof(double))) || (rc = dcls.alloc(g.nn)) ||
      (rc = dcnt.alloc(nb * sizeof(int))) || (rc = doff.alloc(nb * sizeof(int))) ||
      (rc = dtot.alloc(2 * sizeof(int))) || (rc = dflags.alloc(sizeof(int))))
    return rc;
  if (hipMemset(dflags.p, 0, sizeof(int)) != hipSuccess) return MG_EHIP;
  hipLaunchKernelGGL(k_classify_nodes, dim3(nb), dim3(256), 0, nullptr, g, phi0, dphi.as<double>(),
                     dcls.as<int8_t>(), dcnt.as<int>(), dflags.as<int>());
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kScanThreads), 0, nullptr, dcnt.as<int>(), nb,
                     doff.as<int>(), dtot.as<int>());
  int total = 0, flags = 0;
  if (hipMemcpy(&total, dtot.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&flags, dflags.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return MG_EHIP;
  if (flags & kFlagNonFinite) return MG_EINVAL;
  DevBuf dlist, drec, dB;
  if ((rc = dlist.alloc((size_t)total * sizeof(int32_t))) ||
      (rc = drec.alloc((size_t)total * sizeof(GhostRec))) ||
      (rc = dB.alloc((size_t)total * 3 * sizeof(double))))
    return rc;
  if (total > 0) {
    hipLaunchKernelGGL(k_list_ghosts, dim3(nb), dim3(256), 0, nullptr, g.nn, dcls.as<int8_t>(),
                       doff.as<int>(), dlist.as<int32_t>());
    const mg_bc_rule none{};
    const int blocks = (total + 255) / 256;
    if (D == 2)
      hipLaunchKernelGGL(k_ghost_records<2>, dim3(blocks), dim3(256), 0, nullptr, g, total,
                         dlist.as<int32_t>(), dphi.as<double>(), dcls.as<int8_t>(), rule ? *rule : none,
                         rule ? 1 : 0, drec.as<GhostRec>(), dB.as<double>(), dflags.as<int>());
    else
      hipLaunchKernelGGL(k_ghost_records<3>, dim3(blocks), dim3(256), 0, nullptr, g, total,
                         dlist.as<int32_t>(), dphi.as<double>(), dcls.as<int8_t>(), rule ? *rule : none,
                         rule ? 1 : 0, drec.as<GhostRec>(), dB.as<double>(), dflags.as<int>());
  }
  if (hipGetLastError() != hipSuccess) return MG_EHIP;
  out.phi.resize((size_t)g.nn);
  out.cls.resize((size_t)g.nn);
  out.gh.resize((size_t)total);
  out.B.resize((size_t)total * 3);
  if (hipMemcpy(out.phi.data(), dphi.p, g.nn * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(out.cls.data(), dcls.p, g.nn, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(out.gh.data(), drec.p, (size_t)total * sizeof(GhostRec), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(out.B.data(), dB.p, (size_t)total * 3 * sizeof(double), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(&flags, dflags.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return MG_EHIP;
  if (flags & kFlagGeom) return MG_EGEOM;
  bool any_in = false;
  for (int8_t c : out.cls)
    if (c == kIn) {
      any_in = true;
      break;
    }
  return any_in ? MG_OK : MG_EGEOM;
}

}  // namespace ghostmg
