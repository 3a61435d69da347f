// Device kernels of the ghost-cell multigrid cycle (gfx950, wave64).
//
// Node arrays hold one level of every problem of the batch, padded rows (pitch multiple of
// 16), x fastest.  Node-parallel kernels walk a list of active tiles (tiles that hold at
// least one unknown); list kernels walk the compact ghost / band / extension records.
// Workgroups of a tile kernel are mapped so that each of the 8 XCDs takes a contiguous run
// of tiles (the dispatcher deals workgroups to XCDs round-robin), which keeps the halo
// rows a tile shares with its neighbours in one L2.
#include "kernels.h"

namespace ghostmg {

__device__ __forceinline__ int xcd_tile(int b, int nb) {
  // nb is a multiple of 8: XCD k = b % 8 gets tiles [k nb/8, (k+1) nb/8)
  return (b & 7) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ bool in_box(int x, int y, int z, int np, int D) {
  return x >= 0 && x < np && y >= 0 && y < np && (D == 2 || (z >= 0 && z < np));
}

// Max of non-negative doubles through their IEEE bit patterns (order preserving).
__device__ __forceinline__ void atomic_max_pos(uint64_t* dst, double v) {
  if (!(v == v)) v = __longlong_as_double(0x7ff0000000000000LL);  // NaN -> +inf
  atomicMax((unsigned long long*)dst, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) v = fmax(v, red[i]);
  }
  return v;
}

// ---------------------------------------------------------------------------------------
// red-black relaxation of the interior rows, Eq. (jac2d), one tile per workgroup
// ---------------------------------------------------------------------------------------
// The tile and a ring of two nodes are staged in LDS.  Red nodes of tile + ring one are
// relaxed first (they read only black, ghost or outside values, which this pass leaves
// unchanged), then the black nodes of the tile (which read the fresh red values); every
// workgroup writes back only its own tile.  The result is the global red sweep followed
// by the global black sweep.  The update is written as a correction,
// u_P += (h^2 f_P + sum_nb (u_nb - u_P)) / (2D).
template <int D, typename T>
__global__ void __launch_bounds__(256) k_smooth(const int4* __restrict__ tiles, int ntiles,
                                                 Geo g, const int8_t* __restrict__ cls,
                                                 T* __restrict__ u, const T* __restrict__ rhs,
                                                 T h2, T inv2d) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  constexpr int UX = TX + 4, UY = TY + 4, UZ = D == 3 ? TZ + 4 : 1;
  constexpr int FX = TX + 2, FY = TY + 2, FZ = D == 3 ? TZ + 2 : 1;
  __shared__ T su[UZ * UY * UX];
  __shared__ T sf[FZ * FY * FX];
  __shared__ int8_t sc[FZ * FY * FX];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  const int ox = t.y * TX, oy = t.z * TY, oz = t.w * TZ;
  for (int i = threadIdx.x; i < UZ * UY * UX; i += 256) {
    const int x = i % UX, y = (i / UX) % UY, z = i / (UX * UY);
    const int gx = ox + x - 2, gy = oy + y - 2, gz = D == 3 ? oz + z - 2 : 0;
    T v = 0;
    if (in_box(gx, gy, gz, g.np, D)) v = u[base + gx + g.st[1] * gy + g.st[2] * gz];
    su[i] = v;
  }
  for (int i = threadIdx.x; i < FZ * FY * FX; i += 256) {
    const int x = i % FX, y = (i / FX) % FY, z = i / (FX * FY);
    const int gx = ox + x - 1, gy = oy + y - 1, gz = D == 3 ? oz + z - 1 : 0;
    T f = 0;
    int8_t c = 0;
    if (in_box(gx, gy, gz, g.np, D)) {
      const int64_t gi = base + gx + g.st[1] * gy + g.st[2] * gz;
      c = cls[gi];
      if (c == 1) f = rhs[gi];
    }
    sf[i] = f;
    sc[i] = c;
  }
  __syncthreads();
  constexpr int SY = UX, SZ = UX * UY;
  for (int i = threadIdx.x; i < FZ * FY * FX; i += 256) {
    if (sc[i] != 1) continue;
    const int x = i % FX, y = (i / FX) % FY, z = i / (FX * FY);
    const int gx = ox + x - 1, gy = oy + y - 1, gz = D == 3 ? oz + z - 1 : 0;
    if ((gx + gy + gz) & 1) continue;
    const int ui = (x + 1) + SY * (y + 1) + (D == 3 ? SZ * (z + 1) : 0);
    const T c = su[ui];
    T s = (su[ui - 1] - c) + (su[ui + 1] - c);
    s += (su[ui - SY] - c) + (su[ui + SY] - c);
    if (D == 3) s += (su[ui - SZ] - c) + (su[ui + SZ] - c);
    su[ui] = c + (h2 * sf[i] + s) * inv2d;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
    const int fi = (x + 1) + FX * (y + 1) + (D == 3 ? FX * FY * (z + 1) : 0);
    if (sc[fi] != 1) continue;
    const int gx = ox + x, gy = oy + y, gz = D == 3 ? oz + z : 0;
    if (!((gx + gy + gz) & 1)) continue;
    const int ui = (x + 2) + SY * (y + 2) + (D == 3 ? SZ * (z + 2) : 0);
    const T c = su[ui];
    T s = (su[ui - 1] - c) + (su[ui + 1] - c);
    s += (su[ui - SY] - c) + (su[ui + SY] - c);
    if (D == 3) s += (su[ui - SZ] - c) + (su[ui + SZ] - c);
    su[ui] = c + (h2 * sf[fi] + s) * inv2d;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
    const int fi = (x + 1) + FX * (y + 1) + (D == 3 ? FX * FY * (z + 1) : 0);
    if (sc[fi] != 1) continue;
    const int ui = (x + 2) + SY * (y + 2) + (D == 3 ? SZ * (z + 2) : 0);
    u[base + (ox + x) + g.st[1] * (oy + y) + g.st[2] * (D == 3 ? oz + z : 0)] = su[ui];
  }
}

// ---------------------------------------------------------------------------------------
// ghost rows: Eqs. (dir2d) / (neu2d) and the boundary part of the defect
// ---------------------------------------------------------------------------------------
template <int D, typename T>
__device__ __forceinline__ double ghost_apply(const GhostRec& r, const Geo& g,
                                              const T* __restrict__ u, double inv_h) {
  constexpr int K = Pow3<D>::value;
  double w[K];
  const uint32_t used = ghost_row<D>(r, inv_h, w);
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (!(used >> t & 1u)) continue;
    acc += w[t] * (double)u[r.node + template_offset<D>(t, r.s, g.st)];
  }
  return acc;
}

template <int D, typename T>
__device__ __forceinline__ T ghost_new_value(const GhostRec& r, const Geo& g,
                                             const T* __restrict__ u, const T* __restrict__ rhs,
                                             double inv_h, double cD, double cNh) {
  const double Lu = ghost_apply<D, T>(r, g, u, inv_h);
  const double c = r.type ? cD : cNh;
  return (T)((double)u[r.node] + c * ((double)rhs[r.node] - Lu));
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_ghost_new(const GhostRec* __restrict__ gs, int ng, Geo g,
                                                   const T* __restrict__ u, const T* __restrict__ rhs,
                                                   T* __restrict__ tmp, double inv_h, double cD,
                                                   double cNh) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ng) return;
  tmp[i] = ghost_new_value<D, T>(gs[i], g, u, rhs, inv_h, cD, cNh);
}

template <typename T>
__global__ void __launch_bounds__(256) k_ghost_store(const GhostRec* __restrict__ gs, int ng,
                                                     const T* __restrict__ tmp, T* __restrict__ u) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ng) return;
  u[gs[i].node] = tmp[i];
}

template <int D, typename T>
__device__ __forceinline__ void relax_node(int64_t P, const Geo& g, T* __restrict__ u,
                                           const T* __restrict__ rhs, T h2, T inv2d) {
  const T c = u[P];
  T s = (u[P - 1] - c) + (u[P + 1] - c);
  s += (u[P - g.st[1]] - c) + (u[P + g.st[1]] - c);
  if (D == 3) s += (u[P - g.st[2]] - c) + (u[P + g.st[2]] - c);
  u[P] = c + (h2 * rhs[P] + s) * inv2d;
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_relax_list(const int32_t* __restrict__ list, int n, Geo g,
                                                    T* __restrict__ u, const T* __restrict__ rhs,
                                                    T h2, T inv2d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  relax_node<D, T>(list[i], g, u, rhs, h2, inv2d);
}

// Ghost relaxation followed by lambda sweeps over the boundary band (Sec. 3.2), one
// workgroup per problem: every phase (red band, black band, all ghosts from the same state)
// is separated by a workgroup barrier, so the whole sequence is one launch.
template <int D, typename T>
__global__ void __launch_bounds__(1024) k_band(BandArgs<T> a) {
  const int p = blockIdx.x;
  const int g0 = a.ghost_off[p], g1 = a.ghost_off[p + 1];
  const int r0 = a.red_off[p], r1 = a.red_off[p + 1];
  const int b0 = a.black_off[p], b1 = a.black_off[p + 1];
  const int tid = threadIdx.x;
  for (int k = 0; k <= a.lambda; ++k) {
    if (k > 0) {
      for (int i = r0 + tid; i < r1; i += 1024) relax_node<D, T>(a.red[i], a.g, a.u, a.rhs, a.h2, a.inv2d);
      __syncthreads();
      for (int i = b0 + tid; i < b1; i += 1024) relax_node<D, T>(a.black[i], a.g, a.u, a.rhs, a.h2, a.inv2d);
      __syncthreads();
    }
    for (int i = g0 + tid; i < g1; i += 1024)
      a.tmp[i] = ghost_new_value<D, T>(a.ghosts[i], a.g, a.u, a.rhs, a.inv_h, a.cD, a.cNh);
    __syncthreads();
    for (int i = g0 + tid; i < g1; i += 1024) a.u[a.ghosts[i].node] = a.tmp[i];
    __syncthreads();
  }
}

// Ghost relaxation and lambda band sweeps with the band held in LDS: one workgroup per
// chunk runs all 1 + 3 lambda phases (ghosts; then red band, black band, ghosts, lambda
// times) on the chunk's dependency-closed node set, with workgroup barriers between phases,
// and stores the results of the nodes it owns.  k_band_scatter then writes them to u (no
// chunk may overwrite a value another chunk is still loading).
template <int D, typename T>
__global__ void __launch_bounds__(256) k_band_chunk(BandChunkArgs<T> a) {
  constexpr int K = Pow3<D>::value;
  extern __shared__ double lds_d[];
  const int c = blockIdx.x;
  const int s0 = a.off[c], ns = a.off[c + 1] - s0;
  const int g0 = a.goff[c], ngc = a.goff[c + 1] - g0;
  const int32_t* ops_off = a.ops_off + (int64_t)c * (a.phases + 1);
  const int o_base = ops_off[0], nops = ops_off[a.phases] - o_base;
  // LDS layout: ghost weights, ghost constants (FP64); u, rhs, new ghost values (T);
  // neighbour ids, ghost stencil ids, ghost entry ids, op lists (int16)
  double* gw = lds_d;
  double* gc = gw + (size_t)a.gmax * K;
  T* su = (T*)(gc + a.gmax);
  T* sr = su + a.smax;
  T* st = sr + a.smax;
  int16_t* nb = (int16_t*)(st + a.gmax);
  int16_t* gs = nb + (size_t)a.smax * 2 * D;
  int16_t* ge = gs + (size_t)a.gmax * K;
  int16_t* ops = ge + a.gmax;
  for (int i = threadIdx.x; i < ns; i += 256) {
    const int32_t v = a.node[s0 + i];
    su[i] = a.u[v];
    sr[i] = a.rhs[v];
  }
  for (int i = threadIdx.x; i < ns * 2 * D; i += 256) nb[i] = a.nbr[(int64_t)s0 * 2 * D + i];
  for (int i = threadIdx.x; i < ngc * K; i += 256) gs[i] = a.gsten[(int64_t)g0 * K + i];
  for (int i = threadIdx.x; i < nops; i += 256) ops[i] = a.ops[o_base + i];
  for (int j = threadIdx.x; j < ngc; j += 256) {
    const GhostRec r = a.ghosts[a.gidx[g0 + j]];
    double w[K];
    const uint32_t used = ghost_row<D>(r, a.inv_h, w);
#pragma unroll
    for (int t = 0; t < K; ++t) gw[(size_t)j * K + t] = (used >> t & 1u) ? w[t] : 0.0;
    gc[j] = r.type ? a.cD : a.cNh;
    ge[j] = a.gent[g0 + j];
  }
  __syncthreads();
  for (int p = 0; p < a.phases; ++p) {
    const int kind = p == 0 ? 3 : ((p - 1) % 3 == 0 ? 1 : ((p - 1) % 3 == 1 ? 2 : 3));
    const int o0 = ops_off[p] - o_base, o1 = ops_off[p + 1] - o_base;
    if (kind != 3) {
      for (int i = o0 + threadIdx.x; i < o1; i += 256) {
        const int v = ops[i];
        const int16_t* n = nb + v * (2 * D);
        const T cv = su[v];
        T sum = (su[n[0]] - cv) + (su[n[1]] - cv);
        sum += (su[n[2]] - cv) + (su[n[3]] - cv);
        if (D == 3) sum += (su[n[4]] - cv) + (su[n[5]] - cv);
        su[v] = cv + (a.h2 * sr[v] + sum) * a.inv2d;
      }
    } else {
      for (int i = o0 + threadIdx.x; i < o1; i += 256) {
        const int j = ops[i];
        const int v = ge[j];
        const double* w = gw + (size_t)j * K;
        const int16_t* sn = gs + (size_t)j * K;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < K; ++t)
          if (sn[t] >= 0) acc += w[t] * (double)su[sn[t]];
        st[j] = (T)((double)su[v] + gc[j] * ((double)sr[v] - acc));
      }
      __syncthreads();
      for (int i = o0 + threadIdx.x; i < o1; i += 256) su[ge[ops[i]]] = st[ops[i]];
    }
    __syncthreads();
  }
  const int own = a.own[c], out0 = a.out_off[c];
  for (int i = threadIdx.x; i < own; i += 256) a.out[out0 + i] = su[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_band_scatter(const int32_t* __restrict__ node, int n,
                                                      const T* __restrict__ out, T* __restrict__ u) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[node[i]] = out[i];
}

// ---------------------------------------------------------------------------------------
// defect (Sec. 2.4 step 3) with per-problem infinity norms
// ---------------------------------------------------------------------------------------
// One launch: workgroups [0, nbt) take the active tiles (interior rows), the rest take the
// ghost records (boundary rows).  Per-problem maxima of |r| go to norms[2p] (interior) and
// norms[2p + 1] (ghosts) through order-independent integer maxima, so the result is
// deterministic.
template <int D, typename T, typename TO>
__global__ void __launch_bounds__(256) k_defect(const int4* __restrict__ tiles, int ntiles, int nbt,
                                                const GhostRec* __restrict__ gs, int ng, Geo g,
                                                const int8_t* __restrict__ cls,
                                                const T* __restrict__ u, const T* __restrict__ rhs,
                                                TO* __restrict__ r, T inv_h2, double inv_h,
                                                uint64_t* __restrict__ norms) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  __shared__ double red[4];
  if ((int)blockIdx.x < nbt) {
    const int tile = xcd_tile(blockIdx.x, nbt);
    if (tile >= ntiles) return;
    const int4 t = tiles[tile];
    const int64_t base = (int64_t)t.x * g.npp;
    double m = 0.0;
    for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
      const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
      const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
      if (!in_box(x, y, z, g.np, D)) continue;
      const int64_t P = base + x + g.st[1] * y + g.st[2] * z;
      if (cls[P] != 1) continue;
      const T c = u[P];
      T s = (u[P - 1] - c) + (u[P + 1] - c);
      s += (u[P - g.st[1]] - c) + (u[P + g.st[1]] - c);
      if (D == 3) s += (u[P - g.st[2]] - c) + (u[P + g.st[2]] - c);
      const T v = rhs[P] + s * inv_h2;
      r[P] = (TO)v;
      m = fmax(m, fabs((double)v));
      if (!(v == v)) m = __longlong_as_double(0x7ff0000000000000LL);
    }
    if (norms) {
      m = block_max(m, red);
      if (threadIdx.x == 0) atomic_max_pos(&norms[2 * t.x], m);
    }
    return;
  }
  const int i = ((int)blockIdx.x - nbt) * 256 + threadIdx.x;
  if (i >= ng) return;
  const GhostRec rec = gs[i];
  const double v = (double)rhs[rec.node] - ghost_apply<D, T>(rec, g, u, inv_h);
  r[rec.node] = (TO)v;
  if (norms) atomic_max_pos(&norms[2 * (rec.node / g.npp) + 1], fabs(v));
}

// ||(f_h, g_h)||_inf per problem: max |rhs| over the unknowns
template <int D>
__global__ void __launch_bounds__(256) k_rhs_norm(const int4* __restrict__ tiles, int ntiles, Geo g,
                                                  const int8_t* __restrict__ cls,
                                                  const double* __restrict__ rhs,
                                                  uint64_t* __restrict__ norms) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  __shared__ double red[4];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  double m = 0.0;
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    if (!in_box(x, y, z, g.np, D)) continue;
    const int64_t P = base + x + g.st[1] * y + g.st[2] * z;
    if (cls[P] == 0) continue;
    m = fmax(m, fabs(rhs[P]));
    if (!(rhs[P] == rhs[P])) m = __longlong_as_double(0x7ff0000000000000LL);
  }
  m = block_max(m, red);
  if (threadIdx.x == 0) atomic_max_pos(&norms[2 * t.x], m);
}

// ---------------------------------------------------------------------------------------
// extension of the defect outside Omega_h, Eq. (exp) in its steady state
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void extend_one(const ExtRec& e, T* __restrict__ r) {
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (e.src[a] < 0) continue;
    num += e.wt[a] * (double)r[e.src[a]];
    den += e.wt[a];
  }
  r[e.node] = (T)(den > 0.0 ? num / den : 0.0);
}

// one workgroup per problem, DAG levels separated by barriers
template <typename T>
__global__ void __launch_bounds__(1024) k_extend_wg(const ExtRec* __restrict__ ext,
                                                    const int32_t* __restrict__ dag_off,
                                                    const int32_t* __restrict__ dag_start,
                                                    T* __restrict__ r) {
  const int p = blockIdx.x;
  const int s0 = dag_start[p], s1 = dag_start[p + 1];
  for (int d = s0; d + 1 < s1; ++d) {
    for (int i = dag_off[d] + threadIdx.x; i < dag_off[d + 1]; i += 1024) extend_one<T>(ext[i], r);
    __syncthreads();
  }
}

// chunked extension: the chunk's ghost defects are read into LDS, its extension nodes are
// computed DAG level by DAG level in LDS, and only the owned nodes are written back
template <typename T>
__global__ void __launch_bounds__(256) k_extend_chunk(const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ own,
                                                      const int32_t* __restrict__ next,
                                                      const int32_t* __restrict__ node,
                                                      const int16_t* __restrict__ src,
                                                      const double* __restrict__ wt,
                                                      const int16_t* __restrict__ ops,
                                                      const int32_t* __restrict__ lvl,
                                                      const int32_t* __restrict__ lvl_start,
                                                      T* __restrict__ r) {
  extern __shared__ double ext_lds[];
  const int c = blockIdx.x;
  const int s0 = off[c], ns = off[c + 1] - s0, ne = next[c];
  double* sv = ext_lds;
  for (int i = threadIdx.x; i < ns; i += 256) sv[i] = i >= ne ? (double)r[node[s0 + i]] : 0.0;
  __syncthreads();
  for (int d = lvl_start[c]; d + 1 < lvl_start[c + 1]; ++d) {
    for (int k = lvl[d] + threadIdx.x; k < lvl[d + 1]; k += 256) {
      const int i = ops[k];
      double num = 0.0, den = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int q = src[(int64_t)(s0 + i) * 3 + a];
        if (q < 0) continue;
        const double w = wt[(int64_t)(s0 + i) * 3 + a];
        num += w * sv[q];
        den += w;
      }
      sv[i] = den > 0.0 ? num / den : 0.0;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < own[c]; i += 256) r[node[s0 + i]] = (T)sv[i];
}

// all problems' nodes of one DAG level
template <typename T>
__global__ void __launch_bounds__(256) k_extend_level(const ExtRec* __restrict__ ext, int a, int b,
                                                      T* __restrict__ r) {
  const int i = a + blockIdx.x * 256 + threadIdx.x;
  if (i >= b) return;
  extend_one<T>(ext[i], r);
}

// ---------------------------------------------------------------------------------------
// restriction I = I~(w, D_h - Omega_h, I~(w, Omega_h, 0)) (Sec. 2.5): every coarse
// unknown sums the fine defect over its box with the tensor weights of Eqs. (restI),
// (restL), (restR); the coarse correction is reset to zero in the same pass
// ---------------------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(256) k_restrict(const int4* __restrict__ tiles, int ntiles, Geo gc,
                                                  Geo gf, const uint8_t* __restrict__ code,
                                                  const T* __restrict__ rf, T* __restrict__ rhsc,
                                                  T* __restrict__ uc) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t basec = (int64_t)t.x * gc.npp, basef = (int64_t)t.x * gf.npp;
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    if (!in_box(x, y, z, gc.np, D)) continue;
    const int64_t X = basec + x + gc.st[1] * y + gc.st[2] * z;
    uc[X] = (T)0;
    const uint8_t c = code[X];
    if (c == kNoUnknown) continue;
    const int lx = (c & 1) ? -1 : 0, hx = (c & 2) ? 1 : 0;
    const int ly = (c & 4) ? -1 : 0, hy = (c & 8) ? 1 : 0;
    const int lz = D == 3 && (c & 16) ? -1 : 0, hz = D == 3 && (c & 32) ? 1 : 0;
    const int64_t F0 = basef + 2 * x + gf.st[1] * 2 * y + gf.st[2] * 2 * z;
    T s = 0;
    for (int kx = lx; kx <= hx; ++kx)
      for (int ky = ly; ky <= hy; ++ky)
        for (int kz = lz; kz <= hz; ++kz) {
          const T w = (T)(restrict_w1d(lx, hx, kx) * restrict_w1d(ly, hy, ky) *
                          (D == 3 ? restrict_w1d(lz, hz, kz) : 1.0));
          s += w * rf[F0 + kx + gf.st[1] * ky + gf.st[2] * kz];
        }
    rhsc[X] = s;
  }
}

// ---------------------------------------------------------------------------------------
// interpolation of the coarse error and correction of the fine unknowns (Sec. 2.6.1):
// multilinear weights renormalised over the coarse nodes that carry an unknown
// ---------------------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(256) k_prolong(const int4* __restrict__ tiles, int ntiles, Geo gf,
                                                 Geo gc, const int8_t* __restrict__ clsf,
                                                 const int8_t* __restrict__ clsc,
                                                 const T* __restrict__ uc, T* __restrict__ uf) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t basef = (int64_t)t.x * gf.npp, basec = (int64_t)t.x * gc.npp;
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    if (!in_box(x, y, z, gf.np, D)) continue;
    const int64_t P = basef + x + gf.st[1] * y + gf.st[2] * z;
    if (clsf[P] == 0) continue;
    const int j[3] = {x, y, z};
    T num = 0, den = 0;
#pragma unroll
    for (int m = 0; m < (1 << D); ++m) {
      bool skip = false;
      T w = 1;
      int64_t X = basec;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int bit = (m >> a) & 1;
        int jc;
        if ((j[a] & 1) == 0) {
          if (bit) skip = true;
          jc = j[a] >> 1;
        } else {
          jc = bit ? (j[a] + 1) >> 1 : (j[a] - 1) >> 1;
          w *= (T)0.5;
        }
        X += gc.st[a] * jc;
      }
      if (skip) continue;
      if (clsc[X] == 0) continue;
      num += w * uc[X];
      den += w;
    }
    if (den > (T)0) uf[P] += num / den;
  }
}

// ---------------------------------------------------------------------------------------
// exact solve on the coarsest grid: e = A_c^{-1} r (FP64), several row blocks per problem
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_coarse(const int32_t* __restrict__ umap,
                                                const int32_t* __restrict__ umap_off,
                                                const int64_t* __restrict__ ainv_off,
                                                const double* __restrict__ ainv,
                                                const T* __restrict__ rhs, T* __restrict__ u) {
  extern __shared__ double bsh[];
  const int p = blockIdx.y;
  const int a = umap_off[p], nu = umap_off[p + 1] - a;
  const int row0 = blockIdx.x * kCoarseRows;
  if (row0 >= nu) return;
  for (int i = threadIdx.x; i < nu; i += 256) bsh[i] = (double)rhs[umap[a + i]];
  __syncthreads();
  const double* A = ainv + ainv_off[p];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row1 = min(row0 + kCoarseRows, nu);
  for (int r = row0 + w; r < row1; r += 4) {
    double acc = 0.0;
    const double* Ar = A + (int64_t)r * nu;
    for (int j = lane; j < nu; j += 64) acc += Ar[j] * bsh[j];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) u[umap[a + r]] = (T)acc;
  }
}

// ---------------------------------------------------------------------------------------
// plumbing: fills, packing of the caller's arrays, defect-correction updates
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int D>
__global__ void __launch_bounds__(256) k_pack(const int4* __restrict__ tiles, int ntiles, Geo g,
                                              const int8_t* __restrict__ cls,
                                              const double* __restrict__ f,
                                              const double* __restrict__ gv,
                                              const double* __restrict__ uin,
                                              double* __restrict__ rhs, double* __restrict__ u) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  const int64_t nnu = D == 3 ? (int64_t)g.np * g.np * g.np : (int64_t)g.np * g.np;
  const int64_t ubase = (int64_t)t.x * nnu;
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    if (!in_box(x, y, z, g.np, D)) continue;
    const int64_t P = base + x + g.st[1] * y + g.st[2] * z;
    const int64_t Q = ubase + x + (int64_t)g.np * (y + (int64_t)g.np * z);
    const int8_t c = cls[P];
    rhs[P] = c == 1 ? f[Q] : (c == 2 ? gv[Q] : 0.0);
    if (uin) u[P] = c ? uin[Q] : 0.0;
  }
}

template <int D>
__global__ void __launch_bounds__(256) k_unpack(int64_t total, Geo g, const int8_t* __restrict__ cls,
                                                const double* __restrict__ src,
                                                double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t nnu = D == 3 ? (int64_t)g.np * g.np * g.np : (int64_t)g.np * g.np;
  const int64_t p = i / nnu;
  int64_t q = i - p * nnu;
  const int x = (int)(q % g.np);
  q /= g.np;
  const int y = (int)(q % g.np);
  const int z = (int)(q / g.np);
  const int64_t P = p * g.npp + x + g.st[1] * y + g.st[2] * z;
  dst[i] = cls[P] ? src[P] : 0.0;
}

// u64 += u32 at the unknowns (defect correction), and u32 reset for the next step
template <int D>
__global__ void __launch_bounds__(256) k_dc_update(const int4* __restrict__ tiles, int ntiles, Geo g,
                                                   const int8_t* __restrict__ cls,
                                                   double* __restrict__ u64, float* __restrict__ u32) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  for (int i = threadIdx.x; i < TZ * TY * TX; i += 256) {
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    if (!in_box(x, y, z, g.np, D)) continue;
    const int64_t P = base + x + g.st[1] * y + g.st[2] * z;
    if (cls[P] == 0) continue;
    u64[P] += (double)u32[P];
    u32[P] = 0.0f;
  }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
static inline int tile_grid(int ntiles) { return (ntiles + 7) / 8 * 8; }
static inline int lin_grid(int64_t n) { return (int)((n + 255) / 256); }

template <int D, typename T>
void launch_smooth(const DevLevel& L, T* u, const T* rhs, hipStream_t s) {
  if (!L.ntiles) return;
  const T h2 = (T)(L.g.h * L.g.h), inv2d = (T)(1.0 / (2.0 * D));
  hipLaunchKernelGGL((k_smooth<D, T>), dim3(tile_grid(L.ntiles)), dim3(256), 0, s, L.tiles,
                     L.ntiles, L.g, L.cls, u, rhs, h2, inv2d);
}

template <int D, typename T>
void launch_band(const DevLevel& L, const mg_grid& G, T* u, const T* rhs, T* tmp, bool single_wg,
                 int batch, hipStream_t s) {
  const double inv_h = 1.0 / L.g.h, cNh = G.cN * L.g.h;
  const T h2 = (T)(L.g.h * L.g.h), inv2d = (T)(1.0 / (2.0 * D));
  if (single_wg) {
    BandArgs<T> a;
    a.g = L.g;
    a.ghosts = L.ghosts;
    a.ghost_off = L.ghost_off;
    a.red = L.red;
    a.black = L.black;
    a.red_off = L.red_off;
    a.black_off = L.black_off;
    a.u = u;
    a.rhs = rhs;
    a.tmp = tmp;
    a.h2 = h2;
    a.inv2d = inv2d;
    a.inv_h = inv_h;
    a.cD = G.cD;
    a.cNh = cNh;
    a.lambda = G.lambda;
    hipLaunchKernelGGL((k_band<D, T>), dim3(batch), dim3(1024), 0, s, a);
    return;
  }
  auto ghosts = [&]() {
    if (!L.nghost) return;
    hipLaunchKernelGGL((k_ghost_new<D, T>), dim3(lin_grid(L.nghost)), dim3(256), 0, s, L.ghosts,
                       L.nghost, L.g, (const T*)u, rhs, tmp, inv_h, G.cD, cNh);
    hipLaunchKernelGGL((k_ghost_store<T>), dim3(lin_grid(L.nghost)), dim3(256), 0, s, L.ghosts,
                       L.nghost, (const T*)tmp, u);
  };
  ghosts();
  for (int k = 0; k < G.lambda; ++k) {
    if (L.nred)
      hipLaunchKernelGGL((k_relax_list<D, T>), dim3(lin_grid(L.nred)), dim3(256), 0, s, L.red,
                         L.nred, L.g, u, rhs, h2, inv2d);
    if (L.nblack)
      hipLaunchKernelGGL((k_relax_list<D, T>), dim3(lin_grid(L.nblack)), dim3(256), 0, s, L.black,
                         L.nblack, L.g, u, rhs, h2, inv2d);
    ghosts();
  }
}

template <int D, typename T>
void launch_band_chunks(const DevLevel& L, const mg_grid& G, T* u, const T* rhs, T* out,
                        hipStream_t s) {
  if (!L.nchunks) return;
  BandChunkArgs<T> a;
  a.off = L.bc_off;
  a.own = L.bc_own;
  a.out_off = L.bc_out_off;
  a.node = L.bc_node;
  a.nbr = L.bc_nbr;
  a.goff = L.bc_goff;
  a.gidx = L.bc_gidx;
  a.gent = L.bc_gent;
  a.gsten = L.bc_gsten;
  a.ops = L.bc_ops;
  a.ops_off = L.bc_ops_off;
  a.ghosts = L.ghosts;
  a.u = u;
  a.rhs = rhs;
  a.out = out;
  a.smax = L.bc_smax;
  a.gmax = L.bc_gmax;
  a.opsmax = L.bc_opsmax;
  a.phases = L.bc_phases;
  a.h2 = (T)(L.g.h * L.g.h);
  a.inv2d = (T)(1.0 / (2.0 * D));
  a.inv_h = 1.0 / L.g.h;
  a.cD = G.cD;
  a.cNh = G.cN * L.g.h;
  constexpr int K = Pow3<D>::value;
  const size_t lds = (size_t)L.bc_gmax * (K + 1) * sizeof(double) +
                     (size_t)(2 * L.bc_smax + L.bc_gmax) * sizeof(T) +
                     ((size_t)L.bc_smax * 2 * D + (size_t)L.bc_gmax * (K + 1) + L.bc_opsmax) *
                         sizeof(int16_t);
  hipLaunchKernelGGL((k_band_chunk<D, T>), dim3(L.nchunks), dim3(256), lds, s, a);
  hipLaunchKernelGGL((k_band_scatter<T>), dim3(lin_grid(L.bc_nown)), dim3(256), 0, s, L.bc_own_node,
                     L.bc_nown, (const T*)out, u);
}

template <int D, typename T, typename TO>
void launch_defect(const DevLevel& L, const T* u, const T* rhs, TO* r, uint64_t* norms,
                   hipStream_t s) {
  const int nbt = L.ntiles ? tile_grid(L.ntiles) : 0;
  const int nb = nbt + (L.nghost ? lin_grid(L.nghost) : 0);
  if (!nb) return;
  hipLaunchKernelGGL((k_defect<D, T, TO>), dim3(nb), dim3(256), 0, s, L.tiles, L.ntiles, nbt,
                     L.ghosts, L.nghost, L.g, L.cls, u, rhs, r, (T)(1.0 / (L.g.h * L.g.h)),
                     1.0 / L.g.h, norms);
}

template <int D>
void launch_rhs_norm(const DevLevel& L, const double* rhs, uint64_t* norms, hipStream_t s) {
  if (L.ntiles)
    hipLaunchKernelGGL((k_rhs_norm<D>), dim3(tile_grid(L.ntiles)), dim3(256), 0, s, L.tiles,
                       L.ntiles, L.g, L.cls, rhs, norms);
}

template <typename T>
void launch_extend(const DevLevel& L, T* r, bool single_wg, int batch, hipStream_t s) {
  if (!L.next) return;
  if (single_wg) {
    hipLaunchKernelGGL((k_extend_wg<T>), dim3(batch), dim3(1024), 0, s, L.ext, L.dag_off,
                       L.dag_start, r);
    return;
  }
  for (size_t d = 0; d + 1 < L.gdag_off.size(); ++d) {
    const int a = L.gdag_off[d], b = L.gdag_off[d + 1];
    if (b > a)
      hipLaunchKernelGGL((k_extend_level<T>), dim3(lin_grid(b - a)), dim3(256), 0, s,
                         L.ext_merged, a, b, r);
  }
}

template <typename T>
void launch_extend_chunks(const DevLevel& L, T* r, hipStream_t s) {
  if (!L.nechunks) return;
  hipLaunchKernelGGL((k_extend_chunk<T>), dim3(L.nechunks), dim3(256), L.ec_smax * sizeof(double), s,
                     L.ec_off, L.ec_own, L.ec_next, L.ec_node, L.ec_src, L.ec_wt, L.ec_ops, L.ec_lvl,
                     L.ec_lvl_start, r);
}

template <int D, typename T>
void launch_restrict(const DevLevel& F, const DevLevel& C, const T* rf, T* rhsc, T* uc,
                     hipStream_t s) {
  if (C.ntiles)
    hipLaunchKernelGGL((k_restrict<D, T>), dim3(tile_grid(C.ntiles)), dim3(256), 0, s, C.tiles,
                       C.ntiles, C.g, F.g, C.rcode, rf, rhsc, uc);
}

template <int D, typename T>
void launch_prolong(const DevLevel& F, const DevLevel& C, const T* uc, T* uf, hipStream_t s) {
  if (F.ntiles)
    hipLaunchKernelGGL((k_prolong<D, T>), dim3(tile_grid(F.ntiles)), dim3(256), 0, s, F.tiles,
                       F.ntiles, F.g, C.g, F.cls, C.cls, uc, uf);
}

template <typename T>
void launch_coarse(const DevLevel& C, const T* rhs, T* u, int batch, hipStream_t s) {
  const int blocks = (C.nu_max + kCoarseRows - 1) / kCoarseRows;
  hipLaunchKernelGGL((k_coarse<T>), dim3(blocks, batch), dim3(256), C.nu_max * sizeof(double), s,
                     C.umap, C.umap_off, C.ainv_off, C.ainv, rhs, u);
}

template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_fill<T>), dim3(lin_grid(n)), dim3(256), 0, s, p, n, v);
}

template <int D>
void launch_pack(const DevLevel& L, const double* f, const double* g, const double* uin,
                 double* rhs, double* u, hipStream_t s) {
  if (L.ntiles)
    hipLaunchKernelGGL((k_pack<D>), dim3(tile_grid(L.ntiles)), dim3(256), 0, s, L.tiles, L.ntiles,
                       L.g, L.cls, f, g, uin, rhs, u);
}

template <int D>
void launch_unpack(const DevLevel& L, int batch, const double* src, double* dst, hipStream_t s) {
  const int64_t nnu = D == 3 ? (int64_t)L.g.np * L.g.np * L.g.np : (int64_t)L.g.np * L.g.np;
  const int64_t total = nnu * batch;
  hipLaunchKernelGGL((k_unpack<D>), dim3(lin_grid(total)), dim3(256), 0, s, total, L.g, L.cls, src,
                     dst);
}

template <int D>
void launch_dc_update(const DevLevel& L, double* u64, float* u32, hipStream_t s) {
  if (L.ntiles)
    hipLaunchKernelGGL((k_dc_update<D>), dim3(tile_grid(L.ntiles)), dim3(256), 0, s, L.tiles,
                       L.ntiles, L.g, L.cls, u64, u32);
}

#define GHOSTMG_INST(D, T)                                                                    \
  template void launch_smooth<D, T>(const DevLevel&, T*, const T*, hipStream_t);             \
  template void launch_band_chunks<D, T>(const DevLevel&, const mg_grid&, T*, const T*, T*,   \
                                         hipStream_t);                                        \
  template void launch_band<D, T>(const DevLevel&, const mg_grid&, T*, const T*, T*, bool, int, \
                                  hipStream_t);                                               \
  template void launch_defect<D, T, T>(const DevLevel&, const T*, const T*, T*, uint64_t*,    \
                                       hipStream_t);                                          \
  template void launch_restrict<D, T>(const DevLevel&, const DevLevel&, const T*, T*, T*,     \
                                      hipStream_t);                                           \
  template void launch_prolong<D, T>(const DevLevel&, const DevLevel&, const T*, T*, hipStream_t);

GHOSTMG_INST(2, double)
GHOSTMG_INST(2, float)
GHOSTMG_INST(3, double)
GHOSTMG_INST(3, float)
template void launch_defect<2, double, float>(const DevLevel&, const double*, const double*, float*,
                                              uint64_t*, hipStream_t);
template void launch_defect<3, double, float>(const DevLevel&, const double*, const double*, float*,
                                              uint64_t*, hipStream_t);
template void launch_extend<double>(const DevLevel&, double*, bool, int, hipStream_t);
template void launch_extend<float>(const DevLevel&, float*, bool, int, hipStream_t);
template void launch_extend_chunks<double>(const DevLevel&, double*, hipStream_t);
template void launch_extend_chunks<float>(const DevLevel&, float*, hipStream_t);
template void launch_coarse<double>(const DevLevel&, const double*, double*, int, hipStream_t);
template void launch_coarse<float>(const DevLevel&, const float*, float*, int, hipStream_t);
template void launch_fill<double>(double*, int64_t, double, hipStream_t);
template void launch_fill<float>(float*, int64_t, float, hipStream_t);
template void launch_fill<uint64_t>(uint64_t*, int64_t, uint64_t, hipStream_t);
template void launch_rhs_norm<2>(const DevLevel&, const double*, uint64_t*, hipStream_t);
template void launch_rhs_norm<3>(const DevLevel&, const double*, uint64_t*, hipStream_t);
template void launch_pack<2>(const DevLevel&, const double*, const double*, const double*, double*,
                             double*, hipStream_t);
template void launch_pack<3>(const DevLevel&, const double*, const double*, const double*, double*,
                             double*, hipStream_t);
template void launch_unpack<2>(const DevLevel&, int, const double*, double*, hipStream_t);
template void launch_unpack<3>(const DevLevel&, int, const double*, double*, hipStream_t);
template void launch_dc_update<2>(const DevLevel&, double*, float*, hipStream_t);
template void launch_dc_update<3>(const DevLevel&, double*, float*, hipStream_t);

}  // namespace ghostmg
