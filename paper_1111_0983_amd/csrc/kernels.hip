// Device kernels of the ghost-cell multigrid cycle (gfx950, wave64).
//
// Node arrays hold one level of every problem of the batch, padded rows (pitch multiple of
// 16), x fastest.  Node-parallel kernels walk a list of active tiles (tiles that hold at
// least one unknown); list kernels walk the compact ghost / band / extension records.
// Workgroups of a tile kernel are mapped so that each of the 8 XCDs takes a contiguous run
// of tiles (the dispatcher deals workgroups to XCDs round-robin), which keeps the halo
// rows a tile shares with its neighbours in one L2.
#include <algorithm>

#include "kernels.h"

namespace ghostmg {

__device__ __forceinline__ int xcd_tile(int b, int nb) {
  // nb is a multiple of 8: XCD k = b % 8 gets tiles [k nb/8, (k+1) nb/8)
  return (b & 7) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ bool in_box(int x, int y, int z, int np, int D) {
  return x >= 0 && x < np && y >= 0 && y < np && (D == 2 || (z >= 0 && z < np));
}

// Max of non-negative doubles through their IEEE bit patterns (order preserving).  The
// stored maximum only grows, so a value not above the one read first cannot change it: the
// atomic is skipped then (thousands of tiles of one problem would otherwise queue on one
// address), and the result is the same.
__device__ __forceinline__ void atomic_max_pos(uint64_t* dst, double v) {
  if (!(v == v)) v = __longlong_as_double(0x7ff0000000000000LL);  // NaN -> +inf
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const unsigned long long cur =
      __hip_atomic_load((unsigned long long*)dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (bits > cur) atomicMax((unsigned long long*)dst, bits);
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
// the two node updates of a relaxation, shared by every path that applies them
// ---------------------------------------------------------------------------------------
// interior node, Eq. (jac2d) as a correction: u_P + (h^2 f_P + sum_nb (u_nb - u_P)) / (2D);
// nb holds the neighbour values in the order x-, x+, y-, y+ (, z-, z+)
template <int D, typename T>
__device__ __forceinline__ T interior_update(T c, const T* nb, T f, T h2, T inv2d) {
  T s = (nb[0] - c) + (nb[1] - c);
  s += (nb[2] - c) + (nb[3] - c);
  if (D == 3) s += (nb[4] - c) + (nb[5] - c);
  return c + (h2 * f + s) * inv2d;
}

// ghost node, Eqs. (dir2d) / (neu2d): u_G + c_G (g_G - L_G u), with L_G u accumulated over
// the taps of nonzero weight in template order
template <typename T>
__device__ __forceinline__ T ghost_update(T uG, T gG, double Lu, double cG) {
  return (T)((double)uG + cG * ((double)gG - Lu));
}

// L_G u of ghost i from the global arrays
template <int D, typename T>
__device__ __forceinline__ double ghost_apply(const GhostRec& r, const double* __restrict__ w,
                                              const Geo& g, const T* __restrict__ u) {
  constexpr int K = Pow3<D>::value;
  // all weights, then all values (taps of zero weight read the ghost itself), then the sum
  double wv[K];
  T uv[K];
#pragma unroll
  for (int t = 0; t < K; ++t) wv[t] = w[t];
#pragma unroll
  for (int t = 0; t < K; ++t)
    uv[t] = u[wv[t] != 0.0 ? r.node + template_offset<D>(t, r.s, g.st) : r.node];
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < K; ++t)
    if (wv[t] != 0.0) acc += wv[t] * (double)uv[t];
  return acc;
}

// ---------------------------------------------------------------------------------------
// interpolation of the coarse error (Sec. 2.6.1): multilinear weights renormalised over the
// coarse nodes that carry an unknown; shared by the interpolation kernel and the relaxation
// that takes the correction while it stages its values
// ---------------------------------------------------------------------------------------
// num / den for the renormalised interpolation weights: den is 2^-k times the number of
// candidates that carry an unknown, so when it is a power of two the quotient is exactly a
// multiplication (the same bits as the division); only the other counts divide
template <typename T>
__device__ __forceinline__ T renorm_quotient(T num, T den) {
  if (den == (T)1) return num;
  if (den == (T)0.5) return num * (T)2;
  if (den == (T)0.25) return num * (T)4;
  if (den == (T)0.125) return num * (T)8;
  return num / den;
}

// u + sum_m w_m e_m / sum_m w_m over the candidates with an unknown (u unchanged if none)
template <int D, typename T>
__device__ __forceinline__ T prolong_correct(T u, const T* w, const int8_t* cc, const T* ec) {
  T num = 0, den = 0;
#pragma unroll
  for (int m = 0; m < (1 << D); ++m) {
    if (w[m] == (T)0 || cc[m] == 0) continue;
    num += w[m] * ec[m];
    den += w[m];
  }
  return den > (T)0 ? u + renorm_quotient<T>(num, den) : u;
}

// coarse patch under a tile and its 2-node ring (fused interpolation)
// The block of nodes one relaxation workgroup takes: a whole tile (SUB = 1) or, on levels
// with few tiles, one of the SUB^D parts of a tile halved along every axis (more workgroups,
// each with fewer serial passes; part origins stay even)
template <int D, int SUB>
struct RTile {
  static constexpr int X = Tile<D>::X / SUB, Y = Tile<D>::Y / SUB;
  static constexpr int Z = D == 3 ? Tile<D>::Z / SUB : 1;
  static constexpr int N = D == 3 ? SUB * SUB * SUB : SUB * SUB;  // parts per tile
};

// the coarse nodes the interpolation into a block (and its two-node ring) reads
template <int D, int SUB>
struct CPatch {
  static constexpr int X = RTile<D, SUB>::X / 2 + 3, Y = RTile<D, SUB>::Y / 2 + 3;
  static constexpr int Z = D == 3 ? RTile<D, SUB>::Z / 2 + 3 : 1;
};

constexpr int kRelaxPlain = 0, kRelaxProlong = 1, kRelaxRestrict = 2;

// bytes of the tile workgroup's auxiliary LDS area in each mode
template <int D, typename T, int MODE, int SUB>
constexpr size_t tile_aux_bytes() {
  using B = RTile<D, SUB>;
  constexpr int FX = B::X + 2, FY = B::Y + 2, FZ = D == 3 ? B::Z + 2 : 1;
  using CP = CPatch<D, SUB>;
  constexpr size_t coarse = (size_t)CP::X * CP::Y * CP::Z * sizeof(T);
  constexpr size_t fine = MODE == kRelaxRestrict
                              ? (size_t)(2 * FX + 1) * (2 * FY + 1) * sizeof(T) + FZ * FY * FX
                              : 0;
  return ((coarse > fine ? coarse : fine) + 15) / 16 * 16;
}

template <int D, typename T, int MODE, int SUB>
constexpr size_t tile_lds() {
  using B = RTile<D, SUB>;
  constexpr int UX = B::X + 4, UY = B::Y + 4, UZ = D == 3 ? B::Z + 4 : 1;
  constexpr int FX = B::X + 2, FY = B::Y + 2, FZ = D == 3 ? B::Z + 2 : 1;
  constexpr int NCN = CPatch<D, SUB>::X * CPatch<D, SUB>::Y * CPatch<D, SUB>::Z;
  return (size_t)(UZ * UY * UX + FZ * FY * FX) * sizeof(T) + tile_aux_bytes<D, T, MODE, SUB>() +
         (size_t)UZ * UY * UX + NCN;
}

// ---------------------------------------------------------------------------------------
// restriction of one coarse unknown (Sec. 2.5): the fine defect over the node's box with
// the tensor weights of Eqs. (restI), (restL), (restR).  rr holds the 3^D fine values around
// (2x, 2y, 2z) with x slowest; values outside the box get weight 0, which leaves the sum
// over the box, taken in the same order, unchanged.
// ---------------------------------------------------------------------------------------
template <int D, typename T>
__device__ __forceinline__ T restrict_box(uint8_t c, const T* rr) {
  constexpr int KT = Pow3<D>::value;
  // per axis the 1D factors of offsets -1, 0, +1 (0 outside the box): the same exact
  // products of (1,2,1)/4, (2,2)/4 or 1 as the box rule, in the same summation order
  T f[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool lo = a < D && (c >> (2 * a)) & 1, hi = a < D && (c >> (2 * a + 1)) & 1;
    f[a][0] = lo ? (hi ? (T)0.25 : (T)0.5) : (T)0;
    f[a][1] = lo && hi ? (T)0.5 : (lo || hi ? (T)0.5 : (T)1);
    f[a][2] = hi ? (lo ? (T)0.25 : (T)0.5) : (T)0;
  }
  T s = 0;
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int kx = q / (D == 3 ? 9 : 3), ky = (q / (D == 3 ? 3 : 1)) % 3;
    const int kz = D == 3 ? q % 3 : 1;
    const T w = D == 3 ? f[0][kx] * f[1][ky] * f[2][kz] : f[0][kx] * f[1][ky];
    s += w * rr[q];
  }
  return s;
}

// the 3^D fine values restrict_box reads for the coarse node whose (2x, 2y, 2z) is fine node
// F0; taps outside the node's box (which may lie outside the grid) read F0 itself
template <int D, typename T>
__device__ __forceinline__ void restrict_gather(const T* __restrict__ rf, int64_t F0,
                                                const Geo& gf, uint8_t c, T* rr) {
  constexpr int KT = Pow3<D>::value;
  const int lx = (c & 1) ? -1 : 0, hx = (c & 2) ? 1 : 0;
  const int ly = (c & 4) ? -1 : 0, hy = (c & 8) ? 1 : 0;
  const int lz = D == 3 && (c & 16) ? -1 : 0, hz = D == 3 && (c & 32) ? 1 : 0;
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int kx = q / (D == 3 ? 9 : 3) - 1, ky = (q / (D == 3 ? 3 : 1)) % 3 - 1;
    const int kz = D == 3 ? q % 3 - 1 : 0;
    const bool inbox = kx >= lx && kx <= hx && ky >= ly && ky <= hy && kz >= lz && kz <= hz;
    rr[q] = rf[inbox ? F0 + kx + gf.st[1] * ky + gf.st[2] * kz : F0];
  }
}

// One colour phase of a tile workgroup over the N nodes of one colour in a region that starts
// O nodes inside the U region along every axis and whose rows (y, z) hold HX nodes of that
// colour, HY rows per z: node r of the phase lies at x = 2 (r mod HX) + ((y + z + PAR) & 1)
// of its row.  Nodes whose code is not an interior one (1, 3) are left alone.
template <int D, typename T, int N, int HX, int HY, int O, int PAR, int NT = 256>
__device__ __forceinline__ void tile_colour_phase(T* su, const int8_t* sc, const T* sf, int FX,
                                                  int FY, int SY, int SZ, T h2, T inv2d,
                                                  int skip_band) {
  constexpr int K = (N + NT - 1) / NT;
  int ui[K];
  int8_t cd[K];
  T cv[K], fv[K], nb[K][2 * D];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r0 = (int)threadIdx.x + NT * k, r = r0 < N ? r0 : 0;
    const int row = r / HX, y = row % HY, z = row / HY;
    const int x = 2 * (r % HX) + ((y + z + PAR) & 1);
    // F index of the node (the F region starts one node inside the U region)
    const int fi = (x + O - 1) + FX * ((y + O - 1) + (D == 3 ? FY * (z + O - 1) : 0));
    ui[k] = (x + O) + SY * (y + O) + (D == 3 ? SZ * (z + O) : 0);
    cd[k] = r0 < N ? sc[ui[k]] : (int8_t)0;
    cv[k] = su[ui[k]];
    fv[k] = sf[fi];
    nb[k][0] = su[ui[k] - 1];
    nb[k][1] = su[ui[k] + 1];
    nb[k][2] = su[ui[k] - SY];
    nb[k][3] = su[ui[k] + SY];
    if constexpr (D == 3) {
      nb[k][4] = su[ui[k] - SZ];
      nb[k][5] = su[ui[k] + SZ];
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (cd[k] == 1 || (cd[k] == 3 && !skip_band))
      su[ui[k]] = interior_update<D, T>(cv[k], nb[k], fv[k], h2, inv2d);
}

// ---------------------------------------------------------------------------------------
// relaxation, interior tiles: red-black sweep of Eq. (jac2d), one tile per workgroup
// ---------------------------------------------------------------------------------------
// The tile and a ring of two nodes of uin are staged in LDS (with the coarse correction
// added when the relaxation follows an interpolation).  Red interior nodes of tile + ring
// one are relaxed first (they read only black, ghost or outside values, which this pass
// leaves unchanged), then the black interior nodes of the tile (which read the fresh red
// values).  The result is the global red sweep followed by the global black sweep; every
// workgroup writes its own block of uout (a tile, or a part of one: RTile): the interior
// nodes off the boundary band (the relaxation chunks write the band and the ghosts), or,
// with write_all, every unknown.
template <int D, typename T, int MODE, int SUB, int NT = 256>
__device__ void relax_tile(const RelaxArgs<T>& a, int tb, unsigned char* lds) {
  constexpr bool PROLONG = MODE == kRelaxProlong, RESTRICT = MODE == kRelaxRestrict;
  static_assert(!RESTRICT || D == 2, "the restriction is fused in 2D only");
  using B = RTile<D, SUB>;
  constexpr int TX = B::X, TY = B::Y, TZ = B::Z;
  constexpr int UX = TX + 4, UY = TY + 4, UZ = D == 3 ? TZ + 4 : 1;
  constexpr int FX = TX + 2, FY = TY + 2, FZ = D == 3 ? TZ + 2 : 1;
  constexpr int CX = CPatch<D, SUB>::X, CY = CPatch<D, SUB>::Y, CZ = CPatch<D, SUB>::Z;
  constexpr int NUN = UZ * UY * UX, NFN = FZ * FY * FX, NCN = CZ * CY * CX;
  T* su = (T*)lds;
  T* sf = su + NUN;
  // auxiliary area: the coarse patch (interpolation) or the fine defect patch and the
  // restriction codes (restriction)
  unsigned char* aux = (unsigned char*)(sf + NFN);
  T* sce = (T*)aux;
  int8_t* sc = (int8_t*)(aux + tile_aux_bytes<D, T, MODE, SUB>());  // codes of the U region
  int8_t* scc = sc + NUN;  // coarse classes of the patch
  // the parts of one tile are consecutive block numbers (the same XCD)
  const int part = xcd_tile(tb, a.nbt);
  if (part >= a.ntiles * B::N) return;
  const int tile = part / B::N, q = part % B::N;
  const Geo& g = a.g;
  const int4 t = a.tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  const int ox = t.y * Tile<D>::X + TX * (q % SUB), oy = t.z * Tile<D>::Y + TY * ((q / SUB) % SUB);
  const int oz = D == 3 ? t.w * Tile<D>::Z + TZ * (q / (SUB * SUB)) : 0;
  // every global load of the thread is issued before the first is used: positions outside
  // the box read the tile's first node and are replaced by zero afterwards
  constexpr int NU = (NUN + NT - 1) / NT, NF = (NFN + NT - 1) / NT, NC = (NCN + NT - 1) / NT;
  // fine defect patch under the F region (restriction): fine x from 2 ox - 3 to 2 ox + 2 TX + 1
  constexpr int RX = 2 * FX + 1, RY = 2 * FY + 1, NRN = RESTRICT ? RX * RY : 1;
  constexpr int NR = (NRN + NT - 1) / NT;
  T uv[NU], fv[NF], ev[NC], rpv[NR];
  int8_t cv[NU], fc[NF], ccv[NC];
  uint8_t rcv[NF];
  bool uok[NU], fok[NF], cok[NC];
  // the coarse patch first: it is staged after the U region, so it must not arrive last
  if constexpr (PROLONG) {
    const Geo& gc = a.gc;
    const int64_t cbase = (int64_t)t.x * gc.npp;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = threadIdx.x + NT * k;
      const int x = i % CX, y = (i / CX) % CY, z = i / (CX * CY);
      const int cx = ox / 2 - 1 + x, cy = oy / 2 - 1 + y, cz = D == 3 ? oz / 2 - 1 + z : 0;
      cok[k] = i < NCN && in_box(cx, cy, cz, gc.np, D);
      const int64_t ci = cok[k] ? cbase + cx + gc.st[1] * cy + gc.st[2] * cz : cbase;
      ev[k] = a.uc[ci];
      ccv[k] = a.clsc[ci];
    }
  }
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int i = threadIdx.x + NT * k;
    const int x = i % UX, y = (i / UX) % UY, z = i / (UX * UY);
    const int gx = ox + x - 2, gy = oy + y - 2, gz = D == 3 ? oz + z - 2 : 0;
    uok[k] = i < NUN && in_box(gx, gy, gz, g.np, D);
    const int64_t gi = uok[k] ? base + gx + g.st[1] * gy + g.st[2] * gz : base;
    uv[k] = RESTRICT ? (T)0 : a.uin[gi];
    cv[k] = a.rcls[gi];
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int i = threadIdx.x + NT * k;
    const int x = i % FX, y = (i / FX) % FY, z = i / (FX * FY);
    const int gx = ox + x - 1, gy = oy + y - 1, gz = D == 3 ? oz + z - 1 : 0;
    fok[k] = i < NFN && in_box(gx, gy, gz, g.np, D);
    const int64_t gi = fok[k] ? base + gx + g.st[1] * gy + g.st[2] * gz : base;
    fc[k] = a.rcls[gi];
    if constexpr (RESTRICT)
      rcv[k] = a.rcode[gi];
    else
      fv[k] = a.rhs[gi];
  }
  if constexpr (RESTRICT) {
    const int64_t fbase = (int64_t)t.x * a.gf.npp;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int i = threadIdx.x + NT * k;
      const int fx = 2 * ox - 3 + i % RX, fy = 2 * oy - 3 + i / RX;
      const bool ok = i < NRN && in_box(fx, fy, 0, a.gf.np, 2);
      rpv[k] = a.rf[ok ? fbase + fx + a.gf.st[1] * fy : fbase];
    }
  }
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < NUN) {
      su[i] = uok[k] ? uv[k] : (T)0;
      sc[i] = uok[k] ? cv[k] : (int8_t)0;
    }
  }
  if constexpr (RESTRICT) {
    // restricted right-hand side at every unknown of the F region, from the staged patch
    T* sr = (T*)aux;
    uint8_t* src = (uint8_t*)(sr + NRN);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int i = threadIdx.x + NT * k;
      if (i < NRN) sr[i] = rpv[k];
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int i = threadIdx.x + NT * k;
      if (i < NFN) src[i] = fok[k] ? rcv[k] : kNoUnknown;
    }
    __syncthreads();
    // two nodes per pass, every patch read issued before the first use (the 3 x 3 fine
    // neighbourhood of each F node lies inside the patch)
    for (int i0 = threadIdx.x; i0 < NFN; i0 += 512) {
      uint8_t c[2];
      T rr[2][9];
      int ii[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        ii[h] = i0 + NT * h < NFN ? i0 + NT * h : i0;
        c[h] = i0 + NT * h < NFN ? src[ii[h]] : kNoUnknown;
        const int x = ii[h] % FX, y = ii[h] / FX;
        const T* pp = sr + (2 * x + 1) + RX * (2 * y + 1);
#pragma unroll
        for (int q = 0; q < 9; ++q) rr[h][q] = pp[(q / 3 - 1) + RX * (q % 3 - 1)];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (i0 + NT * h < NFN) sf[ii[h]] = c[h] != kNoUnknown ? restrict_box<2, T>(c[h], rr[h]) : (T)0;
    }
    __syncthreads();  // sf is read below at positions other threads computed
    // the restricted right-hand side of the tile's unknowns, for the level's later launches
    for (int i = threadIdx.x; i < TX * TY; i += NT) {
      const int x = i % TX, y = i / TX;
      const int fi = (x + 1) + FX * (y + 1);
      if (src[fi] == kNoUnknown) continue;
      a.rhs_w[base + (ox + x) + g.st[1] * (oy + y)] = sf[fi];
    }
  } else {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int i = threadIdx.x + NT * k;
      if (i < NFN) {
        const int8_t c = fok[k] ? fc[k] : (int8_t)0;
        sf[i] = (c == 1 || c == 3) ? fv[k] : (T)0;
      }
    }
  }
  if constexpr (PROLONG) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = threadIdx.x + NT * k;
      if (i < NCN) {
        sce[i] = cok[k] ? ev[k] : (T)0;
        scc[i] = cok[k] ? ccv[k] : (int8_t)0;
      }
    }
    __syncthreads();
    // u + interpolated correction at every unknown of the U region.  Node j takes the coarse
    // nodes floor(j / 2) and, along each odd coordinate, the next one up (weight 2^-(odd
    // coordinates) each), over those that carry an unknown (Sec. 2.6.1).  Block origins are
    // even, so the U region splits into cells of 2^D fine nodes (x, y, z in {2c, 2c + 1}) that
    // all draw on the same 2^D coarse nodes c .. c + 1: a thread takes a cell, reads those
    // coarse values and codes once and corrects the cell's nodes.
    constexpr int CS[3] = {1, CX, CX * CY};
    constexpr int NCD = 1 << D;
    constexpr int KX = UX / 2, KY = UY / 2, KZ = D == 3 ? UZ / 2 : 1;
    constexpr int FS[3] = {1, UX, UX * UY};
    for (int cell = threadIdx.x; cell < KX * KY * KZ; cell += NT) {
      const int cx = cell % KX, cy = (cell / KX) % KY, cz = cell / (KX * KY);
      const int li0 = cx * CS[0] + cy * CS[1] + cz * CS[2];
      const int ui0 = 2 * cx * FS[0] + 2 * cy * FS[1] + 2 * cz * FS[2];
      int8_t cc[NCD], ucl[NCD];
      T ce[NCD], uo[NCD];
#pragma unroll
      for (int m = 0; m < NCD; ++m) {
        int li = li0, ui = ui0;
#pragma unroll
        for (int q = 0; q < D; ++q)
          if ((m >> q) & 1) li += CS[q], ui += FS[q];
        cc[m] = scc[li];
        ce[m] = sce[li];
        ucl[m] = sc[ui];
        uo[m] = su[ui];
      }
#pragma unroll
      for (int f = 0; f < NCD; ++f) {
        // fine node f of the cell: bit q set where its coordinate q is odd
        const int nodd = __builtin_popcount(f);  // 2^-(odd coordinates), exactly
        const T w1 = nodd == 0 ? (T)1 : nodd == 1 ? (T)0.5 : nodd == 2 ? (T)0.25 : (T)0.125;
        T num = 0, den = 0;
#pragma unroll
        for (int m = 0; m < NCD; ++m) {
          if ((m & f) != m) continue;  // candidate m moves along an even coordinate
          const bool ex = cc[m] != 0;
          num += ex ? w1 * ce[m] : (T)0;
          den += ex ? w1 : (T)0;
        }
        if (den > (T)0) num = renorm_quotient<T>(num, den);
        int ui = ui0;
#pragma unroll
        for (int q = 0; q < D; ++q)
          if ((f >> q) & 1) ui += FS[q];
        if (ucl[f] != 0 && den > (T)0) su[ui] = uo[f] + num;
      }
    }
  }
  __syncthreads();
  constexpr int SY = UX, SZ = UX * UY;
  // red nodes of the F region only (tile origins are even: node x of row (y, z) is red when
  // x + y + z + D is even), FX / 2 per row; then the black nodes of the tile only (x + y + z
  // odd), TX / 2 per row.  A thread issues the reads of all its nodes of a colour (codes
  // included) before the first update: a node of one colour reads only values of the other
  // colour, ghosts or outside nodes, which the phase leaves unchanged.
  constexpr int FXH = FX / 2, TXH = TX / 2;
  constexpr int NRED = FXH * FY * FZ, NBLK = TXH * TY * TZ;
  tile_colour_phase<D, T, NRED, FXH, FY, 1, (D & 1), NT>(su, sc, sf, FX, FY, SY, SZ, a.h2, a.inv2d,
                                                     a.skip_band);
  __syncthreads();
  tile_colour_phase<D, T, NBLK, TXH, TY, 2, 1, NT>(su, sc, sf, FX, FY, SY, SZ, a.h2, a.inv2d,
                                               a.skip_band);
  __syncthreads();
  // the block's nodes to uout: every code and value read before the first store
  constexpr int NST = TZ * TY * TX, KS = (NST + NT - 1) / NT;
  int8_t cst[KS];
  T vst[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int i0 = threadIdx.x + NT * k, i = i0 < NST ? i0 : 0;
    const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
    const int ui = (x + 2) + SY * (y + 2) + (D == 3 ? SZ * (z + 2) : 0);
    cst[k] = i0 < NST ? sc[ui] : (int8_t)0;
    vst[k] = su[ui];
  }
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int i = threadIdx.x + NT * k;
    const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
    if (cst[k] == 0 || (cst[k] != 1 && !a.write_all)) continue;
    a.uout[base + (ox + x) + g.st[1] * (oy + y) + g.st[2] * (D == 3 ? oz + z : 0)] = vst[k];
  }
}


// ---------------------------------------------------------------------------------------
// relaxation, boundary chunks: the whole relaxation of one chunk's node set
// ---------------------------------------------------------------------------------------
// The chunk's node set is closed under the dependencies of its owned nodes (band and
// ghost nodes) through the 3 + 3 lambda phases (red interior, black interior, ghosts; then
// lambda times red band, black band, ghosts, Sec. 3.2).  Its entries come in runs: updated
// ghosts, red-updated, black-updated, read-only; a thread holds one ghost, band_colour_slots(D)
// red and black entries and band_halo_slots(D) read-only entries (slot s of a run: entry
// tid + s * band_chunk_threads(D) of the run), with their node index, phase mask, neighbour ids,
// right-hand side and current value in registers (the ghost also its stencil ids, weights
// and constant); only the values are shared, in LDS.  A phase updates at most
// band_colour_slots(D) entries per thread (one ghost in a ghost phase) and issues all its LDS
// reads before its writes: no update reads a value of its own phase (red reads black and
// ghosts, black reads red and ghosts, the ghosts read the values before their phase).
// Phases are separated by workgroup barriers; a ghost phase computes every new ghost value
// before any is stored.  The owned entries are written to uout.
// One red or black phase of a relaxation chunk over the NC slots from S0: every active slot
// reads its neighbours (all reads before any write), then updates and stores its value.
template <int D, typename T, int NC, int S0, int NS>
__device__ __forceinline__ void band_colour_phase(int p, const uint32_t (&mask)[NS],
                                                  const int (&nbi)[NS][2 * D],
                                                  const int (&e_of)[NS], T (&uv)[NS],
                                                  const T (&rv)[NS], T* su, T h2, T inv2d) {
  bool act[NC];
  T nv[NC][2 * D];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    act[j] = (mask[S0 + j] >> p) & 1u;
    if (act[j]) {
#pragma unroll
      for (int q = 0; q < 2 * D; ++q) nv[j][q] = su[nbi[S0 + j][q]];
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    if (!act[j]) continue;
    uv[S0 + j] = interior_update<D, T>(uv[S0 + j], nv[j], rv[S0 + j], h2, inv2d);
    su[e_of[S0 + j]] = uv[S0 + j];
  }
}

template <int D, typename T, int MODE>
__device__ void relax_chunk(const RelaxArgs<T>& a, int c, unsigned char* lds) {
  constexpr bool PROLONG = MODE == kRelaxProlong, RESTRICT = MODE == kRelaxRestrict;
  constexpr int K = Pow3<D>::value;
  constexpr int NC = band_colour_slots(D), NH = band_halo_slots(D);
  constexpr int NS = 1 + 2 * NC + NH;  // slots: ghost, red, black, read-only
  constexpr int NCAND = 1 << D;
  constexpr bool FIXED = band_fixed_layout(D);
  constexpr int W = band_chunk_threads(D);
  const int cu = __builtin_amdgcn_readfirstlane(c);
  // packed layout: the header gives the entry count, the run lengths and the offsets; fixed
  // layout: every offset is a constant of the level and every run has its full slots
  int32_t hd[kBandHdr];
  if constexpr (FIXED) {
    const BandFixed F = band_fixed(D, true, true);  // offsets below PC / RS do not depend on them
    const int32_t base = cu * a.stride;
    hd[0] = F.NSW;
    hd[1] = 0;
    hd[2] = base;
    hd[3] = base + F.GID;
    hd[4] = base + F.GW;
    hd[5] = base + F.GC;
    hd[6] = base + F.PC;
    hd[7] = base + F.RS;
  } else {
#pragma unroll
    for (int q = 0; q < kBandHdr; ++q) hd[q] = a.hdr[(int64_t)cu * kBandHdr + q];
  }
  const uint32_t cnt = (uint32_t)hd[1];
  const int ns = hd[0];
  const int ng = FIXED ? W : (int)(cnt & 1023u), nr = FIXED ? NC * W : (int)((cnt >> 10) & 2047u);
  const int nb = FIXED ? NC * W : (int)(cnt >> 21);
  const int32_t* E = a.data + hd[2];
  const int tid = threadIdx.x;
  // slot s: its run start and length
  int e_of[NS];
  bool ok_of[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    int start, len, j;
    if (s == 0) {
      start = 0, len = ng, j = 0;
    } else if (s <= NC) {
      start = ng, len = nr, j = s - 1;
    } else if (s <= 2 * NC) {
      start = ng + nr, len = nb, j = s - 1 - NC;
    } else {
      start = ng + nr + nb, len = ns - ng - nr - nb, j = s - 1 - 2 * NC;
    }
    const int i = tid + j * W;
    ok_of[s] = i < len;
    e_of[s] = ok_of[s] ? start + i : 0;
  }
  int32_t node[NS];
  uint32_t mask[NS];
  int32_t nbw[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int ec = e_of[s];
    node[s] = E[ec];
    if constexpr (FIXED) {
      // empty slot positions hold node -1: they read node 0 (a valid index) and are never
      // stored (mask 0)
      ok_of[s] = node[s] >= 0;
      if (!ok_of[s]) node[s] = 0;
    }
    const uint32_t mk = (uint32_t)E[ns + ec];
    mask[s] = ok_of[s] ? mk : 0u;
    if (s >= 1 && s <= 2 * NC) {
#pragma unroll
      for (int q = 0; q < D; ++q) nbw[s][q] = E[2 * ns + ec * D + q];
    }
  }
  const bool ghost = ok_of[0];
  int32_t pcb[NS];
  int32_t rf0[NS], rcd[NS];
  if constexpr (RESTRICT) {
    // fine node index of (2x, 2y, 2z) and restriction code of every updated entry
    const int32_t* RS = a.data + hd[7];
#pragma unroll
    for (int s = 0; s < NS - NH; ++s) {
      rf0[s] = RS[2 * e_of[s]];
      rcd[s] = RS[2 * e_of[s] + 1];
    }
  }
  if constexpr (PROLONG) {
    // coarse index of every entry's interpolation candidate 0
    const int32_t* PC = a.data + hd[6];
#pragma unroll
    for (int s = 0; s < NS; ++s) pcb[s] = PC[e_of[s]];
  }
  T rv[NS], uv[NS];
  T* su = (T*)lds;
  if constexpr (RESTRICT) {
    // the relaxation starts from zero with the right-hand side restricted from the finer
    // level's defect (the tiles store it for the level's later launches)
    constexpr int KT = Pow3<D>::value;
    T rr[NS - NH][KT];
#pragma unroll
    for (int s = 0; s < NS - NH; ++s)
      restrict_gather<D, T>(a.rf, rf0[s], a.gf, (uint8_t)rcd[s], rr[s]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      uv[s] = 0;
      rv[s] = s < NS - NH ? restrict_box<D, T>((uint8_t)rcd[s], rr[s]) : (T)0;
    }
  } else {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      uv[s] = (((mask[s] >> 30) & 1u) ? a.uband : a.uin)[node[s]];
      rv[s] = s < NS - NH ? a.rhs[node[s]] : (T)0;
    }
  }
  if constexpr (PROLONG) {
    // candidate bits from the mask (odd coordinates, candidates with an unknown)
    const int P = a.phases;
    T pe[NS][NCAND];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const uint32_t cb = mask[s] >> (P + D);
#pragma unroll
      for (int m = 0; m < NCAND; ++m) {
        int idx = pcb[s];
#pragma unroll
        for (int q = 0; q < D; ++q)
          if ((m >> q) & 1) idx += (int)a.gc.st[q];
        pe[s][m] = a.uc[(cb >> m) & 1u ? idx : 0];
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      T w1 = 1;
      const int nodd = __popc((mask[s] >> P) & ((1u << D) - 1u));
      for (int q = 0; q < nodd; ++q) w1 *= (T)0.5;
      const uint32_t cb = mask[s] >> (P + D);
      T w[NCAND];
      int8_t cc[NCAND];
#pragma unroll
      for (int m = 0; m < NCAND; ++m) {
        w[m] = (cb >> m) & 1u ? w1 : (T)0;
        cc[m] = (cb >> m) & 1u ? 1 : 0;
      }
      uv[s] = prolong_correct<D, T>(uv[s], w, cc, pe[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (ok_of[s]) su[e_of[s]] = uv[s];
  // gs: the ghost values before the current ghost phase (the ghost rows read other ghosts
  // there, so that a ghost phase can store its new values into su without a second barrier)
  T* gs = su + ns;
  if (ghost) gs[tid] = uv[0];
  // the ghost rows are first needed in phase 2: loaded after the values (registers): the
  // LDS address of every tap (two per word) and the weights in the cycle's precision
  constexpr int KP = (K + 1) / 2;
  uint32_t gadp[KP];
  T gwt[K];
  double gc = 0.0;
  if (ng > 0) {
    const int tg = ghost ? tid : 0;
    const uint32_t* gi = (const uint32_t*)(a.data + hd[3]);
    const T* gw = (const T*)(a.data + hd[4]);
#pragma unroll
    for (int q = 0; q < KP; ++q) gadp[q] = gi[q * ng + tg];
#pragma unroll
    for (int q = 0; q < K; ++q) gwt[q] = gw[q * ng + tg];
    gc = ((const double*)(a.data + hd[5]))[tg];
  }
  __syncthreads();
  // neighbour ids of the red and black slots, decoded once
  int nbi[NS][2 * D];
#pragma unroll
  for (int s = 1; s <= 2 * NC; ++s)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      nbi[s][2 * q] = (int)(int16_t)((uint32_t)nbw[s][q] & 0xffffu);
      nbi[s][2 * q + 1] = (int)(int16_t)((uint32_t)nbw[s][q] >> 16);
    }
  // phases p, p + 1, p + 2 of every sweep: red, black, ghosts (the colour of a phase is
  // fixed, so every slot index below is a compile-time constant)
  for (int p = 0; p < a.phases; p += 3) {
    // the previous ghost phase's values become the snapshot (nothing reads gs until the
    // next ghost phase, two barriers later)
    if (ghost) gs[tid] = uv[0];
    band_colour_phase<D, T, NC, 1, NS>(p, mask, nbi, e_of, uv, rv, su, a.h2, a.inv2d);
    __syncthreads();
    band_colour_phase<D, T, NC, 1 + NC, NS>(p + 1, mask, nbi, e_of, uv, rv, su, a.h2, a.inv2d);
    __syncthreads();
    if (ghost && ((mask[0] >> (p + 2)) & 1u)) {
      // the row in groups of 9 taps, in tap order: the values of one group are read before
      // its products, and no more than one group is held (the whole 27-tap row would double
      // the registers of the 3D kernel and halve its occupancy)
      constexpr int KG = 9;
      T acc = 0;
#pragma unroll
      for (int q0 = 0; q0 < K; q0 += KG) {
        T gv[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q)
          gv[q] = su[(gadp[(q0 + q) >> 1] >> (16 * ((q0 + q) & 1))) & 0xffffu];
#pragma unroll
        for (int q = 0; q < KG; ++q) acc += gwt[q0 + q] * gv[q];
        __builtin_amdgcn_sched_barrier(0);
      }
      uv[0] = ghost_update<T>(uv[0], rv[0], (double)acc, gc);
      su[tid] = uv[0];
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < NS - NH; ++s)
    if (mask[s] >> 31) a.uout[node[s]] = uv[s];
}

// CHUNKS (2D): the launch also runs the level's relaxation chunks (workgroups
// [0, nchunks)).  MODE kRelaxProlong: the relaxation starts from the iterate plus the
// interpolated coarse correction; kRelaxRestrict: it starts from zero with the right-hand
// side restricted from the finer level's defect (and stores that right-hand side).  Each
// variant holds only the registers of the paths it runs.
template <int D, typename T, bool CHUNKS, int MODE, int SUB>
__global__ void __launch_bounds__(256) k_relax(RelaxArgs<T> a) {
  extern __shared__ __align__(16) unsigned char relax_smem[];
  static_assert(!CHUNKS || band_chunk_threads(D) == 256, "chunks sharing a launch with tiles");
  if constexpr (CHUNKS) {
    if ((int)blockIdx.x < a.nchunks) {
      relax_chunk<D, T, MODE>(a, blockIdx.x, relax_smem);
      return;
    }
  }
  relax_tile<D, T, MODE, SUB>(a, (int)blockIdx.x - (CHUNKS ? a.nchunks : 0), relax_smem);
}

// relaxation chunks in a launch of their own (3D: wider workgroups than the tiles')
template <int D, typename T>
__global__ void __launch_bounds__(band_chunk_threads(D)) k_relax_chunks(RelaxArgs<T> a) {
  extern __shared__ __align__(16) unsigned char relax_smem[];
  relax_chunk<D, T, kRelaxPlain>(a, blockIdx.x, relax_smem);
}

// 3D levels with few tiles: the tiles and the first launch's relaxation chunks share one
// launch of chunk-wide workgroups (workgroups [0, nchunks) the chunks, the rest one tile
// each, relaxed by all the workgroup's threads).  There the launch does not fill the chip,
// so the chunks' registers cost the tiles nothing, and a launch of its own is saved.
template <typename T>
__global__ void __launch_bounds__(band_chunk_threads(3)) k_relax_shared3(RelaxArgs<T> a) {
  extern __shared__ __align__(16) unsigned char relax_smem[];
  if ((int)blockIdx.x < a.nchunks)
    relax_chunk<3, T, kRelaxPlain>(a, blockIdx.x, relax_smem);
  else
    relax_tile<3, T, kRelaxPlain, 1, band_chunk_threads(3)>(a, (int)blockIdx.x - a.nchunks,
                                                             relax_smem);
}

// ---------------------------------------------------------------------------------------
// boundary relaxation one phase per launch (levels without relaxation chunks), in place
// ---------------------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(256) k_ghost_new(const GhostRec* __restrict__ gs,
                                                   const double* __restrict__ gw, int ng, Geo g,
                                                   const T* __restrict__ u, const T* __restrict__ rhs,
                                                   T* __restrict__ tmp, double cD, double cNh) {
  constexpr int K = Pow3<D>::value;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ng) return;
  const GhostRec r = gs[i];
  const double Lu = ghost_apply<D, T>(r, gw + (size_t)i * K, g, u);
  tmp[i] = ghost_update<T>(u[r.node], rhs[r.node], Lu, r.type ? cD : cNh);
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
  T nb[2 * D];
  nb[0] = u[P - 1];
  nb[1] = u[P + 1];
  nb[2] = u[P - g.st[1]];
  nb[3] = u[P + g.st[1]];
  if (D == 3) {
    nb[4] = u[P - g.st[2]];
    nb[5] = u[P + g.st[2]];
  }
  u[P] = interior_update<D, T>(u[P], nb, rhs[P], h2, inv2d);
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
  constexpr int K = Pow3<D>::value;
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
    for (int i = g0 + tid; i < g1; i += 1024) {
      const GhostRec r = a.ghosts[i];
      const double Lu = ghost_apply<D, T>(r, a.gw + (size_t)i * K, a.g, a.u);
      a.tmp[i] = ghost_update<T>(a.u[r.node], a.rhs[r.node], Lu, r.type ? a.cD : a.cNh);
    }
    __syncthreads();
    for (int i = g0 + tid; i < g1; i += 1024) a.u[a.ghosts[i].node] = a.tmp[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// the boundary relaxations the paper compares its own with (Sec. 3.3), one workgroup per
// problem: the band (interior nodes within delta, and the ghosts) colour by colour, a
// barrier between colours; no two rows (Kaczmarz) or blocks of a colour share an unknown, so
// the threads of a colour never touch the same value
// ---------------------------------------------------------------------------------------
// the taps of a ghost's stencil St_G (every rung's template, also where a weight vanishes)
template <int D>
__device__ __forceinline__ uint32_t used_taps(const GhostRec& r) {
  constexpr int K = Pow3<D>::value;
  uint32_t m = 0;
  if (r.rung <= 2) {
    for (int t = 0; t < K; ++t) {
      bool ok = true;
      int tt = t;
      for (int a = D - 1; a >= 0; --a) {
        if (r.rung == 2 && tt % 3 == 2) ok = false;
        tt /= 3;
      }
      if (ok) m |= 1u << t;
    }
  } else {
    m |= 1u;
    for (int a = 0; a < D; ++a) {
      if (r.rung == 4 && a != r.axis) continue;
      int ta = 1;
      for (int c = D - 1; c > a; --c) ta *= 3;
      m |= 1u << ta;
    }
  }
  return m;
}

// the equation of one node of Eq. (discr) as (node, weight) pairs: interior -Delta_h u = f as
// (2d u_P - sum of the neighbours) / h^2, ghost L_h u = g over its stencil; returns the count
template <int D>
__device__ __forceinline__ int node_row(int32_t P, int gid, const GhostRec* __restrict__ ghosts,
                                        const double* __restrict__ gw, const Geo& g, double ih2,
                                        int64_t* nd, double* w) {
  constexpr int K = Pow3<D>::value;
  if (gid < 0) {
    nd[0] = P;
    w[0] = 2.0 * D * ih2;
    int m = 1;
    for (int a = 0; a < D; ++a) {
      nd[m] = P - g.st[a];
      w[m++] = -ih2;
      nd[m] = P + g.st[a];
      w[m++] = -ih2;
    }
    return m;
  }
  const GhostRec r = ghosts[gid];
  const uint32_t used = used_taps<D>(r);
  int m = 0;
  for (int t = 0; t < K; ++t) {
    if (!((used >> t) & 1u)) continue;
    nd[m] = r.node + template_offset<D>(t, r.s, g.st);
    w[m++] = gw[(int64_t)gid * K + t];
  }
  return m;
}

// lambda Kaczmarz sweeps: u <- u + (f_j - <l_j, u>) / |l_j|^2 l_j row by row (the orthogonal
// projection onto the row's hyperplane), in FP64
template <int D, typename T>
__global__ void __launch_bounds__(256) k_band_kaczmarz(Geo g, const int2* __restrict__ list,
                                                       const int32_t* __restrict__ off, int ncol,
                                                       const GhostRec* __restrict__ ghosts,
                                                       const double* __restrict__ gw, T* u,
                                                       const T* __restrict__ rhs, int sweeps) {
  constexpr int K = Pow3<D>::value;
  const int32_t* o = off + (int64_t)blockIdx.x * (ncol + 1);
  const double ih2 = 1.0 / (g.h * g.h);
  for (int k = 0; k < sweeps; ++k)
    for (int c = 0; c < ncol; ++c) {
      for (int i = o[c] + (int)threadIdx.x; i < o[c + 1]; i += 256) {
        const int2 e = list[i];
        int64_t nd[K];
        double w[K];
        const int m = node_row<D>(e.x, e.y, ghosts, gw, g, ih2, nd, w);
        double dot = 0.0, n2 = 0.0;
        for (int q = 0; q < m; ++q) {
          dot += w[q] * (double)u[nd[q]];
          n2 += w[q] * w[q];
        }
        if (!(n2 > 0.0)) continue;
        const double a = ((double)rhs[e.x] - dot) / n2;
        for (int q = 0; q < m; ++q) u[nd[q]] = (T)((double)u[nd[q]] + a * w[q]);
      }
      __syncthreads();
    }
}

// index of the ghost at node P among ghosts [lo, hi) (ordered by node), or -1
__device__ __forceinline__ int find_ghost(const GhostRec* __restrict__ ghosts, int lo, int hi,
                                          int64_t P) {
  const int end = hi;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (ghosts[mid].node < P)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < end && ghosts[lo].node == P ? lo : -1;
}

// one block relaxation of every band node (2D): the unknowns of St_P (interior P: its 3 x 3
// neighbourhood within Omega_h u Gamma_h; ghost P: St_G) take the values that satisfy their
// own equations with every other unknown fixed (dense elimination with partial pivoting, in
// FP64 in LDS; a singular block is left unchanged)
constexpr int kBlockThreads = 64;
template <typename T>
__global__ void __launch_bounds__(kBlockThreads) k_band_block(Geo g, const int2* __restrict__ list,
                                                              const int32_t* __restrict__ off,
                                                              int ncol,
                                                              const GhostRec* __restrict__ ghosts,
                                                              const int32_t* __restrict__ ghost_off,
                                                              const double* __restrict__ gw,
                                                              const int8_t* __restrict__ cls, T* u,
                                                              const T* __restrict__ rhs) {
  constexpr int MB = 9;
  __shared__ double sA[kBlockThreads][MB][MB + 1];
  double(*A)[MB + 1] = sA[threadIdx.x];
  const int p = blockIdx.x;
  const int32_t* o = off + (int64_t)p * (ncol + 1);
  const int g0 = ghost_off[p], g1 = ghost_off[p + 1];
  const double ih2 = 1.0 / (g.h * g.h);
  const int64_t base = (int64_t)p * g.npp;
  for (int c = 0; c < ncol; ++c) {
    for (int i = o[c] + (int)threadIdx.x; i < o[c + 1]; i += kBlockThreads) {
      const int2 e = list[i];
      int64_t blk[MB];
      int m = 0;
      if (e.y < 0) {
        const int64_t loc = e.x - base;
        const int y = (int)(loc / g.st[1]), x = (int)(loc - y * g.st[1]);
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int xx = x + dx, yy = y + dy;
            if (xx < 0 || yy < 0 || xx > g.n || yy > g.n) continue;
            const int64_t Q = base + xx + g.st[1] * yy;
            if (cls[Q] != 0) blk[m++] = Q;
          }
      } else {
        const GhostRec r = ghosts[e.y];
        const uint32_t used = used_taps<2>(r);
        for (int t = 0; t < 9; ++t)
          if ((used >> t) & 1u) blk[m++] = r.node + template_offset<2>(t, r.s, g.st);
      }
      for (int q = 0; q < m; ++q) {
        const int gid = cls[blk[q]] == 2 ? find_ghost(ghosts, g0, g1, blk[q]) : -1;
        int64_t nd[9];
        double w[9];
        const int nr = node_row<2>((int32_t)blk[q], gid, ghosts, gw, g, ih2, nd, w);
        for (int cc = 0; cc <= m; ++cc) A[q][cc] = 0.0;
        A[q][m] = (double)rhs[blk[q]];
        for (int k = 0; k < nr; ++k) {
          int col = -1;
          for (int b = 0; b < m; ++b)
            if (blk[b] == nd[k]) col = b;
          if (col >= 0)
            A[q][col] += w[k];
          else
            A[q][m] -= w[k] * (double)u[nd[k]];
        }
      }
      bool singular = false;
      for (int k = 0; k < m && !singular; ++k) {
        int pv = k;
        for (int r = k + 1; r < m; ++r)
          if (fabs(A[r][k]) > fabs(A[pv][k])) pv = r;
        if (A[pv][k] == 0.0) {
          singular = true;
          break;
        }
        if (pv != k)
          for (int cc = 0; cc <= m; ++cc) {
            const double t = A[k][cc];
            A[k][cc] = A[pv][cc];
            A[pv][cc] = t;
          }
        for (int r = k + 1; r < m; ++r) {
          const double f = A[r][k] / A[k][k];
          for (int cc = k; cc <= m; ++cc) A[r][cc] -= f * A[k][cc];
        }
      }
      if (singular) continue;
      double x[MB];
      for (int r = m - 1; r >= 0; --r) {
        double t = A[r][m];
        for (int cc = r + 1; cc < m; ++cc) t -= A[r][cc] * x[cc];
        x[r] = t / A[r][r];
      }
      for (int q = 0; q < m; ++q) u[blk[q]] = (T)x[q];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// defect (Sec. 2.4 step 3) with per-problem infinity norms, and its extension outside
// Omega_h, Eq. (exp) in its steady state
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

// Extension chunk: the chunk's terms are staged in LDS while the defects of its ghost
// sources are evaluated from u (the same arithmetic as the ghost rows of the defect, rounded
// to the defect's type as when stored), one per thread; then every owned extension node
// takes its composed combination of them (FP64, terms in ascending ghost order) and is
// written to r.
template <int D, typename T, typename TO>
__device__ void extend_chunk(const DefectArgs<T, TO>& a, int c, unsigned char* lds) {
  constexpr int K = Pow3<D>::value;
  constexpr int NK = kExtPerThread;
  constexpr int NT = kExtMaxTerms / kExtThreads;
  const int cu = __builtin_amdgcn_readfirstlane(c);
  // fixed layout: every address below is known before the header (the counts) arrives
  constexpr ExtFixed F = ext_fixed(D);
  constexpr int GS = kExtMaxGhosts;
  const int32_t* E = a.data + (int64_t)cu * a.stride;
  const int32_t* N = E;
  const int32_t* TOF = E + F.TO;
  const int32_t* TS = E + F.TS;
  const double* TW = (const double*)(E + F.TW);
  const int32_t* gn = E + F.GN;
  const double* gw = (const double*)(E + F.GW);
  const int tid = threadIdx.x;
  // every global load of the chunk is issued before the first use (positions beyond the
  // counts hold node 0, weight 0 and the last term offset)
  int32_t node[NK], t0[NK], t1[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int e = tid + k * kExtThreads;
    node[k] = N[GS + e];
    t0[k] = TOF[e];
    t1[k] = TOF[e + 1];
  }
  double tw[NT];
  int32_t ts[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int i = tid + j * kExtThreads;
    tw[j] = TW[i];
    ts[j] = TS[i];
  }
  // the first pass of ghost rows (sources tid)
  int32_t gnode[K];
  double gwt[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    gnode[q] = gn[q * GS + tid];
    gwt[q] = gw[q * GS + tid];
  }
  const int32_t self0 = N[tid];
  const int ne = a.hdr[(int64_t)cu * kExtHdr], ngs = a.hdr[(int64_t)cu * kExtHdr + 1];
  const int nterms = TOF[ne];
  double* sv = (double*)lds;
  double* lw = sv + ngs;
  int32_t* ls = (int32_t*)(lw + nterms);
  // ghost sources tid, tid + kExtThreads, ... (a second pass only where a chunk has more
  // sources than threads)
  for (int g0 = 0; g0 < ngs; g0 += kExtThreads) {
    const bool gsrc = g0 + tid < ngs;
    const int tg = g0 + tid;  // < kExtMaxGhosts: positions beyond ngs hold zeros
    if (g0 > 0) {
#pragma unroll
      for (int q = 0; q < K; ++q) {
        gnode[q] = gn[q * GS + tg];
        gwt[q] = gw[q * GS + tg];
      }
    }
    const int32_t self = g0 > 0 ? N[tg] : self0;
    double uq[K];
#pragma unroll
    for (int q = 0; q < K; ++q) uq[q] = (double)a.u[gnode[q]];
    const double rG = (double)a.rhs[self];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q)
      if (gwt[q] != 0.0) acc += gwt[q] * uq[q];
    if (gsrc) sv[g0 + tid] = (double)(TO)(rG - acc);
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int i = tid + j * kExtThreads;
    if (i < nterms) {
      lw[i] = tw[j];
      ls[i] = ts[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (tid + k * kExtThreads >= ne) continue;
    double v = 0.0;
    for (int t = t0[k]; t < t1[k]; ++t) v += lw[t] * sv[ls[t]];
    a.r[node[k]] = (TO)v;
  }
}

// Interior rows of one 3D tile: u over the tile and a one-node ring is staged in LDS (one
// coalesced round of loads, 1.76 values per node instead of up to seven global loads per
// node), f and the node codes are read directly.  Nodes outside the box are never read by
// an interior node (the domain does not touch the box), so ring positions outside it hold
// any value.  The arithmetic and its order are those of the direct path.
template <typename T, typename TO>
__device__ void defect_tile3(const DefectArgs<T, TO>& a, int b, double* red) {
  constexpr int TX = Tile<3>::X, TY = Tile<3>::Y, TZ = Tile<3>::Z;
  constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2, NS = SX * SY * SZ;
  constexpr int NL = (NS + 255) / 256, NK = TX * TY * TZ / 256;
  __shared__ T su[NS];
  const int tile = xcd_tile(b, a.nbt);
  if (tile >= a.ntiles) return;
  const Geo& g = a.g;
  const int4 t = a.tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  const int ox = t.y * TX - 1, oy = t.z * TY - 1, oz = t.w * TZ - 1;
  T lv[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = ox + i % SX, y = oy + (i / SX) % SY, z = oz + i / (SX * SY);
    const bool in = i < NS && in_box(x, y, z, g.np, 3);
    lv[k] = a.u[in ? base + x + g.st[1] * y + g.st[2] * z : base];
  }
  int64_t P[NK];
  bool ok[NK];
  int8_t cl[NK];
  T f[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY, z = t.w * TZ + i / (TX * TY);
    ok[k] = in_box(x, y, z, g.np, 3);
    P[k] = ok[k] ? base + x + g.st[1] * y + g.st[2] * z : base;
    cl[k] = a.cls[P[k]];
    f[k] = a.rhs[P[k]];
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NS) su[i] = lv[k];
  }
  __syncthreads();
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (!ok[k] || cl[k] != 1) continue;
    const int i = threadIdx.x + 256 * k;
    const int li = (i % TX + 1) + SX * ((i / TX) % TY + 1) + SX * SY * (i / (TX * TY) + 1);
    const T c = su[li];
    T s = (su[li - 1] - c) + (su[li + 1] - c);
    s += (su[li - SX] - c) + (su[li + SX] - c);
    s += (su[li - SX * SY] - c) + (su[li + SX * SY] - c);
    const T v = f[k] + s * a.inv_h2;
    a.r[P[k]] = (TO)v;
    m = fmax(m, fabs((double)v));
    if (!(v == v)) m = __longlong_as_double(0x7ff0000000000000LL);
  }
  if (a.norms) {
    m = block_max(m, red);
    if (threadIdx.x == 0) atomic_max_pos(&a.norms[2 * t.x], m);
  }
}

// One launch: extension chunks, then the active tiles (interior rows), then the ghost
// records (boundary rows).  Per-problem maxima of |r| go to norms[2p] (interior) and
// norms[2p + 1] (ghosts) through order-independent integer maxima, so the result is
// deterministic.
template <int D, typename T, typename TO>
__global__ void __launch_bounds__(256) k_defect(DefectArgs<T, TO> a) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  constexpr int K = Pow3<D>::value;
  extern __shared__ __align__(16) unsigned char defect_smem[];
  __shared__ double red[4];
  int b = blockIdx.x;
  // extension chunks exist in 2D only (3D extends with a gather after this launch); keeping
  // their registers out of the 3D instantiation leaves its tiles at full occupancy
  if constexpr (D == 2) {
    if (b < a.nechunks) {
      extend_chunk<D, T, TO>(a, b, defect_smem);
      return;
    }
    b -= a.nechunks;
  }
  const Geo& g = a.g;
  if constexpr (D == 3) {
    if (b < a.nbt) {
      defect_tile3<T, TO>(a, b, red);
      return;
    }
  }
  if (b < a.nbt) {
    const int tile = xcd_tile(b, a.nbt);
    if (tile >= a.ntiles) return;
    const int4 t = a.tiles[tile];
    const int64_t base = (int64_t)t.x * g.npp;
    constexpr int NK = TZ * TY * TX / 256;
    int64_t P[NK];
    bool ok[NK];
    int8_t cl[NK];
    T uc[NK], f[NK], un[NK][2 * D];
    // all loads first (neighbours outside the box read the node itself)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int i = threadIdx.x + 256 * k;
      const int j[3] = {t.y * TX + i % TX, t.z * TY + (i / TX) % TY, D == 3 ? t.w * TZ + i / (TX * TY) : 0};
      ok[k] = in_box(j[0], j[1], j[2], g.np, D);
      P[k] = ok[k] ? base + j[0] + g.st[1] * j[1] + g.st[2] * j[2] : base;
      cl[k] = a.cls[P[k]];
      uc[k] = a.u[P[k]];
      f[k] = a.rhs[P[k]];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        un[k][2 * q] = a.u[ok[k] && j[q] > 0 ? P[k] - g.st[q] : P[k]];
        un[k][2 * q + 1] = a.u[ok[k] && j[q] < g.np - 1 ? P[k] + g.st[q] : P[k]];
      }
    }
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      if (!ok[k] || cl[k] != 1) continue;
      const T c = uc[k];
      T s = (un[k][0] - c) + (un[k][1] - c);
      s += (un[k][2] - c) + (un[k][3] - c);
      if (D == 3) s += (un[k][4] - c) + (un[k][5] - c);
      const T v = f[k] + s * a.inv_h2;
      a.r[P[k]] = (TO)v;
      m = fmax(m, fabs((double)v));
      if (!(v == v)) m = __longlong_as_double(0x7ff0000000000000LL);
    }
    if (a.norms) {
      m = block_max(m, red);
      if (threadIdx.x == 0) atomic_max_pos(&a.norms[2 * t.x], m);
    }
    return;
  }
  const int i = (b - a.nbt) * 256 + threadIdx.x;
  int p = -1;
  double m = 0.0;
  if (i < a.nghost) {
    const GhostRec rec = a.ghosts[i];
    const double v = (double)a.rhs[rec.node] - ghost_apply<D, T>(rec, a.gw + (size_t)i * K, g, a.u);
    a.r[rec.node] = (TO)v;
    if (a.rg) a.rg[i] = (TO)v;
    p = (int)(rec.node / g.npp);
    m = fabs(v);
    if (!(m == m)) m = __longlong_as_double(0x7ff0000000000000LL);
  }
  if (!a.norms) return;
  // one atomic per wave when its ghosts all belong to one problem (ghosts are ordered by
  // problem, so this is the common case)
  const int p0 = __shfl(p, 0);
  if (__all(p == p0 || p < 0)) {
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0 && p0 >= 0) atomic_max_pos(&a.norms[2 * p0 + 1], m);
  } else if (p >= 0) {
    atomic_max_pos(&a.norms[2 * p + 1], m);
  }
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
  constexpr int NK = TZ * TY * TX / 256;
  bool ok[NK];
  int8_t c[NK];
  double f[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    ok[k] = in_box(x, y, z, g.np, D);
    const int64_t P = ok[k] ? base + x + g.st[1] * y + g.st[2] * z : base;
    c[k] = cls[P];
    f[k] = rhs[P];
  }
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (!ok[k] || c[k] == 0) continue;
    m = fmax(m, fabs(f[k]));
    if (!(f[k] == f[k])) m = __longlong_as_double(0x7ff0000000000000LL);
  }
  m = block_max(m, red);
  if (threadIdx.x == 0) atomic_max_pos(&norms[2 * t.x], m);
}

// extension without chunks: one workgroup per problem with DAG levels separated by
// barriers, or one launch per DAG level
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
  constexpr int KT = Pow3<D>::value;
  constexpr int NK = TZ * TY * TX / 256;
  constexpr int NB = D == 2 ? NK : 1;  // coarse nodes whose fine taps are loaded together
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t basec = (int64_t)t.x * gc.npp, basef = (int64_t)t.x * gf.npp;
#pragma unroll
  for (int k0 = 0; k0 < NK; k0 += NB) {
    int64_t X[NB];
    bool ok[NB];
    uint8_t cd[NB];
    T rv[NB][KT];
    // the 3^D fine neighbourhood of every coarse node is loaded before any is used (taps
    // outside the fine box read the centre); taps outside the node's box get weight 0,
    // which leaves the sum over the box, taken in the same order, unchanged
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int i = threadIdx.x + 256 * (k0 + k);
      const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
      const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
      ok[k] = in_box(x, y, z, gc.np, D);
      X[k] = ok[k] ? basec + x + gc.st[1] * y + gc.st[2] * z : basec;
      cd[k] = code[X[k]];
      const int fx = 2 * x, fy = 2 * y, fz = 2 * z;
      const int64_t F0 = basef + fx + gf.st[1] * fy + gf.st[2] * fz;
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        const int kx = q / (D == 3 ? 9 : 3) - 1, ky = (q / (D == 3 ? 3 : 1)) % 3 - 1;
        const int kz = D == 3 ? q % 3 - 1 : 0;
        const bool in = ok[k] && in_box(fx + kx, fy + ky, fz + kz, gf.np, D);
        rv[k][q] = rf[in ? F0 + kx + gf.st[1] * ky + gf.st[2] * kz : (ok[k] ? F0 : basef)];
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!ok[k]) continue;
      uc[X[k]] = (T)0;
      const uint8_t c = cd[k];
      if (c == kNoUnknown) continue;
      rhsc[X[k]] = restrict_box<D, T>(c, rv[k]);
    }
  }
}

// 3D: one workgroup per part of a coarse tile (RTile<D, 2>: 8 x 4 x 4 coarse nodes): the
// fine defect patch under the part (fine nodes 2o - 1 .. 2(o + B) - 1 per axis) is staged in
// LDS in one round of loads, then a thread restricts one coarse node from it (values outside
// the fine grid are staged as 0; they, like every tap outside a node's box, get weight 0).
template <int D, typename T>
__global__ void __launch_bounds__(256) k_restrict_parts(const int4* __restrict__ tiles, int ntiles,
                                                        Geo gc, Geo gf,
                                                        const uint8_t* __restrict__ code,
                                                        const T* __restrict__ rf,
                                                        T* __restrict__ rhsc, T* __restrict__ uc) {
  using B = RTile<D, 2>;
  constexpr int BX = B::X, BY = B::Y, BZ = B::Z;
  static_assert(BX * BY * BZ <= 256, "one coarse node per thread");
  constexpr int PX = 2 * BX + 1, PY = 2 * BY + 1, PZ = D == 3 ? 2 * BZ + 1 : 1;
  constexpr int NP = PX * PY * PZ, NL = (NP + 255) / 256;
  constexpr int KT = Pow3<D>::value;
  __shared__ T sp[NP];
  const int part = xcd_tile(blockIdx.x, gridDim.x);
  if (part >= ntiles * B::N) return;
  const int tile = part / B::N, q = part % B::N;
  const int4 t = tiles[tile];
  const int64_t basec = (int64_t)t.x * gc.npp, basef = (int64_t)t.x * gf.npp;
  const int ox = t.y * Tile<D>::X + BX * (q % 2), oy = t.z * Tile<D>::Y + BY * ((q / 2) % 2);
  const int oz = D == 3 ? t.w * Tile<D>::Z + BZ * (q / 4) : 0;
  T pv[NL];
  bool pok[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int fx = 2 * ox - 1 + i % PX, fy = 2 * oy - 1 + (i / PX) % PY;
    const int fz = D == 3 ? 2 * oz - 1 + i / (PX * PY) : 0;
    pok[k] = i < NP && in_box(fx, fy, fz, gf.np, D);
    pv[k] = rf[pok[k] ? basef + fx + gf.st[1] * fy + gf.st[2] * fz : basef];
  }
  const int lx = threadIdx.x % BX, ly = (threadIdx.x / BX) % BY, lz = threadIdx.x / (BX * BY);
  const int cx = ox + lx, cy = oy + ly, cz = D == 3 ? oz + lz : 0;
  const bool cok = (int)threadIdx.x < BX * BY * BZ && in_box(cx, cy, cz, gc.np, D);
  const int64_t X = cok ? basec + cx + gc.st[1] * cy + gc.st[2] * cz : basec;
  const uint8_t cd = code[X];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NP) sp[i] = pok[k] ? pv[k] : (T)0;
  }
  __syncthreads();
  if (!cok) return;
  uc[X] = (T)0;
  if (cd == kNoUnknown) return;
  // the 3^D fine values around (2x, 2y, 2z), x slowest (the order restrict_box takes)
  T rr[KT];
#pragma unroll
  for (int qq = 0; qq < KT; ++qq) {
    const int kx = qq / (D == 3 ? 9 : 3), ky = (qq / (D == 3 ? 3 : 1)) % 3;
    const int kz = D == 3 ? qq % 3 : 0;
    rr[qq] = sp[(2 * lx + kx) + PX * ((2 * ly + ky) + PY * (D == 3 ? 2 * lz + kz : 0))];
  }
  rhsc[X] = restrict_box<D, T>(cd, rr);
}

// ---------------------------------------------------------------------------------------
// interpolation of the coarse error and correction of the fine unknowns (Sec. 2.6.1):
// multilinear weights renormalised over the coarse nodes that carry an unknown
// ---------------------------------------------------------------------------------------
// One workgroup per fine tile: the tile's values and codes and the coarse patch under it
// (coarse nodes o/2 .. o/2 + T/2 per axis, tile origins o even) are staged in LDS; a thread
// takes a coarse cell, whose 2^D fine nodes (coordinates 2c, 2c + 1) all draw on the same 2^D
// coarse nodes, and corrects them; the tile is then stored back.
template <int D, typename T>
__global__ void __launch_bounds__(256) k_prolong(const int4* __restrict__ tiles, int ntiles, Geo gf,
                                                 Geo gc, const int8_t* __restrict__ clsf,
                                                 const int8_t* __restrict__ clsc,
                                                 const T* __restrict__ uc, T* __restrict__ uf) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  constexpr int NF = TZ * TY * TX, NK = NF / 256;
  constexpr int CX = TX / 2 + 1, CY = TY / 2 + 1, CZ = D == 3 ? TZ / 2 + 1 : 1;
  constexpr int NC = CX * CY * CZ, KC = (NC + 255) / 256;
  constexpr int NCD = 1 << D;
  __shared__ T sfu[NF];
  __shared__ int8_t sfc[NF];
  __shared__ T scu[NC];
  __shared__ int8_t scc[NC];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t basef = (int64_t)t.x * gf.npp, basec = (int64_t)t.x * gc.npp;
  const int ox = t.y * TX, oy = t.z * TY, oz = D == 3 ? t.w * TZ : 0;
  // every global load first (positions outside the box read the first node, code 0)
  int64_t P[NK];
  bool ok[NK];
  T fv[NK];
  int8_t fc[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = ox + i % TX, y = oy + (i / TX) % TY, z = D == 3 ? oz + i / (TX * TY) : 0;
    ok[k] = in_box(x, y, z, gf.np, D);
    P[k] = ok[k] ? basef + x + gf.st[1] * y + gf.st[2] * z : basef;
    fv[k] = uf[P[k]];
    fc[k] = clsf[P[k]];
  }
  T cv[KC];
  int8_t ccv[KC];
  bool cok[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = ox / 2 + i % CX, y = oy / 2 + (i / CX) % CY, z = D == 3 ? oz / 2 + i / (CX * CY) : 0;
    cok[k] = i < NC && in_box(x, y, z, gc.np, D);
    const int64_t X = cok[k] ? basec + x + gc.st[1] * y + gc.st[2] * z : basec;
    cv[k] = uc[X];
    ccv[k] = clsc[X];
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    sfu[i] = fv[k];
    sfc[i] = ok[k] ? fc[k] : (int8_t)0;
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NC) {
      scu[i] = cok[k] ? cv[k] : (T)0;
      scc[i] = cok[k] ? ccv[k] : (int8_t)0;
    }
  }
  __syncthreads();
  constexpr int KX = TX / 2, KY = TY / 2, KZ = D == 3 ? TZ / 2 : 1;
  constexpr int CS[3] = {1, CX, CX * CY}, FS[3] = {1, TX, TX * TY};
  for (int cell = threadIdx.x; cell < KX * KY * KZ; cell += 256) {
    const int cx = cell % KX, cy = (cell / KX) % KY, cz = cell / (KX * KY);
    const int li0 = cx * CS[0] + cy * CS[1] + cz * CS[2];
    const int fi0 = 2 * cx * FS[0] + 2 * cy * FS[1] + 2 * cz * FS[2];
    int8_t cc[NCD], ucl[NCD];
    T ce[NCD], uo[NCD];
#pragma unroll
    for (int m = 0; m < NCD; ++m) {
      int li = li0, fi = fi0;
#pragma unroll
      for (int q = 0; q < D; ++q)
        if ((m >> q) & 1) li += CS[q], fi += FS[q];
      cc[m] = scc[li];
      ce[m] = scu[li];
      ucl[m] = sfc[fi];
      uo[m] = sfu[fi];
    }
#pragma unroll
    for (int f = 0; f < NCD; ++f) {
      // fine node f of the cell (bit q: odd coordinate q), weight 2^-(odd coordinates) on
      // each candidate that carries an unknown, renormalised (the order of prolong_correct)
      const int nodd = __builtin_popcount(f);
      const T w1 = nodd == 0 ? (T)1 : nodd == 1 ? (T)0.5 : nodd == 2 ? (T)0.25 : (T)0.125;
      T num = 0, den = 0;
#pragma unroll
      for (int m = 0; m < NCD; ++m) {
        if ((m & f) != m || cc[m] == 0) continue;
        num += w1 * ce[m];
        den += w1;
      }
      int fi = fi0;
#pragma unroll
      for (int q = 0; q < D; ++q)
        if ((f >> q) & 1) fi += FS[q];
      if (ucl[f] != 0 && den > (T)0) sfu[fi] = uo[f] + renorm_quotient<T>(num, den);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (ok[k] && fc[k] != 0) uf[P[k]] = sfu[i];
  }
}

// ---------------------------------------------------------------------------------------
// exact solve on the coarsest grid: e = A_c^{-1} b in FP64 in either cycle precision (the
// FP32 cycles of the defect correction round only the result into their iterate), one row
// per wave, kCoarseRows rows per workgroup, b (FP64, compact by unknown) staged in LDS.
// When the level has just been entered, b is first restricted (Sec. 2.5) from the finer
// level's defect by k_coarse_restrict, one thread per coarse unknown (its finer node
// (2x, 2y, 2z) and restriction code precomputed), the box sum taken in FP64; on a hierarchy
// of one level, k_coarse_gather takes b from the level's right-hand side.
// ---------------------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(256) k_coarse_restrict(CoarseArgs<T> a, int ntot) {
  constexpr int KT = Pow3<D>::value;
  const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (i >= ntot) return;
  const uint8_t c = a.ucode[i];
  T rr[KT];
  restrict_gather<D, T>(a.rf, a.ufine[i], a.gf, c, rr);
  double rd[KT];
#pragma unroll
  for (int q = 0; q < KT; ++q) rd[q] = (double)rr[q];
  a.rhsc[i] = restrict_box<D, double>(c, rd);
}

template <typename T>
__global__ void __launch_bounds__(256) k_coarse_gather(CoarseArgs<T> a, int ntot) {
  const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (i < ntot) a.rhsc[i] = (double)a.rhs[a.umap[i]];
}

template <typename T>
__global__ void __launch_bounds__(kCoarseRows * 64) k_coarse(CoarseArgs<T> a) {
  constexpr int NT = kCoarseRows * 64;
  constexpr int NQ = 16;  // loads of the row in flight per lane (the stream is latency-bound)
  extern __shared__ double bsh[];
  const int p = blockIdx.y;
  const int a0 = a.umap_off[p], nu = a.umap_off[p + 1] - a0;
  const int row0 = (int)blockIdx.x * kCoarseRows;
  if (row0 >= nu) return;
  for (int i = (int)threadIdx.x; i < nu; i += NT) bsh[i] = a.rhsc[a0 + i];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = row0 + w;
  if (r >= nu) return;
  const double* Ar = a.ainv + a.ainv_off[p] + (int64_t)r * nu;
  double acc = 0.0;
  for (int j0 = 0; j0 < nu; j0 += NQ * 64) {
    double av[NQ], bv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = j0 + lane + 64 * q;
      av[q] = j < nu ? Ar[j] : 0.0;
      bv[q] = j < nu ? bsh[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc += av[q] * bv[q];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) a.u[a.umap[a0 + r]] = (T)acc;
}

// ---------------------------------------------------------------------------------------
// plumbing: fills, packing of the caller's arrays, defect-correction updates
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_scale(T* __restrict__ p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] *= v;
}

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
  constexpr int NK = TZ * TY * TX / 256;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  const int64_t nnu = D == 3 ? (int64_t)g.np * g.np * g.np : (int64_t)g.np * g.np;
  const int64_t ubase = (int64_t)t.x * nnu;
  int64_t P[NK];
  bool ok[NK];
  int8_t c[NK];
  double fv[NK], gvv[NK], uv[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    ok[k] = in_box(x, y, z, g.np, D);
    P[k] = base + x + g.st[1] * y + g.st[2] * z;
    const int64_t Q = ok[k] ? ubase + x + (int64_t)g.np * (y + (int64_t)g.np * z) : ubase;
    c[k] = cls[ok[k] ? P[k] : base];
    fv[k] = f[Q];
    gvv[k] = gv[Q];
    uv[k] = uin ? uin[Q] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (!ok[k]) continue;
    rhs[P[k]] = c[k] == 1 ? fv[k] : (c[k] == 2 ? gvv[k] : 0.0);
    if (uin) u[P[k]] = c[k] ? uv[k] : 0.0;
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
  const int8_t c = cls[P];
  const double v = src[P];
  dst[i] = c ? v : 0.0;
}

// Warm start of a new hierarchy from the solution u of a previous one on the same grid (caller
// layout, (n+1)^D values per problem): every node that is an unknown now but was not before
// takes the mean of the linear extrapolations 2 u(Q1) - u(Q2) along the axis directions where
// Q1 = P -+ e_a and Q2 = P -+ 2 e_a are unknowns of both hierarchies; with no such direction,
// the mean of its axis neighbours that are; else 0.  Nodes that are unknowns of both keep
// their value.  Writes happen only at new nodes and reads only at old ones, so the update is
// in place.
template <int D>
__global__ void __launch_bounds__(256) k_warm_start(int64_t total, Geo g,
                                                    const int8_t* __restrict__ cls,
                                                    const int8_t* __restrict__ cls_prev,
                                                    double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t nnu = D == 3 ? (int64_t)g.np * g.np * g.np : (int64_t)g.np * g.np;
  const int64_t p = i / nnu;
  int64_t q = i - p * nnu;
  int j[3];
  j[0] = (int)(q % g.np);
  q /= g.np;
  j[1] = (int)(q % g.np);
  j[2] = (int)(q / g.np);
  const int64_t base = p * g.npp;
  const int64_t P = base + j[0] + g.st[1] * j[1] + g.st[2] * j[2];
  if (!cls[P] || cls_prev[P]) return;
  const int64_t ust[3] = {1, g.np, (int64_t)g.np * g.np};
  double lin = 0.0, cst = 0.0;
  int nlin = 0, ncst = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      const int j1 = j[a] + sgn, j2 = j[a] + 2 * sgn;
      if (j1 < 0 || j1 > g.n) continue;
      const int64_t Q1 = P + sgn * g.st[a];
      if (!(cls[Q1] && cls_prev[Q1])) continue;
      const double u1 = u[i + sgn * ust[a]];
      cst += u1;
      ++ncst;
      if (j2 < 0 || j2 > g.n) continue;
      const int64_t Q2 = P + 2 * sgn * g.st[a];
      if (!(cls[Q2] && cls_prev[Q2])) continue;
      lin += 2.0 * u1 - u[i + 2 * sgn * ust[a]];
      ++nlin;
    }
  }
  u[i] = nlin ? lin / nlin : (ncst ? cst / ncst : 0.0);
}

template <int D>
void launch_warm_start(const DevLevel& L, const DevLevel& Lprev, int batch, double* u,
                       hipStream_t s) {
  const int64_t nnu = D == 3 ? (int64_t)L.g.np * L.g.np * L.g.np : (int64_t)L.g.np * L.g.np;
  const int64_t total = nnu * batch;
  hipLaunchKernelGGL((k_warm_start<D>), dim3((int)((total + 255) / 256)), dim3(256), 0, s, total, L.g,
                     L.cls, Lprev.cls, u);
}
template void launch_warm_start<2>(const DevLevel&, const DevLevel&, int, double*, hipStream_t);
template void launch_warm_start<3>(const DevLevel&, const DevLevel&, int, double*, hipStream_t);

// u64 += u32 at the unknowns (defect correction), and u32z (the buffer the next step's
// FP32 cycles start from; it may be u32 itself) reset to zero
template <int D>
__global__ void __launch_bounds__(256) k_dc_update(const int4* __restrict__ tiles, int ntiles, Geo g,
                                                   const int8_t* __restrict__ cls,
                                                   double* __restrict__ u64, const float* u32,
                                                   float* u32z) {
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, TZ = Tile<D>::Z;
  constexpr int NK = TZ * TY * TX / 256;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int4 t = tiles[tile];
  const int64_t base = (int64_t)t.x * g.npp;
  int64_t P[NK];
  bool ok[NK];
  int8_t c[NK];
  double uv[NK];
  float ev[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int x = t.y * TX + i % TX, y = t.z * TY + (i / TX) % TY;
    const int z = D == 3 ? t.w * TZ + i / (TX * TY) : 0;
    ok[k] = in_box(x, y, z, g.np, D);
    P[k] = ok[k] ? base + x + g.st[1] * y + g.st[2] * z : base;
    c[k] = cls[P[k]];
    uv[k] = u64[P[k]];
    ev[k] = u32[P[k]];
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (!ok[k] || c[k] == 0) continue;
    u64[P[k]] = uv[k] + (double)ev[k];
    u32z[P[k]] = 0.0f;
  }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
static inline int tile_grid(int ntiles) { return (ntiles + 7) / 8 * 8; }
static inline int lin_grid(int64_t n) { return (int)((n + 255) / 256); }

// per-problem boundary work that one workgroup sweeps within its barriers (levels without
// relaxation chunks); larger boundaries take one launch per phase
constexpr int kSingleWgBand = 8192;
constexpr int kSingleWgExt = 24576;

template <int D, typename T, int MODE, int SUB>
static void launch_relax_sub(RelaxArgs<T> a, const DevLevel& L, hipStream_t s) {
  a.nbt = a.ntiles ? tile_grid(a.ntiles * RTile<D, SUB>::N) : 0;
  const size_t chunk_lds = (size_t)(L.bc_smax + band_chunk_threads(D)) * sizeof(T);
  if constexpr (D == 3) {
    if (MODE == kRelaxPlain && a.nchunks && a.nbt) {
      // tiles and the first launch's chunks together (levels with few tiles, plain mode)
      const size_t lds = std::max(tile_lds<D, T, kRelaxPlain, 1>(), chunk_lds);
      hipLaunchKernelGGL((k_relax_shared3<T>), dim3(a.nchunks + a.nbt), dim3(band_chunk_threads(D)),
                         lds, s, a);
      return;
    }
    // tiles and chunks in launches of their own
    if (a.nbt) {
      RelaxArgs<T> t = a;
      t.nchunks = 0;
      const size_t tlds = tile_lds<D, T, MODE, SUB>();
      hipLaunchKernelGGL((k_relax<D, T, false, MODE, SUB>), dim3(a.nbt), dim3(256), tlds, s, t);
    }
    if (a.nchunks) {
      // (3D interpolation and restriction are launches of their own: chunks relax plainly)
      hipLaunchKernelGGL((k_relax_chunks<D, T>), dim3(a.nchunks), dim3(band_chunk_threads(D)),
                         chunk_lds, s, a);
    }
  } else {
    const int nb = a.nchunks + a.nbt;
    if (!nb) return;
    const size_t lds = std::max(tile_lds<D, T, MODE, SUB>(), chunk_lds);
    if (a.nchunks)
      hipLaunchKernelGGL((k_relax<D, T, true, MODE, SUB>), dim3(nb), dim3(256), lds, s, a);
    else
      hipLaunchKernelGGL((k_relax<D, T, false, MODE, SUB>), dim3(nb), dim3(256), lds, s, a);
  }
}

// tiles split in parts on levels with fewer than kSplitTilesBelow tiles (2D)
constexpr int kSplitTilesBelow = 512;
// 3D levels with at most this many tiles relax their tiles in the launch of the first
// relaxation chunks (k_relax_shared3): levels whose tile launch is a single round of resident
// workgroups (256 CUs x 7 FP32 tiles = 1792), where it costs latency rather than bandwidth
// (tank 384^3: the 192^3 level, 1232 tiles, gains; torus 256^3: the finest level, about
// 1900 tiles, loses when shared)
constexpr int kShareTilesBelow3D = 1536;

template <int D, typename T, int MODE>
static void launch_relax_kernel(const RelaxArgs<T>& a, const DevLevel& L, hipStream_t s) {
  if constexpr (D == 2)
    if (a.ntiles > 0 && a.ntiles < kSplitTilesBelow) return launch_relax_sub<D, T, MODE, 2>(a, L, s);
  launch_relax_sub<D, T, MODE, 1>(a, L, s);
}

size_t defect_lds(const DevLevel& L) { return (size_t)L.ec_smax * sizeof(double); }

template <int D, typename T>
static void launch_band(const DevLevel& L, const mg_grid& G, T* u, const T* rhs, T* tmp,
                        int batch, hipStream_t s) {
  const double cNh = G.cN * L.g.h;
  const T h2 = (T)(L.g.h * L.g.h), inv2d = (T)(1.0 / (2.0 * D));
  if (L.max_bandp + L.max_gp <= kSingleWgBand) {
    BandArgs<T> a;
    a.g = L.g;
    a.ghosts = L.ghosts;
    a.gw = L.gw;
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
    a.cD = G.cD;
    a.cNh = cNh;
    a.lambda = G.lambda;
    hipLaunchKernelGGL((k_band<D, T>), dim3(batch), dim3(1024), 0, s, a);
    return;
  }
  auto ghosts = [&]() {
    if (!L.nghost) return;
    hipLaunchKernelGGL((k_ghost_new<D, T>), dim3(lin_grid(L.nghost)), dim3(256), 0, s, L.ghosts,
                       L.gw, L.nghost, L.g, (const T*)u, rhs, tmp, G.cD, cNh);
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

template <typename T>
struct BandBuf;
template <>
struct BandBuf<double> {
  static double* get(const DevLevel& L) { return L.z64; }
};
template <>
struct BandBuf<float> {
  static float* get(const DevLevel& L) { return L.z32; }
};

template <typename T>
__global__ void __launch_bounds__(256) k_copy_list(const int32_t* __restrict__ list, int n,
                                                   const T* __restrict__ src, T* __restrict__ dst) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[list[i]] = src[list[i]];
}

template <int D, typename T>
void launch_relax(const DevLevel& L, const mg_grid& G, const T* uin, T* uout, const T* rhs,
                  T* tmp, int batch, hipStream_t s, const DevLevel* C, const T* uc,
                  const DevLevel* F, const T* rf) {
  if (F && D != 2) {
    // the restriction is fused in 2D only: restrict, then relax from the zeroed iterate
    launch_restrict<D, T>(*F, L, rf, const_cast<T*>(rhs), const_cast<T*>(uin), s);
    F = nullptr;
  }
  RelaxArgs<T> a;
  a.rf = F ? rf : nullptr;
  a.gf = F ? F->g : L.g;
  a.rcode = L.rcode;
  a.rhs_w = const_cast<T*>(rhs);
  a.prolong = C != nullptr;
  if (C) {
    a.gc = C->g;
    a.uc = uc;
    a.clsc = C->cls;
  } else {
    a.gc = L.g;
    a.uc = uin;
    a.clsc = L.cls;
  }
  a.tiles = L.tiles;
  a.ntiles = L.ntiles;
  a.nbt = 0;  // set by the launch (tiles or parts of tiles)
  a.g = L.g;
  a.rcls = L.rcls;
  a.uin = uin;
  a.uout = uout;
  a.rhs = rhs;
  a.h2 = (T)(L.g.h * L.g.h);
  a.inv2d = (T)(1.0 / (2.0 * D));
  a.uband = uin;
  a.write_all = L.nchunks ? 0 : 1;
  a.skip_band = G.smoother == 2 ? 1 : 0;
  // 2D: the tiles and the first launch's chunks share a launch; 3D chunks (which hold the
  // 27-point ghost rows in registers) get launches of their own, so that the tiles keep
  // their occupancy, except on levels with few tiles (plain relaxations: 3D interpolation and
  // restriction are launches of their own)
  const int k0 = D == 2 || (L.nchunks && L.ntiles > 0 && L.ntiles <= kShareTilesBelow3D) ? 1 : 0;
  a.nchunks = L.nchunks && k0 == 1 ? L.sub[1] - L.sub[0] : 0;
  a.phases = L.bc_phases;
  a.hdr = L.bc_hdr;
  a.data = L.bc_data;
  a.stride = L.bc_stride;
  if ((!L.nchunks || D == 3) && C) {
    // the per-phase boundary path reads u in place, and 3D chunks hold no interpolation
    // data in registers: interpolate first
    launch_prolong<D, T>(L, *C, uc, const_cast<T*>(uin), s);
    a.prolong = 0;
  }
  bool restrict_ = F != nullptr;
  if (!L.nchunks && restrict_) {
    // likewise: restrict (and zero the iterate) first
    launch_restrict<D, T>(*F, L, rf, const_cast<T*>(rhs), const_cast<T*>(uin), s);
    restrict_ = false;
  }
  if (restrict_)
    launch_relax_kernel<D, T, D == 2 ? kRelaxRestrict : kRelaxPlain>(a, L, s);
  else if (a.prolong)
    launch_relax_kernel<D, T, kRelaxProlong>(a, L, s);
  else
    launch_relax_kernel<D, T, kRelaxPlain>(a, L, s);
  if (!L.nchunks) {
    if (G.smoother == 1 && L.alt_ncol) {
      hipLaunchKernelGGL((k_band_kaczmarz<D, T>), dim3(batch), dim3(256), 0, s, L.g, L.alt_list,
                         L.alt_off, L.alt_ncol, L.ghosts, L.gw, uout, rhs, G.lambda);
    } else if (G.smoother == 2 && L.alt_ncol) {
      if constexpr (D == 2)
        hipLaunchKernelGGL((k_band_block<T>), dim3(batch), dim3(kBlockThreads), 0, s, L.g,
                           L.alt_list, L.alt_off, L.alt_ncol, L.ghosts, L.ghost_off, L.gw, L.cls,
                           uout, rhs);
    } else {
      launch_band<D, T>(L, G, uout, rhs, tmp, batch, s);
    }
    return;
  }
  // the relaxation's later launches (chunks only): launch k >= 1 reads the band and ghost
  // values from uout (k odd) or z (k even) and everything else from uout, and writes its
  // owned nodes to z (k odd) or uout (k even)
  T* z = BandBuf<T>::get(L);
  for (int k = k0; k < L.nsub; ++k) {
    RelaxArgs<T> b = a;
    b.ntiles = 0;
    b.nbt = 0;
    b.prolong = 0;
    b.rf = nullptr;
    b.uin = k == 0 ? uin : uout;
    b.uband = k == 0 ? uin : (k & 1) ? uout : z;
    b.uout = k == 0 ? uout : (k & 1) ? z : uout;
    b.nchunks = L.sub[k + 1] - L.sub[k];
    b.hdr = L.bc_hdr + (size_t)L.sub[k] * kBandHdr;
    if (band_fixed_layout(D)) b.data = L.bc_data + (size_t)L.sub[k] * L.bc_stride;
    if (b.nchunks) launch_relax_kernel<D, T, kRelaxPlain>(b, L, s);
  }
  if (!(L.nsub & 1)) {
    // an even number of launches leaves the band and ghost values in z
    if (L.nband_list)
      hipLaunchKernelGGL((k_copy_list<T>), dim3(lin_grid(L.nband_list)), dim3(256), 0, s,
                         L.band_list, L.nband_list, (const T*)z, uout);
  }
}

template <typename T>
static void launch_extend(const DevLevel& L, T* r, int batch, hipStream_t s) {
  if (!L.next) return;
  if (L.max_extp <= kSingleWgExt) {
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

// every extension node takes its composed combination of the ghost defects (rg, by ghost
// id: a compact array that stays in the L2 cache): the kExtLanes lanes of a node take every
// kExtLanes-th term (four loads in flight each), then their partial sums are added pairwise
// across the lanes; weights and sums in the precision of the cycle
constexpr int kExtLanes = 16;
template <typename TO>
__global__ void __launch_bounds__(256) k_ext_terms(int n, const int32_t* __restrict__ node,
                                                   const int32_t* __restrict__ off,
                                                   const int32_t* __restrict__ src,
                                                   const TO* __restrict__ wt,
                                                   const TO* __restrict__ rg, TO* r) {
  const int gid = blockIdx.x * 256 + threadIdx.x;
  const int i = gid / kExtLanes, lane = gid % kExtLanes;
  const int ic = i < n ? i : n - 1;
  const int t0 = off[ic], t1 = i < n ? off[ic + 1] : t0;
  TO v = 0;
  int t = t0 + lane;
  for (; t + 3 * kExtLanes < t1; t += 4 * kExtLanes) {
    TO w[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      w[q] = wt[t + q * kExtLanes];
      x[q] = rg[src[t + q * kExtLanes]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) v += w[q] * x[q];
  }
  for (; t < t1; t += kExtLanes) v += wt[t] * rg[src[t]];
#pragma unroll
  for (int o = kExtLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kExtLanes);
  if (i < n && lane == 0) r[node[i]] = v;
}

template <int D, typename T, typename TO>
void launch_defect(const DevLevel& L, const T* u, const T* rhs, TO* r, uint64_t* norms,
                   bool with_ext, int batch, hipStream_t s) {
  DefectArgs<T, TO> a;
  a.tiles = L.tiles;
  a.ntiles = L.ntiles;
  a.nbt = L.ntiles ? tile_grid(L.ntiles) : 0;
  a.ghosts = L.ghosts;
  a.gw = L.gw;
  a.nghost = L.nghost;
  a.g = L.g;
  a.cls = L.cls;
  a.u = u;
  a.rhs = rhs;
  a.r = r;
  a.inv_h2 = (T)(1.0 / (L.g.h * L.g.h));
  a.norms = norms;
  a.nechunks = with_ext && D == 2 ? L.nechunks : 0;
  // the extension gather reads the ghost defects from the compact array (its weights are in
  // the cycle's precision, which is TO whenever the extension is asked for)
  const bool gather = with_ext && !a.nechunks && L.net > 0;
  a.rg = gather ? (TO*)L.et_rg : nullptr;
  a.hdr = L.ec_hdr;
  a.data = L.ec_data;
  a.stride = L.ec_stride;
  const int nb = a.nechunks + a.nbt + (L.nghost ? lin_grid(L.nghost) : 0);
  if (nb)
    hipLaunchKernelGGL((k_defect<D, T, TO>), dim3(nb), dim3(256),
                       a.nechunks ? defect_lds(L) : 0, s, a);
  if (gather)
    hipLaunchKernelGGL((k_ext_terms<TO>), dim3(lin_grid((int64_t)L.net * kExtLanes)), dim3(256), 0, s,
                       L.net, L.et_node, L.et_off, L.et_src, (const TO*)L.et_wt, (const TO*)L.et_rg, r);
  else if (with_ext && !a.nechunks)
    launch_extend<TO>(L, r, batch, s);
}

template <int D>
void launch_rhs_norm(const DevLevel& L, const double* rhs, uint64_t* norms, hipStream_t s) {
  if (L.ntiles)
    hipLaunchKernelGGL((k_rhs_norm<D>), dim3(tile_grid(L.ntiles)), dim3(256), 0, s, L.tiles,
                       L.ntiles, L.g, L.cls, rhs, norms);
}

template <int D, typename T>
void launch_restrict(const DevLevel& F, const DevLevel& C, const T* rf, T* rhsc, T* uc,
                     hipStream_t s) {
  if (!C.ntiles) return;
  if constexpr (D == 3)
    hipLaunchKernelGGL((k_restrict_parts<D, T>), dim3(tile_grid(C.ntiles * RTile<D, 2>::N)),
                       dim3(256), 0, s, C.tiles, C.ntiles, C.g, F.g, C.rcode, rf, rhsc, uc);
  else
    hipLaunchKernelGGL((k_restrict<D, T>), dim3(tile_grid(C.ntiles)), dim3(256), 0, s, C.tiles,
                       C.ntiles, C.g, F.g, C.rcode, rf, rhsc, uc);
}

template <int D, typename T>
void launch_prolong(const DevLevel& F, const DevLevel& C, const T* uc, T* uf, hipStream_t s) {
  if (F.ntiles)
    hipLaunchKernelGGL((k_prolong<D, T>), dim3(tile_grid(F.ntiles)), dim3(256), 0, s, F.tiles,
                       F.ntiles, F.g, C.g, F.cls, C.cls, uc, uf);
}

template <int D, typename T>
void launch_coarse(const DevLevel& C, const DevLevel* F, const T* rf, T* rhs, T* u, int batch,
                   bool from_rhs, hipStream_t s) {
  if (C.nu_max <= 0) return;
  CoarseArgs<T> a;
  a.umap = C.umap;
  a.umap_off = C.umap_off;
  a.ainv_off = C.ainv_off;
  a.ainv = C.ainv;
  a.gf = F ? F->g : C.g;
  a.ufine = C.ufine;
  a.ucode = C.ucode;
  a.rf = rf;
  a.rhs = rhs;
  a.rhsc = C.rhsc;
  a.u = u;
  if (F && C.nu_total > 0)
    hipLaunchKernelGGL((k_coarse_restrict<D, T>), dim3(lin_grid(C.nu_total)), dim3(256), 0, s, a,
                       C.nu_total);
  else if (from_rhs && C.nu_total > 0)
    hipLaunchKernelGGL((k_coarse_gather<T>), dim3(lin_grid(C.nu_total)), dim3(256), 0, s, a,
                       C.nu_total);
  const int blocks = (C.nu_max + kCoarseRows - 1) / kCoarseRows;
  hipLaunchKernelGGL((k_coarse<T>), dim3(blocks, batch), dim3(kCoarseRows * 64),
                     C.nu_max * sizeof(double), s, a);
}

void launch_scale(double* p, int64_t n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_scale<double>), dim3(lin_grid(n)), dim3(256), 0, s, p, n, v);
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
void launch_dc_update(const DevLevel& L, double* u64, const float* u32, float* u32_zero,
                      hipStream_t s) {
  if (L.ntiles)
    hipLaunchKernelGGL((k_dc_update<D>), dim3(tile_grid(L.ntiles)), dim3(256), 0, s, L.tiles,
                       L.ntiles, L.g, L.cls, u64, u32, u32_zero);
}

#define GHOSTMG_INST(D, T)                                                                    \
  template void launch_relax<D, T>(const DevLevel&, const mg_grid&, const T*, T*, const T*, T*, \
                                   int, hipStream_t, const DevLevel*, const T*,               \
                                   const DevLevel*, const T*);                                \
  template void launch_defect<D, T, T>(const DevLevel&, const T*, const T*, T*, uint64_t*,    \
                                       bool, int, hipStream_t);                               \
  template void launch_restrict<D, T>(const DevLevel&, const DevLevel&, const T*, T*, T*,     \
                                      hipStream_t);                                           \
  template void launch_prolong<D, T>(const DevLevel&, const DevLevel&, const T*, T*, hipStream_t); \
  template void launch_coarse<D, T>(const DevLevel&, const DevLevel*, const T*, T*, T*, int,        \
                                    bool, hipStream_t);                                            \

GHOSTMG_INST(2, double)
GHOSTMG_INST(2, float)
GHOSTMG_INST(3, double)
GHOSTMG_INST(3, float)
template void launch_defect<2, double, float>(const DevLevel&, const double*, const double*, float*,
                                              uint64_t*, bool, int, hipStream_t);
template void launch_defect<3, double, float>(const DevLevel&, const double*, const double*, float*,
                                              uint64_t*, bool, int, hipStream_t);
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
template void launch_dc_update<2>(const DevLevel&, double*, const float*, float*, hipStream_t);
template void launch_dc_update<3>(const DevLevel&, double*, const float*, float*, hipStream_t);

}  // namespace ghostmg
