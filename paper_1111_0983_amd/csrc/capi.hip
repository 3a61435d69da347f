// C ABI of the ghost-cell multigrid solver: hierarchy upload, the cycle driver (captured
// once into HIP graphs), the solve loop with its stopping test, and the query entry points.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "kernels.h"

using namespace ghostmg;

namespace {

#define HIP_TRY(x)                       \
  do {                                   \
    if ((x) != hipSuccess) return MG_EHIP; \
  } while (0)

template <typename T>
int upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return MG_OK;
  if (hipMalloc((void**)dst, src.size() * sizeof(T)) != hipSuccess) return MG_ENOMEM;
  if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return MG_EHIP;
  return MG_OK;
}

template <typename T>
int alloc_zero(T** dst, size_t n) {
  *dst = nullptr;
  if (!n) return MG_OK;
  if (hipMalloc((void**)dst, n * sizeof(T)) != hipSuccess) return MG_ENOMEM;
  if (hipMemset(*dst, 0, n * sizeof(T)) != hipSuccess) return MG_EHIP;
  return MG_OK;
}

int max_span(const std::vector<int32_t>& off) {
  int m = 0;
  for (size_t i = 0; i + 1 < off.size(); ++i) m = std::max(m, off[i + 1] - off[i]);
  return m;
}

// relaxation chunks: owned band and ghost nodes per chunk (2D; twice as many for the wider
// 3D workgroups), and the redundant work (chunk entries per owned node) above which a level
// relaxes its boundary with one launch per phase instead; owned extension nodes per
// extension chunk
constexpr int kChunkOwn = 320;
constexpr double kChunkRedundancy2D = 4.0, kChunkRedundancy3D = 8.0;
constexpr int kExtChunkOwn = 512;

int upload_level(mg_handle_s* H, int l) {
  const HostLevel& S = H->host[l];
  DevLevel& L = H->dev[l];
  const size_t nn = (size_t)H->batch * S.g.npp;
  const bool dc = H->grid.precision == MG_FP32_DC;
  L.g = S.g;
  L.ntiles = (int)S.tiles.size();
  L.nghost = (int)S.ghosts.size();
  L.nred = (int)S.red.size();
  L.nblack = (int)S.black.size();
  L.next = (int)S.ext.size();
  L.gdag_off = S.gdag_off;
  L.max_gp = max_span(S.ghost_off);
  L.max_bandp = max_span(S.red_off) + max_span(S.black_off);
  L.max_extp = max_span(S.ext_off);
  int rc;
  if ((rc = upload(&L.cls, S.cls))) return rc;
  if ((rc = upload(&L.phi, S.phi))) return rc;
  if ((rc = upload(&L.tiles, S.tiles))) return rc;
  if ((rc = upload(&L.ghosts, S.ghosts))) return rc;
  if ((rc = upload(&L.ghost_off, S.ghost_off))) return rc;
  if ((rc = upload(&L.red, S.red))) return rc;
  if ((rc = upload(&L.black, S.black))) return rc;
  if ((rc = upload(&L.red_off, S.red_off))) return rc;
  if ((rc = upload(&L.black_off, S.black_off))) return rc;
  if ((rc = upload(&L.ext, S.ext))) return rc;
  if ((rc = upload(&L.ext_merged, S.ext_merged))) return rc;
  if ((rc = upload(&L.ext_off, S.ext_off))) return rc;
  if ((rc = upload(&L.dag_off, S.dag_off))) return rc;
  if ((rc = upload(&L.dag_start, S.dag_start))) return rc;
  if ((rc = upload(&L.rcode, S.rcode))) return rc;
  if ((rc = upload(&L.rcls, S.rcls))) return rc;
  if ((rc = upload(&L.gw, S.gw))) return rc;
  const bool need64 = !dc || l == 0;
  if (need64) {
    for (int k = 0; k < 2; ++k)
      if ((rc = alloc_zero(&L.u64[k], nn))) return rc;
    if ((rc = alloc_zero(&L.rhs64, nn))) return rc;
    if ((rc = alloc_zero(&L.r64, nn))) return rc;
    if ((rc = alloc_zero(&L.gtmp64, (size_t)L.nghost + 1))) return rc;
  }
  if (dc) {
    for (int k = 0; k < 2; ++k)
      if ((rc = alloc_zero(&L.u32[k], nn))) return rc;
    if ((rc = alloc_zero(&L.rhs32, nn))) return rc;
    if ((rc = alloc_zero(&L.r32, nn))) return rc;
    if ((rc = alloc_zero(&L.gtmp32, (size_t)L.nghost + 1))) return rc;
  }
  if (S.bc_nchunks) {
    L.nchunks = S.bc_nchunks;
    L.bc_smax = S.bc_smax;
    L.bc_stride = S.bc_stride;
    L.bc_phases = S.bc_range;
    L.nsub = (int)S.bc_sub.size() - 1;
    if (L.nsub < 1 || L.nsub > 7) return MG_EINVAL;
    for (int k = 0; k <= L.nsub; ++k) L.sub[k] = S.bc_sub[k];
    if ((rc = upload(&L.bc_hdr, S.bc_hdr))) return rc;
    if ((rc = upload(&L.bc_data, S.bc_data))) return rc;
    if (L.nsub > 1) {
      if (dc ? (rc = alloc_zero(&L.z32, nn)) : (rc = alloc_zero(&L.z64, nn))) return rc;
      if (!(L.nsub & 1)) {
        std::vector<int32_t> bl(S.red.begin(), S.red.end());
        bl.insert(bl.end(), S.black.begin(), S.black.end());
        for (const GhostRec& gr : S.ghosts) bl.push_back((int32_t)gr.node);
        L.nband_list = (int)bl.size();
        if ((rc = upload(&L.band_list, bl))) return rc;
      }
    }
  }
  if (H->grid.smoother != 0 && l < H->L) {
    // band nodes and ghosts of every problem by colour (x mod M) + M (y mod M) + M^2 (z mod M)
    const int M = H->grid.smoother == 1 ? 5 : 7;
    int ncol = 1;
    for (int a = 0; a < H->dim; ++a) ncol *= M;
    const Geo& g = S.g;
    auto colour = [&](int32_t v) {
      const int64_t loc = v % g.npp;
      const int64_t z = H->dim == 3 ? loc / g.st[2] : 0, rem = loc - z * (H->dim == 3 ? g.st[2] : 0);
      const int64_t y = rem / g.st[1], x = rem - y * g.st[1];
      return (int)(x % M + M * (y % M) + (int64_t)M * M * (z % M));
    };
    std::vector<std::vector<int2>> by(H->batch * (size_t)ncol);
    auto add = [&](int32_t v, int gid) {
      by[(size_t)(v / g.npp) * ncol + colour(v)].push_back(make_int2(v, gid));
    };
    for (int32_t v : S.red) add(v, -1);
    for (int32_t v : S.black) add(v, -1);
    for (size_t i = 0; i < S.ghosts.size(); ++i) add(S.ghosts[i].node, (int)i);
    std::vector<int2> list;
    std::vector<int32_t> off;
    for (size_t k = 0; k < by.size(); ++k) {
      if (k % ncol == 0 && k) off.push_back((int32_t)list.size());
      off.push_back((int32_t)list.size());
      list.insert(list.end(), by[k].begin(), by[k].end());
    }
    off.push_back((int32_t)list.size());
    L.alt_ncol = ncol;
    if ((rc = upload(&L.alt_list, list))) return rc;
    if ((rc = upload(&L.alt_off, off))) return rc;
  }
  if (!S.et_node.empty()) {
    L.net = (int)S.et_node.size();
    if ((rc = upload(&L.et_node, S.et_node))) return rc;
    if ((rc = upload(&L.et_off, S.et_off))) return rc;
    if ((rc = upload(&L.et_src, S.et_src))) return rc;
    if (H->grid.precision == MG_FP32_DC) {
      std::vector<float> w32(S.et_wt.begin(), S.et_wt.end());
      float* w = nullptr;
      rc = upload(&w, w32);
      L.et_wt = w;
    } else {
      double* w = nullptr;
      rc = upload(&w, S.et_wt);
      L.et_wt = w;
    }
    if (rc) return rc;
    if (S.nghost && hipMalloc(&L.et_rg, (size_t)S.nghost * sizeof(double)) != hipSuccess)
      return MG_ENOMEM;
  }
  if (S.ec_nchunks) {
    L.nechunks = S.ec_nchunks;
    L.ec_smax = S.ec_smax;
    L.ec_stride = S.ec_stride;
    if ((rc = upload(&L.ec_hdr, S.ec_hdr))) return rc;
    if ((rc = upload(&L.ec_data, S.ec_data))) return rc;
  }
  if (l == H->L) {
    L.nu_max = max_span(S.umap_off);
    L.nu_total = (int)S.umap.size();
    if ((rc = upload(&L.umap, S.umap))) return rc;
    if ((rc = upload(&L.umap_off, S.umap_off))) return rc;
    if ((rc = upload(&L.ainv_off, S.ainv_off))) return rc;
    if ((rc = upload(&L.ainv, S.ainv))) return rc;
    if ((rc = alloc_zero(&L.rhsc, (size_t)L.nu_total))) return rc;
    if (l > 0) {
      // per unknown: the finer level's node (2x, 2y, 2z) and the restriction code (the solve
      // restricts its right-hand side itself)
      const Geo& gc = S.g;
      const Geo& gf = H->host[l - 1].g;
      std::vector<int32_t> uf(S.umap.size());
      std::vector<uint8_t> uc(S.umap.size());
      for (size_t i = 0; i < S.umap.size(); ++i) {
        const int64_t X = S.umap[i], p = X / gc.npp, loc = X - p * gc.npp;
        const int64_t z = H->dim == 3 ? loc / gc.st[2] : 0, rem = loc - z * (H->dim == 3 ? gc.st[2] : 0);
        const int64_t y = rem / gc.st[1], x = rem - y * gc.st[1];
        uf[i] = (int32_t)(p * gf.npp + 2 * x + gf.st[1] * 2 * y + gf.st[2] * 2 * z);
        uc[i] = S.rcode[X];
      }
      if ((rc = upload(&L.ufine, uf))) return rc;
      if ((rc = upload(&L.ucode, uc))) return rc;
    }
  }
  return MG_OK;
}

template <typename T>
struct Arr;
template <>
struct Arr<double> {
  static double* u(DevLevel& L, int k) { return L.u64[k]; }
  static double* rhs(DevLevel& L) { return L.rhs64; }
  static double* r(DevLevel& L) { return L.r64; }
  static double* tmp(DevLevel& L) { return L.gtmp64; }
};
template <>
struct Arr<float> {
  static float* u(DevLevel& L, int k) { return L.u32[k]; }
  static float* rhs(DevLevel& L) { return L.rhs32; }
  static float* r(DevLevel& L) { return L.r32; }
  static float* tmp(DevLevel& L) { return L.gtmp32; }
};

// One relaxation of level l from its current iterate buffer into the other one; with
// prolong, it starts from the iterate plus the interpolated correction of level l + 1; with
// restrict_, from zero with the right-hand side restricted from level l - 1's defect.
template <int D, typename T>
void relax(mg_handle_s* H, int l, hipStream_t s, bool prolong = false, bool restrict_ = false) {
  DevLevel& L = H->dev[l];
  const int c = H->cur[l];
  DevLevel* C = prolong ? &H->dev[l + 1] : nullptr;
  DevLevel* F = restrict_ ? &H->dev[l - 1] : nullptr;
  launch_relax<D, T>(L, H->grid, Arr<T>::u(L, c), Arr<T>::u(L, 1 - c), Arr<T>::rhs(L),
                     Arr<T>::tmp(L), H->batch, s, C, C ? Arr<T>::u(*C, H->cur[l + 1]) : nullptr,
                     F, F ? Arr<T>::r(*F) : nullptr);
  H->cur[l] = 1 - c;
}

// The cycle of Sec. 2.4 from level l (TGCS recursion, gamma = 1 V, 2 W).  H->cur tracks,
// while the launches are recorded, which buffer holds each level's iterate.  fresh: the
// level has just been entered from level l - 1, whose defect still has to be restricted
// (Sec. 2.5) into this level's right-hand side, with a zero iterate; the first relaxation
// does that as it stages its values.
template <int D, typename T>
void cycle(mg_handle_s* H, int l, hipStream_t s, bool fresh = false) {
  DevLevel& L = H->dev[l];
  if (l == H->L) {
    // the coarsest solve, after the restriction into its right-hand side
    DevLevel* F = fresh ? &H->dev[l - 1] : nullptr;
    launch_coarse<D, T>(L, F, F ? Arr<T>::r(*F) : nullptr, Arr<T>::rhs(L), Arr<T>::u(L, H->cur[l]),
                        H->batch, l == 0, s);
    return;
  }
  if (fresh && H->grid.nu1 == 0) {
    DevLevel& F = H->dev[l - 1];
    launch_restrict<D, T>(F, L, Arr<T>::r(F), Arr<T>::rhs(L), Arr<T>::u(L, H->cur[l]), s);
    fresh = false;
  }
  for (int i = 0; i < H->grid.nu1; ++i) relax<D, T>(H, l, s, false, fresh && i == 0);
  launch_defect<D, T, T>(L, Arr<T>::u(L, H->cur[l]), Arr<T>::rhs(L), Arr<T>::r(L), nullptr, true,
                         H->batch, s);
  DevLevel& C = H->dev[l + 1];
  H->cur[l + 1] = 0;
  for (int k = 0; k < H->grid.gamma; ++k) cycle<D, T>(H, l + 1, s, k == 0);
  // interpolation + correction, taken by the first post-relaxation as it stages its values
  if (H->grid.nu2 == 0)
    launch_prolong<D, T>(L, C, Arr<T>::u(C, H->cur[l + 1]), Arr<T>::u(L, H->cur[l]), s);
  for (int i = 0; i < H->grid.nu2; ++i) relax<D, T>(H, l, s, i == 0);
}

template <int D>
void defect_norm64(mg_handle_s* H, int c, hipStream_t s) {
  DevLevel& L = H->dev[0];
  launch_fill<uint64_t>(H->norms, 2 * H->batch, 0, s);
  launch_defect<D, double, double>(L, L.u64[c], L.rhs64, L.r64, H->norms, false, H->batch, s);
}

// FP64 defect of u64 written as the FP32 right-hand side of the correction problem
template <int D>
void dc_defect(mg_handle_s* H, hipStream_t s) {
  DevLevel& L = H->dev[0];
  launch_fill<uint64_t>(H->norms, 2 * H->batch, 0, s);
  launch_defect<D, double, float>(L, L.u64[0], L.rhs64, L.rhs32, H->norms, false, H->batch, s);
}

// one FP64 cycle from finest buffer c, then (with norm) the defect norm of its result
template <int D>
void record_cycle(mg_handle_s* H, int c, bool norm, hipStream_t s) {
  H->cur[0] = c;
  cycle<D, double>(H, 0, s);
  if (norm) defect_norm64<D>(H, H->cur[0], s);
}

// ncyc FP32 cycles on the correction (from zero in FP32 buffer 0), u64 += the correction,
// FP32 buffer 0 cleared for the next step, then the new FP64 defect
template <int D>
void record_dc(mg_handle_s* H, int ncyc, hipStream_t s) {
  H->cur[0] = 0;
  for (int k = 0; k < ncyc; ++k) cycle<D, float>(H, 0, s);
  DevLevel& L = H->dev[0];
  launch_dc_update<D>(L, L.u64[0], L.u32[H->cur[0]], L.u32[0], s);
  dc_defect<D>(H, s);
}

hipStream_t stream_of(mg_handle_s* H) { return H->stream; }

// Record one cycle (FP64 from finest buffer c, with or without the defect norm, or one
// defect-correction step of dc FP32 cycles) into a graph.
int capture(mg_handle_s* H, int dc, int c, bool norm, hipGraphExec_t* out) {
  if (*out) return MG_OK;
  hipStream_t s = stream_of(H);
  hipGraph_t graph;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  if (H->dim == 2)
    dc ? record_dc<2>(H, dc, s) : record_cycle<2>(H, c, norm, s);
  else
    dc ? record_dc<3>(H, dc, s) : record_cycle<3>(H, c, norm, s);
  if (hipStreamEndCapture(s, &graph) != hipSuccess) return MG_EHIP;
  const hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  const hipError_t d = hipGraphDestroy(graph);  // the executable graph does not need it
  return e == hipSuccess && d == hipSuccess ? MG_OK : MG_EHIP;
}

// finest FP64 buffer after one FP64 cycle that starts in buffer c
int after_cycle(const mg_handle_s* H, int c) { return (c + H->grid.nu1 + H->grid.nu2) & 1; }

// Read the per-problem norms; returns the max over problems of max(interior, ghost) / r0.
int read_rel(mg_handle_s* H, double* rel) {
  hipStream_t s = stream_of(H);
  HIP_TRY(hipMemcpyAsync(H->norms_host, H->norms, 2 * H->batch * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double m = 0.0;
  for (int p = 0; p < H->batch; ++p) {
    const double v = std::max(H->norms_host[2 * p], H->norms_host[2 * p + 1]) / H->r0[p];
    if (!(v == v)) {
      m = NAN;
      break;
    }
    m = std::max(m, v);
  }
  *rel = m;
  return MG_OK;
}

int check_ptrs(const void* a, const void* b, const void* c) {
  return (!a || !b || !c) ? MG_EINVAL : MG_OK;
}

template <int D>
int pack(mg_handle_s* H, const double* f, const double* g, const double* u) {
  hipStream_t s = stream_of(H);
  DevLevel& L = H->dev[0];
  launch_pack<D>(L, f, g, u, L.rhs64, L.u64[0], s);
  H->cur0 = 0;
  if (H->grid.precision == MG_FP32_DC) launch_fill<float>(L.u32[0], (int64_t)H->batch * L.g.npp, 0.f, s);
  // r0 = ||(f_h, g_h)||_inf per problem
  launch_fill<uint64_t>(H->norms, 2 * H->batch, 0, s);
  launch_rhs_norm<D>(L, L.rhs64, H->norms, s);
  HIP_TRY(hipMemcpyAsync(H->norms_host, H->norms, 2 * H->batch * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int p = 0; p < H->batch; ++p) {
    const double v = H->norms_host[2 * p];
    if (!(v == v) || std::isinf(v)) return MG_EINVAL;
    H->r0[p] = v > 0.0 ? v : 1.0;
  }
  return MG_OK;
}

int solve_impl(mg_handle_s* H, const double* f, const double* g, double* u, double tol,
               int fixed_cycles, mg_stats* st) {
  int rc = check_ptrs(f, g, u);
  if (rc) return rc;
  const bool dc = H->grid.precision == MG_FP32_DC;
  hipStream_t s = stream_of(H);
  auto t0 = std::chrono::steady_clock::now();
  rc = H->dim == 2 ? pack<2>(H, f, g, u) : pack<3>(H, f, g, u);
  if (rc) return rc;
  if (dc) {
    if ((rc = capture(H, H->grid.inner_cycles, 0, true, &H->graph_dc))) return rc;
    H->graph_dc_short.resize(H->grid.inner_cycles, nullptr);
    for (int r = 1; r < H->grid.inner_cycles; ++r)
      if ((rc = capture(H, r, 0, true, &H->graph_dc_short[r]))) return rc;
  } else {
    for (int c = 0; c < (after_cycle(H, 0) == 1 ? 2 : 1); ++c)
      for (int nm = 0; nm < 2; ++nm)
        if ((rc = capture(H, 0, c, nm == 1, &H->graph_cycle[c][nm]))) return rc;
  }
  // defect of the initial guess
  if (H->dim == 2)
    dc ? dc_defect<2>(H, s) : defect_norm64<2>(H, 0, s);
  else
    dc ? dc_defect<3>(H, s) : defect_norm64<3>(H, 0, s);
  double rel;
  if ((rc = read_rel(H, &rel))) return rc;
  H->history.clear();
  H->history.push_back(rel);
  int cycles = 0, steps = 0, grew = 0, status = MG_OK, last_cycles = 1;
  double prev = rel;
  const int per = dc ? H->grid.inner_cycles : 1;
  for (;;) {
    if (fixed_cycles >= 0) {
      if (steps >= fixed_cycles) break;
    } else {
      if (rel <= tol) break;
      if (!(rel < INFINITY) || grew >= 5) {
        status = MG_EDIVERGED;
        break;
      }
      if (cycles + per > H->grid.max_cycles) {
        status = MG_ENOCONV;
        break;
      }
    }
    // Once the history gives a convergence factor per cycle (the last read-back's reduction
    // over the cycles queued before it), queue the steps that the factor says are still
    // needed, minus one, before reading the residual back: the stopping test is unchanged,
    // only host round trips are saved.  In defect correction, a last step that needs fewer
    // cycles than a full one (with a factor 2 on the tolerance to spare) runs only those.
    // A fixed number of steps is queued at once, with one read-back at the end.
    int k = fixed_cycles >= 0 ? std::max(1, fixed_cycles - steps) : 1;
    int r_short = 0;
    if (fixed_cycles < 0 && H->history.size() >= 3) {
      const double r1 = H->history[H->history.size() - 1], r2 = H->history[H->history.size() - 2];
      const double rho = std::pow(r1 / r2, 1.0 / last_cycles);
      if (rho > 0.0 && std::pow(rho, per) < 0.9 && rel > tol) {
        const double need_c = std::log(tol / rel) / std::log(rho);
        const int need = (int)std::ceil(need_c / per);
        k = std::max(1, std::min(need - 1, 16));
        if (need == 1 && per > 1) {
          const int r = (int)std::ceil(std::log(0.5 * tol / rel) / std::log(rho));
          if (r >= 1 && r < per) r_short = r;
        }
      }
      k = std::min(k, std::max(1, (H->grid.max_cycles - cycles) / per));
    }
    if (r_short) {
      HIP_TRY(hipGraphLaunch(H->graph_dc_short[r_short], s));
      k = 1;
    } else {
      for (int i = 0; i < k; ++i) {
        if (dc) {
          HIP_TRY(hipGraphLaunch(H->graph_dc, s));
        } else {
          // only the last cycle before a read-back needs its defect norm
          HIP_TRY(hipGraphLaunch(H->graph_cycle[H->cur0][i == k - 1 ? 1 : 0], s));
          H->cur0 = after_cycle(H, H->cur0);
        }
      }
    }
    last_cycles = r_short ? r_short : per * k;
    cycles += last_cycles;
    steps += k;
    if ((rc = read_rel(H, &rel))) return rc;
    H->history.push_back(rel);
    grew = rel > prev ? grew + 1 : 0;
    prev = rel;
  }
  if (H->dim == 2)
    launch_unpack<2>(H->dev[0], H->batch, H->dev[0].u64[dc ? 0 : H->cur0], u, s);
  else
    launch_unpack<3>(H->dev[0], H->batch, H->dev[0].u64[dc ? 0 : H->cur0], u, s);
  HIP_TRY(hipStreamSynchronize(s));
  if (hipGetLastError() != hipSuccess) return MG_EHIP;
  auto t1 = std::chrono::steady_clock::now();
  if (st) {
    st->status = status;
    st->cycles = cycles;
    st->outer = dc ? steps : 0;
    st->rel_residual = rel;
    st->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    st->history = H->history.data();
    st->history_len = (int)H->history.size();
  }
  return status;
}

// The convergence factor of Sec. 3: the homogeneous problem (f = g = 0) from the initial
// iterate u0, rho^(m) = ||r^(m)||_inf / ||r^(m-1)||_inf (max over the batch and over the
// interior and ghost parts), the iterate rescaled by 1 / ||r^(m)|| after every cycle (the
// iteration is linear), stopped when |rho^(m) - rho^(m-1)| / rho^(m) < rtol, when the
// defect vanishes or stops being finite, when rho^(m) > 1e3, or after max_cycles cycles.
int rho_impl(mg_handle_s* H, const double* u0, int max_cycles, double rtol, double* rho,
             double* hist, int* ncycles) {
  hipStream_t s = stream_of(H);
  // f, g and u all read from u0 (valid memory); the right-hand side is then cleared
  int rc = H->dim == 2 ? pack<2>(H, u0, u0, u0) : pack<3>(H, u0, u0, u0);
  if (rc) return rc;
  DevLevel& L = H->dev[0];
  const int64_t nn = (int64_t)H->batch * L.g.npp;
  launch_fill<double>(L.rhs64, nn, 0.0, s);
  for (int c = 0; c < (after_cycle(H, 0) == 1 ? 2 : 1); ++c)
    if ((rc = capture(H, 0, c, true, &H->graph_cycle[c][1]))) return rc;
  auto norm = [&](double* out) -> int {
    HIP_TRY(hipMemcpyAsync(H->norms_host, H->norms, 2 * H->batch * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double m = 0.0;
    for (int p = 0; p < 2 * H->batch; ++p) {
      const double v = H->norms_host[p];
      if (!(v == v)) {
        m = NAN;
        break;
      }
      m = std::max(m, v);
    }
    *out = m;
    return MG_OK;
  };
  if (H->dim == 2)
    defect_norm64<2>(H, 0, s);
  else
    defect_norm64<3>(H, 0, s);
  double rprev;
  if ((rc = norm(&rprev))) return rc;
  if (!(rprev > 0.0) || !(rprev < INFINITY)) return MG_EINVAL;
  launch_scale(L.u64[0], nn, 1.0 / rprev, s);
  H->cur0 = 0;
  double rr = 0.0, prev_rho = -1.0;
  int m = 0;
  while (m < max_cycles) {
    HIP_TRY(hipGraphLaunch(H->graph_cycle[H->cur0][1], s));
    H->cur0 = after_cycle(H, H->cur0);
    ++m;
    double rn;
    if ((rc = norm(&rn))) return rc;
    rr = rn;  // the previous iterate's defect norm is 1 after the rescaling
    if (hist) hist[m - 1] = rr;
    if (!(rn > 0.0) || !(rn < INFINITY)) break;
    launch_scale(L.u64[H->cur0], nn, 1.0 / rn, s);
    if (prev_rho > 0.0 && std::fabs(rr - prev_rho) / rr < rtol) break;
    if (rr > 1e3) break;
    prev_rho = rr;
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (hipGetLastError() != hipSuccess) return MG_EHIP;
  *rho = rr;
  *ncycles = m;
  return MG_OK;
}

void free_level(DevLevel& L) {
  void* ptrs[] = {L.alt_list, L.alt_off, L.bc_hdr, L.bc_data, L.z64, L.z32, L.band_list, L.ec_hdr, L.ec_data,
                  L.et_node, L.et_off, L.et_src, L.et_wt, L.et_rg, L.rcls, L.gw,
                  L.cls, L.phi, L.tiles, L.ghosts, L.ghost_off, L.red, L.black, L.red_off, L.black_off,
                  L.ext, L.ext_merged, L.ext_off, L.dag_off, L.dag_start, L.rcode, L.u64[0],
                  L.u64[1], L.rhs64, L.r64, L.gtmp64, L.u32[0], L.u32[1], L.rhs32, L.r32, L.gtmp32,
                  L.umap, L.umap_off, L.ainv_off, L.ainv, L.rhsc, L.ufine, L.ucode};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  L = DevLevel();
}

template <int D, typename T>
void time_launch(mg_handle_s* h, int kernel, int level, int i, hipStream_t s) {
  DevLevel& L = h->dev[level];
  T* u = Arr<T>::u(L, i & 1);
  switch (kernel) {
    case 0:
      launch_relax<D, T>(L, h->grid, u, Arr<T>::u(L, 1 - (i & 1)), Arr<T>::rhs(L), Arr<T>::tmp(L),
                         h->batch, s);
      break;
    case 1:
      launch_defect<D, T, T>(L, u, Arr<T>::rhs(L), Arr<T>::r(L), nullptr, true, h->batch, s);
      break;
    case 2: {
      DevLevel& C = h->dev[level + 1];
      launch_restrict<D, T>(L, C, Arr<T>::r(L), Arr<T>::rhs(C), Arr<T>::u(C, 0), s);
      break;
    }
    case 3: {
      DevLevel& C = h->dev[level + 1];
      launch_prolong<D, T>(L, C, Arr<T>::u(C, 0), u, s);
      break;
    }
    case 5: {  // relaxation taking the interpolated correction of level + 1
      DevLevel& C = h->dev[level + 1];
      launch_relax<D, T>(L, h->grid, u, Arr<T>::u(L, 1 - (i & 1)), Arr<T>::rhs(L), Arr<T>::tmp(L),
                         h->batch, s, &C, Arr<T>::u(C, 0));
      break;
    }
    case 6: {  // relaxation from zero with the right-hand side restricted from level - 1
      DevLevel& F = h->dev[level - 1];
      launch_relax<D, T>(L, h->grid, u, Arr<T>::u(L, 1 - (i & 1)), Arr<T>::rhs(L), Arr<T>::tmp(L),
                         h->batch, s, nullptr, nullptr, &F, Arr<T>::r(F));
      break;
    }
    case 7: {  // coarsest solve, restricting from level - 1 (if any) as in a cycle
      DevLevel* F = level > 0 ? &h->dev[level - 1] : nullptr;
      launch_coarse<D, T>(L, F, F ? Arr<T>::r(*F) : nullptr, Arr<T>::rhs(L), Arr<T>::u(L, 0),
                          h->batch, level == 0, s);
      break;
    }
    default:
      launch_defect<D, T, T>(L, u, Arr<T>::rhs(L), Arr<T>::r(L), h->norms, false, h->batch, s);
  }
}

}  // namespace

extern "C" {

int mg_grid_default(mg_grid* g, int dim, int n, int n_coarse) {
  if (!g) return MG_EINVAL;
  std::memset(g, 0, sizeof(*g));
  g->dim = dim;
  g->n = n;
  g->lo = -1.0;
  g->hi = 1.0;
  g->n_coarse = n_coarse;
  g->nu1 = 2;
  g->nu2 = 1;
  g->gamma = 1;
  g->lambda = 5;
  g->delta_h = 3.0;
  g->cD = 0.9;
  g->cN = 0.9 * 2.0 / (3.0 * std::sqrt((double)dim));
  g->split = 1;
  g->precision = MG_FP64;
  g->inner_cycles = 3;
  g->max_cycles = 100;
  g->batch = 1;
  return MG_OK;
}

namespace {

int setup_impl(const double* phi, const mg_bc_rule* bc, mg_bc_fn fn, void* ctx,
               const mg_grid* grid, mg_handle_t* out);

}  // namespace

int mg_setup(const double* phi, const mg_bc_rule* bc, const mg_grid* grid, mg_handle_t* out) {
  if (!bc) return MG_EINVAL;
  return setup_impl(phi, bc, nullptr, nullptr, grid, out);
}

int mg_setup_partition(const double* phi, mg_bc_fn fn, void* ctx, const mg_grid* grid,
                       mg_handle_t* out) {
  if (!fn) return MG_EINVAL;
  return setup_impl(phi, nullptr, fn, ctx, grid, out);
}

}  // extern "C"

namespace {

int setup_impl(const double* phi, const mg_bc_rule* bc, mg_bc_fn fn, void* ctx,
               const mg_grid* grid, mg_handle_t* out) {
  if (!phi || !grid || !out) return MG_EINVAL;
  *out = nullptr;
  const mg_grid& G = *grid;
  if ((G.dim != 2 && G.dim != 3) || G.n < 4 || G.n_coarse < 2 || !(G.hi > G.lo) || G.batch < 1 ||
      G.nu1 < 0 || G.nu2 < 0 || G.gamma < 1 || G.gamma > 2 || G.lambda < 0 || G.max_cycles < 0 ||
      (G.precision != MG_FP64 && G.precision != MG_FP32_DC) ||
      (G.precision == MG_FP32_DC && G.inner_cycles < 1) || G.smoother < 0 || G.smoother > 2 ||
      (G.smoother == 2 && G.dim != 2))
    return MG_EINVAL;
  int L = 0, nn = G.n;
  while (nn > G.n_coarse) {
    if (nn % 2) return MG_EINVAL;
    nn /= 2;
    ++L;
  }
  if (nn != G.n_coarse || L >= kMaxLevels) return MG_EINVAL;
  int64_t nodes = 1;
  for (int a = 0; a < G.dim; ++a) nodes *= (int64_t)G.n + 1;
  const int64_t padded = (int64_t)((G.n + 1 + 15) / 16 * 16) * nodes / (G.n + 1);
  if (padded * G.batch >= ((int64_t)1 << 31)) return MG_EINVAL;

  mg_handle_s* H = new (std::nothrow) mg_handle_s();
  if (!H) return MG_ENOMEM;
  H->grid = G;
  if (bc) H->bc.assign(bc, bc + G.batch);
  H->bc_fn = fn;
  H->bc_ctx = ctx;
  H->L = L;
  H->batch = G.batch;
  H->dim = G.dim;
  // the classification runs on the GPU: phi in host memory is uploaded first
  hipPointerAttribute_t attr;
  bool on_device = false;
  if (hipPointerGetAttributes(&attr, phi) == hipSuccess && attr.type == hipMemoryTypeDevice)
    on_device = true;
  (void)hipGetLastError();
  double* phi_up = nullptr;
  if (!on_device) {
    const size_t bytes = (size_t)nodes * G.batch * sizeof(double);
    if (hipMalloc((void**)&phi_up, bytes) != hipSuccess) {
      delete H;
      return MG_ENOMEM;
    }
    if (hipMemcpy(phi_up, phi, bytes, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(phi_up);
      delete H;
      return MG_EHIP;
    }
  }
  int rc = build_hierarchy(H, on_device ? phi : phi_up);
  if (phi_up) (void)hipFree(phi_up);
  // relaxation and extension chunks (levels that relax: all but the coarsest); a level
  // whose chunks cannot be built keeps the per-phase boundary launches
  if (!rc)
    for (int l = 0; l < L; ++l) {
      HostLevel& S = H->host[l];
      // the largest number of phases per launch whose chunks fit (all of a relaxation in
      // one launch where possible); the comparison relaxations sweep the band on their own
      // (no chunks)
      const int P = 3 + 3 * H->grid.lambda;
      const bool built =
          H->grid.smoother == 0 &&
          build_band_chunks(H, l, kChunkOwn * (H->dim == 2 ? 1 : 2),
                            H->dim == 2 ? kChunkRedundancy2D : kChunkRedundancy3D, P);
      if (!built) {
        S.bc_nchunks = 0;
        S.bc_hdr.clear();
        S.bc_data.clear();
        S.bc_sub.clear();
      }
      // 2D: extension chunks (each evaluates the few ghost defects it needs); 3D (an
      // extension node's terms reach hundreds of 27-tap ghost rows) and where chunks cannot
      // be built: a gather of the ghost defects the defect launch has written
      if (H->dim == 3 || !build_ext_chunks(H, l, kExtChunkOwn)) {
        S.ec_nchunks = 0;
        S.ec_hdr.clear();
        S.ec_data.clear();
        build_ext_terms(H, l);
      }
    }
  // the coarsest right-hand side of one problem is staged in 64 KB of LDS
  if (!rc && max_span(H->host[L].umap_off) > kMaxCoarseUnknowns) rc = MG_EINVAL;
  if (!rc) {
    H->dev.assign(L + 1, DevLevel());
    for (int l = 0; l <= L && !rc; ++l) rc = upload_level(H, l);
  }
  if (!rc && hipMalloc((void**)&H->norms, 2 * G.batch * sizeof(uint64_t)) != hipSuccess) rc = MG_ENOMEM;
  if (!rc && hipHostMalloc((void**)&H->norms_host, 2 * G.batch * sizeof(double)) != hipSuccess)
    rc = MG_ENOMEM;
  if (!rc && hipStreamCreate(&H->own_stream) != hipSuccess) rc = MG_EHIP;
  H->stream = H->own_stream;
  if (!rc && (hipEventCreate(&H->ev0) != hipSuccess || hipEventCreate(&H->ev1) != hipSuccess))
    rc = MG_EHIP;
  if (!rc && hipDeviceSynchronize() != hipSuccess) rc = MG_EHIP;
  H->r0 = new (std::nothrow) double[G.batch];
  if (!rc && !H->r0) rc = MG_ENOMEM;
  if (rc) {
    mg_free(H);
    return rc;
  }
  H->bc_fn = nullptr;  // the caller's function is not called after setup
  H->bc_ctx = nullptr;
  *out = H;
  return MG_OK;
}

}  // namespace

extern "C" {

int mg_set_stream(mg_handle_t h, void* hip_stream) {
  if (!h) return MG_EINVAL;
  // captured graphs are stream independent: only the stream they are launched on changes
  h->stream = hip_stream ? (hipStream_t)hip_stream : h->own_stream;
  return MG_OK;
}

int mg_query_level(mg_handle_t h, int level, int64_t* info) {
  if (!h || !info || level < 0 || level > h->L) return MG_EINVAL;
  const HostLevel& S = h->host[level];
  info[0] = S.g.n;
  info[1] = S.nint;
  info[2] = S.nghost;
  info[3] = S.nband;
  info[4] = (int64_t)S.ext.size();
  info[5] = (int64_t)S.tiles.size();
  info[6] = level == h->L ? (int64_t)S.umap.size() : 0;
  info[7] = h->L + 1;
  return MG_OK;
}

int mg_query_ghosts(mg_handle_t h, int problem, int level, int64_t* count, int64_t* node,
                    double* B, double* nB, int8_t* type, int8_t* rung) {
  if (!h || !count || problem < 0 || problem >= h->batch || level < 0 || level > h->L)
    return MG_EINVAL;
  const HostLevel& S = h->host[level];
  const int a = S.ghost_off[problem], b = S.ghost_off[problem + 1];
  *count = b - a;
  if (!node) return MG_OK;
  const Geo& g = S.g;
  for (int i = a; i < b; ++i) {
    const GhostRec& r = S.ghosts[i];
    int64_t loc = r.node - (int64_t)problem * g.npp;
    const int64_t z = h->dim == 3 ? loc / g.st[2] : 0;
    loc -= z * g.st[2];
    const int64_t y = loc / g.st[1], x = loc - y * g.st[1];
    node[i - a] = x + (int64_t)g.np * (y + (int64_t)g.np * z);
    for (int c = 0; c < 3; ++c) {
      if (B) B[3 * (i - a) + c] = S.gB[3 * i + c];
      if (nB) nB[3 * (i - a) + c] = r.type ? 0.0 : r.nb[c];
    }
    if (type) type[i - a] = r.type;
    if (rung) rung[i - a] = r.rung;
  }
  return MG_OK;
}

int mg_query_classes(mg_handle_t h, int problem, int level, int8_t* cls) {
  if (!h || !cls || problem < 0 || problem >= h->batch || level < 0 || level > h->L)
    return MG_EINVAL;
  const HostLevel& S = h->host[level];
  const Geo& g = S.g;
  const int nz = h->dim == 3 ? g.np : 1;
  int64_t q = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < g.np; ++y)
      for (int x = 0; x < g.np; ++x)
        cls[q++] = S.cls[(size_t)problem * g.npp + x + g.st[1] * y + g.st[2] * z];
  return MG_OK;
}

int mg_solve(mg_handle_t h, const double* f, const double* g, double* u, double tol,
             mg_stats* st) {
  if (!h || !(tol >= 0.0)) return MG_EINVAL;
  return solve_impl(h, f, g, u, tol, -1, st);
}

int mg_cycles(mg_handle_t h, const double* f, const double* g, double* u, int ncycles) {
  if (!h || ncycles < 0) return MG_EINVAL;
  return solve_impl(h, f, g, u, 0.0, ncycles, nullptr);
}

int mg_rho(mg_handle_t h, const double* u0, int max_cycles, double rtol, double* rho,
           double* hist, int* ncycles) {
  if (!h || !u0 || !rho || !ncycles || max_cycles < 1 || !(rtol >= 0.0) ||
      h->grid.precision != MG_FP64)
    return MG_EINVAL;
  return rho_impl(h, u0, max_cycles, rtol, rho, hist, ncycles);
}

int mg_warm_start(mg_handle_t h, mg_handle_t prev, double* u) {
  if (!h || !prev || !u || h->dim != prev->dim || h->batch != prev->batch ||
      h->grid.n != prev->grid.n || h->grid.lo != prev->grid.lo || h->grid.hi != prev->grid.hi)
    return MG_EINVAL;
  hipStream_t s = stream_of(h);
  // the previous hierarchy's work must be done before its classes are read on this stream
  if (prev->stream != s) HIP_TRY(hipStreamSynchronize(prev->stream));
  if (h->dim == 2)
    launch_warm_start<2>(h->dev[0], prev->dev[0], h->batch, u, s);
  else
    launch_warm_start<3>(h->dev[0], prev->dev[0], h->batch, u, s);
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_residual(mg_handle_t h, const double* f, const double* g, const double* u, double* r,
                double* norms) {
  if (!h || !f || !g || !u) return MG_EINVAL;
  hipStream_t s = stream_of(h);
  int rc = h->dim == 2 ? pack<2>(h, f, g, u) : pack<3>(h, f, g, u);
  if (rc) return rc;
  DevLevel& L = h->dev[0];
  launch_fill<double>(L.r64, (int64_t)h->batch * L.g.npp, 0.0, s);
  if (h->dim == 2)
    defect_norm64<2>(h, 0, s);
  else
    defect_norm64<3>(h, 0, s);
  HIP_TRY(hipMemcpyAsync(h->norms_host, h->norms, 2 * h->batch * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, s));
  if (r) {
    if (h->dim == 2)
      launch_unpack<2>(L, h->batch, L.r64, r, s);
    else
      launch_unpack<3>(L, h->batch, L.r64, r, s);
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (norms)
    for (int i = 0; i < 2 * h->batch; ++i) norms[i] = h->norms_host[i];
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

int mg_time_kernel(mg_handle_t h, int kernel, int level, int reps, double* avg_ms, double* bytes) {
  // the coarsest level is solved directly (kernel 7 only), the others relax
  if (!h || level < 0 || level > h->L || reps < 1 || kernel < 0 || kernel > 7) return MG_EINVAL;
  if ((kernel == 7) != (level == h->L)) return MG_EINVAL;
  if (kernel == 6 && level == 0) return MG_EINVAL;
  hipStream_t s = stream_of(h);
  DevLevel& L = h->dev[level];
  const HostLevel& S = h->host[level];
  const bool dc = h->grid.precision == MG_FP32_DC;
  const double sz = dc ? 4.0 : 8.0;
  if (dc ? !L.u32[0] : !L.u64[0]) return MG_EINVAL;
  auto run = [&](int i) {
    if (h->dim == 2)
      dc ? time_launch<2, float>(h, kernel, level, i, s) : time_launch<2, double>(h, kernel, level, i, s);
    else
      dc ? time_launch<3, float>(h, kernel, level, i, s) : time_launch<3, double>(h, kernel, level, i, s);
  };
  run(0);
  HIP_TRY(hipEventRecord(h->ev0, s));
  for (int i = 1; i <= reps; ++i) run(i);
  HIP_TRY(hipEventRecord(h->ev1, s));
  HIP_TRY(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (avg_ms) *avg_ms = ms / reps;
  if (bytes) {
    // algorithmic bytes: every array element the kernel must touch, once (iterate read and
    // written, right-hand side and node code read per unknown; ghost row weights)
    const double nu = (double)S.nint + (double)S.nghost, ng = (double)S.nghost;
    const double K = h->dim == 2 ? 9.0 : 27.0;
    // the relaxation chunks hold the ghost weights in the cycle's precision, the per-phase
    // launches of levels without chunks read the FP64 rows
    const double gws = L.nchunks > 0 ? sz : 8.0;
    double b = 0.0;
    if (kernel == 0) b = nu * (3.0 * sz + 1.0) + ng * K * gws;
    if (kernel == 5) {
      const HostLevel& C = h->host[level + 1];
      b = nu * (3.0 * sz + 1.0) + ng * K * gws + (double)(C.nint + C.nghost) * (sz + 1.0);
    }
    if (kernel == 6) {
      // no iterate read; the right-hand side is written; the finer defect is read
      const HostLevel& F = h->host[level - 1];
      b = nu * (2.0 * sz + 2.0) + ng * K * gws +
          ((double)F.nint + (double)F.nghost + (double)F.ext.size()) * sz;
    }
    if (kernel == 1) b = nu * (3.0 * sz + 1.0) + ng * K * 8.0 + (double)S.ext.size() * (sz + 24.0);
    if (kernel == 7) {
      // the FP64 inverse of every problem, the unknowns' indices and codes, the FP64
      // right-hand side written and read, u written, and (below the finest level) the finer
      // defect read
      b = 0.0;
      for (int p = 0; p < h->batch; ++p) {
        const double m = (double)(S.umap_off[p + 1] - S.umap_off[p]);
        b += 8.0 * m * m + m * (16.0 + sz + 5.0);
      }
      if (level > 0) {
        const HostLevel& F = h->host[level - 1];
        b += ((double)F.nint + (double)F.nghost + (double)F.ext.size()) * sz;
      }
    }
    if (kernel == 4) b = nu * (3.0 * sz + 1.0) + ng * K * 8.0;
    if (kernel == 2) {
      const HostLevel& C = h->host[level + 1];
      b = (nu + (double)S.ext.size()) * sz + (double)(C.nint + C.nghost) * (2.0 * sz + 1.0);
    }
    if (kernel == 3) {
      const HostLevel& C = h->host[level + 1];
      b = nu * (2.0 * sz + 1.0) + (double)(C.nint + C.nghost) * (sz + 1.0);
    }
    *bytes = b;
  }
  return hipGetLastError() == hipSuccess ? MG_OK : MG_EHIP;
}

void mg_free(mg_handle_t h) {
  if (!h) return;
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < 2; ++k)
      if (h->graph_cycle[c][k]) (void)hipGraphExecDestroy(h->graph_cycle[c][k]);
  if (h->graph_dc) (void)hipGraphExecDestroy(h->graph_dc);
  for (hipGraphExec_t gx : h->graph_dc_short)
    if (gx) (void)hipGraphExecDestroy(gx);
  for (DevLevel& L : h->dev) free_level(L);
  if (h->norms) (void)hipFree(h->norms);
  if (h->norms_host) (void)hipHostFree(h->norms_host);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete[] h->r0;
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
}

const char* mg_strerror(int code) {
  switch (code) {
    case MG_OK: return "ok";
    case MG_EINVAL: return "invalid argument";
    case MG_ENOMEM: return "out of memory";
    case MG_EHIP: return "HIP runtime error";
    case MG_EGEOM: return "unusable geometry";
    case MG_ENOCONV: return "cycle budget exhausted before the tolerance";
    case MG_EDIVERGED: return "iteration diverged";
    default: return "unknown error";
  }
}

}  // extern "C"
