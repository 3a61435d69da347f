// Launchers of the multigrid kernels (kernels.hip).
#pragma once
#include "ghostmg_impl.h"

namespace ghostmg {

constexpr int kCoarseRows = 16;  // rows of the coarsest inverse per workgroup

template <typename T>
struct BandArgs {
  Geo g;
  const GhostRec* ghosts;
  const int32_t *ghost_off, *red, *black, *red_off, *black_off;
  T* u;
  const T* rhs;
  T* tmp;
  T h2, inv2d;
  double inv_h, cD, cNh;
  int lambda;
};

template <typename T>
struct BandChunkArgs {
  const int32_t *off, *own, *out_off, *node, *goff, *gidx, *ops_off;
  const int16_t *nbr, *gent, *gsten, *ops;
  const GhostRec* ghosts;
  T* u;
  const T* rhs;
  T* out;
  int smax, gmax, opsmax, phases;
  T h2, inv2d;
  double inv_h, cD, cNh;
};

template <int D, typename T>
void launch_band_chunks(const DevLevel& L, const mg_grid& G, T* u, const T* rhs, T* out,
                        hipStream_t s);
template <int D, typename T>
void launch_smooth(const DevLevel& L, T* u, const T* rhs, hipStream_t s);
template <int D, typename T>
void launch_band(const DevLevel& L, const mg_grid& G, T* u, const T* rhs, T* tmp, bool single_wg,
                 int batch, hipStream_t s);
template <int D, typename T, typename TO>
void launch_defect(const DevLevel& L, const T* u, const T* rhs, TO* r, uint64_t* norms,
                   hipStream_t s);
template <int D>
void launch_rhs_norm(const DevLevel& L, const double* rhs, uint64_t* norms, hipStream_t s);
template <typename T>
void launch_extend(const DevLevel& L, T* r, bool single_wg, int batch, hipStream_t s);
template <int D, typename T>
void launch_restrict(const DevLevel& F, const DevLevel& C, const T* rf, T* rhsc, T* uc,
                     hipStream_t s);
template <int D, typename T>
void launch_prolong(const DevLevel& F, const DevLevel& C, const T* uc, T* uf, hipStream_t s);
template <typename T>
void launch_coarse(const DevLevel& C, const T* rhs, T* u, int batch, hipStream_t s);
template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t s);
template <int D>
void launch_pack(const DevLevel& L, const double* f, const double* g, const double* uin,
                 double* rhs, double* u, hipStream_t s);
template <int D>
void launch_unpack(const DevLevel& L, int batch, const double* src, double* dst, hipStream_t s);
template <int D>
void launch_dc_update(const DevLevel& L, double* u64, float* u32, hipStream_t s);

int build_hierarchy(mg_handle_s* H, const double* phi);
bool build_band_chunks(mg_handle_s* H, int l, int own_target, int lds_budget,
                       double max_redundancy);
bool build_ext_chunks(mg_handle_s* H, int l, int own_target, int max_entries);
template <typename T>
void launch_extend_chunks(const DevLevel& L, T* r, hipStream_t s);

}  // namespace ghostmg
