// Launchers of the multigrid kernels (kernels.hip).
#pragma once
#include "ghostmg_impl.h"

namespace ghostmg {

constexpr int kCoarseRows = 16;  // rows of the coarsest inverse per workgroup (one per wave)
// unknowns per problem on the coarsest grid (its right-hand side is staged in 64 KB of LDS)
constexpr int kMaxCoarseUnknowns = 8192;

// Per-phase boundary relaxation (levels without relaxation chunks), in place on u.
template <typename T>
struct BandArgs {
  Geo g;
  const GhostRec* ghosts;
  const double* gw;
  const int32_t *ghost_off, *red, *black, *red_off, *black_off;
  T* u;
  const T* rhs;
  T* tmp;
  T h2, inv2d;
  double cD, cNh;
  int lambda;
};

// One relaxation from uin into uout: workgroups [0, nchunks) run the relaxation chunks,
// the rest the interior tiles.
template <typename T>
struct RelaxArgs {
  const int4* tiles;
  int ntiles, nbt;
  Geo g;
  const int8_t* rcls;
  const T* uin;
  T* uout;
  const T* rhs;
  // chunk entries of band and ghost nodes (mask bit 30) start from uband, the others from uin
  const T* uband;
  T h2, inv2d;
  int write_all;  // tiles also write band interior and ghost nodes (levels without chunks)
  int skip_band;  // tiles leave the band interior nodes unrelaxed (block relaxation owns them)
  int nchunks, phases;
  // packed layout: chunk c's header at hdr[c * kBandHdr], offsets into data; fixed layout
  // (band_fixed_layout): chunk c's data at data + c * stride, the header is not read
  const int32_t *hdr, *data;
  int stride;
  // interpolation of the coarse correction uc (level with geometry gc and classes clsc)
  // applied to uin before relaxing (prolong != 0)
  int prolong;
  Geo gc;
  const T* uc;
  const int8_t* clsc;
  // restriction of the finer level's defect rf (geometry gf) with this level's codes, into
  // rhs_w (the level's right-hand side), fused into a relaxation that starts from zero
  const T* rf;
  Geo gf;
  const uint8_t* rcode;
  T* rhs_w;
};

// Coarsest solve: the explicit FP64 inverse of every problem (rows of nu doubles at
// ainv_off[p]) times the FP64 right-hand side rhsc (compact, by unknown), which is first
// restricted from rf (geometry gf, the next finer level) when rf is set, or gathered from the
// level's right-hand side rhs; the product is rounded into the iterate u of the cycle's
// precision
template <typename T>
struct CoarseArgs {
  const int32_t *umap, *umap_off;
  const int64_t* ainv_off;
  const double* ainv;
  Geo gf;
  const int32_t* ufine;  // per unknown: finer node (2x, 2y, 2z) and restriction code
  const uint8_t* ucode;
  const T* rf;
  const T* rhs;
  double* rhsc;
  T* u;
};

// Defect r = rhs - A u: workgroups [0, nechunks) run the extension chunks (Eq. (exp)),
// then nbt workgroups the interior tiles, then the ghost rows.
template <typename T, typename TO>
struct DefectArgs {
  const int4* tiles;
  int ntiles, nbt;
  const GhostRec* ghosts;
  const double* gw;
  int nghost;
  Geo g;
  const int8_t* cls;
  const T* u;
  const T* rhs;
  TO* r;
  TO* rg;  // when not null: the ghost defects also stored by ghost id (extension gather)
  T inv_h2;
  uint64_t* norms;
  int nechunks;
  const int32_t *hdr, *data;  // extension chunk c: counts at hdr[c * kExtHdr], data at c * stride
  int stride;
};

// One complete relaxation (Sec. 2.4 step 1 with the boundary sweeps of Sec. 3.2): reads
// uin, writes every unknown of uout (uin != uout).  With C, the relaxation starts from
// uin + the interpolation of the coarse correction uc (Sec. 2.6.1, step 6 of the cycle).
// With F, the relaxation starts from zero, with the right-hand side restricted from the
// finer level F's defect rf (Sec. 2.5, steps 4-5 of the cycle), which it also stores in rhs.
template <int D, typename T>
void launch_relax(const DevLevel& L, const mg_grid& G, const T* uin, T* uout, const T* rhs,
                  T* tmp, int batch, hipStream_t s, const DevLevel* C = nullptr,
                  const T* uc = nullptr, const DevLevel* F = nullptr, const T* rf = nullptr);
// Defect of u into r; with_ext also extends it outside Omega_h (Eq. (exp)).  norms, when
// given, receives the per-problem infinity norms (no extension then).
template <int D, typename T, typename TO>
void launch_defect(const DevLevel& L, const T* u, const T* rhs, TO* r, uint64_t* norms,
                   bool with_ext, int batch, hipStream_t s);
template <int D>
void launch_rhs_norm(const DevLevel& L, const double* rhs, uint64_t* norms, hipStream_t s);
template <int D, typename T>
void launch_restrict(const DevLevel& F, const DevLevel& C, const T* rf, T* rhsc, T* uc,
                     hipStream_t s);
template <int D, typename T>
void launch_prolong(const DevLevel& F, const DevLevel& C, const T* uc, T* uf, hipStream_t s);
// coarsest solve; with F (the next finer level) its FP64 right-hand side is first restricted
// from rf, F's defect (a launch of its own); without F it is the one last restricted, or,
// with from_rhs (a hierarchy of one level), it is taken from rhs
template <int D, typename T>
void launch_coarse(const DevLevel& C, const DevLevel* F, const T* rf, T* rhs, T* u, int batch,
                   bool from_rhs, hipStream_t s);
template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t s);
void launch_scale(double* p, int64_t n, double v, hipStream_t s);
template <int D>
void launch_pack(const DevLevel& L, const double* f, const double* g, const double* uin,
                 double* rhs, double* u, hipStream_t s);
template <int D>
void launch_unpack(const DevLevel& L, int batch, const double* src, double* dst, hipStream_t s);
template <int D>
void launch_warm_start(const DevLevel& L, const DevLevel& Lprev, int batch, double* u,
                       hipStream_t s);
template <int D>
void launch_dc_update(const DevLevel& L, double* u64, const float* u32, float* u32_zero,
                      hipStream_t s);

// dynamic LDS bytes of launch_defect for a level
size_t defect_lds(const DevLevel& L);

// phi: device memory
int build_hierarchy(mg_handle_s* H, const double* phi);
// relaxation chunks of level l with the largest phase count per launch, at most Rmax, that
// fits (HostLevel::bc_range); false when none fits
bool build_band_chunks(mg_handle_s* H, int l, int own_target, double max_redundancy, int Rmax);
bool build_ext_chunks(mg_handle_s* H, int l, int own_target);
bool build_ext_terms(mg_handle_s* H, int l);

}  // namespace ghostmg
