// Internal data structures of the ghost-cell multigrid library (host side and the views
// the kernels receive).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ghostmg.h"
#include "stencil.h"

namespace ghostmg {

constexpr int kMaxLevels = 16;

// Tile shapes of the node-parallel kernels: 64 x 16 nodes in 2D, 16 x 8 x 8 in 3D.
template <int D>
struct Tile;
template <>
struct Tile<2> {
  static constexpr int X = 64, Y = 16, Z = 1;
};
template <>
struct Tile<3> {
  static constexpr int X = 16, Y = 8, Z = 8;
};

struct ExtRec {       // 40 bytes: one extension node and its upwind sources (Eq. (exp))
  int32_t node;
  int32_t src[3];     // -1 where absent
  double wt[3];       // |n_a| of the available sources
};
static_assert(sizeof(ExtRec) == 40, "ExtRec layout");

// Geometry of one level as seen by a kernel.
struct Geo {
  int n;              // intervals per axis
  int np;             // n + 1
  int pitch;          // x stride (>= np, multiple of 16)
  int64_t st[3];      // strides of x, y, z
  int64_t npp;        // nodes per problem (padded)
  double h;
};

// Host-side product of the setup for one level (all problems of the batch).
struct HostLevel {
  Geo g;
  std::vector<int8_t> cls;              // batch * npp
  std::vector<double> phi;              // batch * npp (levels >= 1: network features)
  std::vector<GhostRec> ghosts;         // ordered by (problem, node)
  std::vector<double> gB;               // 3 per ghost (closest points, for queries)
  std::vector<int32_t> ghost_off;       // batch + 1
  std::vector<int32_t> red, black;      // interior band nodes by colour
  std::vector<int32_t> red_off, black_off;
  std::vector<ExtRec> ext;              // extension towards level + 1, by (problem, DAG level)
  std::vector<int32_t> ext_off;         // batch + 1
  std::vector<int32_t> dag_off;         // per problem: DAG level boundaries, flattened
  std::vector<int32_t> dag_start;       // batch + 1: index of the problem's first boundary
  std::vector<int32_t> gdag_off;        // DAG level boundaries over all problems merged
  std::vector<ExtRec> ext_merged;       // ext ordered by (DAG level, problem)
  std::vector<uint8_t> rcode;           // restriction code of every node of this level
  std::vector<int4> tiles;              // (problem, tx, ty, tz) of tiles holding unknowns
  int64_t nint = 0, nghost = 0, nband = 0;
  // boundary band in LDS-resident chunks: each chunk owns band/ghost nodes and carries
  // every node its owned results depend on through the 1 + 3 lambda relaxation phases
  std::vector<int32_t> bc_off;          // chunks + 1: offsets into bc_node
  std::vector<int32_t> bc_own;          // chunks: owned nodes (the first entries of the chunk)
  std::vector<int32_t> bc_out_off;      // chunks + 1: offsets of the owned results
  std::vector<int32_t> bc_node;         // node of every chunk entry
  std::vector<int16_t> bc_nbr;          // 2D local neighbour ids per entry (-1 unused)
  std::vector<int32_t> bc_goff;         // chunks + 1: offsets into the ghost slots
  std::vector<int16_t> bc_gent;         // per ghost slot: its local entry id
  std::vector<int32_t> bc_gidx;         // per ghost slot: ghost record index
  std::vector<int16_t> bc_gsten;        // per ghost slot: 3^D local stencil ids (-1 unused)
  std::vector<int16_t> bc_ops;          // per phase: local entry ids (interior phases) or
                                        // ghost slots (ghost phases)
  std::vector<int32_t> bc_ops_off;      // chunks * (phases + 1)
  std::vector<int32_t> bc_own_node;     // owned nodes in output order
  int bc_smax = 0, bc_gmax = 0, bc_opsmax = 0;  // largest chunk, ghost slots, op list
  // defect extension in LDS-resident chunks: owned extension nodes, the extension nodes
  // they depend on, then the ghost defects they read
  std::vector<int32_t> ec_off;          // chunks + 1: offsets into ec_node
  std::vector<int32_t> ec_own;          // chunks: owned entries (first)
  std::vector<int32_t> ec_next;         // chunks: extension entries (owned + dependencies)
  std::vector<int32_t> ec_node;         // node of every entry
  std::vector<int16_t> ec_src;          // 3 local source ids per entry (-1 absent)
  std::vector<double> ec_wt;            // 3 weights per entry
  std::vector<int16_t> ec_ops;          // extension entries by DAG level
  std::vector<int32_t> ec_lvl;          // DAG level boundaries into ec_ops, flattened
  std::vector<int32_t> ec_lvl_start;    // chunks + 1: first boundary of each chunk
  int ec_smax = 0;
  // coarsest level
  std::vector<int32_t> umap;            // unknown node indices, by problem
  std::vector<int32_t> umap_off;        // batch + 1
  std::vector<int64_t> ainv_off;        // batch + 1 offsets into ainv
  std::vector<double> ainv;             // explicit inverse of each coarsest matrix
};

struct DevLevel {
  Geo g;
  int ntiles = 0, nghost = 0, nred = 0, nblack = 0, next = 0, ndag = 0;
  int max_gp = 0, max_bandp = 0, max_extp = 0;   // largest per-problem list sizes
  int nchunks = 0, bc_smax = 0, bc_gmax = 0, bc_opsmax = 0, bc_nown = 0, bc_phases = 0;
  int32_t *bc_off = nullptr, *bc_own = nullptr, *bc_out_off = nullptr, *bc_node = nullptr,
          *bc_goff = nullptr, *bc_gidx = nullptr, *bc_ops_off = nullptr, *bc_own_node = nullptr;
  int16_t *bc_nbr = nullptr, *bc_gent = nullptr, *bc_gsten = nullptr, *bc_ops = nullptr;
  double* bc_out64 = nullptr;
  float* bc_out32 = nullptr;
  int nechunks = 0, ec_smax = 0;
  int32_t *ec_off = nullptr, *ec_own = nullptr, *ec_next = nullptr, *ec_node = nullptr,
          *ec_lvl = nullptr, *ec_lvl_start = nullptr;
  int16_t *ec_src = nullptr, *ec_ops = nullptr;
  double* ec_wt = nullptr;
  int8_t* cls = nullptr;
  double* phi = nullptr;
  int4* tiles = nullptr;
  GhostRec* ghosts = nullptr;
  int32_t *ghost_off = nullptr, *red = nullptr, *black = nullptr, *red_off = nullptr,
          *black_off = nullptr;
  ExtRec *ext = nullptr, *ext_merged = nullptr;
  int32_t *ext_off = nullptr, *dag_off = nullptr, *dag_start = nullptr;
  std::vector<int32_t> gdag_off;        // host copy for the per-DAG-level launches
  uint8_t* rcode = nullptr;
  // arrays [batch * npp]
  double *u64 = nullptr, *rhs64 = nullptr, *r64 = nullptr, *gtmp64 = nullptr;
  float *u32 = nullptr, *rhs32 = nullptr, *r32 = nullptr, *gtmp32 = nullptr;
  // coarsest level
  int nu_max = 0;
  int32_t *umap = nullptr, *umap_off = nullptr;
  int64_t* ainv_off = nullptr;
  double* ainv = nullptr;
};

}  // namespace ghostmg

struct mg_handle_s {
  mg_grid grid;
  std::vector<mg_bc_rule> bc;
  int L = 0;                          // index of the coarsest level
  int batch = 1;
  int dim = 2;
  hipStream_t stream = nullptr;      // stream all work is ordered on
  hipStream_t own_stream = nullptr;  // the handle's own stream (used when none is set)
  std::vector<ghostmg::HostLevel> host;
  std::vector<ghostmg::DevLevel> dev;
  uint64_t* norms = nullptr;          // device: [batch][2] interior / ghost max |r| bits
  double* norms_host = nullptr;       // pinned host mirror
  double* r0 = nullptr;               // per problem ||(f_h, g_h)||_inf (host)
  std::vector<double> history;
  hipGraphExec_t graph_cycle = nullptr;  // one FP64 cycle + defect norm
  hipGraphExec_t graph_dc = nullptr;     // one defect-correction step + defect norm
  const double* graph_f = nullptr;       // arrays the graphs were captured with
  bool band_single_wg = true;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
