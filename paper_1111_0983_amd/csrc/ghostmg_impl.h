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
// header words of a relaxation chunk and of an extension chunk
constexpr int kBandHdr = 8;
constexpr int kExtHdr = 8;
// extension chunks: workgroup size, extension nodes per thread
constexpr int kExtThreads = 256;
constexpr int kExtPerThread = 4;
constexpr int kExtMaxEntries = kExtPerThread * kExtThreads;
constexpr int kExtMaxTerms = 6 * kExtThreads;   // composed extension terms per chunk
constexpr int kExtMaxGhosts = 2 * kExtThreads;  // ghost sources per extension chunk
// relaxation chunks: workgroup size (larger in 3D, where a band patch must be wide for its
// closure over several phases to stay a small multiple of it); per thread one updated
// ghost, band_colour_slots(D) red and as many black entries, band_halo_slots(D) entries
// that are read but never updated (more in 3D, where a band patch's closure has more of
// them).  In 2D a thread updates one entry per colour phase (short phases, more chunks); in
// 3D two (the level-0 chunk work is large and more chunks would add redundant entries)
constexpr int band_chunk_threads(int D) { return D == 2 ? 256 : 512; }
constexpr int band_colour_slots(int D) { return D == 2 ? 1 : 2; }
constexpr int kBandHaloSlots2D = 1, kBandHaloSlots3D = 4;
constexpr int band_halo_slots(int D) { return D == 2 ? kBandHaloSlots2D : kBandHaloSlots3D; }
constexpr int band_max_entries(int D) {
  return (1 + 2 * band_colour_slots(D) + band_halo_slots(D)) * band_chunk_threads(D);
}
// 2D chunks use the fixed layout: every chunk's data has the level's size (bc_stride words)
// and every entry sits at its slot position, so that a workgroup finds its data at
// chunk * bc_stride without first reading the chunk's header (one dependent load fewer
// before the first phase).  3D keeps the packed layout (its chunks are half full, and
// a fixed layout would double the data the launch reads).
constexpr bool band_fixed_layout(int D) { return D == 2; }
// Extension chunks always use a fixed layout (offsets in int32 words, every chunk
// ext_fixed(D).stride words at chunk * stride): ghost-source nodes [0, kExtMaxGhosts) and the
// extension nodes after them, the term offsets (kExtMaxEntries + 1), the term source ids, the
// term weights (FP64), the ghost stencil nodes and weights (tap-major, stride
// kExtMaxGhosts); positions beyond a chunk's counts hold node 0, weight 0 and the last term
// offset, so a workgroup issues its first loads before its header (the counts) arrives.
struct ExtFixed {
  int NODES, TO, TS, TW, GN, GW, stride;
};
constexpr ExtFixed ext_fixed(int D) {
  const int K = D == 2 ? 9 : 27, GS = kExtMaxGhosts, NE = kExtMaxEntries, MT = kExtMaxTerms;
  const int TO = GS + NE, TS = TO + (NE + 1 + 1) / 2 * 2, TW = TS + (MT + 1) / 2 * 2;
  const int GN = TW + 2 * MT, GW = GN + (K * GS + 1) / 2 * 2;
  return ExtFixed{0, TO, TS, TW, GN, GW, GW + 2 * K * GS};
}
// Offsets (int32 words) of the fixed layout: slots S = 1 + 2 band_colour_slots(D) +
// band_halo_slots(D), W = band_chunk_threads(D), NSW = S W entries: node (-1 where empty),
// mask, D neighbour words per entry, then the ghost rows (LDS tap addresses two per word, and
// weights in the cycle's precision, tap-major with stride W; the regions keep the size of
// one word per tap and FP64 weights), c_G per ghost slot, the interpolation candidates and
// the restriction pairs (per entry, where the level has them).
struct BandFixed {
  int NSW, W, GID, GW, GC, PC, RS, stride;
};
constexpr BandFixed band_fixed(int D, bool pc, bool rs) {
  const int W = band_chunk_threads(D), NSW = band_max_entries(D), K = D == 2 ? 9 : 27;
  const int GID = (2 + D) * NSW, GW = GID + (K * W + 1) / 2 * 2, GC = GW + 2 * K * W;
  const int PC = GC + 2 * W, RS = PC + (pc ? NSW : 0);
  return BandFixed{NSW, W, GID, GW, GC, PC, RS, RS + (rs ? 2 * NSW : 0)};
}

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
  // node codes of the relaxation: 0 outside, 1 interior off the band, 2 ghost, 3 interior
  // band node (the boundary band of Sec. 3.2)
  std::vector<int8_t> rcls;
  std::vector<double> gw;               // Pow3<D> row weights per ghost (0 for unused taps)
  // Relaxation chunks: each chunk owns band and ghost nodes and carries every node that
  // their values after a launch's phases depend on; a relaxation is 3 + 3 lambda phases (red
  // interior, black interior, ghosts; lambda times red band, black band, ghosts), taken
  // bc_range at a time, with a chunk set per launch.
  // Entries come in four runs (W = band_chunk_threads(D)): the updated ghosts (at most W),
  // the entries the red phases update, those the black phases update (at most
  // band_colour_slots(D) * W each), and the entries only read (at most band_halo_slots(D) *
  // W); entry i of a run belongs to thread i % W.  Chunk c: header
  // bc_hdr[c * kBandHdr ..] = {entries, updated ghosts | red << 10 | black << 21, offsets
  // into bc_data of: the per-entry arrays, the ghost stencil ids, the ghost
  // weights, the ghost constants, the interpolation candidates (-1 on the coarsest level)
  // and the restriction data (-1 on the finest level)}: per entry the coarse node index of
  // its interpolation candidate 0 (candidate m adds the coarse stride of each axis q with bit
  // q of m), and 2 words: the fine node index of (2x, 2y, 2z) and the restriction code.
  // Per-entry arrays (int32 words): node index; mask (bit p < R: updated in phase p of the
  // launch's R phases; bits [R, R + D): odd coordinates; bits [R + D, R + D + 2^D):
  // interpolation candidate m exists and carries an unknown; bit 30: band or ghost node;
  // bit 31: owned, written to the output); D words of
  // (minus, plus) int16 local neighbour ids per axis.  Per ghost (tap-major, ghost fastest):
  // the LDS addresses of its Pow3<D> taps, two 16-bit addresses per word (a tap on a ghost
  // entry reads that ghost's value before the ghost phase, held at ns + its id; any other tap
  // the entry's value at its id; taps of zero weight name the ghost's own earlier value), and
  // the weights (0 for those taps) in the precision of the cycles (FP32 with FP32 cycles);
  // one FP64 constant c_G.  That is the packed layout (3D); in 2D
  // (band_fixed_layout) the same arrays sit at the fixed offsets of band_fixed(), entry i of a
  // run at its slot position, the ghost rows with stride W, and the header's first word is
  // the slot count.
  std::vector<int32_t> bc_hdr;
  std::vector<int32_t> bc_data;
  int bc_nchunks = 0, bc_smax = 0, bc_nown = 0;
  // phases per launch (whole sweeps dividing 3 + 3 lambda) and the first chunk of each
  // launch's set (bc_sub[k] .. bc_sub[k + 1])
  int bc_range = 0;
  std::vector<int> bc_sub;
  int bc_stride = 0;  // band_fixed_layout: words per chunk (chunk c's data at c * bc_stride)
  int64_t bc_entries = 0;               // sum of chunk sizes (redundant work included)
  // Extension chunks.  The steady state of Eq. (exp) on the upwind graph is linear in the
  // ghost defects: every extension value is a fixed combination of the defects of the ghost
  // nodes its upwind paths start from, with weights composed on the host.  Each chunk owns a
  // run of extension nodes (at most kExtMaxEntries) and evaluates the defects of the ghost
  // sources they need (at most kExtMaxGhosts).  Chunk c: header
  // ec_hdr[c * kExtHdr ..] = {extension nodes, ghost sources, offsets into ec_data of: the node
  // indices (ghost sources, then extension nodes), the term offsets (per extension node and
  // one past the end, relative to the chunk's first term), the term source ids (local ghost
  // ids), the term weights (FP64), the ghost stencil nodes (tap-major), the ghost row
  // weights (FP64, tap-major)}; at most kExtMaxTerms terms, stored at the fixed offsets of
  // ext_fixed() (chunk c at c * ec_stride).  ec_smax: the largest chunk's LDS in doubles
  // (ghost values, term weights, term ids).
  std::vector<int32_t> ec_hdr;
  std::vector<int32_t> ec_data;
  int ec_nchunks = 0, ec_smax = 0, ec_stride = 0;
  // the same composed terms as flat arrays (3D: a gather after the defect, which has already
  // written the ghost defects): extension node, term offsets (records + 1), ghost index (in
  // the level's ghost list) and weight of every term
  std::vector<int32_t> et_node, et_off, et_src;
  std::vector<double> et_wt;
  // coarsest level
  std::vector<int32_t> umap;            // unknown node indices, by problem
  std::vector<int32_t> umap_off;        // batch + 1
  std::vector<int64_t> ainv_off;        // batch + 1 offsets into ainv
  std::vector<double> ainv;             // explicit inverse of each coarsest matrix
};

// One level of one problem classified on the GPU: the level's phi (unpadded node order, x
// fastest), node classes (0 outside, 1 interior, 2 ghost), ghost records in node order (node =
// unpadded local index) and their closest points B (3 per ghost).  phi0: the level-0 phi of
// every problem in device memory; rule: the problem's half-space rule, or null when a caller's
// partition decides the types (the records then have type 0, a normal for every ghost that
// has one, and pad0 = 1 where it has none).  MG_EINVAL for a non-finite phi, MG_EGEOM for
// geometry the discretisation does not cover.
struct LevelClass {
  std::vector<double> phi;
  std::vector<int8_t> cls;
  std::vector<GhostRec> gh;
  std::vector<double> B;
};
int classify_level_gpu(const double* phi0, int D, int n0, int l, int problem, double lo, double h,
                       const mg_bc_rule* rule, LevelClass& out);

struct DevLevel {
  Geo g;
  int ntiles = 0, nghost = 0, nred = 0, nblack = 0, next = 0, ndag = 0;
  int max_gp = 0, max_bandp = 0, max_extp = 0;   // largest per-problem list sizes
  int nchunks = 0, bc_phases = 0, bc_smax = 0, bc_stride = 0;
  // launches per relaxation (bc_phases each) and their chunk ranges; z64 / z32: the band
  // values between launches when there is more than one
  int nsub = 0;
  int sub[8] = {};
  double* z64 = nullptr;
  float* z32 = nullptr;
  int32_t* band_list = nullptr;  // band and ghost nodes (copied back after an even count)
  int nband_list = 0;
  int32_t *bc_hdr = nullptr, *bc_data = nullptr;
  int nechunks = 0, ec_smax = 0, ec_stride = 0;
  int32_t *ec_hdr = nullptr, *ec_data = nullptr;
  int net = 0;
  int32_t *et_node = nullptr, *et_off = nullptr, *et_src = nullptr;
  // term weights in the precision of the cycles (FP32 with FP32 cycles), and the ghost
  // defects by ghost id (nghost values of that precision), written by the defect launch
  void* et_wt = nullptr;
  void* et_rg = nullptr;
  int8_t* rcls = nullptr;
  double* gw = nullptr;
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
  // boundary relaxations of the comparison (grid.smoother 1, 2): the band nodes and ghosts
  // (node, ghost index or -1) by problem and colour; alt_off[p * (alt_ncol + 1) + c]
  int alt_ncol = 0;
  int2* alt_list = nullptr;
  int32_t* alt_off = nullptr;
  // arrays [batch * npp]; the iterate has two buffers, a relaxation reads one and writes
  // the other
  double *u64[2] = {nullptr, nullptr}, *rhs64 = nullptr, *r64 = nullptr, *gtmp64 = nullptr;
  float *u32[2] = {nullptr, nullptr}, *rhs32 = nullptr, *r32 = nullptr, *gtmp32 = nullptr;
  // coarsest level
  int nu_max = 0, nu_total = 0;  // largest per-problem and total unknown counts
  int32_t *umap = nullptr, *umap_off = nullptr;
  int64_t* ainv_off = nullptr;
  double* ainv = nullptr;
  double* rhsc = nullptr;   // FP64 right-hand side by unknown (nu_total), either precision
  // per coarsest unknown: the next finer level's node (2x, 2y, 2z) and the restriction code
  int32_t* ufine = nullptr;
  uint8_t* ucode = nullptr;
};

}  // namespace ghostmg

struct mg_handle_s {
  mg_grid grid;
  std::vector<mg_bc_rule> bc;
  mg_bc_fn bc_fn = nullptr;            // caller's partition (setup only), else the rules
  void* bc_ctx = nullptr;
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
  // one FP64 cycle starting from finest iterate buffer 0 or 1 (a cycle with an odd number
  // of finest relaxations ends in the other buffer), [c][1] followed by the defect norm of
  // its result, [c][0] without it
  hipGraphExec_t graph_cycle[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t graph_dc = nullptr;     // one defect-correction step + defect norm
  // the same step with r < inner_cycles FP32 cycles at index r (a last step that needs
  // less than a full one)
  std::vector<hipGraphExec_t> graph_dc_short;
  int cur0 = 0;                          // buffer holding the finest FP64 iterate
  int cur[ghostmg::kMaxLevels] = {};     // per level current buffer while recording
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
