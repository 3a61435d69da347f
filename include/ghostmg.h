/*
 * ghostmg.h -- C ABI of the MI355X (gfx950) ghost-cell multigrid Poisson solver.
 *
 * The solver computes the unique solution of the discrete system of Coco and Russo,
 * arXiv 1111.0983, Eq. (discr): the 5-point (2D) or 7-point (3D) Laplacian
 * -Delta_h u = f at the interior nodes Omega_h = {phi < 0} and the boundary rows
 * L_h u = g at the ghost nodes Gamma_h (Sec. 2.3, Eqs. (clpt), (St_G), (discrBC)),
 * for a domain given by a signed distance function phi sampled at the nodes of the box
 * [lo, hi]^dim (Sec. 2.2).  It iterates the multigrid cycle of Sec. 2.4 - 2.6 (red-black
 * relaxation of Eqs. (jac2d), (dir2d), (neu2d), the lambda extra boundary sweeps of
 * Sec. 3.2, defect extension Eq. (exp), partial full-weighting restriction
 * Eqs. (Fstencil)-(Fstencil22), multilinear interpolation, exact coarsest solve) on the
 * GPU until ||r||_inf / ||(f_h, g_h)||_inf <= tol.
 *
 * Layout of every node array: (n+1)^dim FP64 values per problem, x fastest, then y, then
 * z; problems of a batch are consecutive.  Node j has coordinates lo + h j, h = (hi-lo)/n.
 *
 * Ownership: the caller owns every pointer it passes; the handle owns all level data and
 * keeps no reference to caller memory after a call returns.  Calls on one handle are not
 * thread-safe; work is ordered on the handle's stream (mg_set_stream, default the null
 * stream).  Every call returns MG_OK (0) or a negative mg_status; no C++ exception
 * crosses this interface.  mg_strerror() names a code.
 */
#ifndef GHOSTMG_H
#define GHOSTMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_handle_s* mg_handle_t;

enum mg_status {
  MG_OK = 0,
  MG_EINVAL = -1,     /* bad argument: grid sizes, NaN input, null pointer */
  MG_ENOMEM = -2,     /* host or device allocation failed */
  MG_EHIP = -3,       /* a HIP runtime call failed */
  MG_EGEOM = -4,      /* unusable geometry: empty coarsest level, zero normal, singular
                         coarsest matrix (e.g. a component with no Dirichlet ghost) */
  MG_ENOCONV = -5,    /* max_cycles reached before the tolerance */
  MG_EDIVERGED = -6   /* non-finite residual, or growth over five consecutive cycles */
};

enum mg_precision {
  MG_FP64 = 0,        /* every cycle in FP64 */
  MG_FP32_DC = 1      /* FP32 cycles on the correction inside an FP64 defect correction */
};

typedef struct {
  int dim;            /* 2 or 3 */
  int n;              /* intervals per axis on the finest grid */
  double lo, hi;      /* the box [lo, hi]^dim; the domain must not touch its faces */
  int n_coarse;       /* intervals on the coarsest grid; n = n_coarse * 2^L */
  int nu1, nu2;       /* pre- and post-relaxations (V(2,1): 2, 1) */
  int gamma;          /* 1 = V-cycle, 2 = W-cycle (Sec. 1.3, Remarks 1-2) */
  int lambda;         /* extra boundary sweeps per relaxation (Sec. 3.2: 5) */
  double delta_h;     /* band width in units of h (Sec. 3.2: 3) */
  double cD;          /* mu_D dt of Eq. (dir2d) (0.9) */
  double cN;          /* mu_N dt = cN h of Eq. (neu2d) (0.9 * 2 / (3 sqrt(dim))) */
  int split;          /* 1: Dirichlet and Neumann defects are extended and restricted
                         separately; 0: one outside pass over D_h - Omega_h */
  int precision;      /* mg_precision */
  int inner_cycles;   /* FP32 cycles per defect-correction step (MG_FP32_DC); mg_solve's
                         last step runs fewer when the measured convergence factor says
                         they reach tol with a factor 2 to spare */
  int max_cycles;     /* cycle budget of mg_solve (FP64 cycles, or FP32 cycles in DC) */
  int batch;          /* independent problems solved together (>= 1) */
  int smoother;       /* boundary relaxation (Sec. 3.3): 0 = ghost relaxation with lambda
                         extra band sweeps (the paper's method); 1 = lambda Kaczmarz sweeps
                         over the band after the interior sweep; 2 = one block relaxation of
                         every band node after a sweep of the interior off the band (2D).
                         1 and 2 sweep the band colour by colour (colour (x mod M) + M (y mod M)
                         + M^2 (z mod M), M = 5 / 7), one workgroup per problem: meant for the
                         comparison of Sec. 3.3 on small grids */
} mg_grid;

/* Dirichlet at a ghost iff a . B + c > 0 (strict) or >= 0 (not strict), B its closest
 * boundary point (Sec. 2.1: the partition of the boundary into Gamma_D and Gamma_N). */
typedef struct {
  double a[3];
  double c;
  int strict;
} mg_bc_rule;

typedef struct {
  int status;           /* the call's return code */
  int cycles;           /* multigrid cycles run (FP32 cycles in DC mode) */
  int outer;            /* defect-correction steps (DC mode), else 0 */
  double rel_residual;  /* final max over problems of ||r||_inf / ||(f_h, g_h)||_inf */
  double solve_ms;      /* wall time of the call on its stream */
  const double* history;/* relative residual (max over problems) at each residual check:
                           before the first cycle, after every cycle (or DC step) until a
                           convergence factor is known, then after the batch of cycles the
                           factor predicts are still needed minus one; owned by the handle,
                           valid until the next solve or mg_free */
  int history_len;
} mg_stats;

/* A caller-defined partition of the boundary (Sec. 2.1: the boundary is the union of
 * Gamma_D and Gamma_N): returns nonzero when the boundary point B (3 coordinates, unused
 * ones 0) of problem `problem` belongs to Gamma_D, 0 when it belongs to Gamma_N. */
typedef int (*mg_bc_fn)(int problem, const double* B, void* ctx);

/* Fill *g with the paper's constants (lambda 5, delta 3h, mu dt 0.9 / 0.9 * 2h/(3 sqrt d)),
 * V(2,1), FP64 (3 inner cycles per step if precision is set to MG_FP32_DC), batch 1,
 * box [-1, 1]^dim. */
int mg_grid_default(mg_grid* g, int dim, int n, int n_coarse);

/* Build the level hierarchy (Sec. 2.4: each grid rediscretises the problem from phi at its
 * nodes).  phi: batch * (n+1)^dim values, host or device memory, negative inside.
 * bc: batch rules (host memory).  On success *out receives a new handle. */
int mg_setup(const double* phi, const mg_bc_rule* bc, const mg_grid* grid, mg_handle_t* out);

/* mg_setup with the Dirichlet/Neumann partition given by fn instead of half-space rules.
 * fn is called on the host during this call only (never afterwards), with ctx, at the
 * closest boundary point of every ghost and of every outside node of the defect extension,
 * on every level; it must be deterministic.  MG_EINVAL when fn is NULL. */
int mg_setup_partition(const double* phi, mg_bc_fn fn, void* ctx, const mg_grid* grid,
                       mg_handle_t* out);

/* Order all later work of the handle on this hipStream_t (NULL = null stream). */
int mg_set_stream(mg_handle_t h, void* hip_stream);

/* Level sizes: info[0] n, [1] interior nodes, [2] ghost nodes, [3] interior band nodes,
 * [4] extension nodes, [5] tiles, [6] coarsest unknowns (last level only), [7] levels;
 * summed over the batch. */
int mg_query_level(mg_handle_t h, int level, int64_t* info);

/* Ghost points of one problem on one level, in increasing node index.  Two-call use: with
 * node == NULL only *count is written.  node: node index within the problem; B, nB: 3
 * values per ghost (closest point, unit normal at B used by Neumann rows); type: 1
 * Dirichlet, 0 Neumann; rung: stencil rung 1..4.  Host memory. */
int mg_query_ghosts(mg_handle_t h, int problem, int level, int64_t* count, int64_t* node,
                    double* B, double* nB, int8_t* type, int8_t* rung);

/* Node classes of one problem on one level: 0 outside, 1 interior, 2 ghost (host memory,
 * (n_level+1)^dim bytes). */
int mg_query_classes(mg_handle_t h, int problem, int level, int8_t* cls);

/* Solve to ||r||_inf <= tol ||(f_h, g_h)||_inf.  f: read on Omega_h; g: read on Gamma_h
 * (g(B) at ghost G); u: in/out initial guess, on return the solution on Omega_h u Gamma_h
 * and 0 elsewhere.  Device memory, batch * (n+1)^dim FP64 each.  st may be NULL. */
int mg_solve(mg_handle_t h, const double* f, const double* g, double* u, double tol,
             mg_stats* st);

/* Exactly ncycles cycles from u, no tolerance test (iterate-level checks). */
int mg_cycles(mg_handle_t h, const double* f, const double* g, double* u, int ncycles);

/* Warm start for a moving domain (a sequence of problems on one grid): u (device, batch *
 * (n+1)^dim FP64, in place) holds the solution computed with handle `prev`; every node that
 * is an unknown of h but was not one of prev (a node the boundary has moved over, typically
 * a new ghost) takes the mean of the linear extrapolations 2 u(Q1) - u(Q2) from the axis
 * directions where Q1, Q2 (one and two nodes inward) are unknowns of both handles, or the
 * mean of such axis neighbours, or 0.  Other values are kept.  Without it the new nodes hold
 * 0 and their interior neighbours' rows start with defects of order u / h^2.  Both handles
 * must have the same grid and batch (MG_EINVAL otherwise). */
int mg_warm_start(mg_handle_t h, mg_handle_t prev, double* u);

/* Convergence factor of the cycle (Sec. 3): the homogeneous problem (f = g = 0) iterated
 * from u0 (device, batch * (n+1)^dim FP64, read only), rho^(m) = ||r^(m)||_inf /
 * ||r^(m-1)||_inf (max over the batch, interior and ghost parts), the iterate rescaled after
 * every cycle; stops when |rho^(m) - rho^(m-1)| / rho^(m) < rtol (rtol 0: never), when
 * rho^(m) > 1e3 or the defect vanishes or is not finite, or after max_cycles.  *rho: the
 * last factor; hist (host, max_cycles values, may be NULL): rho^(m) for m = 1..*ncycles.
 * The two-grid cycle of the paper is a hierarchy of two levels (n_coarse = n / 2).
 * FP64 handles only (MG_EINVAL otherwise); MG_EINVAL also for a zero initial defect. */
int mg_rho(mg_handle_t h, const double* u0, int max_cycles, double rtol, double* rho,
           double* hist, int* ncycles);

/* Defect r = (f + Delta_h u on Omega_h, g - L_h u on Gamma_h, 0 elsewhere) of the finest
 * level (Sec. 2.4 step 3); r may be NULL.  norms (host, 2 * batch values): the infinity
 * norms of the interior and ghost parts per problem. */
int mg_residual(mg_handle_t h, const double* f, const double* g, const double* u, double* r,
                double* norms);

/* Time one launch of the cycle at one level on the handle's stream with HIP events, run
 * reps times after one warm-up; kernel 0 = one relaxation (red-black interior sweep with the
 * ghost relaxation and the lambda boundary sweeps of Sec. 3.2; one launch on levels with
 * relaxation chunks), 1 = defect with its extension, Eq. (exp), 2 = restriction,
 * 3 = interpolation + correction, 4 = defect with its norms (the stopping test), 5 = a
 * relaxation that first takes the interpolated correction of level + 1 (the cycle's first
 * post-relaxation), 6 = a relaxation from zero with the right-hand side restricted from
 * level - 1 (the cycle's first pre-relaxation on a coarse level; 2D, else a restriction
 * launch followed by a relaxation), 7 = the coarsest solve (its right-hand side restricted
 * from level - 1's defect, as in a cycle, then the inverse times it).
 * level runs from 0 to the level above the coarsest (6: from 1; 7: the coarsest level only),
 * else MG_EINVAL.  The level's iterate,
 * defect and coarse arrays are overwritten; a later mg_solve is unaffected.  avg_ms: mean duration; bytes: the
 * algorithmic HBM bytes per launch (every array element it must read or write once: per
 * unknown the iterate read and written, the right-hand side and the node code; per ghost
 * its row weights; per extension node its value and weights). */
int mg_time_kernel(mg_handle_t h, int kernel, int level, int reps, double* avg_ms,
                   double* bytes);

/* Level-set reinitialisation, Eq. (sdf) (Sec. 2.2): `iters` forward-Euler steps (dt = h / 2)
 * of d phi / d t = sgn(phi0) (1 - |grad phi|) from phi = phi0, which turn a level-set function
 * into a signed distance function near its zero set, as mg_setup assumes (a few mesh widths
 * per step pair; the zero set does not move).  Upwind (Godunov) |grad phi| away from the
 * boundary; nodes next to it (phi0 changes sign or vanishes towards an axis neighbour) relax
 * towards phi0 / |grad phi0|.  phi0, phi, tmp: device memory, batch * (n+1)^dim FP64 each on
 * the box [lo, hi]^dim (x fastest), three distinct buffers; phi receives the result, tmp is
 * scratch.  Work is ordered on `stream` (hipStream_t, NULL = null stream). */
int mg_reinit(int dim, int n, int batch, double lo, double hi, const double* phi0, int iters,
              double* phi, double* tmp, void* stream);

void mg_free(mg_handle_t h);

const char* mg_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GHOSTMG_H */
