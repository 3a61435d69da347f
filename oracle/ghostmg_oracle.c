/*
 * ghostmg_oracle.c -- plain FP64 CPU oracle for the ghost-cell multigrid method of
 * A. Coco and G. Russo, "A Finite Difference Ghost-cell Multigrid approach for Poisson
 * Equation with mixed Boundary Conditions in Arbitrary Domain" (arXiv 1111.0983).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library; the two are written independently from the paper.
 *
 * Everything is dimension-generic (d = 1, 2, 3), slow and direct:
 *   - discretisation: interior rows Eq. (jac2d) / 5- or 7-point Delta_h (Sec. 2.3),
 *     ghost rows Eq. (discrBC) built from the closest point Eq. (clpt) and the upwind
 *     stencil Eq. (St_G), reduced stencils of Remark 3;
 *   - relaxation: Eqs. (jac2d), (dir2d), (neu2d) in GS-LEX order (Sec. 2.4) or in a
 *     red-black order with Jacobi ghost updates (the ordering the GPU uses), followed by
 *     lambda extra sweeps on the boundary band (Sec. 3.2);
 *   - defect (Sec. 2.4 step 3), extension of the defect Eq. (exp) (Sec. 2.6),
 *     partial restriction Eqs. (Fstencil), (Fstencil23), (Fstencil22) and the composite
 *     restriction (Sec. 2.5), bilinear interpolation (Sec. 2.6.1);
 *   - TGCS / V / W cycles (Sec. 1.2 remarks, Sec. 2.4), exact coarsest solve by dense
 *     LU with partial pivoting (Sec. 3.3);
 *   - convergence factor rho = ||r^(m)|| / ||r^(m-1)|| (Sec. 3).
 * Built with OpenMP, the red-black passes, the defect, the restriction and the
 * interpolation split their per-node loops over threads; every node's arithmetic is the
 * same, so the results are bit for bit those of one thread.  GS-LEX stays sequential.
 *
 * Readings where the paper is silent or garbled (listed in the design notes):
 *   grid nodes lo + h*j, j in {0..N}^d; interior iff phi < 0; one-sided second-order
 *   gradient of phi on the faces of the box; sign ties |B_a - G_a| <= 1e-12 h resolved to
 *   the side of the smaller-phi neighbour; reduced-stencil ladder 3^d -> 2^d -> (d+1)
 *   -> 2 points; extension as the steady state of Eq. (exp) with the upwind difference
 *   taken with a minus sign, processed once in increasing phi; restriction boxes chosen
 *   with a fixed tie order; bilinear interpolation renormalised over present coarse nodes.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXLEV 24
enum { ORC_OUT = 0, ORC_IN = 1, ORC_GHOST = 2 };
enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENOMEM = -2,
  ORC_EGEOM = -4,
  ORC_ENOCONV = -5,
  ORC_EDIVERGED = -6
};

typedef struct {
  int dim;          /* 1, 2 or 3 */
  int n;            /* intervals per axis on the finest grid */
  double lo, hi;    /* the box [lo, hi]^dim */
  int n_coarse;     /* intervals per axis on the coarsest grid; n = n_coarse * 2^L */
  int nu1, nu2;     /* pre- and post-relaxations */
  int gamma;        /* 1 = V-cycle, 2 = W-cycle */
  int lambda;       /* extra boundary sweeps after every relaxation (Sec. 3.2) */
  double delta_h;   /* band width delta in units of h (Sec. 3.2: delta = 3h) */
  double cD;        /* mu_D * dt */
  double cN;        /* mu_N * dt = cN * h */
  int ordering;     /* 0 = GS-LEX (the paper), 1 = red-black interior + Jacobi ghosts */
  int split;        /* 0: outside pass over all of D_h - Omega_h (the paper's composite
                       restriction); 1: Dirichlet- and Neumann-labelled outside nodes are
                       extended and restricted separately */
  int smoother;     /* boundary relaxation (Sec. 3.3): 0 = the paper's ghost relaxation with
                       lambda extra sweeps; 1 = lambda Kaczmarz sweeps over the band after an
                       interior sweep; 2 = block relaxation of the band after a sweep of the
                       interior off the band.  With ordering 0 every sweep is lexicographic;
                       with ordering 1 the interior sweeps are red-black and the band is swept
                       colour by colour (colour (x mod M) + M (y mod M) + M^2 (z mod M), M = 5
                       for Kaczmarz, 7 for blocks: no two rows or blocks of a colour touch the
                       same unknowns, so a colour may be swept in any order) */
} orc_grid;

/* Dirichlet iff a.B + c > 0 (strict) or >= 0 (not strict), evaluated at the closest point B. */
typedef struct {
  double a[3];
  double c;
  int strict;
} orc_bc_rule;

typedef struct {
  int n;
  double h;
  int64_t np, nn, st[3];
  double* phi;
  int8_t* cls;
  int64_t* gid;
  /* ghost records, in increasing node index */
  int64_t ng;
  int64_t* gnode;
  int8_t *gtype, *grung, *gsgn, *gaxis;
  double *gB, *gnG, *gnB, *gxi, *gc;
  int64_t* gwn; /* ng * 3^d stencil node indices, -1 where unused */
  double* gw;   /* ng * 3^d weights of the boundary operator L_h */
  int8_t* band;
  int8_t* lab; /* outside nodes: BC type of their closest boundary point (1 D, 0 N), else -1 */
  int64_t nint, nband;
  /* defect extension towards the next coarser level */
  int64_t ne;
  int64_t *enode, *esrc;
  double* ewt;
  /* restriction boxes for the nodes of the next coarser level */
  int8_t *rlo, *rhi;
  /* coarsest level */
  int64_t nu;
  int64_t *umap, *piv;
  double* lu;
  /* work arrays */
  double *u, *rhs, *r, *tmp;
} olev;

/* A general partition of the boundary (Sec. 2.1): nonzero when B lies on Gamma_D. */
typedef int (*orc_bc_fn)(const double* B, void* ctx);

typedef struct {
  orc_grid g;
  orc_bc_rule bc;
  orc_bc_fn bc_fn; /* when set, replaces the half-space rule */
  void* bc_ctx;
  int L; /* index of the coarsest level */
  int K; /* 3^dim */
  olev lev[ORC_MAXLEV];
} ohandle;

/* Gamma_D or Gamma_N at the boundary point B (dimension d; unused coordinates are 0). */
static int on_dirichlet(const ohandle* H, int d, const double* B) {
  if (H->bc_fn) {
    double b[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) b[a] = B[a];
    return H->bc_fn(b, H->bc_ctx) != 0;
  }
  double v = H->bc.c;
  for (int a = 0; a < d; ++a) v += H->bc.a[a] * B[a];
  return H->bc.strict ? (v > 0.0) : (v >= 0.0);
}

/* ------------------------------------------------------------------------------------ */
/* indexing helpers                                                                     */
/* ------------------------------------------------------------------------------------ */

static void to_j(const olev* L, int d, int64_t idx, int j[3]) {
  j[0] = j[1] = j[2] = 0;
  for (int a = 0; a < d; ++a) {
    j[a] = (int)(idx % L->np);
    idx /= L->np;
  }
}

static int in_box(const olev* L, int d, const int j[3]) {
  for (int a = 0; a < d; ++a)
    if (j[a] < 0 || j[a] > L->n) return 0;
  return 1;
}

static int64_t to_idx(const olev* L, int d, const int j[3]) {
  int64_t idx = 0;
  for (int a = d - 1; a >= 0; --a) idx = idx * L->np + j[a];
  return idx;
}

static double coord(const ohandle* H, const olev* L, int j) { return H->g.lo + L->h * (double)j; }

/* Second-order gradient of phi at node j: central differences (Eq. (clpt) asks for a
 * second-order accurate gradient), one-sided second-order on the faces of the box. */
static void grad_phi(const olev* L, int d, const int j[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  int64_t c = to_idx(L, d, j);
  for (int a = 0; a < d; ++a) {
    int64_t s = L->st[a];
    if (j[a] > 0 && j[a] < L->n)
      g[a] = (L->phi[c + s] - L->phi[c - s]) / (2.0 * L->h);
    else if (j[a] == 0)
      g[a] = (-3.0 * L->phi[c] + 4.0 * L->phi[c + s] - L->phi[c + 2 * s]) / (2.0 * L->h);
    else
      g[a] = (3.0 * L->phi[c] - 4.0 * L->phi[c - s] + L->phi[c - 2 * s]) / (2.0 * L->h);
  }
}

/* ------------------------------------------------------------------------------------ */
/* ghost-point boundary operator (Sec. 2.3)                                             */
/* ------------------------------------------------------------------------------------ */

/* one-dimensional Lagrange bases on the nodes 0, 1, 2 of the upwind stencil */
static void basis1d(int rung, double t, double b[3], double db[3]) {
  if (rung == 1) { /* quadratic, Eq. (St_G) nine-point (3^d) stencil */
    b[0] = 0.5 * (t - 1.0) * (t - 2.0);
    b[1] = t * (2.0 - t);
    b[2] = 0.5 * t * (t - 1.0);
    db[0] = t - 1.5;
    db[1] = 2.0 - 2.0 * t;
    db[2] = t - 0.5;
  } else { /* linear, the 2x2 (2^d) reduced stencil of Remark 3 */
    b[0] = 1.0 - t;
    b[1] = t;
    b[2] = 0.0;
    db[0] = -1.0;
    db[1] = 1.0;
    db[2] = 0.0;
  }
}

/* template position t <-> k in {0,1,2}^d with k_x the slowest digit */
static void t_to_k(int d, int t, int k[3]) {
  k[0] = k[1] = k[2] = 0;
  for (int a = d - 1; a >= 0; --a) {
    k[a] = t % 3;
    t /= 3;
  }
}

/* Value weights wv[t] and gradient weights wg[a][t] of the interpolant on the stencil of
 * the given rung at the local coordinates xi (xi_a = s_a (B_a - G_a) / h).
 * rung 1: 3^d tensor quadratic; rung 2: 2^d tensor linear; rung 3: d+1 points
 * {G, G + s_a e_a}; rung 4: the two points {G, G + s_ax e_ax}.  Returns the mask of used
 * template positions. */
static void interp_weights(int d, int rung, int axis, const int8_t* s, const double* xi, double h,
                           double* wv, double wg[3][27], int8_t* used) {
  int K = 1;
  for (int a = 0; a < d; ++a) K *= 3;
  for (int t = 0; t < K; ++t) {
    wv[t] = 0.0;
    wg[0][t] = wg[1][t] = wg[2][t] = 0.0;
    used[t] = 0;
  }
  if (rung == 1 || rung == 2) {
    double b[3][3], db[3][3];
    for (int a = 0; a < d; ++a) basis1d(rung, xi[a], b[a], db[a]);
    for (int t = 0; t < K; ++t) {
      int k[3];
      t_to_k(d, t, k);
      int ok = 1;
      for (int a = 0; a < d; ++a)
        if (rung == 2 && k[a] == 2) ok = 0;
      if (!ok) continue;
      used[t] = 1;
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= b[a][k[a]];
      wv[t] = v;
      for (int a = 0; a < d; ++a) {
        double gcomp = (double)s[a] / h * db[a][k[a]];
        for (int c = 0; c < d; ++c)
          if (c != a) gcomp *= b[c][k[c]];
        wg[a][t] = gcomp;
      }
    }
  } else {
    /* linear interpolant through G and G + s_a e_a (for the listed axes) */
    int tG = 0;
    used[tG] = 1;
    double sumxi = 0.0;
    for (int a = 0; a < d; ++a) {
      if (rung == 4 && a != axis) continue;
      int ta = 1;
      for (int c = d - 1; c > a; --c) ta *= 3; /* k = e_a */
      used[ta] = 1;
      wv[ta] = xi[a];
      sumxi += xi[a];
      wg[a][tG] = -(double)s[a] / h;
      wg[a][ta] = (double)s[a] / h;
    }
    wv[tG] = 1.0 - sumxi;
  }
}

static int64_t template_node(const olev* L, int d, int64_t G, const int8_t* s, int t) {
  int k[3];
  t_to_k(d, t, k);
  int64_t off = 0;
  for (int a = 0; a < d; ++a) off += (int64_t)s[a] * k[a] * L->st[a];
  return G + off;
}

static int template_contained(const olev* L, int d, const int jG[3], const int8_t* s, int t) {
  int k[3], j[3];
  t_to_k(d, t, k);
  for (int a = 0; a < 3; ++a) j[a] = jG[a];
  for (int a = 0; a < d; ++a) j[a] = jG[a] + s[a] * k[a];
  if (!in_box(L, d, j)) return 0;
  int8_t c = L->cls[to_idx(L, d, j)];
  return c == ORC_IN || c == ORC_GHOST;
}

static int build_ghosts(ohandle* H, int l) {
  olev* L = &H->lev[l];
  const int d = H->g.dim, K = H->K;
  int64_t ng = 0;
  for (int64_t i = 0; i < L->nn; ++i) ng += (L->cls[i] == ORC_GHOST);
  L->ng = ng;
  L->gnode = (int64_t*)calloc(ng + 1, sizeof(int64_t));
  L->gtype = (int8_t*)calloc(ng + 1, 1);
  L->grung = (int8_t*)calloc(ng + 1, 1);
  L->gaxis = (int8_t*)calloc(ng + 1, 1);
  L->gsgn = (int8_t*)calloc(3 * ng + 3, 1);
  L->gB = (double*)calloc(3 * ng + 3, sizeof(double));
  L->gnG = (double*)calloc(3 * ng + 3, sizeof(double));
  L->gnB = (double*)calloc(3 * ng + 3, sizeof(double));
  L->gxi = (double*)calloc(3 * ng + 3, sizeof(double));
  L->gc = (double*)calloc(ng + 1, sizeof(double));
  L->gwn = (int64_t*)malloc((size_t)(K * ng + K) * sizeof(int64_t));
  L->gw = (double*)calloc((size_t)(K * ng + K), sizeof(double));
  L->gid = (int64_t*)malloc((size_t)L->nn * sizeof(int64_t));
  if (!L->gnode || !L->gwn || !L->gw || !L->gid || !L->gsgn) return ORC_ENOMEM;
  for (int64_t i = 0; i < L->nn; ++i) L->gid[i] = -1;

  int64_t q = 0;
  for (int64_t G = 0; G < L->nn; ++G) {
    if (L->cls[G] != ORC_GHOST) continue;
    L->gid[G] = q;
    L->gnode[q] = G;
    int jG[3];
    to_j(L, d, G, jG);
    /* closest boundary point, Eq. (clpt) */
    double gr[3];
    grad_phi(L, d, jG, gr);
    double nrm2 = 0.0;
    for (int a = 0; a < d; ++a) nrm2 += gr[a] * gr[a];
    double nrm = sqrt(nrm2);
    if (!(nrm > 0.0)) return ORC_EGEOM;
    double B[3] = {0, 0, 0}, xG[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
      double na = gr[a] / nrm;
      xG[a] = coord(H, L, jG[a]);
      L->gnG[3 * q + a] = na;
      B[a] = xG[a] - na * L->phi[G];
      L->gB[3 * q + a] = B[a];
    }
    /* boundary-condition type at B */
    int dir = on_dirichlet(H, d, B);
    L->gtype[q] = (int8_t)dir;
    L->gc[q] = dir ? H->g.cD : H->g.cN * L->h;

    /* upwind signs, Eq. (St_G), with the tie rule */
    int8_t pref[3] = {1, 1, 1};
    int tied[3] = {0, 0, 0}, ntied = 0, tiedax[3];
    for (int a = 0; a < d; ++a) {
      double df = B[a] - xG[a];
      if (fabs(df) > 1e-12 * L->h) {
        pref[a] = df > 0.0 ? 1 : -1;
      } else {
        tied[a] = 1;
        tiedax[ntied++] = a;
        double pm = INFINITY, pp = INFINITY;
        if (jG[a] > 0) pm = L->phi[G - L->st[a]];
        if (jG[a] < L->n) pp = L->phi[G + L->st[a]];
        pref[a] = (pm < pp) ? -1 : 1;
      }
    }
    (void)tied;
    /* reduced-stencil ladder of Remark 3 */
    int rung_found = 0, axis = 0;
    int8_t s[3] = {1, 1, 1};
    for (int rung = 1; rung <= 3 && !rung_found; ++rung) {
      for (int m = 0; m < (1 << ntied) && !rung_found; ++m) {
        for (int a = 0; a < 3; ++a) s[a] = pref[a];
        for (int b = 0; b < ntied; ++b)
          if (m & (1 << b)) s[tiedax[b]] = (int8_t)-pref[tiedax[b]];
        int ok = 1;
        for (int t = 0; t < K && ok; ++t) {
          int k[3];
          t_to_k(d, t, k);
          int need = 0;
          if (rung == 1) need = 1;
          else if (rung == 2) {
            need = 1;
            for (int a = 0; a < d; ++a)
              if (k[a] == 2) need = 0;
          } else {
            int nz = 0, big = 0;
            for (int a = 0; a < d; ++a) {
              nz += (k[a] != 0);
              big += (k[a] > 1);
            }
            need = (nz <= 1 && big == 0);
          }
          if (need && !template_contained(L, d, jG, s, t)) ok = 0;
        }
        if (ok) rung_found = rung;
      }
    }
    if (!rung_found) {
      /* last rung: two points along the axis to the interior neighbour of least phi */
      double best = INFINITY;
      int ba = -1, bs = 0;
      for (int a = 0; a < d; ++a) {
        for (int dirn = -1; dirn <= 1; dirn += 2) {
          int j2[3] = {jG[0], jG[1], jG[2]};
          j2[a] += dirn;
          if (!in_box(L, d, j2)) continue;
          int64_t Q = to_idx(L, d, j2);
          if (L->cls[Q] != ORC_IN) continue;
          if (L->phi[Q] < best) {
            best = L->phi[Q];
            ba = a;
            bs = dirn;
          }
        }
      }
      if (ba < 0) return ORC_EGEOM;
      for (int a = 0; a < 3; ++a) s[a] = pref[a];
      s[ba] = (int8_t)bs;
      axis = ba;
      rung_found = 4;
    }
    L->grung[q] = (int8_t)rung_found;
    L->gaxis[q] = (int8_t)axis;
    double xi[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
      L->gsgn[3 * q + a] = s[a];
      xi[a] = (double)s[a] * (B[a] - xG[a]) / L->h;
      L->gxi[3 * q + a] = xi[a];
    }
    /* weights of L_h, Eq. (discrBC) */
    double wv[27], wg[3][27];
    int8_t used[27];
    interp_weights(d, rung_found, axis, s, xi, L->h, wv, wg, used);
    for (int t = 0; t < K; ++t) L->gwn[K * q + t] = used[t] ? template_node(L, d, G, s, t) : -1;
    if (dir) {
      for (int t = 0; t < K; ++t) L->gw[K * q + t] = used[t] ? wv[t] : 0.0;
    } else {
      /* normal at B from the same interpolant of phi, Eq. (neu2d) */
      double gp[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a)
        for (int t = 0; t < K; ++t)
          if (used[t]) gp[a] += wg[a][t] * L->phi[L->gwn[K * q + t]];
      double gn2 = 0.0;
      for (int a = 0; a < d; ++a) gn2 += gp[a] * gp[a];
      double gn = sqrt(gn2);
      if (!(gn > 0.0)) return ORC_EGEOM;
      double nB[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) {
        nB[a] = gp[a] / gn;
        L->gnB[3 * q + a] = nB[a];
      }
      for (int t = 0; t < K; ++t) {
        double w = 0.0;
        if (used[t])
          for (int a = 0; a < d; ++a) w += nB[a] * wg[a][t];
        L->gw[K * q + t] = w;
      }
    }
    ++q;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* level construction                                                                   */
/* ------------------------------------------------------------------------------------ */

static int build_level_geometry(ohandle* H, int l) {
  olev* L = &H->lev[l];
  const int d = H->g.dim;
  /* interior nodes: phi < 0 (Sec. 2.2, 2.3) */
  for (int64_t i = 0; i < L->nn; ++i) L->cls[i] = (L->phi[i] < 0.0) ? ORC_IN : ORC_OUT;
  /* ghost points: outside nodes with an interior neighbour (Sec. 2.3) */
  L->nint = 0;
  for (int64_t i = 0; i < L->nn; ++i) {
    if (L->cls[i] == ORC_IN) {
      L->nint++;
      continue;
    }
    int j[3];
    to_j(L, d, i, j);
    for (int a = 0; a < d; ++a) {
      for (int dirn = -1; dirn <= 1; dirn += 2) {
        int j2[3] = {j[0], j[1], j[2]};
        j2[a] += dirn;
        if (!in_box(L, d, j2)) continue;
        if ((L->phi[to_idx(L, d, j2)] < 0.0)) L->cls[i] = ORC_GHOST;
      }
    }
  }
  if (L->nint == 0) return ORC_EGEOM;
  /* the domain must not touch the faces of the box (Sec. 2.1) */
  for (int64_t i = 0; i < L->nn; ++i) {
    if (L->cls[i] != ORC_IN) continue;
    int j[3];
    to_j(L, d, i, j);
    for (int a = 0; a < d; ++a)
      if (j[a] == 0 || j[a] == L->n) return ORC_EGEOM;
  }
  int rc = build_ghosts(H, l);
  if (rc) return rc;
  L->lab = (int8_t*)malloc((size_t)L->nn);
  if (!L->lab) return ORC_ENOMEM;
  for (int64_t i = 0; i < L->nn; ++i) L->lab[i] = -1;
  for (int64_t q = 0; q < L->ng; ++q) L->lab[L->gnode[q]] = L->gtype[q];
  /* band for the extra relaxations: ghosts and interior nodes within delta (Sec. 3.2) */
  L->band = (int8_t*)calloc((size_t)L->nn, 1);
  if (!L->band) return ORC_ENOMEM;
  double delta = H->g.delta_h * L->h;
  L->nband = 0;
  for (int64_t i = 0; i < L->nn; ++i) {
    if (L->cls[i] == ORC_GHOST) L->band[i] = 1;
    if (L->cls[i] == ORC_IN && L->phi[i] >= -delta) {
      L->band[i] = 1;
      L->nband++;
    }
  }
  return ORC_OK;
}

typedef struct {
  double phi;
  int64_t idx;
} keyed;

static int cmp_keyed(const void* x, const void* y) {
  const keyed* a = (const keyed*)x;
  const keyed* b = (const keyed*)y;
  if (a->phi < b->phi) return -1;
  if (a->phi > b->phi) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Nodes and upwind sources of the extension of the defect, Eq. (exp), Sec. 2.6. */
static int build_extension(ohandle* H, int l) {
  olev* F = &H->lev[l];
  olev* C = &H->lev[l + 1];
  const int d = H->g.dim;
  int64_t* rank = (int64_t*)malloc((size_t)F->nn * sizeof(int64_t));
  if (!rank) return ORC_ENOMEM;
  for (int64_t i = 0; i < F->nn; ++i) rank[i] = -1;
  int64_t ne = 0;
  for (int64_t X = 0; X < C->nn; ++X) {
    if (C->cls[X] != ORC_GHOST) continue;
    int jc[3];
    to_j(C, d, X, jc);
    int nnb = 1;
    for (int a = 0; a < d; ++a) nnb *= 3;
    for (int o = 0; o < nnb; ++o) {
      int j[3] = {0, 0, 0}, oo = o;
      for (int a = 0; a < d; ++a) {
        j[a] = 2 * jc[a] + (oo % 3) - 1;
        oo /= 3;
      }
      if (!in_box(F, d, j)) continue;
      int64_t P = to_idx(F, d, j);
      if (F->cls[P] == ORC_OUT && rank[P] < 0) {
        rank[P] = 0;
        ++ne;
      }
    }
  }
  keyed* ks = (keyed*)malloc((size_t)(ne + 1) * sizeof(keyed));
  if (!ks) {
    free(rank);
    return ORC_ENOMEM;
  }
  int64_t q = 0;
  for (int64_t i = 0; i < F->nn; ++i)
    if (rank[i] == 0) {
      ks[q].phi = F->phi[i];
      ks[q].idx = i;
      ++q;
    }
  /* Gauss-Seidel order by distance from the boundary (Sec. 2.6) */
  qsort(ks, (size_t)ne, sizeof(keyed), cmp_keyed);
  for (int64_t e = 0; e < ne; ++e) rank[ks[e].idx] = e;
  F->ne = ne;
  F->enode = (int64_t*)malloc((size_t)(ne + 1) * sizeof(int64_t));
  F->esrc = (int64_t*)malloc((size_t)(3 * ne + 3) * sizeof(int64_t));
  F->ewt = (double*)calloc((size_t)(3 * ne + 3), sizeof(double));
  if (!F->enode || !F->esrc || !F->ewt) {
    free(ks);
    free(rank);
    return ORC_ENOMEM;
  }
  for (int64_t e = 0; e < ne; ++e) {
    int64_t P = ks[e].idx;
    F->enode[e] = P;
    int j[3];
    to_j(F, d, P, j);
    double gr[3];
    grad_phi(F, d, j, gr);
    double nrm = 0.0;
    for (int a = 0; a < d; ++a) nrm += gr[a] * gr[a];
    nrm = sqrt(nrm);
    for (int a = 0; a < 3; ++a) {
      F->esrc[3 * e + a] = -1;
      F->ewt[3 * e + a] = 0.0;
    }
    if (!(nrm > 0.0)) {
      F->lab[P] = 1;
      continue;
    }
    {
      /* label: boundary-condition type at the closest boundary point of P */
      double Bp[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < d; ++a) Bp[a] = coord(H, F, j[a]) - gr[a] / nrm * F->phi[P];
      F->lab[P] = (int8_t)on_dirichlet(H, d, Bp);
    }
    int nsame = 0;
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1 && (!H->g.split || nsame > 0)) break;
    for (int a = 0; a < d; ++a) {
      double na = gr[a] / nrm;
      if (na == 0.0) continue;
      /* upwind neighbour Q_a = P - sgn(n_a) h e_a */
      int jq[3] = {j[0], j[1], j[2]};
      jq[a] -= (na > 0.0) ? 1 : -1;
      if (!in_box(F, d, jq)) continue;
      int64_t Q = to_idx(F, d, jq);
      int avail = (F->cls[Q] == ORC_GHOST) || (rank[Q] >= 0 && rank[Q] < e);
      if (!avail) continue;
      /* split transfer: first only sources with the label of P; if there are none, all */
      if (H->g.split && pass == 0 && F->lab[Q] != F->lab[P]) continue;
      if (pass == 0) ++nsame;
      F->esrc[3 * e + a] = Q;
      F->ewt[3 * e + a] = fabs(na);
    }
    }
  }
  free(ks);
  free(rank);
  return ORC_OK;
}

/* node set I_h of the partial transfer: interior (inside pass) or outside (outside pass) */
static int member(const olev* F, int64_t P, int inside, int lab) {
  if (inside) return F->cls[P] == ORC_IN;
  return F->cls[P] != ORC_IN && (lab < 0 || F->lab[P] == lab);
}

/* Maximal full rectangle T in the 3^d neighbourhood whose nodes all lie in I_h (Sec. 2.5). */
static void choose_box(const olev* F, int d, const int jf[3], int inside, int lab, int8_t lo[3],
                       int8_t hi[3]) {
  int best_key[7] = {0, 0, 0, 0, 0, 0, 0};
  int have = 0;
  int ncand = 1;
  for (int a = 0; a < d; ++a) ncand *= 4;
  for (int c = 0; c < ncand; ++c) {
    int a_[3] = {0, 0, 0}, b_[3] = {0, 0, 0}, cc = c;
    for (int a = 0; a < d; ++a) {
      int code = cc % 4;
      cc /= 4;
      a_[a] = (code & 1) ? -1 : 0;
      b_[a] = (code & 2) ? 1 : 0;
    }
    /* all nodes of the box in the grid and in I_h */
    int ok = 1;
    int ext[3] = {1, 1, 1};
    int cnt = 1;
    for (int a = 0; a < d; ++a) {
      ext[a] = b_[a] - a_[a] + 1;
      cnt *= ext[a];
    }
    for (int t = 0; t < cnt && ok; ++t) {
      int j[3] = {jf[0], jf[1], jf[2]}, tt = t;
      for (int a = 0; a < d; ++a) {
        j[a] = jf[a] + a_[a] + (tt % ext[a]);
        tt /= ext[a];
      }
      if (!in_box(F, d, j) || !member(F, to_idx(F, d, j), inside, lab)) ok = 0;
    }
    if (!ok) continue;
    int key[7] = {cnt, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      key[1 + a] = (a < d) ? ext[a] : 0;
      key[4 + a] = (a < d) ? (a_[a] == -1) : 0;
    }
    int better = !have;
    if (have) {
      for (int m = 0; m < 7; ++m) {
        if (key[m] != best_key[m]) {
          better = key[m] > best_key[m];
          break;
        }
      }
    }
    if (better) {
      have = 1;
      memcpy(best_key, key, sizeof(key));
      for (int a = 0; a < 3; ++a) {
        lo[a] = (int8_t)((a < d) ? a_[a] : 0);
        hi[a] = (int8_t)((a < d) ? b_[a] : 0);
      }
    }
  }
  if (!have) { /* cannot happen: the centre node is always a member */
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = 0;
  }
}

static int build_restriction(ohandle* H, int l) {
  olev* F = &H->lev[l];
  olev* C = &H->lev[l + 1];
  const int d = H->g.dim;
  F->rlo = (int8_t*)calloc((size_t)(3 * C->nn), 1);
  F->rhi = (int8_t*)calloc((size_t)(3 * C->nn), 1);
  if (!F->rlo || !F->rhi) return ORC_ENOMEM;
  for (int64_t X = 0; X < C->nn; ++X) {
    if (C->cls[X] == ORC_OUT) continue;
    int jc[3], jf[3] = {0, 0, 0};
    to_j(C, d, X, jc);
    for (int a = 0; a < d; ++a) jf[a] = 2 * jc[a];
    int inside = C->cls[X] == ORC_IN;
    int lab = (!inside && H->g.split) ? F->lab[to_idx(F, d, jf)] : -1;
    choose_box(F, d, jf, inside, lab, &F->rlo[3 * X], &F->rhi[3 * X]);
  }
  return ORC_OK;
}

/* dense LU with partial pivoting of the coarsest system (exact solver, Sec. 3.3) */
static int build_coarse(ohandle* H) {
  olev* C = &H->lev[H->L];
  const int d = H->g.dim, K = H->K;
  int64_t nu = 0;
  for (int64_t i = 0; i < C->nn; ++i) nu += (C->cls[i] != ORC_OUT);
  C->nu = nu;
  C->umap = (int64_t*)malloc((size_t)(nu + 1) * sizeof(int64_t));
  C->piv = (int64_t*)malloc((size_t)(nu + 1) * sizeof(int64_t));
  C->lu = (double*)calloc((size_t)(nu * nu + 1), sizeof(double));
  int64_t* col = (int64_t*)malloc((size_t)C->nn * sizeof(int64_t));
  if (!C->umap || !C->piv || !C->lu || !col) return ORC_ENOMEM;
  int64_t q = 0;
  for (int64_t i = 0; i < C->nn; ++i) {
    col[i] = -1;
    if (C->cls[i] != ORC_OUT) {
      C->umap[q] = i;
      col[i] = q++;
    }
  }
  double* A = C->lu;
  double ih2 = 1.0 / (C->h * C->h);
  for (int64_t r = 0; r < nu; ++r) {
    int64_t P = C->umap[r];
    if (C->cls[P] == ORC_IN) {
      A[r * nu + r] += 2.0 * d * ih2;
      for (int a = 0; a < d; ++a) {
        A[r * nu + col[P - C->st[a]]] -= ih2;
        A[r * nu + col[P + C->st[a]]] -= ih2;
      }
    } else {
      int64_t g = C->gid[P];
      for (int t = 0; t < K; ++t) {
        int64_t nd = C->gwn[K * g + t];
        if (nd >= 0) A[r * nu + col[nd]] += C->gw[K * g + t];
      }
    }
  }
  free(col);
  double amax = 0.0;
  for (int64_t i = 0; i < nu * nu; ++i)
    if (fabs(A[i]) > amax) amax = fabs(A[i]);
  for (int64_t k = 0; k < nu; ++k) {
    int64_t p = k;
    double pv = fabs(A[k * nu + k]);
    for (int64_t i = k + 1; i < nu; ++i)
      if (fabs(A[i * nu + k]) > pv) {
        pv = fabs(A[i * nu + k]);
        p = i;
      }
    C->piv[k] = p;
    if (!(pv > 1e-13 * amax)) return ORC_EGEOM;
    if (p != k)
      for (int64_t j = 0; j < nu; ++j) {
        double t = A[k * nu + j];
        A[k * nu + j] = A[p * nu + j];
        A[p * nu + j] = t;
      }
    for (int64_t i = k + 1; i < nu; ++i) {
      double m = A[i * nu + k] / A[k * nu + k];
      A[i * nu + k] = m;
      if (m != 0.0)
        for (int64_t j = k + 1; j < nu; ++j) A[i * nu + j] -= m * A[k * nu + j];
    }
  }
  return ORC_OK;
}

static void free_level(olev* L) {
  free(L->phi); free(L->cls); free(L->gid);
  free(L->gnode); free(L->gtype); free(L->grung); free(L->gsgn); free(L->gaxis);
  free(L->gB); free(L->gnG); free(L->gnB); free(L->gxi); free(L->gc);
  free(L->gwn); free(L->gw); free(L->band); free(L->lab);
  free(L->enode); free(L->esrc); free(L->ewt);
  free(L->rlo); free(L->rhi);
  free(L->umap); free(L->piv); free(L->lu);
  free(L->u); free(L->rhs); free(L->r); free(L->tmp);
  memset(L, 0, sizeof(*L));
}

void orc_free(void* h) {
  ohandle* H = (ohandle*)h;
  if (!H) return;
  for (int l = 0; l <= H->L && l < ORC_MAXLEV; ++l) free_level(&H->lev[l]);
  free(H);
}

static void* setup_impl(const double* phi, const orc_bc_rule* bc, orc_bc_fn fn, void* ctx,
                        const orc_grid* g, int* err);

/* phi: node values on the finest grid, (n+1)^dim, x fastest. */
void* orc_setup(const double* phi, const orc_bc_rule* bc, const orc_grid* g, int* err) {
  *err = ORC_EINVAL;
  if (!bc) return NULL;
  return setup_impl(phi, bc, NULL, NULL, g, err);
}

/* orc_setup with the partition of the boundary given by fn (called during setup only). */
void* orc_setup_fn(const double* phi, orc_bc_fn fn, void* ctx, const orc_grid* g, int* err) {
  *err = ORC_EINVAL;
  if (!fn) return NULL;
  return setup_impl(phi, NULL, fn, ctx, g, err);
}

static void* setup_impl(const double* phi, const orc_bc_rule* bc, orc_bc_fn fn, void* ctx,
                        const orc_grid* g, int* err) {
  *err = ORC_EINVAL;
  if (!phi || !g) return NULL;
  if (g->dim < 1 || g->dim > 3 || g->n < 2 || g->n_coarse < 2 || g->hi <= g->lo) return NULL;
  if (g->gamma < 1 || g->gamma > 2 || g->nu1 < 0 || g->nu2 < 0 || g->lambda < 0) return NULL;
  if (g->smoother < 0 || g->smoother > 2) return NULL;
  int L = 0;
  int nn_ = g->n;
  while (nn_ > g->n_coarse) {
    if (nn_ % 2) return NULL;
    nn_ /= 2;
    ++L;
  }
  if (nn_ != g->n_coarse || L >= ORC_MAXLEV) return NULL;
  ohandle* H = (ohandle*)calloc(1, sizeof(ohandle));
  if (!H) {
    *err = ORC_ENOMEM;
    return NULL;
  }
  H->g = *g;
  if (bc) H->bc = *bc;
  H->bc_fn = fn;
  H->bc_ctx = ctx;
  H->L = L;
  H->K = 1;
  for (int a = 0; a < g->dim; ++a) H->K *= 3;
  const int d = g->dim;
  for (int l = 0; l <= L; ++l) {
    olev* V = &H->lev[l];
    V->n = g->n >> l;
    V->h = (g->hi - g->lo) / (double)V->n;
    V->np = V->n + 1;
    V->nn = 1;
    for (int a = 0; a < 3; ++a) V->st[a] = 0;
    for (int a = 0; a < d; ++a) {
      V->st[a] = V->nn;
      V->nn *= V->np;
    }
    V->phi = (double*)malloc((size_t)V->nn * sizeof(double));
    V->cls = (int8_t*)malloc((size_t)V->nn);
    V->u = (double*)calloc((size_t)V->nn, sizeof(double));
    V->rhs = (double*)calloc((size_t)V->nn, sizeof(double));
    V->r = (double*)calloc((size_t)V->nn, sizeof(double));
    V->tmp = (double*)calloc((size_t)V->nn, sizeof(double));
    if (!V->phi || !V->cls || !V->u || !V->rhs || !V->r || !V->tmp) {
      *err = ORC_ENOMEM;
      orc_free(H);
      return NULL;
    }
    /* coarse grids take phi at their nodes, which are nodes of the finest grid */
    int64_t stride = (int64_t)1 << l;
    for (int64_t i = 0; i < V->nn; ++i) {
      int j[3];
      to_j(V, d, i, j);
      int64_t fi = 0, np0 = g->n + 1;
      for (int a = d - 1; a >= 0; --a) fi = fi * np0 + (int64_t)j[a] * stride;
      V->phi[i] = phi[fi];
    }
    int rc = build_level_geometry(H, l);
    if (rc) {
      *err = rc;
      orc_free(H);
      return NULL;
    }
  }
  for (int l = 0; l < L; ++l) {
    int rc = build_extension(H, l);
    if (!rc) rc = build_restriction(H, l);
    if (rc) {
      *err = rc;
      orc_free(H);
      return NULL;
    }
  }
  int rc = build_coarse(H);
  if (rc) {
    *err = rc;
    orc_free(H);
    return NULL;
  }
  *err = ORC_OK;
  return H;
}

/* ------------------------------------------------------------------------------------ */
/* operators                                                                            */
/* ------------------------------------------------------------------------------------ */

static double ghost_apply(const ohandle* H, const olev* L, int64_t g, const double* u) {
  double s = 0.0;
  for (int t = 0; t < H->K; ++t) {
    int64_t nd = L->gwn[H->K * g + t];
    if (nd >= 0) s += L->gw[H->K * g + t] * u[nd];
  }
  return s;
}

/* defect, Sec. 2.4 step 3: f + Delta_h u inside, g - L_h u at ghosts; zero elsewhere.
 * The Laplacian is evaluated as sum_nb (u_nb - u_P) / h^2, which is Delta_h u written
 * so that the subtraction of nearly equal neighbours is exact. */
static void defect(const ohandle* H, int l, const double* u, const double* rhs, double* r,
                   double* nin, double* ngh) {
  const olev* L = &H->lev[l];
  const int d = H->g.dim;
  double h2 = L->h * L->h, mi = 0.0, mg = 0.0;
  /* rows are independent; each thread keeps its own maxima (a NaN is kept), combined below */
#pragma omp parallel
  {
    double ti = 0.0, tg = 0.0;
#pragma omp for schedule(static)
    for (int64_t P = 0; P < L->nn; ++P) {
      if (L->cls[P] == ORC_IN) {
        double s = 0.0;
        for (int a = 0; a < d; ++a) {
          s += u[P - L->st[a]] - u[P];
          s += u[P + L->st[a]] - u[P];
        }
        r[P] = rhs[P] + s / h2;
        if (fabs(r[P]) > ti || r[P] != r[P]) ti = (r[P] != r[P]) ? NAN : fabs(r[P]);
      } else if (L->cls[P] == ORC_GHOST) {
        r[P] = rhs[P] - ghost_apply(H, L, L->gid[P], u);
        if (fabs(r[P]) > tg || r[P] != r[P]) tg = (r[P] != r[P]) ? NAN : fabs(r[P]);
      } else {
        r[P] = 0.0;
      }
    }
#pragma omp critical
    {
      if (ti != ti || mi != mi) mi = NAN; else if (ti > mi) mi = ti;
      if (tg != tg || mg != mg) mg = NAN; else if (tg > mg) mg = tg;
    }
  }
  if (nin) *nin = mi;
  if (ngh) *ngh = mg;
}

/* interior relaxation, Eq. (jac2d): u_P = (h^2 f_P + sum of the 2d neighbours) / (2d),
 * evaluated as u_P + (h^2 f_P + sum_nb (u_nb - u_P)) / (2d).  The two are equal in exact
 * arithmetic; the correction form lets the iteration settle on a rounding of the discrete
 * solution whose residual is a few ulps of u / h^2 instead of the noise of a full sum. */
static void relax_interior(const ohandle* H, const olev* L, int64_t P, double* u,
                           const double* rhs) {
  const int d = H->g.dim;
  double s = 0.0;
  for (int a = 0; a < d; ++a) s += (u[P - L->st[a]] - u[P]) + (u[P + L->st[a]] - u[P]);
  u[P] = u[P] + (L->h * L->h * rhs[P] + s) / (2.0 * d);
}

/* ghost relaxation, Eqs. (dir2d) and (neu2d): u_G += mu dt (g(B) - L_h u (G)) */
static double relax_ghost_value(const ohandle* H, const olev* L, int64_t G, const double* u,
                                const double* rhs) {
  int64_t g = L->gid[G];
  return u[G] + L->gc[g] * (rhs[G] - ghost_apply(H, L, g, u));
}

static int parity(const olev* L, int d, int64_t P) {
  int j[3];
  to_j(L, d, P, j);
  return (j[0] + j[1] + j[2]) & 1;
}

/* one pass of the relaxation over Omega_h u Gamma_h (or over the band only) */
static void relax_pass(ohandle* H, int l, double* u, const double* rhs, int band_only) {
  olev* L = &H->lev[l];
  const int d = H->g.dim;
  if (H->g.ordering == 0) {
    /* GS-LEX: x slowest, then y, then z (Sec. 2.4) */
    int64_t np = L->np;
    int64_t n1 = d > 1 ? np : 1, n2 = d > 2 ? np : 1;
    for (int64_t i0 = 0; i0 < np; ++i0)
      for (int64_t i1 = 0; i1 < n1; ++i1)
        for (int64_t i2 = 0; i2 < n2; ++i2) {
          int64_t P = i0 + L->st[1] * i1 + L->st[2] * i2;
          if (band_only && !L->band[P]) continue;
          if (L->cls[P] == ORC_IN)
            relax_interior(H, L, P, u, rhs);
          else if (L->cls[P] == ORC_GHOST)
            u[P] = relax_ghost_value(H, L, P, u, rhs);
        }
  } else {
    /* red interior, black interior, then every ghost from the same state (Jacobi); a node
     * of one colour reads only the other colour, ghosts and outside nodes, so each of the
     * three passes may run its nodes in any order (here: on several threads) */
    for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
      for (int64_t P = 0; P < L->nn; ++P) {
        if (L->cls[P] != ORC_IN) continue;
        if (band_only && !L->band[P]) continue;
        if (parity(L, d, P) != colour) continue;
        relax_interior(H, L, P, u, rhs);
      }
    }
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < L->ng; ++g)
      L->tmp[g] = relax_ghost_value(H, L, L->gnode[g], u, rhs);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < L->ng; ++g) u[L->gnode[g]] = L->tmp[g];
  }
}

/* Coefficients of the equation of node P of Eq. (discr) (interior: -Delta_h u = f, written
 * as (2d u_P - sum of the neighbours) / h^2; ghost: L_h u = g): up to 3^d nodes and weights;
 * returns their number. */
static int row_of(const ohandle* H, const olev* L, int64_t P, int64_t* nd, double* w) {
  const int d = H->g.dim;
  if (L->cls[P] == ORC_IN) {
    const double h2 = L->h * L->h;
    int m = 0;
    nd[m] = P;
    w[m++] = 2.0 * d / h2;
    for (int a = 0; a < d; ++a) {
      nd[m] = P - L->st[a];
      w[m++] = -1.0 / h2;
      nd[m] = P + L->st[a];
      w[m++] = -1.0 / h2;
    }
    return m;
  }
  const int64_t g = L->gid[P];
  int m = 0;
  for (int t = 0; t < H->K; ++t) {
    if (L->gwn[H->K * g + t] < 0) continue;
    nd[m] = L->gwn[H->K * g + t];
    w[m++] = L->gw[H->K * g + t];
  }
  return m;
}

/* Kaczmarz step on the equation of node P (Sec. 3.3): u <- u + (f_P - <l_P, u>) / |l_P|^2 l_P,
 * the orthogonal projection of u onto the hyperplane of that equation. */
static void kaczmarz_row(const ohandle* H, const olev* L, int64_t P, double* u,
                         const double* rhs) {
  int64_t nd[27];
  double w[27];
  const int m = row_of(H, L, P, nd, w);
  double dot = 0.0, n2 = 0.0;
  for (int i = 0; i < m; ++i) {
    dot += w[i] * u[nd[i]];
    n2 += w[i] * w[i];
  }
  if (!(n2 > 0.0)) return;
  const double a = (rhs[P] - dot) / n2;
  for (int i = 0; i < m; ++i) u[nd[i]] += a * w[i];
}

/* Block relaxation at node P (Sec. 3.3): the unknowns of St_P (interior P: its 3^d
 * neighbourhood within Omega_h u Gamma_h; ghost P: its stencil St_G) take the values that
 * satisfy their own equations with every other unknown fixed, u_1 = A_11^{-1} (f_1 - A_12 u_2);
 * dense elimination with partial pivoting; a singular block is left unchanged.  Returns 0 when
 * it was solved. */
static int block_solve(const ohandle* H, const olev* L, int64_t P, double* u, const double* rhs) {
  const int d = H->g.dim;
  int64_t blk[27];
  int m = 0;
  if (L->cls[P] == ORC_IN) {
    int j[3];
    to_j(L, d, P, j);
    int nb = 1;
    for (int a = 0; a < d; ++a) nb *= 3;
    for (int o = 0; o < nb; ++o) {
      int jj[3] = {j[0], j[1], j[2]}, oo = o;
      for (int a = 0; a < d; ++a) {
        jj[a] += oo % 3 - 1;
        oo /= 3;
      }
      if (!in_box(L, d, jj)) continue;
      const int64_t Q = to_idx(L, d, jj);
      if (L->cls[Q] != ORC_OUT) blk[m++] = Q;
    }
  } else {
    const int64_t g = L->gid[P];
    for (int t = 0; t < H->K; ++t)
      if (L->gwn[H->K * g + t] >= 0) blk[m++] = L->gwn[H->K * g + t];
  }
  double A[27][28];
  for (int i = 0; i < m; ++i) {
    int64_t nd[27];
    double w[27];
    const int q = row_of(H, L, blk[i], nd, w);
    for (int c = 0; c <= m; ++c) A[i][c] = 0.0;
    A[i][m] = rhs[blk[i]];
    for (int k = 0; k < q; ++k) {
      int c = -1;
      for (int b = 0; b < m; ++b)
        if (blk[b] == nd[k]) c = b;
      if (c >= 0)
        A[i][c] += w[k];
      else
        A[i][m] -= w[k] * u[nd[k]];
    }
  }
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
    if (A[p][k] == 0.0) return 1;
    if (p != k)
      for (int c = 0; c <= m; ++c) {
        const double t = A[k][c];
        A[k][c] = A[p][c];
        A[p][c] = t;
      }
    for (int i = k + 1; i < m; ++i) {
      const double f = A[i][k] / A[k][k];
      for (int c = k; c <= m; ++c) A[i][c] -= f * A[k][c];
    }
  }
  double x[27];
  for (int i = m - 1; i >= 0; --i) {
    double t = A[i][m];
    for (int c = i + 1; c < m; ++c) t -= A[i][c] * x[c];
    x[i] = t / A[i][i];
  }
  for (int i = 0; i < m; ++i) u[blk[i]] = x[i];
  return 0;
}

/* nodes in GS-LEX order (x slowest, then y, then z; Sec. 2.4), as a callback walk */
#define FOR_LEX(L, d, P)                                                   \
  for (int64_t i0_ = 0; i0_ < (L)->np; ++i0_)                              \
    for (int64_t i1_ = 0; i1_ < ((d) > 1 ? (L)->np : 1); ++i1_)            \
      for (int64_t i2_ = 0; i2_ < ((d) > 2 ? (L)->np : 1); ++i2_)          \
        for (int64_t P = i0_ + (L)->st[1] * i1_ + (L)->st[2] * i2_, once_ = 1; once_; once_ = 0)

/* one relaxation followed by lambda extra sweeps on the boundary band (Sec. 3.2); or one of
 * the two alternatives of Sec. 3.3 that the paper compares it with: a Gauss-Seidel sweep of
 * the interior followed by lambda Kaczmarz sweeps over the band (ghosts and interior nodes
 * within delta of the boundary), or a Gauss-Seidel sweep of the interior off the band
 * followed by one block relaxation of every band node */
static int colour_of(const olev* L, int d, int64_t P, int M) {
  int j[3] = {0, 0, 0};
  to_j(L, d, P, j);
  int c = 0;
  for (int a = d - 1; a >= 0; --a) c = c * M + j[a] % M;
  return c;
}

/* interior red-black sweep (ordering 1) over every interior node, or over those off the band */
static void rb_interior(ohandle* H, olev* L, double* u, const double* rhs, int off_band) {
  const int d = H->g.dim;
  for (int colour = 0; colour < 2; ++colour)
    for (int64_t P = 0; P < L->nn; ++P) {
      if (L->cls[P] != ORC_IN || (off_band && L->band[P])) continue;
      if (parity(L, d, P) != colour) continue;
      relax_interior(H, L, P, u, rhs);
    }
}

static void relax(ohandle* H, int l, double* u, const double* rhs) {
  olev* L = &H->lev[l];
  const int d = H->g.dim;
  if (H->g.smoother != 0 && H->g.ordering == 1) {
    const int kac = H->g.smoother == 1, M = kac ? 5 : 7;
    int nc = 1;
    for (int a = 0; a < d; ++a) nc *= M;
    rb_interior(H, L, u, rhs, !kac);
    for (int k = 0; k < (kac ? H->g.lambda : 1); ++k)
      for (int c = 0; c < nc; ++c)
        for (int64_t P = 0; P < L->nn; ++P) {
          if (!L->band[P] || colour_of(L, d, P, M) != c) continue;
          if (kac)
            kaczmarz_row(H, L, P, u, rhs);
          else
            (void)block_solve(H, L, P, u, rhs);
        }
    return;
  }
  if (H->g.smoother == 1) {
    FOR_LEX(L, d, P) {
      if (L->cls[P] == ORC_IN) relax_interior(H, L, P, u, rhs);
    }
    for (int k = 0; k < H->g.lambda; ++k) {
      FOR_LEX(L, d, P) {
        if (L->band[P]) kaczmarz_row(H, L, P, u, rhs);
      }
    }
    return;
  }
  if (H->g.smoother == 2) {
    FOR_LEX(L, d, P) {
      if (L->cls[P] == ORC_IN && !L->band[P]) relax_interior(H, L, P, u, rhs);
    }
    FOR_LEX(L, d, P) {
      if (L->band[P]) (void)block_solve(H, L, P, u, rhs);
    }
    return;
  }
  relax_pass(H, l, u, rhs, 0);
  for (int k = 0; k < H->g.lambda; ++k) relax_pass(H, l, u, rhs, 1);
}

/* extension of the defect outside Omega_h, steady state of Eq. (exp) in phi order */
static void extend(const ohandle* H, int l, double* r) {
  const olev* F = &H->lev[l];
  for (int64_t e = 0; e < F->ne; ++e) {
    double num = 0.0, den = 0.0;
    for (int a = 0; a < 3; ++a) {
      int64_t Q = F->esrc[3 * e + a];
      if (Q < 0) continue;
      num += F->ewt[3 * e + a] * r[Q];
      den += F->ewt[3 * e + a];
    }
    r[F->enode[e]] = den > 0.0 ? num / den : 0.0;
  }
}

static double w1d(int lo, int hi, int k) {
  if (lo == -1 && hi == 1) return k == 0 ? 0.5 : 0.25; /* Eq. (restI): (1,2,1)/4 */
  if (lo == hi) return 1.0;                             /* single node */
  return 0.5;                                           /* Eqs. (restL), (restR) */
}

/* composite restriction I = I~(w, D_h - Omega_h, I~(w, Omega_h, 0)) (Sec. 2.5) */
static void restrict_defect(const ohandle* H, int l, const double* r, double* rc) {
  const olev* F = &H->lev[l];
  const olev* C = &H->lev[l + 1];
  const int d = H->g.dim;
#pragma omp parallel for schedule(static)
  for (int64_t X = 0; X < C->nn; ++X) {
    rc[X] = 0.0;
    if (C->cls[X] == ORC_OUT) continue;
    int jc[3];
    to_j(C, d, X, jc);
    const int8_t* lo = &F->rlo[3 * X];
    const int8_t* hi = &F->rhi[3 * X];
    int ext[3] = {1, 1, 1}, cnt = 1;
    for (int a = 0; a < d; ++a) {
      ext[a] = hi[a] - lo[a] + 1;
      cnt *= ext[a];
    }
    double s = 0.0;
    for (int t = 0; t < cnt; ++t) {
      /* k_x slowest */
      int k[3] = {0, 0, 0}, tt = t;
      for (int a = d - 1; a >= 0; --a) {
        k[a] = lo[a] + tt % ext[a];
        tt /= ext[a];
      }
      int j[3] = {0, 0, 0};
      double w = 1.0;
      for (int a = 0; a < d; ++a) {
        j[a] = 2 * jc[a] + k[a];
        w *= w1d(lo[a], hi[a], k[a]);
      }
      s += w * r[to_idx(F, d, j)];
    }
    rc[X] = s;
  }
}

/* bilinear (multilinear) interpolation of the coarse error, renormalised over the coarse
 * nodes that carry an unknown, and correction of the fine unknowns (Sec. 2.6.1) */
static void prolong_correct(const ohandle* H, int l, const double* ec, double* u) {
  const olev* F = &H->lev[l];
  const olev* C = &H->lev[l + 1];
  const int d = H->g.dim;
#pragma omp parallel for schedule(static)
  for (int64_t P = 0; P < F->nn; ++P) {
    if (F->cls[P] == ORC_OUT) continue;
    int j[3];
    to_j(F, d, P, j);
    int ncomb = 1 << d;
    double num = 0.0, den = 0.0;
    for (int m = 0; m < ncomb; ++m) {
      int jc[3] = {0, 0, 0};
      double w = 1.0;
      int skip = 0;
      for (int a = 0; a < d; ++a) {
        int bit = (m >> a) & 1;
        if (j[a] % 2 == 0) {
          if (bit) {
            skip = 1;
            break;
          }
          jc[a] = j[a] / 2;
        } else {
          jc[a] = bit ? (j[a] + 1) / 2 : (j[a] - 1) / 2;
          w *= 0.5;
        }
      }
      if (skip) continue;
      int64_t X = to_idx(C, d, jc);
      if (C->cls[X] == ORC_OUT) continue;
      num += w * ec[X];
      den += w;
    }
    if (den > 0.0) u[P] += num / den;
  }
}

static void coarse_solve(const ohandle* H, double* u, const double* rhs) {
  const olev* C = &H->lev[H->L];
  int64_t nu = C->nu;
  double* x = C->tmp;
  for (int64_t i = 0; i < nu; ++i) x[i] = rhs[C->umap[i]];
  for (int64_t k = 0; k < nu; ++k) {
    int64_t p = C->piv[k];
    if (p != k) {
      double t = x[k];
      x[k] = x[p];
      x[p] = t;
    }
  }
  for (int64_t i = 0; i < nu; ++i) {
    double s = x[i];
    for (int64_t j = 0; j < i; ++j) s -= C->lu[i * nu + j] * x[j];
    x[i] = s;
  }
  for (int64_t i = nu - 1; i >= 0; --i) {
    double s = x[i];
    for (int64_t j = i + 1; j < nu; ++j) s -= C->lu[i * nu + j] * x[j];
    x[i] = s / C->lu[i * nu + i];
  }
  for (int64_t i = 0; i < C->nn; ++i) u[i] = 0.0;
  for (int64_t i = 0; i < nu; ++i) u[C->umap[i]] = x[i];
}

/* TGCS / V / W cycle (Sec. 2.4, Remarks 1-2 of Sec. 1.3) */
static void cycle(ohandle* H, int l, double* u, const double* rhs) {
  olev* F = &H->lev[l];
  if (l == H->L) {
    coarse_solve(H, u, rhs);
    return;
  }
  for (int i = 0; i < H->g.nu1; ++i) relax(H, l, u, rhs);
  defect(H, l, u, rhs, F->r, NULL, NULL);
  extend(H, l, F->r);
  olev* C = &H->lev[l + 1];
  restrict_defect(H, l, F->r, C->rhs);
  memset(C->u, 0, (size_t)C->nn * sizeof(double));
  for (int k = 0; k < H->g.gamma; ++k) cycle(H, l + 1, C->u, C->rhs);
  prolong_correct(H, l, C->u, u);
  for (int i = 0; i < H->g.nu2; ++i) relax(H, l, u, rhs);
}

/* ------------------------------------------------------------------------------------ */
/* exported entry points                                                                */
/* ------------------------------------------------------------------------------------ */

int orc_num_levels(void* h) { return ((ohandle*)h)->L + 1; }

/* Threads of the red-black passes, the defect, the restriction and the interpolation (the
 * results do not depend on it); returns the number in use.  n <= 0 only queries. */
int orc_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* out: n, nn, nint, ng, nband(interior part), ne, nu(coarsest only) */
int orc_level_info(void* h, int l, int64_t* out) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  olev* L = &H->lev[l];
  out[0] = L->n;
  out[1] = L->nn;
  out[2] = L->nint;
  out[3] = L->ng;
  out[4] = L->nband;
  out[5] = L->ne;
  out[6] = (l == H->L) ? L->nu : 0;
  return ORC_OK;
}

int orc_get_cls(void* h, int l, int8_t* cls, int8_t* band) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  olev* L = &H->lev[l];
  if (cls) memcpy(cls, L->cls, (size_t)L->nn);
  if (band) memcpy(band, L->band, (size_t)L->nn);
  return ORC_OK;
}

/* BC labels of the nodes of level l: the type (1 D, 0 N) of the closest boundary point of
 * every ghost and extension node, -1 elsewhere */
int orc_get_labels(void* h, int l, int8_t* lab) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L || !lab) return ORC_EINVAL;
  memcpy(lab, H->lev[l].lab, (size_t)H->lev[l].nn);
  return ORC_OK;
}

int orc_get_ghosts(void* h, int l, int64_t* node, int8_t* type, int8_t* rung, int8_t* sgn,
                   double* B, double* nG, double* nB, double* xi, double* c, int64_t* wn,
                   double* w) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  olev* L = &H->lev[l];
  int64_t ng = L->ng;
  if (node) memcpy(node, L->gnode, (size_t)ng * sizeof(int64_t));
  if (type) memcpy(type, L->gtype, (size_t)ng);
  if (rung) memcpy(rung, L->grung, (size_t)ng);
  if (sgn) memcpy(sgn, L->gsgn, (size_t)(3 * ng));
  if (B) memcpy(B, L->gB, (size_t)(3 * ng) * sizeof(double));
  if (nG) memcpy(nG, L->gnG, (size_t)(3 * ng) * sizeof(double));
  if (nB) memcpy(nB, L->gnB, (size_t)(3 * ng) * sizeof(double));
  if (xi) memcpy(xi, L->gxi, (size_t)(3 * ng) * sizeof(double));
  if (c) memcpy(c, L->gc, (size_t)ng * sizeof(double));
  if (wn) memcpy(wn, L->gwn, (size_t)(H->K * ng) * sizeof(int64_t));
  if (w) memcpy(w, L->gw, (size_t)(H->K * ng) * sizeof(double));
  return ORC_OK;
}

int orc_get_extension(void* h, int l, int64_t* node, int64_t* src, double* wt) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l >= H->L) return ORC_EINVAL;
  olev* L = &H->lev[l];
  if (node) memcpy(node, L->enode, (size_t)L->ne * sizeof(int64_t));
  if (src) memcpy(src, L->esrc, (size_t)(3 * L->ne) * sizeof(int64_t));
  if (wt) memcpy(wt, L->ewt, (size_t)(3 * L->ne) * sizeof(double));
  return ORC_OK;
}

/* restriction boxes (lo, hi per axis) for every node of level l+1 */
int orc_get_boxes(void* h, int l, int8_t* lo, int8_t* hi) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l >= H->L) return ORC_EINVAL;
  olev* F = &H->lev[l];
  olev* C = &H->lev[l + 1];
  memcpy(lo, F->rlo, (size_t)(3 * C->nn));
  memcpy(hi, F->rhi, (size_t)(3 * C->nn));
  return ORC_OK;
}

int orc_defect(void* h, int l, const double* u, const double* rhs, double* r, double* norms) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  defect(H, l, u, rhs, r, &norms[0], &norms[1]);
  return ORC_OK;
}

int orc_relax(void* h, int l, double* u, const double* rhs, int band_only) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  if (band_only < 0)
    relax(H, l, u, rhs);
  else
    relax_pass(H, l, u, rhs, band_only);
  return ORC_OK;
}

/* One Kaczmarz step (kind 1) or one block relaxation (kind 2) at node P of level l. */
int orc_boundary_step(void* h, int l, int64_t P, double* u, const double* rhs, int kind) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  const olev* L = &H->lev[l];
  if (P < 0 || P >= L->nn || L->cls[P] == ORC_OUT) return ORC_EINVAL;
  if (kind == 1) {
    kaczmarz_row(H, L, P, u, rhs);
    return ORC_OK;
  }
  if (kind == 2) return block_solve(H, L, P, u, rhs) ? ORC_EGEOM : ORC_OK;
  return ORC_EINVAL;
}

/* Smoothing factor of Sec. 3.3: the relaxation alone (no coarse grid) on the homogeneous
 * problem from u, mu^(m) = ||r^(m)||_inf / ||r^(m-1)||_inf for m = 1..iters (in hist). */
int orc_smoothing(void* h, double* u, int iters, double* hist) {
  ohandle* H = (ohandle*)h;
  olev* F = &H->lev[0];
  double* zero = (double*)calloc((size_t)F->nn, sizeof(double));
  if (!zero) return ORC_ENOMEM;
  double ni, ngh;
  defect(H, 0, u, zero, F->r, &ni, &ngh);
  double prev = ni > ngh ? ni : ngh;
  for (int m = 0; m < iters; ++m) {
    relax(H, 0, u, zero);
    defect(H, 0, u, zero, F->r, &ni, &ngh);
    const double rn = ni > ngh ? ni : ngh;
    hist[m] = rn / prev;
    prev = rn;
  }
  free(zero);
  return ORC_OK;
}

int orc_extend(void* h, int l, double* r) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l >= H->L) return ORC_EINVAL;
  extend(H, l, r);
  return ORC_OK;
}

int orc_restrict(void* h, int l, const double* r, double* rc) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l >= H->L) return ORC_EINVAL;
  restrict_defect(H, l, r, rc);
  return ORC_OK;
}

int orc_prolong(void* h, int l, const double* ec, double* u) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l >= H->L) return ORC_EINVAL;
  prolong_correct(H, l, ec, u);
  return ORC_OK;
}

int orc_coarse_solve(void* h, double* u, const double* rhs) {
  coarse_solve((ohandle*)h, u, rhs);
  return ORC_OK;
}

/* one cycle on the finest level */
int orc_cycle(void* h, double* u, const double* rhs) {
  cycle((ohandle*)h, 0, u, rhs);
  return ORC_OK;
}

/* Cycles until ||r||_inf / ||(f_h, g_h)||_inf <= tol.  hist[m] = relative residual
 * before cycle m (hist must hold max_cycles + 1 entries). */
int orc_solve(void* h, double* u, const double* rhs, double tol, int max_cycles, double* hist,
              int* ncycles) {
  ohandle* H = (ohandle*)h;
  olev* F = &H->lev[0];
  double r0 = 0.0;
  for (int64_t P = 0; P < F->nn; ++P)
    if (F->cls[P] != ORC_OUT && fabs(rhs[P]) > r0) r0 = fabs(rhs[P]);
  if (r0 == 0.0) r0 = 1.0;
  double prev = INFINITY;
  int grew = 0;
  for (int m = 0;; ++m) {
    double ni, ngh;
    defect(H, 0, u, rhs, F->r, &ni, &ngh);
    double rel = (ni > ngh ? ni : ngh) / r0;
    if (ni != ni || ngh != ngh) rel = NAN;
    if (hist) hist[m] = rel;
    *ncycles = m;
    if (rel <= tol) return ORC_OK;
    /* divergence: a non-finite residual, or growth over five consecutive cycles */
    grew = (rel > prev) ? grew + 1 : 0;
    if (!(rel < INFINITY) || grew >= 5) return ORC_EDIVERGED;
    prev = rel;
    if (m >= max_cycles) return ORC_ENOCONV;
    cycle(H, 0, u, rhs);
  }
}

/* Convergence factor of Sec. 3 on the homogeneous problem from the initial guess u:
 * rho^(m) = ||r^(m)|| / ||r^(m-1)||, stopped when |rho^(m) - rho^(m-1)| / rho^(m) < rtol.
 * u is rescaled after every cycle (the iteration is linear and homogeneous).  Returns the
 * last factor in *rho; hist receives rho^(m) for m = 1..ncycles. */
int orc_rho(void* h, double* u, int max_cycles, double rtol, double* rho, double* hist,
            int* ncycles) {
  ohandle* H = (ohandle*)h;
  olev* F = &H->lev[0];
  double* zero = (double*)calloc((size_t)F->nn, sizeof(double));
  if (!zero) return ORC_ENOMEM;
  double ni, ngh;
  defect(H, 0, u, zero, F->r, &ni, &ngh);
  double rprev = ni > ngh ? ni : ngh, rho_prev = -1.0, rr = 0.0;
  int m;
  for (m = 1; m <= max_cycles; ++m) {
    cycle(H, 0, u, zero);
    defect(H, 0, u, zero, F->r, &ni, &ngh);
    double rn = ni > ngh ? ni : ngh;
    rr = rn / rprev;
    if (hist) hist[m - 1] = rr;
    if (!(rn > 0.0) || rn != rn) break;
    for (int64_t P = 0; P < F->nn; ++P) u[P] /= rn;
    rprev = 1.0;
    if (rho_prev > 0.0 && fabs(rr - rho_prev) / rr < rtol) break;
    if (rr > 1e3) break;
    rho_prev = rr;
  }
  free(zero);
  *rho = rr;
  *ncycles = m > max_cycles ? max_cycles : m;
  return ORC_OK;
}

/* Sparse rows of the system Eq. (discr) on level l, in CSR over the unknowns ordered by
 * node index.  Call with indptr == NULL to get the number of unknowns and non-zeros. */
int orc_assemble(void* h, int l, int64_t* nrows, int64_t* nnz, int64_t* rowmap, int64_t* indptr,
                 int64_t* indices, double* data) {
  ohandle* H = (ohandle*)h;
  if (l < 0 || l > H->L) return ORC_EINVAL;
  olev* L = &H->lev[l];
  const int d = H->g.dim, K = H->K;
  int64_t nu = 0, nz = 0;
  for (int64_t P = 0; P < L->nn; ++P) {
    if (L->cls[P] == ORC_IN) {
      ++nu;
      nz += 2 * d + 1;
    } else if (L->cls[P] == ORC_GHOST) {
      ++nu;
      int64_t g = L->gid[P];
      for (int t = 0; t < K; ++t) nz += (L->gwn[K * g + t] >= 0);
    }
  }
  *nrows = nu;
  *nnz = nz;
  if (!indptr) return ORC_OK;
  int64_t* col = (int64_t*)malloc((size_t)L->nn * sizeof(int64_t));
  if (!col) return ORC_ENOMEM;
  int64_t q = 0;
  for (int64_t P = 0; P < L->nn; ++P) {
    col[P] = -1;
    if (L->cls[P] != ORC_OUT) {
      rowmap[q] = P;
      col[P] = q++;
    }
  }
  double ih2 = 1.0 / (L->h * L->h);
  int64_t k = 0;
  for (int64_t r = 0; r < nu; ++r) {
    int64_t P = rowmap[r];
    indptr[r] = k;
    if (L->cls[P] == ORC_IN) {
      /* -Delta_h u = f */
      indices[k] = col[P];
      data[k++] = 2.0 * d * ih2;
      for (int a = 0; a < d; ++a) {
        indices[k] = col[P - L->st[a]];
        data[k++] = -ih2;
        indices[k] = col[P + L->st[a]];
        data[k++] = -ih2;
      }
    } else {
      /* L_h u = g */
      int64_t g = L->gid[P];
      for (int t = 0; t < K; ++t) {
        int64_t nd = L->gwn[K * g + t];
        if (nd < 0) continue;
        indices[k] = col[nd];
        data[k++] = L->gw[K * g + t];
      }
    }
  }
  indptr[nu] = k;
  free(col);
  return ORC_OK;
}
