// Host construction of the multigrid hierarchy: node classes, ghost records, boundary
// bands, defect-extension lists, restriction codes, active tiles and the coarsest-grid
// inverse.  FP64 throughout; built with -ffp-contract=off so every geometric decision
// (interior / ghost, boundary-condition type, upwind signs, processing order) is an exact
// function of phi.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "ghostmg_impl.h"

namespace ghostmg {
namespace {

enum { OUT = 0, IN = 1, GHOST = 2 };

// One level of one problem in unpadded node order (x fastest).
struct PL {
  int D = 2, n = 0, np = 0;
  double h = 0.0, lo = -1.0;
  int64_t nn = 0, st[3] = {0, 0, 0};
  std::vector<double> phi;
  std::vector<int8_t> cls;
  std::vector<int32_t> gid;   // node -> ghost index, -1 otherwise
  std::vector<int8_t> lab;    // boundary-condition label of outside nodes, -1 otherwise
  std::vector<GhostRec> gh;   // node field holds the local unpadded index here
  std::vector<double> B;      // 3 per ghost
};

inline void jof(const PL& L, int64_t idx, int j[3]) {
  j[0] = j[1] = j[2] = 0;
  for (int a = 0; a < L.D; ++a) {
    j[a] = (int)(idx % L.np);
    idx /= L.np;
  }
}
inline int64_t iof(const PL& L, const int j[3]) {
  int64_t idx = 0;
  for (int a = L.D - 1; a >= 0; --a) idx = idx * L.np + j[a];
  return idx;
}
inline bool inbox(const PL& L, const int j[3]) {
  for (int a = 0; a < L.D; ++a)
    if (j[a] < 0 || j[a] > L.n) return false;
  return true;
}

// Gradient of phi: central differences, one-sided second order on the box faces.
void gradient(const PL& L, const int j[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  const int64_t c = iof(L, j);
  for (int a = 0; a < L.D; ++a) {
    const int64_t s = L.st[a];
    if (j[a] > 0 && j[a] < L.n)
      g[a] = (L.phi[c + s] - L.phi[c - s]) / (2.0 * L.h);
    else if (j[a] == 0)
      g[a] = (-3.0 * L.phi[c] + 4.0 * L.phi[c + s] - L.phi[c + 2 * s]) / (2.0 * L.h);
    else
      g[a] = (3.0 * L.phi[c] - 4.0 * L.phi[c - s] + L.phi[c - 2 * s]) / (2.0 * L.h);
  }
}

// The partition of the boundary into Gamma_D and Gamma_N (Sec. 2.1), evaluated at a closest
// boundary point: a half-space rule, or the caller's function.
struct BcPartition {
  const mg_bc_rule* rule;
  mg_bc_fn fn;
  void* ctx;
  int problem;
  bool dirichlet(int D, const double* B) const {
    if (fn) {
      double b[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < D; ++a) b[a] = B[a];
      return fn(problem, b, ctx) != 0;
    }
    double v = rule->c;
    for (int a = 0; a < D; ++a) v += rule->a[a] * B[a];
    return rule->strict ? (v > 0.0) : (v >= 0.0);
  }
};

template <int D>
void row_weights(const GhostRec& g, double inv_h, double* w) {
  ghost_row<D>(g, inv_h, w);
}

// The host side of a level's classification (the classes, ghost records and closest points
// come from classify_level_gpu): the node -> ghost index map, the boundary-condition labels of
// the ghosts and, with a caller's partition, the ghosts' types (Dirichlet ghosts keep no
// normal; a Neumann ghost needs one).
int finish_classes(PL& L, const BcPartition& part) {
  L.gid.assign(L.nn, -1);
  L.lab.assign(L.nn, -1);
  for (size_t q = 0; q < L.gh.size(); ++q) {
    GhostRec& r = L.gh[q];
    if (part.fn) {
      r.type = part.dirichlet(L.D, &L.B[3 * q]) ? 1 : 0;
      if (r.type) {
        for (int a = 0; a < 3; ++a) r.nb[a] = 0.0;
      } else if (r.pad0) {
        return MG_EGEOM;  // no normal at B
      }
    }
    r.pad0 = 0;
    L.gid[r.node] = (int32_t)q;
    L.lab[r.node] = r.type;
  }
  return MG_OK;
}

struct Ext {
  int64_t node;
  int64_t src[3];
  double wt[3];
  int dag;
};

// Nodes of the defect extension for the transfer from F to the next coarser level C
// (Sec. 2.6): every outside non-ghost node of F in the 3^D neighbourhood of a ghost of C,
// processed once in increasing phi, each averaging its available upwind neighbours
// Q_a = P - sgn(n_a) e_a with weights |n_a| (the steady state of Eq. (exp)).
int extension(PL& F, const PL& C, const mg_grid& G, const BcPartition& part,
              std::vector<Ext>& out) {
  const int D = F.D;
  int nnb = 1;
  for (int a = 0; a < D; ++a) nnb *= 3;
  // the extension nodes: outside fine nodes under the coarse ghosts, each once (ids, in
  // increasing node index); a node's rank (its position in increasing phi) and DAG level
  // are kept per id, looked up by binary search (the fine level has far more nodes than
  // extension nodes)
  std::vector<int64_t> ids;
  for (int64_t X = 0; X < C.nn; ++X) {
    if (C.cls[X] != GHOST) continue;
    int jc[3];
    jof(C, X, jc);
    for (int o = 0; o < nnb; ++o) {
      int j[3] = {0, 0, 0}, oo = o;
      for (int a = 0; a < D; ++a) {
        j[a] = 2 * jc[a] + oo % 3 - 1;
        oo /= 3;
      }
      if (!inbox(F, j)) continue;
      const int64_t P = iof(F, j);
      if (F.cls[P] == OUT) ids.push_back(P);
    }
  }
  std::sort(ids.begin(), ids.end());
  ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
  auto slot = [&](int64_t P) -> int64_t {  // position of P in ids, -1 when absent
    const auto it = std::lower_bound(ids.begin(), ids.end(), P);
    return it != ids.end() && *it == P ? (int64_t)(it - ids.begin()) : -1;
  };
  std::vector<int64_t> nodes(ids);
  std::sort(nodes.begin(), nodes.end(), [&](int64_t a, int64_t b) {
    if (F.phi[a] != F.phi[b]) return F.phi[a] < F.phi[b];
    return a < b;
  });
  std::vector<int64_t> rank(ids.size(), -1);
  for (size_t e = 0; e < nodes.size(); ++e) rank[slot(nodes[e])] = (int64_t)e;
  std::vector<int> dag(ids.size(), 0);
  out.clear();
  out.reserve(nodes.size());
  for (size_t e = 0; e < nodes.size(); ++e) {
    const int64_t P = nodes[e];
    Ext x;
    x.node = P;
    x.dag = 1;
    for (int a = 0; a < 3; ++a) {
      x.src[a] = -1;
      x.wt[a] = 0.0;
    }
    int j[3];
    jof(F, P, j);
    double gr[3];
    gradient(F, j, gr);
    double n2 = 0.0;
    for (int a = 0; a < D; ++a) n2 += gr[a] * gr[a];
    const double nrm = std::sqrt(n2);
    const int64_t sp = slot(P);
    if (!(nrm > 0.0)) {
      F.lab[P] = 1;
      dag[sp] = 1;
      out.push_back(x);
      continue;
    }
    double Bp[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) Bp[a] = (F.lo + F.h * (double)j[a]) - gr[a] / nrm * F.phi[P];
    F.lab[P] = part.dirichlet(D, Bp) ? 1 : 0;
    int nsame = 0;
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1 && (!G.split || nsame > 0)) break;
      for (int a = 0; a < D; ++a) {
        const double na = gr[a] / nrm;
        if (na == 0.0) continue;
        int q[3] = {j[0], j[1], j[2]};
        q[a] -= na > 0.0 ? 1 : -1;
        if (!inbox(F, q)) continue;
        const int64_t Q = iof(F, q);
        const int64_t sq = F.cls[Q] == OUT ? slot(Q) : -1;
        const bool avail = F.cls[Q] == GHOST || (sq >= 0 && rank[sq] < (int64_t)e);
        if (!avail) continue;
        if (G.split && pass == 0 && F.lab[Q] != F.lab[P]) continue;
        if (pass == 0) ++nsame;
        x.src[a] = Q;
        x.wt[a] = std::fabs(na);
      }
    }
    int lvl = 1;
    for (int a = 0; a < 3; ++a)
      if (x.src[a] >= 0 && F.cls[x.src[a]] == OUT) lvl = std::max(lvl, dag[slot(x.src[a])] + 1);
    dag[sp] = lvl;
    x.dag = lvl;
    out.push_back(x);
  }
  return MG_OK;
}

// Box of the partial full-weighting transfer at coarse node X (Sec. 2.5): the largest box
// [lo_a, hi_a], lo in {-1, 0}, hi in {0, 1}, whose fine nodes all lie in I_h; ties go to
// the larger x, then y, then z extent, then to a box starting at -1 in x, then y, then z.
uint8_t box_code(const PL& F, const int jf[3], bool inside, int lab) {
  const int D = F.D;
  int best[7] = {0, 0, 0, 0, 0, 0, 0};
  bool have = false;
  uint8_t code = 0;
  int ncand = 1;
  for (int a = 0; a < D; ++a) ncand *= 4;
  for (int c = 0; c < ncand; ++c) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, cc = c;
    for (int a = 0; a < D; ++a) {
      lo[a] = (cc & 1) ? -1 : 0;
      hi[a] = (cc & 2) ? 1 : 0;
      cc >>= 2;
    }
    int ext[3] = {1, 1, 1}, cnt = 1;
    for (int a = 0; a < D; ++a) {
      ext[a] = hi[a] - lo[a] + 1;
      cnt *= ext[a];
    }
    bool ok = true;
    for (int t = 0; t < cnt && ok; ++t) {
      int j[3] = {jf[0], jf[1], jf[2]}, tt = t;
      for (int a = 0; a < D; ++a) {
        j[a] = jf[a] + lo[a] + tt % ext[a];
        tt /= ext[a];
      }
      if (!inbox(F, j)) {
        ok = false;
        break;
      }
      const int64_t P = iof(F, j);
      if (inside)
        ok = F.cls[P] == IN;
      else
        ok = F.cls[P] != IN && (lab < 0 || F.lab[P] == lab);
    }
    if (!ok) continue;
    int key[7] = {cnt, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < D; ++a) {
      key[1 + a] = ext[a];
      key[4 + a] = lo[a] == -1;
    }
    bool better = !have;
    for (int m = 0; m < 7 && have; ++m)
      if (key[m] != best[m]) {
        better = key[m] > best[m];
        break;
      }
    if (better) {
      have = true;
      std::memcpy(best, key, sizeof(key));
      code = 0;
      for (int a = 0; a < D; ++a) code |= (uint8_t)(((lo[a] == -1) << (2 * a)) | ((hi[a] == 1) << (2 * a + 1)));
    }
  }
  return code;
}

// Explicit inverse of the coarsest system by LU with partial pivoting (FP64).
int invert(std::vector<double>& A, int n, std::vector<double>& inv) {
  // LU with partial pivoting, then the inverse column by column.  The rows of the coarsest
  // system couple nodes a few grid rows apart, so the factors are banded: every loop runs
  // over the nonzero span of its row only (the same operations as the dense loops, minus
  // those on zeros), and the columns of the inverse are solved on several threads.
  std::vector<int> piv(n);
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  auto last_nz = [&](int r) {
    int j = n - 1;
    while (j > r && A[(size_t)r * n + j] == 0.0) --j;
    return j;
  };
  for (int k = 0; k < n; ++k) {
    int p = k;
    double pv = std::fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > pv) {
        pv = std::fabs(A[(size_t)i * n + k]);
        p = i;
      }
    piv[k] = p;
    if (!(pv > 1e-13 * amax)) return MG_EGEOM;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
    const double d = A[(size_t)k * n + k];
    const int ub = last_nz(k);
    for (int i = k + 1; i < n; ++i) {
      if (A[(size_t)i * n + k] == 0.0) continue;
      const double m = A[(size_t)i * n + k] / d;
      A[(size_t)i * n + k] = m;
      double* ri = &A[(size_t)i * n];
      const double* rk = &A[(size_t)k * n];
      for (int j = k + 1; j <= ub; ++j) ri[j] -= m * rk[j];
    }
  }
  // spans of the factors: L row i from lo[i], U row i up to hi[i]
  std::vector<int> lo(n), hi(n);
  for (int i = 0; i < n; ++i) {
    int j = 0;
    while (j < i && A[(size_t)i * n + j] == 0.0) ++j;
    lo[i] = j;
    hi[i] = last_nz(i);
  }
  inv.assign((size_t)n * n, 0.0);
  auto solve_cols = [&](int c0, int c1) {
    std::vector<double> x(n);
    for (int c = c0; c < c1; ++c) {
      for (int i = 0; i < n; ++i) x[i] = 0.0;
      x[c] = 1.0;
      for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(x[k], x[piv[k]]);
      for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int j = lo[i]; j < i; ++j) s -= A[(size_t)i * n + j] * x[j];
        x[i] = s;
      }
      for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j <= hi[i]; ++j) s -= A[(size_t)i * n + j] * x[j];
        x[i] = s / A[(size_t)i * n + i];
      }
      for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = x[i];
    }
  };
  const int nt = n < 512 ? 1 : (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (nt == 1) {
    solve_cols(0, n);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(solve_cols, (int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt));
    for (auto& x : th) x.join();
  }
  return MG_OK;
}

}  // namespace

// Build every level of every problem; phi is device memory, batch * (n+1)^D values.
int build_hierarchy(mg_handle_s* H, const double* phi) {
  const mg_grid& G = H->grid;
  const int D = G.dim, batch = G.batch, L = H->L;
  H->host.assign(L + 1, HostLevel());
  for (int l = 0; l <= L; ++l) {
    Geo& g = H->host[l].g;
    g.n = G.n >> l;
    g.np = g.n + 1;
    g.pitch = (g.np + 15) / 16 * 16;
    g.h = (G.hi - G.lo) / (double)g.n;
    g.st[0] = 1;
    g.st[1] = g.pitch;
    g.st[2] = D == 3 ? (int64_t)g.pitch * g.np : 0;
    g.npp = D == 3 ? (int64_t)g.pitch * g.np * g.np : (int64_t)g.pitch * g.np;
    H->host[l].cls.assign((size_t)batch * g.npp, 0);
    H->host[l].rcode.assign((size_t)batch * g.npp, kNoUnknown);
    H->host[l].ghost_off.assign(1, 0);
    H->host[l].red_off.assign(1, 0);
    H->host[l].black_off.assign(1, 0);
    H->host[l].ext_off.assign(1, 0);
    H->host[l].dag_start.assign(1, 0);
    H->host[l].umap_off.assign(1, 0);
    H->host[l].ainv_off.assign(1, 0);
  }
  for (int p = 0; p < batch; ++p) {
    const BcPartition part{H->bc_fn ? nullptr : &H->bc[p], H->bc_fn, H->bc_ctx, p};
    std::vector<PL> lev(L + 1);
    for (int l = 0; l <= L; ++l) {
      PL& V = lev[l];
      V.D = D;
      V.n = G.n >> l;
      V.np = V.n + 1;
      V.h = (G.hi - G.lo) / (double)V.n;
      V.lo = G.lo;
      V.nn = 1;
      for (int a = 0; a < D; ++a) {
        V.st[a] = V.nn;
        V.nn *= V.np;
      }
      // classes, ghost records and closest points on the GPU (Sec. 2.2-2.3)
      LevelClass lc;
      int rc = classify_level_gpu(phi, D, G.n, l, p, G.lo, V.h, H->bc_fn ? nullptr : &H->bc[p], lc);
      if (rc) return rc;
      V.phi = std::move(lc.phi);
      V.cls = std::move(lc.cls);
      V.gh = std::move(lc.gh);
      V.B = std::move(lc.B);
      if ((rc = finish_classes(V, part))) return rc;
    }
    for (int l = 0; l <= L; ++l) {
      PL& V = lev[l];
      HostLevel& HL = H->host[l];
      const Geo& g = HL.g;
      const int64_t base = (int64_t)p * g.npp;
      auto pad = [&](int64_t local) {
        int j[3];
        jof(V, local, j);
        return base + j[0] + g.st[1] * j[1] + g.st[2] * j[2];
      };
      if (l > 0 && HL.phi.empty()) HL.phi.assign((size_t)batch * g.npp, 0.0);
      for (int64_t i = 0; i < V.nn; ++i) {
        HL.cls[pad(i)] = V.cls[i];
        if (l > 0) HL.phi[pad(i)] = V.phi[i];
        if (V.cls[i] == IN) ++HL.nint;
      }
      // ghosts
      for (size_t q = 0; q < V.gh.size(); ++q) {
        GhostRec r = V.gh[q];
        r.node = (int32_t)pad(r.node);
        HL.ghosts.push_back(r);
        for (int a = 0; a < 3; ++a) HL.gB.push_back(V.B[3 * q + a]);
      }
      HL.nghost += (int64_t)V.gh.size();
      HL.ghost_off.push_back((int32_t)HL.ghosts.size());
      // boundary band: interior nodes within delta = delta_h h of the boundary (Sec. 3.2)
      const double delta = G.delta_h * V.h;
      for (int64_t i = 0; i < V.nn; ++i) {
        if (V.cls[i] != IN || !(V.phi[i] >= -delta)) continue;
        int j[3];
        jof(V, i, j);
        ((j[0] + j[1] + j[2]) & 1 ? HL.black : HL.red).push_back((int32_t)pad(i));
        ++HL.nband;
      }
      HL.red_off.push_back((int32_t)HL.red.size());
      HL.black_off.push_back((int32_t)HL.black.size());
      // tiles holding unknowns
      const int TX = D == 2 ? Tile<2>::X : Tile<3>::X;
      const int TY = D == 2 ? Tile<2>::Y : Tile<3>::Y;
      const int TZ = D == 2 ? 1 : Tile<3>::Z;
      const int ntx = (V.np + TX - 1) / TX, nty = (V.np + TY - 1) / TY;
      const int ntz = D == 2 ? 1 : (V.np + TZ - 1) / TZ;
      for (int tz = 0; tz < ntz; ++tz)
        for (int ty = 0; ty < nty; ++ty)
          for (int tx = 0; tx < ntx; ++tx) {
            bool any = false;
            for (int z = tz * TZ; z < std::min((tz + 1) * TZ, D == 2 ? 1 : V.np) && !any; ++z)
              for (int y = ty * TY; y < std::min((ty + 1) * TY, V.np) && !any; ++y)
                for (int x = tx * TX; x < std::min((tx + 1) * TX, V.np); ++x) {
                  const int64_t i = x + (int64_t)V.np * (y + (int64_t)V.np * z);
                  if (V.cls[i] != OUT) {
                    any = true;
                    break;
                  }
                }
            if (any) HL.tiles.push_back(make_int4(p, tx, ty, tz));
          }
    }
    // extension lists and restriction codes between consecutive levels
    for (int l = 0; l < L; ++l) {
      PL& F = lev[l];
      PL& C = lev[l + 1];
      HostLevel& HF = H->host[l];
      HostLevel& HC = H->host[l + 1];
      std::vector<Ext> ext;
      int rc = extension(F, C, G, part, ext);
      if (rc) return rc;
      const Geo& gf = HF.g;
      const int64_t basef = (int64_t)p * gf.npp;
      auto padf = [&](int64_t local) -> int32_t {
        if (local < 0) return -1;
        int j[3];
        jof(F, local, j);
        return (int32_t)(basef + j[0] + gf.st[1] * j[1] + gf.st[2] * j[2]);
      };
      std::stable_sort(ext.begin(), ext.end(), [](const Ext& a, const Ext& b) { return a.dag < b.dag; });
      int maxdag = 0;
      for (const Ext& x : ext) maxdag = std::max(maxdag, x.dag);
      // problem p's DAG levels: HF.ext[dag_off[dag_start[p] + d - 1], dag_off[... + d])
      const int32_t ebase = (int32_t)HF.ext.size();
      size_t k = 0;
      for (int d = 1; d <= maxdag; ++d) {
        HF.dag_off.push_back(ebase + (int32_t)k);
        while (k < ext.size() && ext[k].dag == d) ++k;
      }
      HF.dag_off.push_back(ebase + (int32_t)ext.size());
      HF.dag_start.push_back((int32_t)HF.dag_off.size());
      for (const Ext& x : ext) {
        ExtRec r;
        r.node = padf(x.node);
        for (int a = 0; a < 3; ++a) {
          r.src[a] = padf(x.src[a]);
          r.wt[a] = x.wt[a];
        }
        HF.ext.push_back(r);
      }
      HF.ext_off.push_back((int32_t)HF.ext.size());
      // restriction codes of the coarse nodes (each node's own box search: split over
      // threads, every thread writing its own nodes)
      const Geo& gc = HC.g;
      const int64_t basec = (int64_t)p * gc.npp;
      auto codes = [&](int64_t X0, int64_t X1) {
        for (int64_t X = X0; X < X1; ++X) {
          if (C.cls[X] == OUT) continue;
          int jc[3], jf[3] = {0, 0, 0};
          jof(C, X, jc);
          for (int a = 0; a < D; ++a) jf[a] = 2 * jc[a];
          const bool inside = C.cls[X] == IN;
          const int lab = (!inside && G.split) ? F.lab[iof(F, jf)] : -1;
          HC.rcode[basec + jc[0] + gc.st[1] * jc[1] + gc.st[2] * jc[2]] = box_code(F, jf, inside, lab);
        }
      };
      const int nt = C.nn < ((int64_t)1 << 16)
                         ? 1
                         : (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
      if (nt == 1) {
        codes(0, C.nn);
      } else {
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t) th.emplace_back(codes, C.nn * t / nt, C.nn * (t + 1) / nt);
        for (auto& x : th) x.join();
      }
    }
    // the coarsest system and its inverse
    {
      PL& C = lev[L];
      HostLevel& HC = H->host[L];
      const Geo& gc = HC.g;
      const int64_t basec = (int64_t)p * gc.npp;
      std::vector<int64_t> col(C.nn, -1);
      std::vector<int64_t> um;
      for (int64_t i = 0; i < C.nn; ++i)
        if (C.cls[i] != OUT) {
          col[i] = (int64_t)um.size();
          um.push_back(i);
        }
      const int nu = (int)um.size();
      std::vector<double> A((size_t)nu * nu, 0.0);
      const double ih2 = 1.0 / (C.h * C.h);
      const double inv_h = 1.0 / C.h;
      for (int r = 0; r < nu; ++r) {
        const int64_t P = um[r];
        if (C.cls[P] == IN) {
          A[(size_t)r * nu + r] += 2.0 * D * ih2;
          for (int a = 0; a < D; ++a) {
            A[(size_t)r * nu + col[P - C.st[a]]] -= ih2;
            A[(size_t)r * nu + col[P + C.st[a]]] -= ih2;
          }
        } else {
          const GhostRec& gr = C.gh[C.gid[P]];
          double w[27];
          uint32_t used = D == 2 ? ghost_row<2>(gr, inv_h, w) : ghost_row<3>(gr, inv_h, w);
          const int K = D == 2 ? 9 : 27;
          for (int t = 0; t < K; ++t) {
            if (!(used >> t & 1u)) continue;
            int64_t off = 0, tt = t;
            for (int c = D - 1; c >= 0; --c) {
              off += (int64_t)gr.s[c] * (tt % 3) * C.st[c];
              tt /= 3;
            }
            A[(size_t)r * nu + col[P + off]] += w[t];
          }
        }
      }
      std::vector<double> inv;
      int rc = invert(A, nu, inv);
      if (rc) return rc;
      for (int r = 0; r < nu; ++r) {
        int j[3];
        jof(C, um[r], j);
        HC.umap.push_back((int32_t)(basec + j[0] + gc.st[1] * j[1] + gc.st[2] * j[2]));
      }
      HC.umap_off.push_back((int32_t)HC.umap.size());
      HC.ainv.insert(HC.ainv.end(), inv.begin(), inv.end());
      HC.ainv_off.push_back((int64_t)HC.ainv.size());
    }
  }
  // extension lists merged over problems by DAG level (for launches per DAG level)
  for (int l = 0; l < L; ++l) {
    HostLevel& HF = H->host[l];
    int maxdag = 0;
    for (int p = 0; p < batch; ++p) maxdag = std::max(maxdag, HF.dag_start[p + 1] - HF.dag_start[p] - 1);
    HF.gdag_off.clear();
    HF.ext_merged.clear();
    for (int d = 1; d <= maxdag; ++d) {
      HF.gdag_off.push_back((int32_t)HF.ext_merged.size());
      for (int p = 0; p < batch; ++p) {
        const int nd = HF.dag_start[p + 1] - HF.dag_start[p] - 1;
        if (d > nd) continue;
        const int32_t a = HF.dag_off[HF.dag_start[p] + d - 1], b = HF.dag_off[HF.dag_start[p] + d];
        HF.ext_merged.insert(HF.ext_merged.end(), HF.ext.begin() + a, HF.ext.begin() + b);
      }
    }
    HF.gdag_off.push_back((int32_t)HF.ext_merged.size());
  }
  // relaxation codes (band interior nodes marked 3) and the row weights of every ghost
  const int K = D == 2 ? 9 : 27;
  for (int l = 0; l <= L; ++l) {
    HostLevel& HL = H->host[l];
    HL.rcls = HL.cls;
    for (int32_t v : HL.red) HL.rcls[v] = 3;
    for (int32_t v : HL.black) HL.rcls[v] = 3;
    HL.gw.assign(HL.ghosts.size() * K, 0.0);
    const double inv_h = 1.0 / HL.g.h;
    for (size_t i = 0; i < HL.ghosts.size(); ++i) {
      double w[27];
      const uint32_t used = D == 2 ? ghost_row<2>(HL.ghosts[i], inv_h, w)
                                   : ghost_row<3>(HL.ghosts[i], inv_h, w);
      for (int t = 0; t < K; ++t)
        if (used >> t & 1u) HL.gw[i * K + t] = w[t];
    }
  }
  return MG_OK;
}

}  // namespace ghostmg

namespace ghostmg {

namespace {

uint64_t spread_bits(uint64_t v, int D) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (D * b);
  return r;
}

void node_coords(const Geo& g, int D, int64_t v, int64_t* p, int j[3]) {
  *p = v / g.npp;
  int64_t loc = v - *p * g.npp;
  const int64_t z = D == 3 ? loc / g.st[2] : 0;
  loc -= z * g.st[2];
  const int64_t y = loc / g.st[1];
  j[0] = (int)(loc - y * g.st[1]);
  j[1] = (int)y;
  j[2] = (int)z;
}

// Morton order within a problem, problems in sequence
uint64_t morton_key(const Geo& g, int D, int64_t v) {
  int64_t p;
  int j[3];
  node_coords(g, D, v, &p, j);
  return ((uint64_t)p << 60) | spread_bits(j[0], D) | (spread_bits(j[1], D) << 1) |
         (spread_bits(j[2], D) << 2);
}

void pad_even(std::vector<int32_t>& v) {
  if (v.size() & 1) v.push_back(0);
}

void put_doubles(std::vector<int32_t>& v, const std::vector<double>& d) {
  const size_t w0 = v.size();
  v.resize(w0 + 2 * d.size());
  if (!d.empty()) std::memcpy(v.data() + w0, d.data(), d.size() * sizeof(double));
}

int32_t pack16(int a, int b) { return (int32_t)(((uint32_t)(uint16_t)a) | ((uint32_t)(uint16_t)b << 16)); }

// The chunk data just written from Dv[off] (packed layout: ns entries in runs of ng ghosts,
// nr red, nbk black, then read-only ones) rewritten in the fixed layout (band_fixed): entry i of
// run r moves to local id (first slot of r + i / W) W + i mod W, and every local id it stores
// (neighbour pairs, ghost tap addresses) is renumbered the same way; the earlier ghost values
// move from ns + j to NSW + j.  w32: the ghost weights are FP32.
void to_fixed_layout(std::vector<int32_t>& Dv, int32_t off, int D, int ns, int ng, int nr, int nbk,
                     int32_t gid_off, int32_t gw_off, int32_t gc_off, int32_t pc_off,
                     int32_t rs_off, bool pc, bool rs, bool w32) {
  const BandFixed F = band_fixed(D, pc, rs);
  const int W = F.W, NC = band_colour_slots(D), K = D == 2 ? 9 : 27;
  const int first_slot[4] = {0, 1, 1 + NC, 1 + 2 * NC};
  const int start[4] = {0, ng, ng + nr, ng + nr + nbk};
  std::vector<int32_t> map(ns);
  for (int e = 0; e < ns; ++e) {
    const int r = e < start[1] ? 0 : e < start[2] ? 1 : e < start[3] ? 2 : 3;
    const int i = e - start[r];
    map[e] = (first_slot[r] + i / W) * W + i % W;
  }
  std::vector<int32_t> X((size_t)F.stride, 0);
  for (int i = 0; i < F.NSW; ++i) X[i] = -1;
  for (int e = 0; e < ns; ++e) {
    const int id = map[e];
    X[id] = Dv[off + e];
    X[F.NSW + id] = Dv[off + ns + e];
    for (int q = 0; q < D; ++q) {
      const uint32_t w = (uint32_t)Dv[off + 2 * ns + e * D + q];
      const int lo = (int16_t)(w & 0xffffu), hi = (int16_t)(w >> 16);
      X[2 * F.NSW + id * D + q] = pack16(map[lo], map[hi]);
    }
    if (pc) X[F.PC + id] = Dv[pc_off + e];
    if (rs) {
      X[F.RS + 2 * id] = Dv[rs_off + 2 * e];
      X[F.RS + 2 * id + 1] = Dv[rs_off + 2 * e + 1];
    }
  }
  auto remap = [&](int a) { return a >= ns ? F.NSW + map[a - ns] : map[a]; };
  for (int q2 = 0; q2 < (K + 1) / 2; ++q2)
    for (int j = 0; j < ng; ++j) {
      const uint32_t w = (uint32_t)Dv[gid_off + q2 * ng + j];
      X[F.GID + q2 * W + j] = pack16(remap((int)(w & 0xffffu)), remap((int)(w >> 16)));
    }
  for (int q = 0; q < K; ++q)
    for (int j = 0; j < ng; ++j) {
      if (w32) {
        X[F.GW + q * W + j] = Dv[gw_off + q * ng + j];
      } else {
        X[F.GW + 2 * (q * W + j)] = Dv[gw_off + 2 * (q * ng + j)];
        X[F.GW + 2 * (q * W + j) + 1] = Dv[gw_off + 2 * (q * ng + j) + 1];
      }
    }
  for (int j = 0; j < ng; ++j) {
    X[F.GC + 2 * j] = Dv[gc_off + 2 * j];
    X[F.GC + 2 * j + 1] = Dv[gc_off + 2 * j + 1];
  }
  Dv.resize(off);
  Dv.insert(Dv.end(), X.begin(), X.end());
}

// initial runs of at most own_target consecutive (Morton-ordered) nodes of one problem
std::vector<std::pair<size_t, size_t>> initial_runs(const std::vector<std::pair<uint64_t, int32_t>>& U,
                                                    int own_target) {
  std::vector<std::pair<size_t, size_t>> runs;
  for (size_t a = 0; a < U.size();) {
    const size_t b = std::min(U.size(), a + (size_t)own_target);
    const uint64_t pa = U[a].first >> 60;
    size_t e = a;
    while (e < b && (U[e].first >> 60) == pa) ++e;
    runs.push_back({a, e});
    a = e;
  }
  std::reverse(runs.begin(), runs.end());
  return runs;
}

}  // namespace

// Relaxation chunks of level l.  A relaxation is P = 3 + 3 lambda phases: 0 red interior,
// 1 black interior, 2 ghosts, then for k = 1..lambda phases 3k (red band), 3k + 1 (black
// band), 3k + 2 (ghosts).  The nodes written by the boundary part (band and ghost nodes) are
// split into Morton-ordered runs.  The phases are taken R at a time (one launch each, whole
// sweeps); for every launch each run's node set is closed backwards over the launch's
// phases: a node whose value after phase t is needed, and which phase t updates, needs the
// values after phase t - 1 of every node it reads.  A chunk with more updated ghosts, red or
// black entries or read-only entries than its threads hold is split in two.  Returns false
// when a small run is still too large, when R does not divide the phases or its mask bits do
// not fit, or when the redundant work exceeds max_redundancy times the owned nodes per launch
// (the caller then tries fewer phases per launch, and the level finally relaxes its boundary
// part with one launch per phase).
bool build_band_chunks(mg_handle_s* H, int l, int own_target, double max_redundancy, int Rmax) {
  HostLevel& HL = H->host[l];
  const int D = H->dim, lambda = H->grid.lambda;
  const Geo& g = HL.g;
  const int K = D == 2 ? 9 : 27;
  const int P = 3 + 3 * lambda;
  const size_t nn = HL.cls.size();
  // FP32 cycles read FP32 ghost weights
  const bool w32 = H->grid.precision == MG_FP32_DC;
  // role of a node: 1 red band, 2 black band, 3 ghost, 4 red interior off the band,
  // 5 black interior off the band
  std::vector<int8_t> role(nn, 0);
  std::vector<int32_t> gidx(nn, -1);
  for (size_t v = 0; v < nn; ++v) {
    if (HL.cls[v] != 1) continue;
    int64_t p;
    int j[3];
    node_coords(g, D, (int64_t)v, &p, j);
    const bool black = (j[0] + j[1] + j[2]) & 1;
    role[v] = HL.rcls[v] == 3 ? (black ? 2 : 1) : (black ? 5 : 4);
  }
  for (size_t i = 0; i < HL.ghosts.size(); ++i) {
    role[HL.ghosts[i].node] = 3;
    gidx[HL.ghosts[i].node] = (int32_t)i;
  }
  auto updates = [&](int r, int p) {
    if (p == 0) return r == 1 || r == 4;
    if (p == 1) return r == 2 || r == 5;
    if (p % 3 == 2) return r == 3;
    return p % 3 == 0 ? r == 1 : r == 2;
  };
  auto tap_node = [&](int32_t v, int t) {
    const GhostRec& r = HL.ghosts[gidx[v]];
    return (int32_t)(v + (D == 2 ? template_offset<2>(t, r.s, g.st) : template_offset<3>(t, r.s, g.st)));
  };
  auto reads = [&](int32_t v, std::vector<int32_t>& out) {
    out.clear();
    out.push_back(v);
    if (role[v] == 3) {
      for (int t = 0; t < K; ++t)
        if (HL.gw[(size_t)gidx[v] * K + t] != 0.0) out.push_back(tap_node(v, t));
    } else {
      for (int a = 0; a < D; ++a) {
        out.push_back((int32_t)(v - g.st[a]));
        out.push_back((int32_t)(v + g.st[a]));
      }
    }
  };
  std::vector<std::pair<uint64_t, int32_t>> U;
  for (size_t v = 0; v < nn; ++v)
    if (role[v] >= 1 && role[v] <= 3) U.push_back({morton_key(g, D, (int64_t)v), (int32_t)v});
  std::sort(U.begin(), U.end());
  const double cNh = H->grid.cN * g.h;
  // the scratch marks of a closure are indexed by a compact id over the interior and ghost
  // nodes (the only nodes a closure reaches); every run restores the marks it set, so a
  // thread's marks serve every attempt below
  const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const std::vector<std::pair<size_t, size_t>> runs0 = initial_runs(U, own_target);
  std::vector<int32_t> cid(nn, -1);
  int32_t ncid = 0;
  for (size_t v = 0; v < nn; ++v)
    if (role[v] != 0) cid[v] = ncid++;
  struct Scratch {
    std::vector<int16_t> need;
    std::vector<int32_t> lid;
    std::vector<char> owned;
  };
  std::vector<Scratch> pool;
  // every launch's chunk set (phases [p0, p0 + R)) is built on threads of its own, into its
  // own arrays, then appended in launch order with its offsets moved: the data is that of a
  // sequential build
  struct RangeOut {
    std::vector<int32_t> hdr, data;
    int nchunks = 0, smax = 0, stride = 0;
    int64_t entries = 0, nown = 0;
    bool ok = true;
  };
  // one attempt: launches of R phases each (whole sweeps); mask bits: R phases, then D + 2^D
  // interpolation bits, bit 30 band or ghost node, bit 31 owned
  auto attempt = [&](int R) -> bool {
  HL.bc_hdr.clear();
  HL.bc_data.clear();
  HL.bc_nchunks = 0;
  HL.bc_smax = 0;
  HL.bc_stride = 0;
  HL.bc_entries = 0;
  HL.bc_nown = 0;
  HL.bc_range = R;
  HL.bc_sub.assign(1, 0);
  const int S = P / R;
  // within a launch, its initial owned runs split in NG groups, one thread each
  const int NG = std::max(1, std::min(hw / S, (int)(runs0.size() / 64)));
  if (pool.size() < (size_t)S * NG) pool.resize((size_t)S * NG);
  std::vector<RangeOut> outs((size_t)S * NG);
  // a failed group ends the others early (the build fails as a whole)
  std::atomic<bool> failed{false};
  auto build_group = [&](int r, int grp) {
  RangeOut& O = outs[(size_t)r * NG + grp];
  const int p0 = r * R, p1 = p0 + R;
  Scratch& sc = pool[(size_t)r * NG + grp];
  if (sc.need.empty()) {
    sc.need.assign(ncid, -2);
    sc.lid.assign(ncid, -1);
    sc.owned.assign(ncid, 0);
  }
  std::vector<int16_t>& need = sc.need;
  std::vector<int32_t>& lid = sc.lid;
  std::vector<char>& owned = sc.owned;
  std::vector<int32_t> touched, rd;
  std::vector<int64_t> keyed;
  // this group's initial runs, processed from the last as the sequential build does
  const size_t g0 = runs0.size() * grp / NG, g1 = runs0.size() * (grp + 1) / NG;
  std::vector<std::pair<size_t, size_t>> pending(runs0.begin() + g0, runs0.begin() + g1);
  while (!pending.empty()) {
    if (failed.load(std::memory_order_relaxed)) {
      O.ok = false;
      return;
    }
    const auto [a, b] = pending.back();
    pending.pop_back();
    touched.clear();
    for (size_t i = a; i < b; ++i) {
      need[cid[U[i].second]] = (int16_t)(p1 - 1);
      owned[cid[U[i].second]] = 1;
      touched.push_back(U[i].second);
    }
    // a closure with more entries than a chunk holds cannot fit (the slot checks below would
    // reject it): it stops growing there and the run is split at once
    bool over = false;
    for (int p = p1 - 1; p >= p0 && !over; --p) {
      const size_t nt = touched.size();
      for (size_t i = 0; i < nt && !over; ++i) {
        const int32_t v = touched[i];
        if (!updates(role[v], p) || need[cid[v]] < p) continue;
        reads(v, rd);
        for (int32_t w : rd) {
          if (need[cid[w]] == -2) touched.push_back(w);
          if (need[cid[w]] < p - 1) need[cid[w]] = (int16_t)(p - 1);
        }
        over = touched.size() > (size_t)band_max_entries(D);
      }
    }
    if (over) {
      for (int32_t v : touched) {
        need[cid[v]] = -2;
        owned[cid[v]] = 0;
      }
      if (b - a <= 16) {
        O.ok = false;
        failed = true;
        return;
      }
      const size_t m = a + (b - a) / 2;
      pending.push_back({m, b});
      pending.push_back({a, m});
      continue;
    }
    // entries: the updated ghosts, the red-updated, the black-updated, the read-only nodes;
    // each run by node index
    auto run_of = [&](int32_t v) {
      for (int p = p0; p < p1; ++p)
        if (updates(role[v], p) && need[cid[v]] >= p) return p % 3 == 2 ? 0 : (p % 3 == 0 ? 1 : 2);
      return 3;
    };
    // (run, node) keys, each run computed once
    keyed.clear();
    for (int32_t v : touched) keyed.push_back(((int64_t)run_of(v) << 32) | (uint32_t)v);
    std::sort(keyed.begin(), keyed.end());
    const int ns = (int)touched.size();
    int cnt[4] = {0, 0, 0, 0};
    for (int i = 0; i < ns; ++i) {
      touched[i] = (int32_t)(keyed[i] & 0xffffffff);
      ++cnt[keyed[i] >> 32];
    }
    const int ng = cnt[0], nr = cnt[1], nbk = cnt[2];
    const int W = band_chunk_threads(D);
    bool ok = ng <= W && nr <= band_colour_slots(D) * W && nbk <= band_colour_slots(D) * W &&
              cnt[3] <= band_halo_slots(D) * W;
    for (int i = ns - cnt[3]; i < ns; ++i)
      if (owned[cid[touched[i]]]) ok = false;  // an owned node is always updated
    if (ok) {
      for (int i = 0; i < ns; ++i) lid[cid[touched[i]]] = i;
      for (int i = 0; i < ns - cnt[3] && ok; ++i) {
        const int32_t v = touched[i];
        if (role[v] == 3) continue;
        for (int a2 = 0; a2 < D; ++a2)
          if (lid[cid[v - g.st[a2]]] < 0 || lid[cid[v + g.st[a2]]] < 0) ok = false;
      }
      for (int j = 0; j < ng && ok; ++j)
        for (int t = 0; t < K; ++t)
          if (HL.gw[(size_t)gidx[touched[j]] * K + t] != 0.0 && lid[cid[tap_node(touched[j], t)]] < 0) ok = false;
    }
    if (!ok) {
      for (int32_t v : touched) {
        need[cid[v]] = -2;
        lid[cid[v]] = -1;
        owned[cid[v]] = 0;
      }
      if (b - a <= 16) {
        O.ok = false;
        failed = true;
        return;
      }
      const size_t m = a + (b - a) / 2;
      pending.push_back({m, b});
      pending.push_back({a, m});
      continue;
    }
    // per-chunk data: node, phase mask (bit 31: owned), interior neighbour pairs, ghost
    // stencil ids and weights (transposed: tap-major), ghost constants
    std::vector<int32_t>& Dv = O.data;
    pad_even(Dv);
    const int32_t off = (int32_t)Dv.size();
    for (int32_t v : touched) Dv.push_back(v);
    for (int32_t v : touched) {
      uint32_t m = owned[cid[v]] ? 0x80000000u : 0u;
      if (role[v] >= 1 && role[v] <= 3) m |= 0x40000000u;
      for (int p = p0; p < p1; ++p)
        if (updates(role[v], p) && need[cid[v]] >= p) m |= 1u << (p - p0);
      Dv.push_back((int32_t)m);
    }
    for (int32_t v : touched)
      for (int a2 = 0; a2 < D; ++a2) {
        const bool relaxed = role[v] != 3 && role[v] != 0;
        const int lo = relaxed && lid[cid[v - g.st[a2]]] >= 0 ? lid[cid[v - g.st[a2]]] : 0;
        const int hi = relaxed && lid[cid[v + g.st[a2]]] >= 0 ? lid[cid[v + g.st[a2]]] : 0;
        Dv.push_back(pack16(lo, hi));
      }
    // interpolation candidates of every entry (Sec. 2.6.1): one word, the coarse node index
    // of candidate 0 (candidate m adds the coarse stride of every axis q with bit q of m);
    // mask bits [P, P + D): the odd coordinates (weight 2^-count), bits [P + D, P + D + 2^D):
    // candidate m exists and carries an unknown
    const int32_t pc_off = (int32_t)Dv.size();
    if (l < H->L) {
      const HostLevel& HC = H->host[l + 1];
      const int NC = 1 << D;
      for (int i = 0; i < ns; ++i) {
        int64_t p;
        int j[3];
        node_coords(g, D, touched[i], &p, j);
        uint32_t bits = 0;
        int jb[3] = {0, 0, 0};
        for (int q = 0; q < D; ++q) {
          if (j[q] & 1) bits |= 1u << q;
          jb[q] = (j[q] & 1) ? (j[q] - 1) >> 1 : j[q] >> 1;
        }
        for (int m = 0; m < NC; ++m) {
          bool exists = true;
          int jc[3] = {jb[0], jb[1], jb[2]};
          for (int q = 0; q < D; ++q) {
            const int bit = (m >> q) & 1;
            if (bit && (j[q] & 1) == 0) exists = false;
            jc[q] += bit;
          }
          if (exists && HC.cls[p * HC.g.npp + jc[0] + HC.g.st[1] * jc[1] + HC.g.st[2] * jc[2]] != 0)
            bits |= 1u << (D + m);
        }
        Dv[off + ns + i] |= (int32_t)(bits << R);
        Dv.push_back((int32_t)(p * HC.g.npp + jb[0] + HC.g.st[1] * jb[1] + HC.g.st[2] * jb[2]));
      }
    }
    // ghost rows: the LDS address each tap reads, two taps per word (tap pair major, ghost
    // fastest): a tap on a ghost entry (local id below ng) reads that ghost's value before the
    // ghost phase, kept at ns + id; any other tap reads the entry's current value at its id;
    // taps of zero weight name the ghost's own earlier value
    const int32_t gid_off = (int32_t)Dv.size();
    auto tap_addr = [&](int j, int t) {
      if (t >= K) return 0;
      const double w = HL.gw[(size_t)gidx[touched[j]] * K + t];
      const int id = w != 0.0 ? lid[cid[tap_node(touched[j], t)]] : j;
      return id < ng ? ns + id : id;
    };
    for (int t = 0; t < K; t += 2)
      for (int j = 0; j < ng; ++j) Dv.push_back(pack16(tap_addr(j, t), tap_addr(j, t + 1)));
    pad_even(Dv);
    // the weights in the precision of the cycles that read them
    const int32_t gw_off = (int32_t)Dv.size();
    std::vector<double> wv;
    for (int t = 0; t < K; ++t)
      for (int j = 0; j < ng; ++j) wv.push_back(HL.gw[(size_t)gidx[touched[j]] * K + t]);
    if (w32) {
      for (double w : wv) {
        const float f = (float)w;
        int32_t bits;
        std::memcpy(&bits, &f, sizeof bits);
        Dv.push_back(bits);
      }
      pad_even(Dv);
    } else {
      put_doubles(Dv, wv);
    }
    const int32_t gc_off = (int32_t)Dv.size();
    wv.clear();
    for (int j = 0; j < ng; ++j) wv.push_back(HL.ghosts[gidx[touched[j]]].type ? H->grid.cD : cNh);
    put_doubles(Dv, wv);
    // restriction data of every entry (levels fed by a finer level): the fine node index
    // of (2x, 2y, 2z) and the node's restriction code
    const int32_t rs_off = (int32_t)Dv.size();
    if (l > 0) {
      const HostLevel& HF = H->host[l - 1];
      for (int i = 0; i < ns; ++i) {
        int64_t p;
        int j[3];
        node_coords(g, D, touched[i], &p, j);
        Dv.push_back((int32_t)(p * HF.g.npp + 2 * j[0] + HF.g.st[1] * 2 * j[1] + HF.g.st[2] * 2 * j[2]));
        Dv.push_back((int32_t)HL.rcode[touched[i]]);
      }
    }
    const uint32_t counts = (uint32_t)ng | ((uint32_t)nr << 10) | ((uint32_t)nbk << 21);
    if (band_fixed_layout(D)) {
      // the header keeps the counts; the data sits at chunk * bc_stride
      const BandFixed F = band_fixed(D, l < H->L, l > 0);
      to_fixed_layout(Dv, off, D, ns, ng, nr, nbk, gid_off, gw_off, gc_off, pc_off, rs_off,
                      l < H->L, l > 0, w32);
      O.stride = F.stride;
      const int32_t hdr[kBandHdr] = {F.NSW, (int32_t)counts, off, off + F.GID, off + F.GW,
                                     off + F.GC, l < H->L ? off + F.PC : -1, l > 0 ? off + F.RS : -1};
      O.hdr.insert(O.hdr.end(), hdr, hdr + kBandHdr);
      O.smax = F.NSW;
    } else {
      const int32_t hdr[kBandHdr] = {ns, (int32_t)counts, off, gid_off, gw_off, gc_off,
                                     l < H->L ? pc_off : -1, l > 0 ? rs_off : -1};
      O.hdr.insert(O.hdr.end(), hdr, hdr + kBandHdr);
      O.smax = std::max(O.smax, ns);
    }
    ++O.nchunks;
    O.entries += ns;
    O.nown += (int64_t)(b - a);
    for (int32_t v : touched) {
      need[cid[v]] = -2;
      lid[cid[v]] = -1;
      owned[cid[v]] = 0;
    }
    // over the whole redundancy budget already: the build fails (early exit; the marks are
    // restored, so the thread's scratch serves the next attempt)
    if ((double)O.entries > max_redundancy * (double)S * (double)U.size()) {
      O.ok = false;
      failed = true;
      return;
    }
  }
  };
  if (S * NG == 1) {
    build_group(0, 0);
  } else {
    std::vector<std::thread> th;
    for (int r = 0; r < S; ++r)
      for (int grp = 0; grp < NG; ++grp) th.emplace_back(build_group, r, grp);
    for (auto& t : th) t.join();
  }
  for (const RangeOut& O : outs)
    if (!O.ok) return false;
  // launch by launch; within a launch the groups from the last (the sequential order)
  for (int r = 0; r < S; ++r) {
  for (int grp = NG - 1; grp >= 0; --grp) {
    const RangeOut& O = outs[(size_t)r * NG + grp];
    pad_even(HL.bc_data);
    const int32_t base = (int32_t)HL.bc_data.size();
    HL.bc_data.insert(HL.bc_data.end(), O.data.begin(), O.data.end());
    // header words 2.. are offsets into the data (-1: absent)
    for (int c = 0; c < O.nchunks; ++c)
      for (int q = 0; q < kBandHdr; ++q) {
        const int32_t v = O.hdr[(size_t)c * kBandHdr + q];
        HL.bc_hdr.push_back(q >= 2 && v >= 0 ? v + base : v);
      }
    HL.bc_nchunks += O.nchunks;
    HL.bc_entries += O.entries;
    HL.bc_nown += (int)O.nown;
    HL.bc_smax = std::max(HL.bc_smax, O.smax);
    if (O.stride) HL.bc_stride = O.stride;
  }
  HL.bc_sub.push_back(HL.bc_nchunks);
  }
  if (!U.empty() && (double)HL.bc_entries > max_redundancy * (double)S * (double)U.size())
    return false;
  return true;
  };
  // the largest number of phases per launch (whole sweeps dividing the relaxation's phases,
  // at most 7 launches) whose chunks fit
  for (int R = std::min(Rmax, P); R >= 3; R -= 3)
    if (P % R == 0 && P / R <= 7 && R + D + (1 << D) <= 30 && attempt(R)) return true;
  HL.bc_hdr.clear();
  HL.bc_data.clear();
  HL.bc_sub.clear();
  HL.bc_nchunks = 0;
  return false;
}

// Composed extension weights of level l.  The records are stored in DAG order per problem,
// so every source that is an extension node has its weights already: a record's weights are
// those of its sources, each scaled by its normalised upwind weight wt_a / sum(wt), merged by
// ghost node (ascending).  A record without sources has no terms (its value is 0).
void compose_extension(const HostLevel& HL, const std::vector<int32_t>& eid,
                       std::vector<int32_t>& off, std::vector<int32_t>& src,
                       std::vector<double>& wt) {
  const size_t ne = HL.ext.size();
  off.assign(ne + 1, 0);
  src.clear();
  wt.clear();
  std::vector<std::pair<int32_t, double>> m;
  for (size_t i = 0; i < ne; ++i) {
    const ExtRec& r = HL.ext[i];
    double den = 0.0;
    for (int a = 0; a < 3; ++a)
      if (r.src[a] >= 0) den += r.wt[a];
    m.clear();
    for (int a = 0; a < 3 && den > 0.0; ++a) {
      const int32_t q = r.src[a];
      if (q < 0) continue;
      const double f = r.wt[a] / den;
      if (eid[q] < 0) {
        m.push_back({q, f});
        continue;
      }
      const int32_t j = eid[q];
      for (int32_t t = off[j]; t < off[j + 1]; ++t) m.push_back({src[t], f * wt[t]});
    }
    std::stable_sort(m.begin(), m.end(),
                     [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                       return x.first < y.first;
                     });
    for (size_t k = 0; k < m.size(); ++k) {
      if (k > 0 && m[k].first == m[k - 1].first) {
        wt.back() += m[k].second;
      } else {
        src.push_back(m[k].first);
        wt.push_back(m[k].second);
      }
    }
    off[i + 1] = (int32_t)src.size();
  }
}

// Composed extension terms of level l as flat arrays, for a gather launch after the defect
// (which also stores the ghost defects by ghost id in a compact array): per extension record
// its node and term range, per term the ghost's index in the level's ghost list and the
// weight.  Returns false when a source is neither extension node nor ghost.
bool build_ext_terms(mg_handle_s* H, int l) {
  HostLevel& HL = H->host[l];
  HL.et_node.clear();
  HL.et_off.clear();
  HL.et_src.clear();
  HL.et_wt.clear();
  if (HL.ext.empty()) return true;
  const size_t nn = HL.cls.size();
  std::vector<int32_t> eid(nn, -1), gidx(nn, -1);
  for (size_t i = 0; i < HL.ext.size(); ++i) eid[HL.ext[i].node] = (int32_t)i;
  for (size_t i = 0; i < HL.ghosts.size(); ++i) gidx[HL.ghosts[i].node] = (int32_t)i;
  for (const ExtRec& r : HL.ext)
    for (int a = 0; a < 3; ++a)
      if (r.src[a] >= 0 && eid[r.src[a]] < 0 && gidx[r.src[a]] < 0) return false;
  compose_extension(HL, eid, HL.et_off, HL.et_src, HL.et_wt);
  for (int32_t& q : HL.et_src) q = gidx[q];
  for (const ExtRec& r : HL.ext) HL.et_node.push_back(r.node);
  return true;
}

// Extension chunks of level l: each chunk owns a Morton-ordered run of extension nodes and
// the ghost nodes their composed weights name.  A chunk with more than kExtMaxEntries
// extension nodes, kExtMaxGhosts ghost sources or kExtMaxTerms terms is split in two;
// returns false when a single node is still too large, or a source is neither extension
// node nor ghost.
bool build_ext_chunks(mg_handle_s* H, int l, int own_target) {
  HostLevel& HL = H->host[l];
  const int D = H->dim;
  const Geo& g = HL.g;
  const int K = D == 2 ? 9 : 27;
  HL.ec_hdr.clear();
  HL.ec_data.clear();
  HL.ec_nchunks = 0;
  HL.ec_smax = 0;
  HL.ec_stride = 0;
  if (HL.ext.empty()) return true;
  const size_t nn = HL.cls.size();
  std::vector<int32_t> eid(nn, -1), gidx(nn, -1);
  for (size_t i = 0; i < HL.ext.size(); ++i) eid[HL.ext[i].node] = (int32_t)i;
  for (size_t i = 0; i < HL.ghosts.size(); ++i) gidx[HL.ghosts[i].node] = (int32_t)i;
  for (const ExtRec& r : HL.ext)
    for (int a = 0; a < 3; ++a)
      if (r.src[a] >= 0 && eid[r.src[a]] < 0 && gidx[r.src[a]] < 0) return false;
  std::vector<int32_t> toff, tsrc;
  std::vector<double> twt;
  compose_extension(HL, eid, toff, tsrc, twt);
  std::vector<std::pair<uint64_t, int32_t>> U;
  for (size_t i = 0; i < HL.ext.size(); ++i)
    U.push_back({morton_key(g, D, HL.ext[i].node), (int32_t)i});
  std::sort(U.begin(), U.end());
  std::vector<std::pair<size_t, size_t>> pending = initial_runs(U, own_target);
  std::vector<int32_t> lid(nn, -1);
  while (!pending.empty()) {
    const auto [a, b] = pending.back();
    pending.pop_back();
    std::vector<int32_t> ghosts_e;
    for (size_t i = a; i < b; ++i) {
      const int32_t e = U[i].second;
      for (int32_t t = toff[e]; t < toff[e + 1]; ++t)
        if (lid[tsrc[t]] == -1) {
          lid[tsrc[t]] = -2;
          ghosts_e.push_back(tsrc[t]);
        }
    }
    const int ne = (int)(b - a), ngs = (int)ghosts_e.size();
    int64_t nt = 0;
    for (size_t i = a; i < b; ++i) nt += toff[U[i].second + 1] - toff[U[i].second];
    if (ne > kExtMaxEntries || ngs > kExtMaxGhosts || nt > kExtMaxTerms) {
      for (int32_t q : ghosts_e) lid[q] = -1;
      if (b - a <= 1) return false;
      const size_t m = a + (b - a) / 2;
      pending.push_back({m, b});
      pending.push_back({a, m});
      continue;
    }
    int k = 0;
    for (int32_t q : ghosts_e) lid[q] = k++;
    std::vector<int32_t>& Dv = HL.ec_data;
    pad_even(Dv);
    const int32_t off = (int32_t)Dv.size();
    for (int32_t q : ghosts_e) Dv.push_back(q);
    for (size_t i = a; i < b; ++i) Dv.push_back(HL.ext[U[i].second].node);
    const int32_t to_off = (int32_t)Dv.size();
    int32_t nterms = 0;
    for (size_t i = a; i < b; ++i) {
      Dv.push_back(nterms);
      nterms += toff[U[i].second + 1] - toff[U[i].second];
    }
    Dv.push_back(nterms);
    const int32_t ts_off = (int32_t)Dv.size();
    std::vector<double> wv;
    for (size_t i = a; i < b; ++i)
      for (int32_t t = toff[U[i].second]; t < toff[U[i].second + 1]; ++t) {
        Dv.push_back(lid[tsrc[t]]);
        wv.push_back(twt[t]);
      }
    pad_even(Dv);
    const int32_t tw_off = (int32_t)Dv.size();
    put_doubles(Dv, wv);
    const int32_t gn_off = (int32_t)Dv.size();
    for (int t = 0; t < K; ++t)
      for (int32_t q : ghosts_e) {
        // taps of zero weight name the ghost itself
        const GhostRec& r = HL.ghosts[gidx[q]];
        const bool used = HL.gw[(size_t)gidx[q] * K + t] != 0.0;
        const int64_t o = D == 2 ? template_offset<2>(t, r.s, g.st) : template_offset<3>(t, r.s, g.st);
        Dv.push_back(used ? (int32_t)(q + o) : q);
      }
    pad_even(Dv);
    const int32_t gw_off = (int32_t)Dv.size();
    wv.clear();
    for (int t = 0; t < K; ++t)
      for (int32_t q : ghosts_e) wv.push_back(HL.gw[(size_t)gidx[q] * K + t]);
    put_doubles(Dv, wv);
    // rewritten in the fixed layout (ext_fixed): the same arrays at fixed offsets, padded
    {
      const ExtFixed F = ext_fixed(D);
      const int GS = kExtMaxGhosts, NE = kExtMaxEntries;
      std::vector<int32_t> X((size_t)F.stride, 0);
      for (int j = 0; j < ngs; ++j) X[j] = Dv[off + j];
      for (int e = 0; e < ne; ++e) X[GS + e] = Dv[off + ngs + e];
      for (int e = 0; e <= NE; ++e) X[F.TO + e] = Dv[to_off + (e < ne ? e : ne)];
      for (int t = 0; t < nterms; ++t) {
        X[F.TS + t] = Dv[ts_off + t];
        X[F.TW + 2 * t] = Dv[tw_off + 2 * t];
        X[F.TW + 2 * t + 1] = Dv[tw_off + 2 * t + 1];
      }
      for (int t = 0; t < K; ++t)
        for (int j = 0; j < ngs; ++j) {
          X[F.GN + t * GS + j] = Dv[gn_off + t * ngs + j];
          X[F.GW + 2 * (t * GS + j)] = Dv[gw_off + 2 * (t * ngs + j)];
          X[F.GW + 2 * (t * GS + j) + 1] = Dv[gw_off + 2 * (t * ngs + j) + 1];
        }
      Dv.resize(off);
      Dv.insert(Dv.end(), X.begin(), X.end());
      HL.ec_stride = F.stride;
    }
    const ExtFixed F = ext_fixed(D);
    const int32_t hdr[kExtHdr] = {ne, ngs, off, off + F.TO, off + F.TS, off + F.TW, off + F.GN, off + F.GW};
    HL.ec_hdr.insert(HL.ec_hdr.end(), hdr, hdr + kExtHdr);
    ++HL.ec_nchunks;
    HL.ec_smax = std::max(HL.ec_smax, ngs + nterms + (nterms + 1) / 2);
    for (int32_t q : ghosts_e) lid[q] = -1;
  }
  return true;
}

}  // namespace ghostmg
