// Host-side setup of the preconditioner (Sec. 3, Sec. 4.1 components 2-4):
// diagonal and V_e blocks of the DG matrix, labels V_J / N, the spaces V_e,
// the conforming prolongation P and the low-order-refined matrix A~ P.
#include <algorithm>
#include <array>
#include <cmath>
#include <exception>
#include <map>
#include <numeric>

#include "internal.hpp"

namespace hpdg {

// ------------------------------------------------------------ penalties
double br2_eta(const Mesh& M, const OpOpts& o) {
  if (o.eta > 0) return o.eta;
  std::vector<int> cnt(M.ne, 0);
  for (const Face& f : M.faces) {
    cnt[f.em]++;
    if (f.ep >= 0) cnt[f.ep]++;
  }
  return 1.0 + *std::max_element(cnt.begin(), cnt.end());
}

static double pi_rule(int p, int rule) { return rule == 0 ? (p + 1.0) * (p + 1.0) : (double)p * p; }

// SIPG: sigma = eta k_e pi(p_e) / h_e (Sec. 2), p_e max, h_e min, k_e max.
// BR2: eta_br2 * k_e (the factor in front of the lifting term, Sec. 4.4).
double penalty_or_br2(const Mesh& M, const OpOpts& o, const Face& f, double eta_br2) {
  int pe;
  double he, ke;
  if (f.ep < 0) { pe = M.p[f.em]; he = M.h[f.em]; ke = M.k[f.em]; }
  else {
    pe = std::max(M.p[f.em], M.p[f.ep]);
    he = std::min(M.h[f.em], M.h[f.ep]);
    ke = std::max(M.k[f.em], M.k[f.ep]);
  }
  if (o.form == 1) return eta_br2 * ke;
  return o.eta * ke * pi_rule(pe, o.penalty_rule) / he;
}

// ------------------------------------------------- face quadrature helpers
struct FaceSide {
  int e, s;          // element and which of its sides (0 lower, 1 upper)
  double js;         // sign of its trace in [[u]].e_m
  double ca;         // weight in the average {k du/dx_m}
  int n;             // p+1
  // per tangential dim j: Lt[j][g*n + i] Lagrange values at the face points
  std::vector<double> Lt[2];
};

struct FaceQuad {
  int m, nt, q;
  int tdim[2];
  std::vector<double> wt[2];   // per tangential dim: weights * length / N
  std::vector<FaceSide> sides;
};

static FaceQuad face_quad(const Mesh& M, const Face& f) {
  FaceQuad Q;
  Q.m = f.m;
  Q.nt = 0;
  for (int t = 0; t < M.dim; ++t)
    if (t != f.m) Q.tdim[Q.nt++] = t;
  int pm = M.p[f.em];
  if (f.ep >= 0) pm = std::max(pm, M.p[f.ep]);
  Q.q = pm + 1;
  std::vector<double> gx, gw;
  gauss_rule(Q.q, gx, gw);
  for (int j = 0; j < Q.nt; ++j) {
    int t = Q.tdim[j];
    Q.wt[j].resize(Q.q);
    for (int g = 0; g < Q.q; ++g) Q.wt[j][g] = gw[g] * (double)(f.hi[t] - f.lo[t]) / (double)M.N;
  }
  auto add_side = [&](int e, int s, double js, double ca) {
    FaceSide S;
    S.e = e; S.s = s; S.js = js; S.ca = ca; S.n = M.p[e] + 1;
    const Basis1D& B = basis(M.p[e]);
    for (int j = 0; j < Q.nt; ++j) {
      int t = Q.tdim[j];
      S.Lt[j].resize(Q.q * S.n);
      for (int g = 0; g < Q.q; ++g) {
        double x = (double)f.lo[t] + (double)(f.hi[t] - f.lo[t]) * gx[g];
        double r = (x - (double)M.lo[3 * e + t]) / (double)M.sz[e];
        lagrange_eval(B.x, r, &S.Lt[j][g * S.n]);
      }
    }
    Q.sides.push_back(std::move(S));
  };
  if (f.ep >= 0) {
    add_side(f.em, 1, 1.0, 0.5);
    add_side(f.ep, 0, -1.0, 0.5);
  } else {
    add_side(f.em, f.side, f.side ? 1.0 : -1.0, 1.0);
  }
  return Q;
}

static inline void multi_index(int64_t r, int n, int dim, int* i) {
  for (int m = 0; m < dim; ++m) { i[m] = (int)(r % n); r /= n; }
}

// ------------------------------------------------------------- diagonal
std::vector<double> dg_diagonal(const Mesh& M, const OpOpts& o) {
  std::vector<double> diag(M.ndof, 0.0);
  int d = M.dim;
  for (int e = 0; e < M.ne; ++e) {
    const Basis1D& B = basis(M.p[e]);
    int n = M.p[e] + 1;
    double sc = M.k[e] * std::pow(M.h[e], d - 2);
    int64_t nd = M.off[e + 1] - M.off[e];
    for (int64_t r = 0; r < nd; ++r) {
      int i[3];
      multi_index(r, n, d, i);
      double s = 0;
      for (int m = 0; m < d; ++m) {
        double t = 1;
        for (int j = 0; j < d; ++j) t *= (j == m ? B.K : B.M)[i[j] * n + i[j]];
        s += t;
      }
      diag[M.off[e] + r] += sc * s;
    }
  }
  double eta2 = o.form == 1 ? br2_eta(M, o) : 0.0;
  for (const Face& f : M.faces) {
    FaceQuad Q = face_quad(M, f);
    double sig = penalty_or_br2(M, o, f, eta2);
    double c2 = f.ep >= 0 ? 0.25 : 1.0;
    for (const FaceSide& A : Q.sides) {
      const Basis1D& Ba = basis(M.p[A.e]);
      int n = A.n;
      int sidx = A.s ? n - 1 : 0;
      double dsd = (A.s ? Ba.D1 : Ba.D0)[sidx] / M.h[A.e];
      // 1D factors per tangential dim and per node index
      std::vector<double> Af[2];
      std::vector<double> Qk[2][2];
      for (int j = 0; j < Q.nt; ++j) {
        Af[j].assign(n, 0.0);
        for (int i = 0; i < n; ++i)
          for (int g = 0; g < Q.q; ++g) Af[j][i] += Q.wt[j][g] * A.Lt[j][g * n + i] * A.Lt[j][g * n + i];
        if (o.form == 1) {
          for (size_t kk = 0; kk < Q.sides.size(); ++kk) {
            const FaceSide& K = Q.sides[kk];
            const Basis1D& Bk = basis(M.p[K.e]);
            int nk = K.n;
            // S[r][i] = sum_g w L^K_r L^A_i ; Q(i) = S[:,i]^T Minv_K S[:,i]
            Qk[kk][j].assign(n, 0.0);
            std::vector<double> S(nk * n, 0.0);
            for (int r = 0; r < nk; ++r)
              for (int i = 0; i < n; ++i)
                for (int g = 0; g < Q.q; ++g) S[r * n + i] += Q.wt[j][g] * K.Lt[j][g * nk + r] * A.Lt[j][g * n + i];
            for (int i = 0; i < n; ++i) {
              double acc = 0;
              for (int r = 0; r < nk; ++r)
                for (int r2 = 0; r2 < nk; ++r2) acc += S[r * n + i] * Bk.Minv[r * nk + r2] * S[r2 * n + i];
              Qk[kk][j][i] = acc;
            }
          }
        }
      }
      double ka = M.k[A.e];
      int64_t nd = M.off[A.e + 1] - M.off[A.e];
      for (int64_t r = 0; r < nd; ++r) {
        int i[3];
        multi_index(r, n, d, i);
        if (i[Q.m] != sidx) continue;
        double P = 1.0;
        for (int j = 0; j < Q.nt; ++j) P *= Af[j][i[Q.tdim[j]]];
        double v = -2.0 * A.js * A.ca * ka * dsd * P;
        if (o.form == 0) v += sig * P;
        else {
          for (size_t kk = 0; kk < Q.sides.size(); ++kk) {
            const FaceSide& K = Q.sides[kk];
            const Basis1D& Bk = basis(M.p[K.e]);
            int sk = K.s ? K.n - 1 : 0;
            double mk = Bk.Minv[sk * K.n + sk] * std::pow(M.h[K.e], -d);
            double t = 1.0;
            for (int j = 0; j < Q.nt; ++j) t *= Qk[kk][j][i[Q.tdim[j]]];
            v += c2 * sig * mk * t;
          }
        }
        diag[M.off[A.e] + r] += v;
      }
    }
  }
  return diag;
}

// ------------------------------------------------------ dense sub-blocks
std::vector<double> dg_submatrix(const Mesh& M, const OpOpts& o, const std::vector<int64_t>& dofs,
                                 double eta2) {
  int d = M.dim;
  size_t nb = dofs.size();
  std::vector<double> S(nb * nb, 0.0);
  std::map<int, std::vector<std::pair<int, int>>> by_elem;   // elem -> (local r, block pos)
  for (size_t a = 0; a < nb; ++a) {
    int e = (int)(std::upper_bound(M.off.begin(), M.off.end(), dofs[a]) - M.off.begin()) - 1;
    by_elem[e].push_back({(int)(dofs[a] - M.off[e]), (int)a});
  }
  for (auto& [e, lst] : by_elem) {
    const Basis1D& B = basis(M.p[e]);
    int n = M.p[e] + 1;
    double sc = M.k[e] * std::pow(M.h[e], d - 2);
    for (auto [ri, ai] : lst)
      for (auto [rj, aj] : lst) {
        int i[3], j[3];
        multi_index(ri, n, d, i);
        multi_index(rj, n, d, j);
        double s = 0;
        for (int m = 0; m < d; ++m) {
          double t = 1;
          for (int l = 0; l < d; ++l) t *= (l == m ? B.K : B.M)[i[l] * n + j[l]];
          s += t;
        }
        S[ai * nb + aj] += sc * s;
      }
  }
  // the faces of the block's elements, each once
  std::vector<int> fl;
  for (auto& kv : by_elem)
    for (int q = M.ef_ptr[kv.first]; q < M.ef_ptr[kv.first + 1]; ++q) fl.push_back(M.ef_idx[q]);
  std::sort(fl.begin(), fl.end());
  fl.erase(std::unique(fl.begin(), fl.end()), fl.end());
  // Face terms. Every integrand is a product over the tangential dimensions
  // (traces and normal derivatives of tensor-product GL functions on a face
  // box), so each face integral is a product of 1D integrals: with the 1D
  // face-mass factors C_j^{XY}[i, i'] = sum_g w_j(g) l^X_i(x_g) l^Y_i'(x_g) of
  // the face's sides X, Y in tangential dimension j,
  //   int [[phi_a]] {k d phi_b / dn} = js_a [a on f] (D_sb(i^b_m) k_b ca_b / h_b) prod_j C_j^{ab}
  //   int [[phi_a]] [[phi_b]]        = js_a js_b [a, b on f] prod_j C_j^{ab}
  //   BR2 lifting through side K     = mk_K js_a js_b [a, b on f] prod_j (C_j^{Ka}' Minv_K C_j^{Kb})
  // (exact: the 1D rules have max(p-, p+) + 1 points), so every block entry
  // costs O(1) once the small factor matrices of the face are formed.
  for (int fi : fl) {
    const Face& f = M.faces[fi];
    FaceQuad Q = face_quad(M, f);
    const int ns = (int)Q.sides.size();
    // block DOFs on each side's element: (block position, multi-index)
    struct Col { int a; int i[3]; };
    std::vector<Col> cols[2];
    bool any = false, anyon = false;
    for (int x = 0; x < ns; ++x) {
      const FaceSide& A = Q.sides[x];
      auto it = by_elem.find(A.e);
      if (it == by_elem.end()) continue;
      const int sidx = A.s ? A.n - 1 : 0;
      for (auto [r, a] : it->second) {
        Col c;
        c.a = a;
        multi_index(r, A.n, d, c.i);
        cols[x].push_back(c);
        any = true;
        anyon |= c.i[Q.m] == sidx;
      }
    }
    // the jump of a column vanishes unless its node lies on the face, so a
    // face without such columns adds nothing
    if (!any || !anyon) continue;
    const double sig = penalty_or_br2(M, o, f, eta2);
    // C[x][y][j]: n_x x n_y
    std::vector<double> C[2][2][2];
    for (int x = 0; x < ns; ++x)
      for (int y = 0; y < ns; ++y)
        for (int j = 0; j < Q.nt; ++j) {
          const int nx = Q.sides[x].n, ny = Q.sides[y].n;
          std::vector<double>& c = C[x][y][j];
          c.assign((size_t)nx * ny, 0.0);
          for (int g = 0; g < Q.q; ++g) {
            const double w = Q.wt[j][g];
            const double* lx = &Q.sides[x].Lt[j][g * nx];
            const double* ly = &Q.sides[y].Lt[j][g * ny];
            for (int i = 0; i < nx; ++i)
              for (int i2 = 0; i2 < ny; ++i2) c[i * ny + i2] += w * lx[i] * ly[i2];
          }
        }
    auto prodC = [&](const std::vector<double>* cj, int ny, const int* ia, const int* ib) {
      double t = 1.0;
      for (int j = 0; j < Q.nt; ++j) t *= cj[j][ia[Q.tdim[j]] * ny + ib[Q.tdim[j]]];
      return t;
    };
    // consistency and symmetry terms
    for (int x = 0; x < ns; ++x) {
      const FaceSide& X = Q.sides[x];
      const int sx = X.s ? X.n - 1 : 0;
      for (int y = 0; y < ns; ++y) {
        const FaceSide& Y = Q.sides[y];
        const Basis1D& By = basis(M.p[Y.e]);
        const std::vector<double>& Dy = Y.s ? By.D1 : By.D0;
        const double fy = Y.ca * M.k[Y.e] / M.h[Y.e];
        for (const Col& ca : cols[x]) {
          if (ca.i[Q.m] != sx) continue;
          for (const Col& cb : cols[y]) {
            const double v = X.js * Dy[cb.i[Q.m]] * fy * prodC(C[x][y], Y.n, ca.i, cb.i);
            S[(size_t)ca.a * nb + cb.a] -= v;
            S[(size_t)cb.a * nb + ca.a] -= v;
          }
        }
      }
    }
    if (o.form == 0) {
      for (int x = 0; x < ns; ++x) {
        const FaceSide& X = Q.sides[x];
        const int sx = X.s ? X.n - 1 : 0;
        for (int y = 0; y < ns; ++y) {
          const FaceSide& Y = Q.sides[y];
          const int sy = Y.s ? Y.n - 1 : 0;
          for (const Col& ca : cols[x]) {
            if (ca.i[Q.m] != sx) continue;
            for (const Col& cb : cols[y]) {
              if (cb.i[Q.m] != sy) continue;
              S[(size_t)ca.a * nb + cb.a] += sig * X.js * Y.js * prodC(C[x][y], Y.n, ca.i, cb.i);
            }
          }
        }
      }
    } else {
      const double c2 = f.ep >= 0 ? 0.25 : 1.0;
      for (int k = 0; k < ns; ++k) {
        const FaceSide& K = Q.sides[k];
        const Basis1D& Bk = basis(M.p[K.e]);
        const int nk = K.n;
        const int sk = K.s ? nk - 1 : 0;
        const double mk = Bk.Minv[sk * nk + sk] * std::pow(M.h[K.e], -d);
        // L[x][y][j] = C_j^{Kx}' Minv_K C_j^{Ky}
        std::vector<double> L[2][2][2];
        for (int x = 0; x < ns; ++x)
          for (int y = 0; y < ns; ++y)
            for (int j = 0; j < Q.nt; ++j) {
              const int nx = Q.sides[x].n, ny = Q.sides[y].n;
              const std::vector<double>& ckx = C[k][x][j];
              const std::vector<double>& cky = C[k][y][j];
              std::vector<double> mc((size_t)nk * ny, 0.0);   // Minv C^{Ky}
              for (int r = 0; r < nk; ++r)
                for (int r2 = 0; r2 < nk; ++r2) {
                  const double mi = Bk.Minv[r * nk + r2];
                  for (int i2 = 0; i2 < ny; ++i2) mc[r * ny + i2] += mi * cky[r2 * ny + i2];
                }
              std::vector<double>& l = L[x][y][j];
              l.assign((size_t)nx * ny, 0.0);
              for (int r = 0; r < nk; ++r)
                for (int i = 0; i < nx; ++i) {
                  const double cv = ckx[r * nx + i];
                  for (int i2 = 0; i2 < ny; ++i2) l[i * ny + i2] += cv * mc[r * ny + i2];
                }
            }
        for (int x = 0; x < ns; ++x) {
          const FaceSide& X = Q.sides[x];
          const int sx = X.s ? X.n - 1 : 0;
          for (int y = 0; y < ns; ++y) {
            const FaceSide& Y = Q.sides[y];
            const int sy = Y.s ? Y.n - 1 : 0;
            const double w = c2 * sig * mk * X.js * Y.js;
            for (const Col& ca : cols[x]) {
              if (ca.i[Q.m] != sx) continue;
              for (const Col& cb : cols[y]) {
                if (cb.i[Q.m] != sy) continue;
                S[(size_t)ca.a * nb + cb.a] += w * prodC(L[x][y], Y.n, ca.i, cb.i);
              }
            }
          }
        }
      }
    }
  }
  return S;
}

// -------------------------------------------------- conforming prolongation
namespace {
using SRow = std::vector<std::pair<int32_t, double>>;

struct Pt { int64_t base[3], scale[3]; double x[3]; };

struct ConfBuilder {
  const Mesh& M;
  std::unordered_map<int, std::vector<SRow>> memo;
  explicit ConfBuilder(const Mesh& m) : M(m) {}

  static void merge(SRow& acc, const SRow& r, double c) {
    if (c == 0.0) return;
    for (auto& [j, v] : r) acc.push_back({j, v * c});
  }
  static void compact(SRow& r) {
    std::sort(r.begin(), r.end(), [](auto& a, auto& b) { return a.first < b.first; });
    SRow out;
    for (auto& [j, v] : r) {
      if (!out.empty() && out.back().first == j) out.back().second += v;
      else out.push_back({j, v});
    }
    out.erase(std::remove_if(out.begin(), out.end(), [](auto& a) { return a.second == 0.0; }), out.end());
    r.swap(out);
  }

  SRow eval(int id, const Pt& pt) {
    const Entity& E = M.ent[id];
    const std::vector<SRow>& C = coef(id);
    int od[3], k = 0;
    for (int m = 0; m < M.dim; ++m)
      if (E.key.v[2 * m + 1] > E.key.v[2 * m]) od[k++] = m;
    int deg = E.deg;
    int n = deg + 1;
    double L[3][kMaxN];
    for (int j = 0; j < k; ++j) {
      int m = od[j];
      int64_t lo = E.key.v[2 * m] / 4, S = (E.key.v[2 * m + 1] - E.key.v[2 * m]) / 4;
      double r = ((double)(pt.base[m] - lo) + (double)pt.scale[m] * pt.x[m]) / (double)S;
      lagrange_eval(basis(deg).x, r, L[j]);
    }
    // only the entity nodes whose 1D factors are all nonzero contribute (a
    // point on the entity's own nodes has one); visited in increasing node
    // order, so the sums are formed in the same order as a full sweep
    int nz[3][kMaxN], nnz[3] = {1, 1, 1}, total = 1;
    for (int j = 0; j < k; ++j) {
      nnz[j] = 0;
      for (int i = 0; i < n; ++i)
        if (L[j][i] != 0.0) nz[j][nnz[j]++] = i;
      total *= nnz[j];
    }
    SRow acc;
    for (int t = 0; t < total; ++t) {
      double c = 1.0;
      int tt = t, g = 0, stride = 1;
      for (int j = 0; j < k; ++j) {
        const int a = nz[j][tt % nnz[j]];
        tt /= nnz[j];
        c *= L[j][a];
        g += a * stride;
        stride *= n;
      }
      if (total == 1 && c == 1.0) return C[g];   // rows in C are already compact
      merge(acc, C[g], c);
    }
    compact(acc);
    return acc;
  }

  const std::vector<SRow>& coef(int id) {
    auto it = memo.find(id);
    if (it != memo.end()) return it->second;
    const Entity E = M.ent[id];
    int od[3], k = 0;
    for (int m = 0; m < M.dim; ++m)
      if (E.key.v[2 * m + 1] > E.key.v[2 * m]) od[k++] = m;
    int deg = E.deg;
    int n = deg + 1;
    int ng = 1;
    for (int j = 0; j < k; ++j) ng *= n;
    std::vector<SRow> C(ng);
    for (int g = 0; g < ng; ++g) {
      int jj[3], gg = g;
      bool interior = true;
      for (int j = 0; j < k; ++j) {
        jj[j] = gg % n;
        gg /= n;
        if (jj[j] == 0 || jj[j] == deg) interior = false;
      }
      if (interior) {
        if (!E.boundary) {
          int64_t li = 0;
          for (int j = k - 1; j >= 0; --j) li = li * (deg - 1) + (jj[j] - 1);
          C[g].push_back({(int32_t)(E.col0 + li), 1.0});
        }
        continue;
      }
      EKey bk = E.key;
      Pt pt;
      for (int m = 0; m < 3; ++m) { pt.base[m] = 0; pt.scale[m] = 0; pt.x[m] = 0.0; }
      for (int m = 0; m < M.dim; ++m) {
        int64_t l4 = E.key.v[2 * m], h4 = E.key.v[2 * m + 1];
        pt.base[m] = l4 / 4;
        if (h4 > l4) {
          int j = 0;
          while (od[j] != m) ++j;
          if (jj[j] == 0) { bk.v[2 * m + 1] = l4; }
          else if (jj[j] == deg) { bk.v[2 * m] = h4; }
          pt.scale[m] = (h4 - l4) / 4;
          pt.x[m] = basis(deg).x[jj[j]];
        }
      }
      auto bi = M.ent_index.find(bk);
      if (bi == M.ent_index.end()) throw Error(-1, "entity boundary not found");
      C[g] = eval(M.resolve(bi->second), pt);
    }
    return memo.emplace(id, std::move(C)).first->second;
  }
};
}  // namespace

CSR prolongation(Mesh& M) {
  M.build_entities();
  // element ranges in parallel, each with its own memo of entity rows (a
  // row does not depend on what the memo already holds); ranges yield
  // consecutive rows
  const int T = std::max(1, setup_threads());
  std::vector<std::vector<int64_t>> len(T);
  std::vector<std::vector<int32_t>> idx(T);
  std::vector<std::vector<double>> val(T);
  std::vector<std::exception_ptr> err(T);
  const Mesh& CM = M;
  const int d = M.dim;
  parallel_chunks(M.ne, [&](int64_t e0, int64_t e1, int t) {
    try {
      ConfBuilder cb(CM);
      for (int64_t e = e0; e < e1; ++e) {
        int p = CM.p[e], n = p + 1;
        const Basis1D& B = basis(p);
        int64_t nd = CM.off[e + 1] - CM.off[e];
        for (int64_t r = 0; r < nd; ++r) {
          int i[3] = {1, 1, 1};
          multi_index(r, n, d, i);
          int ti = 0, mul = 1;
          for (int m = 0; m < d; ++m) {
            const int tm = i[m] == 0 ? 0 : (i[m] == p ? 2 : 1);
            ti += tm * mul;
            mul *= 3;
          }
          int id = CM.resolve(CM.sub[(size_t)e * 27 + ti]);
          Pt pt;
          for (int m = 0; m < 3; ++m) { pt.base[m] = 0; pt.scale[m] = 0; pt.x[m] = 0; }
          for (int m = 0; m < d; ++m) { pt.base[m] = CM.lo[3 * e + m]; pt.scale[m] = CM.sz[e]; pt.x[m] = B.x[i[m]]; }
          SRow row = cb.eval(id, pt);
          for (auto& [j, v] : row) { idx[t].push_back(j); val[t].push_back(v); }
          len[t].push_back((int64_t)row.size());
        }
      }
    } catch (...) {
      err[t] = std::current_exception();
    }
  }, 64);
  for (auto& x : err)
    if (x) std::rethrow_exception(x);
  CSR P;
  P.nrows = M.ndof;
  P.ncols = M.nconf;
  P.ptr.assign(1, 0);
  for (int t = 0; t < T; ++t) {
    for (int64_t l : len[t]) P.ptr.push_back(P.ptr.back() + l);
    P.idx.insert(P.idx.end(), idx[t].begin(), idx[t].end());
    P.val.insert(P.val.end(), val[t].begin(), val[t].end());
  }
  return P;
}

// ----------------------------------------------------------------- labels
static void side_types(int dim, const int t[3], int out[3][3], int& cnt) {
  cnt = 0;
  for (int m = 0; m < dim; ++m)
    if (t[m] != 1) {
      for (int j = 0; j < 3; ++j) out[cnt][j] = 1;
      out[cnt][m] = t[m];
      ++cnt;
    }
}
static int tindex(const int t[3], int dim) {
  int idx = 0, mul = 1;
  for (int m = 0; m < dim; ++m) { idx += t[m] * mul; mul *= 3; }
  return idx;
}

std::vector<int8_t> dof_labels(Mesh& M, int remark_relax) {
  M.build_entities();
  int d = M.dim;
  std::vector<char> not_hp_free(M.ent.size(), 0);
  for (size_t id = 0; id < M.ent.size(); ++id) {
    const Entity& E = M.ent[id];
    if (!E.hanging || E.dim > d - 2) continue;
    auto T = M.touching((int)id);
    int pmin = 1 << 30, pmax = -1;
    for (auto& t : T) { pmin = std::min(pmin, M.p[t.e]); pmax = std::max(pmax, M.p[t.e]); }
    if (pmin == pmax) continue;
    for (auto& t : T) {
      int st[3][3], ns;
      side_types(d, t.t, st, ns);
      for (int s = 0; s < ns; ++s) not_hp_free[M.resolve(M.sub[(size_t)t.e * 27 + tindex(st[s], d)])] = 1;
    }
  }
  // side classes: conforming, uniform degree, coarse degree <= finer degrees
  std::vector<int8_t> cls_done(M.ent.size(), 0), cls_conf(M.ent.size(), 0), cls_uni(M.ent.size(), 0),
      cls_cle(M.ent.size(), 0);
  auto side_class = [&](int id) {
    if (cls_done[id]) return;
    auto T = M.touching(id);
    std::vector<int> full, others;
    for (auto& t : T) {
      int sid = M.sub[(size_t)t.e * 27 + tindex(t.t, d)];
      auto& v = sid == id ? full : others;
      if (std::find(v.begin(), v.end(), t.e) == v.end()) v.push_back(t.e);
    }
    int pmin = 1 << 30, pmax = -1, omin = 1 << 30;
    for (int e : full) { pmin = std::min(pmin, M.p[e]); pmax = std::max(pmax, M.p[e]); }
    for (int e : others) { pmin = std::min(pmin, M.p[e]); pmax = std::max(pmax, M.p[e]); omin = std::min(omin, M.p[e]); }
    cls_conf[id] = others.empty();
    cls_uni[id] = pmin == pmax;
    cls_cle[id] = !others.empty() && full.size() == 1 && M.p[full[0]] <= omin;
    cls_done[id] = 1;
  };
  std::vector<int8_t> lab(M.ndof, 0);
  for (int e = 0; e < M.ne; ++e) {
    int p = M.p[e], n = p + 1;
    int64_t nd = M.off[e + 1] - M.off[e];
    for (int64_t r = 0; r < nd; ++r) {
      int i[3] = {1, 1, 1}, t[3] = {1, 1, 1};
      multi_index(r, n, d, i);
      bool interior = true;
      for (int m = 0; m < d; ++m) {
        t[m] = i[m] == 0 ? 0 : (i[m] == p ? 2 : 1);
        if (t[m] != 1) interior = false;
      }
      if (interior) continue;
      int id = M.sub[(size_t)e * 27 + tindex(t, d)];
      const Entity& E = M.ent[id];
      bool j = false;
      if (E.dim == 0 && !E.hanging) j = true;                        // J1
      else if (E.dim == d - 1 && !E.hanging) {
        side_class(id);
        j = cls_conf[id] && cls_uni[id];                              // J2
      }
      if (!j) {
        int st[3][3], ns;
        side_types(d, t, st, ns);
        for (int s = 0; s < ns && !j; ++s) {
          int sid = M.resolve(M.sub[(size_t)e * 27 + tindex(st[s], d)]);
          if (!not_hp_free[sid]) j = true;                            // J3
          else if (remark_relax) {
            side_class(sid);
            if (cls_cle[sid]) j = true;                               // J4
          }
        }
      }
      lab[M.off[e] + r] = j ? 1 : 2;
    }
  }
  return lab;
}

std::vector<std::vector<int64_t>> edge_spaces(const Mesh& M, const std::vector<int8_t>& lab) {
  std::vector<int64_t> parent(M.ndof, -1);
  for (int64_t g = 0; g < M.ndof; ++g)
    if (lab[g] == 2) parent[g] = g;
  auto find = [&](int64_t a) {
    while (parent[a] != a) { parent[a] = parent[parent[a]]; a = parent[a]; }
    return a;
  };
  int d = M.dim;
  for (const Face& f : M.faces) {
    std::vector<int64_t> mem;
    auto collect = [&](int e, int upper) {
      int p = M.p[e], n = p + 1;
      int64_t nd = M.off[e + 1] - M.off[e];
      for (int64_t r = 0; r < nd; ++r) {
        int i[3];
        multi_index(r, n, d, i);
        if (i[f.m] != (upper ? p : 0)) continue;
        int64_t g = M.off[e] + r;
        if (lab[g] == 2) mem.push_back(g);
      }
    };
    if (f.ep >= 0) { collect(f.em, 1); collect(f.ep, 0); }
    else collect(f.em, f.side);
    for (size_t a = 1; a < mem.size(); ++a) {
      int64_t ra = find(mem[a]), rb = find(mem[0]);
      if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
    }
  }
  std::unordered_map<int64_t, size_t> root_of;
  std::vector<std::vector<int64_t>> comps;
  for (int64_t g = 0; g < M.ndof; ++g) {
    if (parent[g] < 0) continue;
    int64_t r = find(g);
    auto it = root_of.find(r);
    if (it == root_of.end()) { root_of[r] = comps.size(); comps.push_back({g}); }
    else comps[it->second].push_back(g);
  }
  // components in order of their smallest DOF; DOFs ascending (already)
  std::sort(comps.begin(), comps.end(), [](auto& a, auto& b) { return a[0] < b[0]; });
  return comps;
}

// V_e in 3D (Sec. 3.3 treats 2D only): the seed-and-grow process with its
// growth kept inside the master face of the seed, so every space belongs to
// one master face (a conforming side, the full side of the coarser leaf of a
// nonconforming interface, or a boundary side) and holds the N-DOFs on that
// face from the leaves on both of its sides. Built leaf by leaf: each side of
// a leaf contributes its N-DOFs to the space of the side's master face, found
// from the sizes of the neighbours across it. Spaces of different master
// faces overlap on shared element edges and vertices. Order: DOFs ascending
// within a space, duplicates removed, spaces lexicographically.
std::vector<std::vector<int64_t>> face_spaces(const Mesh& M, const std::vector<int8_t>& lab) {
  const int d = M.dim;
  std::map<std::array<int64_t, 3>, std::vector<int64_t>> by_master;
  for (int e = 0; e < M.ne; ++e) {
    const int p = M.p[e], n = p + 1;
    const int64_t nd = M.off[e + 1] - M.off[e];
    for (int m = 0; m < d; ++m)
      for (int s = 0; s < 2; ++s) {
        // neighbours across side (m, s): faces of e with normal m on that side
        int nb = -1;
        bool any = false;
        for (int q = M.ef_ptr[e]; q < M.ef_ptr[e + 1]; ++q) {
          const Face& f = M.faces[M.ef_idx[q]];
          if (f.m != m) continue;
          const int side = f.ep < 0 ? f.side : (f.em == e ? 1 : 0);
          if (side != s) continue;
          any = true;
          if (f.ep >= 0) nb = f.em == e ? f.ep : f.em;
        }
        if (!any) continue;
        std::array<int64_t, 3> key;
        if (nb < 0 || M.sz[nb] < M.sz[e]) key = {e, m, s};         // boundary, or e is the coarse leaf
        else if (M.sz[nb] > M.sz[e]) key = {nb, m, 1 - s};         // the neighbour is the coarse leaf
        else key = s == 1 ? std::array<int64_t, 3>{e, m, 1} : std::array<int64_t, 3>{nb, m, 1};
        std::vector<int64_t>& mem = by_master[key];
        for (int64_t r = 0; r < nd; ++r) {
          int i[3];
          multi_index(r, n, d, i);
          if (i[m] != (s ? p : 0)) continue;
          const int64_t g = M.off[e] + r;
          if (lab[g] == 2) mem.push_back(g);
        }
      }
  }
  std::vector<std::vector<int64_t>> out;
  for (auto& kv : by_master) {
    std::vector<int64_t>& v = kv.second;
    if (v.empty()) continue;
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    out.push_back(std::move(v));
  }
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
  return out;
}

// -------------------------------------------------------------------- LOR
// A~_K: Q1 stiffness on the Cartesian sub-grid of the GL nodes of K, times
// k_K (Sec. 3.4). Each sub-cell box with sides D_m contributes
// sum_m (prod_{j!=m} D_j / D_m) (k1 in dim m, m1 in the other dims).
// LOR element matrix as a 3^d stencil per node: A[r * 3^d + s] couples node r
// with node r + delta(s), delta_m = (s / 3^m) % 3 - 1 (the Q1 sub-cells only
// couple nodes that differ by at most one in each index)
static void lor_elem(const Mesh& M, int e, std::vector<double>& A) {
  int d = M.dim, p = M.p[e], n = p + 1;
  const Basis1D& B = basis(p);
  int nd = 1, ns = 1;
  for (int m = 0; m < d; ++m) { nd *= n; ns *= 3; }
  A.assign((size_t)nd * ns, 0.0);
  const double k1[2][2] = {{1, -1}, {-1, 1}};
  const double m1[2][2] = {{1.0 / 3, 1.0 / 6}, {1.0 / 6, 1.0 / 3}};
  int ncell = 1;
  for (int m = 0; m < d; ++m) ncell *= p;
  int nv = 1 << d;
  for (int c = 0; c < ncell; ++c) {
    int ci[3] = {0, 0, 0}, cc = c;
    for (int m = 0; m < d; ++m) { ci[m] = cc % p; cc /= p; }
    double D[3];
    for (int m = 0; m < d; ++m) D[m] = M.h[e] * (B.x[ci[m] + 1] - B.x[ci[m]]);
    int gidx[8];
    for (int v = 0; v < nv; ++v) {
      int g = 0, mul = 1;
      for (int m = 0; m < d; ++m) { g += (ci[m] + ((v >> m) & 1)) * mul; mul *= n; }
      gidx[v] = g;
    }
    double coef[3];   // product of the other extents over this one
    for (int m = 0; m < d; ++m) {
      coef[m] = 1.0;
      for (int j = 0; j < d; ++j)
        if (j != m) coef[m] *= D[j];
      coef[m] /= D[m];
    }
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b) {
        double s = 0;
        for (int m = 0; m < d; ++m) {
          double t = coef[m];
          for (int j = 0; j < d; ++j) t *= (j == m ? k1 : m1)[(a >> j) & 1][(b >> j) & 1];
          s += t;
        }
        int st = 0, mul = 1;
        for (int m = 0; m < d; ++m) { st += (((b >> m) & 1) - ((a >> m) & 1) + 1) * mul; mul *= 3; }
        A[(size_t)gidx[a] * ns + st] += M.k[e] * s;
      }
  }
}

CSR lor_times(const Mesh& M, const CSR& P) {
  // element ranges in parallel; each range yields consecutive rows
  const int T = std::max(1, setup_threads());
  std::vector<std::vector<int64_t>> len(T);
  std::vector<std::vector<int32_t>> idx(T);
  std::vector<std::vector<double>> val(T);
  parallel_chunks(M.ne, [&](int64_t e0, int64_t e1, int t) {
    std::vector<double> acc(P.ncols, 0.0);
    std::vector<char> used(P.ncols, 0);
    std::vector<int32_t> cols;
    std::vector<double> A;
    for (int64_t e = e0; e < e1; ++e) {
      lor_elem(M, (int)e, A);
      const int64_t nd = M.off[e + 1] - M.off[e];
      const int n = M.p[e] + 1, ns = M.dim == 3 ? 27 : 9;
      const int64_t str[3] = {1, n, (int64_t)n * n};
      for (int64_t r = 0; r < nd; ++r) {
        cols.clear();
        // stencil entries in increasing column order; those off the element
        // are never written and stay zero
        for (int st = 0; st < ns; ++st) {
          double a = A[(size_t)r * ns + st];
          if (a == 0.0) continue;
          int64_t c = r;
          for (int m = 0, q = st; m < M.dim; ++m, q /= 3) c += (q % 3 - 1) * str[m];
          int64_t row = M.off[e] + c;
          for (int64_t q = P.ptr[row]; q < P.ptr[row + 1]; ++q) {
            int32_t j = P.idx[q];
            if (!used[j]) { used[j] = 1; cols.push_back(j); acc[j] = 0.0; }
            acc[j] += a * P.val[q];
          }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t j : cols) { idx[t].push_back(j); val[t].push_back(acc[j]); used[j] = 0; }
        len[t].push_back((int64_t)cols.size());
      }
    }
  }, 16);
  CSR R;
  R.nrows = M.ndof;
  R.ncols = P.ncols;
  R.ptr.assign(1, 0);
  for (int t = 0; t < T; ++t) {
    for (int64_t l : len[t]) R.ptr.push_back(R.ptr.back() + l);
    R.idx.insert(R.idx.end(), idx[t].begin(), idx[t].end());
    R.val.insert(R.val.end(), val[t].begin(), val[t].end());
  }
  return R;
}

}  // namespace hpdg
