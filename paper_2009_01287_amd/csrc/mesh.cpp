// Mesh topology: leaves of a quadtree/octree forest over an n_base^d grid on
// [0,1]^d (Sec. 2: quadrilateral elements with affine maps T_K; the
// hexahedral case is the same construction in 3D).
//
// Faces (mesh skeleton Gamma, Sec. 2): every positive-measure intersection of
// two leaf sides plus the leaf sides on the boundary. Each interior face is
// found once, from the element below it: the cell across a leaf's upper side
// is either a leaf (conforming face), inside a coarser leaf (one face, the
// fine side), or subdivided (one face per finer leaf, found by descending the
// tree along the side).
//
// Sub-entities (vertices, edges, faces, interior) of each leaf are
// deduplicated by geometry. An entity is hanging when its relative interior
// lies inside the relative interior of a strictly larger sub-entity of
// another leaf; the largest such container is its master (Sec. 3.2.1).
#include <algorithm>
#include <array>
#include <cmath>

#include "internal.hpp"

namespace hpdg {

static EKey cell_key(int level, const int64_t* a, int dim) {
  EKey k;
  std::memset(k.v, 0, sizeof(k.v));
  k.v[0] = level;
  for (int m = 0; m < dim; ++m) k.v[1 + m] = a[m];
  return k;
}

Mesh* make_mesh(int dim, int n_base, int64_t n, const int32_t* level, const int32_t* anchor,
                const int32_t* degree, const double* kcoef) {
  if (dim != 2 && dim != 3) throw Error(-1, "dim must be 2 or 3");
  if (n_base < 1 || n < 1) throw Error(-1, "empty mesh");
  Mesh* M = new Mesh();
  try {
    M->dim = dim;
    M->n_base = n_base;
    M->ne = (int)n;
    int L = 0;
    for (int64_t e = 0; e < n; ++e) {
      if (level[e] < 0 || level[e] > 20) throw Error(-1, "level out of range");
      L = std::max(L, (int)level[e]);
    }
    M->L = L;
    M->N = (int64_t)n_base << L;
    M->level.assign(level, level + n);
    M->p.assign(degree, degree + n);
    M->k.assign(kcoef, kcoef + n);
    M->lo.assign(3 * n, 0);
    M->sz.assign(n, 0);
    M->h.assign(n, 0.0);
    M->off.assign(n + 1, 0);
    long double vol = 0.0L;
    for (int64_t e = 0; e < n; ++e) {
      int lev = level[e];
      if (degree[e] < 1 || degree[e] > kMaxP) throw Error(-1, "degree must be in 1..8");
      if (!(kcoef[e] > 0.0) || !std::isfinite(kcoef[e])) throw Error(-1, "coefficient must be positive");
      int64_t a[3] = {0, 0, 0};
      for (int m = 0; m < dim; ++m) {
        a[m] = anchor[e * dim + m];
        if (a[m] < 0 || a[m] >= ((int64_t)n_base << lev)) throw Error(-1, "leaf outside the domain");
      }
      M->sz[e] = (int64_t)1 << (L - lev);
      for (int m = 0; m < dim; ++m) M->lo[3 * e + m] = a[m] * M->sz[e];
      M->h[e] = (double)M->sz[e] / (double)M->N;
      int64_t nd = 1;
      for (int m = 0; m < dim; ++m) nd *= degree[e] + 1;
      M->off[e + 1] = M->off[e] + nd;
      EKey key = cell_key(lev, a, dim);
      if (!M->cells.emplace(key, (int)e).second) throw Error(-1, "duplicate leaf");
      vol += std::pow((long double)M->sz[e], dim);
    }
    M->ndof = M->off[n];
    // no leaf may have another leaf as an ancestor; the volumes must add up
    for (int64_t e = 0; e < n; ++e) {
      int lev = level[e];
      int64_t a[3] = {0, 0, 0};
      for (int m = 0; m < dim; ++m) a[m] = anchor[e * dim + m];
      for (int l = 0; l < lev; ++l) {
        int64_t b[3];
        for (int m = 0; m < dim; ++m) b[m] = a[m] >> (lev - l);
        if (M->cells.count(cell_key(l, b, dim))) throw Error(-1, "overlapping leaves");
      }
    }
    if (vol != std::pow((long double)M->N, dim)) throw Error(-1, "leaves do not tile the domain");
    M->build_faces();
  } catch (...) {
    delete M;
    throw;
  }
  return M;
}

int Mesh::locate(const int64_t y4[3]) const {
  for (int m = 0; m < dim; ++m)
    if (y4[m] < 0 || y4[m] >= 4 * N) return -1;
  for (int l = 0; l <= L; ++l) {
    int64_t s4 = (int64_t)4 << (L - l);
    int64_t a[3] = {0, 0, 0};
    for (int m = 0; m < dim; ++m) a[m] = y4[m] / s4;
    auto it = cells.find(cell_key(l, a, dim));
    if (it != cells.end()) return it->second;
  }
  throw Error(-1, "point not covered by the mesh");
}

int Mesh::leaves_at(const int64_t y4[3], int* out) const {
  int deg[3], nd = 0;
  for (int m = 0; m < dim; ++m)
    if (y4[m] % 4 == 0) deg[nd++] = m;
  int cnt = 0;
  for (int s = 0; s < (1 << nd); ++s) {
    int64_t y[3] = {y4[0], y4[1], y4[2]};
    for (int j = 0; j < nd; ++j) y[deg[j]] += ((s >> j) & 1) ? 1 : -1;
    int e = locate(y);
    if (e < 0) continue;
    bool dup = false;
    for (int i = 0; i < cnt; ++i) dup |= out[i] == e;
    if (!dup) out[cnt++] = e;
  }
  return cnt;
}

void Mesh::build_faces() {
  faces.clear();
  max_dlevel = 0;
  for (int e = 0; e < ne; ++e) {
    int lev = level[e];
    int64_t a[3] = {0, 0, 0};
    for (int m = 0; m < dim; ++m) a[m] = lo[3 * e + m] / sz[e];
    for (int m = 0; m < dim; ++m) {
      for (int side = 0; side < 2; ++side) {
        int64_t c = lo[3 * e + m] + side * sz[e];
        if (c == 0 || c == N) {            // boundary side
          Face f;
          f.m = m; f.em = e; f.ep = -1; f.side = side;
          for (int t = 0; t < 3; ++t) { f.lo[t] = t < dim ? lo[3 * e + t] : 0; f.hi[t] = t < dim ? lo[3 * e + t] + sz[e] : 0; }
          f.lo[m] = f.hi[m] = c;
          faces.push_back(f);
          continue;
        }
        if (side == 0) continue;            // interior faces are found from below
        int64_t b[3] = {a[0], a[1], a[2]};
        b[m] += 1;
        auto emit = [&](int nb) {
          Face f;
          f.m = m; f.em = e; f.ep = nb; f.side = 1;
          for (int t = 0; t < 3; ++t) {
            if (t >= dim) { f.lo[t] = f.hi[t] = 0; continue; }
            f.lo[t] = std::max(lo[3 * e + t], lo[3 * nb + t]);
            f.hi[t] = std::min(lo[3 * e + t] + sz[e], lo[3 * nb + t] + sz[nb]);
          }
          f.lo[m] = f.hi[m] = c;
          faces.push_back(f);
          max_dlevel = std::max(max_dlevel, std::abs(level[nb] - lev));
        };
        auto it = cells.find(cell_key(lev, b, dim));
        if (it != cells.end()) { emit(it->second); continue; }
        bool found = false;
        for (int l = lev - 1; l >= 0 && !found; --l) {
          int64_t bb[3];
          for (int t = 0; t < dim; ++t) bb[t] = b[t] >> (lev - l);
          auto jt = cells.find(cell_key(l, bb, dim));
          if (jt != cells.end()) { emit(jt->second); found = true; }
        }
        if (found) continue;
        // finer neighbours: descend into the children touching the side
        std::vector<std::pair<int, std::array<int64_t, 3>>> stack;
        stack.push_back({lev, {b[0], b[1], b[2]}});
        while (!stack.empty()) {
          auto [l, cc] = stack.back();
          stack.pop_back();
          if (l > L) throw Error(-1, "inconsistent tree");
          for (int ch = 0; ch < (1 << (dim - 1)); ++ch) {
            int64_t nc[3];
            int bit = 0;
            for (int t = 0; t < dim; ++t) {
              if (t == m) { nc[t] = 2 * cc[t]; continue; }   // lower half along m
              nc[t] = 2 * cc[t] + ((ch >> bit) & 1);
              ++bit;
            }
            auto kt = cells.find(cell_key(l + 1, nc, dim));
            if (kt != cells.end()) emit(kt->second);
            else stack.push_back({l + 1, {nc[0], nc[1], dim > 2 ? nc[2] : 0}});
          }
        }
      }
    }
  }
  // faces of every element (CSR)
  ef_ptr.assign(ne + 1, 0);
  for (const Face& f : faces) {
    ef_ptr[f.em + 1]++;
    if (f.ep >= 0) ef_ptr[f.ep + 1]++;
  }
  for (int e = 0; e < ne; ++e) ef_ptr[e + 1] += ef_ptr[e];
  ef_idx.assign(ef_ptr[ne], 0);
  std::vector<int> fill(ef_ptr.begin(), ef_ptr.end() - 1);
  for (int i = 0; i < (int)faces.size(); ++i) {
    ef_idx[fill[faces[i].em]++] = i;
    if (faces[i].ep >= 0) ef_idx[fill[faces[i].ep]++] = i;
  }
}

EKey Mesh::sub_key(int e, const int t[3]) const {
  EKey k;
  std::memset(k.v, 0, sizeof(k.v));
  for (int m = 0; m < dim; ++m) {
    int64_t l4 = 4 * lo[3 * e + m], h4 = 4 * (lo[3 * e + m] + sz[e]);
    if (t[m] == 0) { k.v[2 * m] = l4; k.v[2 * m + 1] = l4; }
    else if (t[m] == 2) { k.v[2 * m] = h4; k.v[2 * m + 1] = h4; }
    else { k.v[2 * m] = l4; k.v[2 * m + 1] = h4; }
  }
  return k;
}

void Mesh::leaf_type_at(int e, const int64_t y4[3], int t[3]) const {
  for (int m = 0; m < 3; ++m) t[m] = 1;
  for (int m = 0; m < dim; ++m) {
    if (y4[m] == 4 * lo[3 * e + m]) t[m] = 0;
    else if (y4[m] == 4 * (lo[3 * e + m] + sz[e])) t[m] = 2;
    else t[m] = 1;
  }
}

static void type_of(int idx, int dim, int t[3]) {
  t[0] = t[1] = t[2] = 1;
  for (int m = 0; m < dim; ++m) { t[m] = idx % 3; idx /= 3; }
}
static int type_index(const int t[3], int dim) {
  int idx = 0, mul = 1;
  for (int m = 0; m < dim; ++m) { idx += t[m] * mul; mul *= 3; }
  return idx;
}

std::vector<Touch> Mesh::touching(int id) const {
  const EKey& k = ent[id].key;
  std::vector<Touch> out;
  int64_t n[3] = {1, 1, 1};
  for (int m = 0; m < dim; ++m)
    if (k.v[2 * m + 1] > k.v[2 * m]) n[m] = (k.v[2 * m + 1] - k.v[2 * m]) / 4;
  for (int64_t a = 0; a < n[0]; ++a)
    for (int64_t b = 0; b < n[1]; ++b)
      for (int64_t c = 0; c < n[2]; ++c) {
        int64_t y[3] = {0, 0, 0};
        int64_t ix[3] = {a, b, c};
        for (int m = 0; m < dim; ++m)
          y[m] = k.v[2 * m + 1] > k.v[2 * m] ? k.v[2 * m] + 2 + 4 * ix[m] : k.v[2 * m];
        int ls[8];
        int cnt = leaves_at(y, ls);
        for (int i = 0; i < cnt; ++i) {
          Touch t;
          t.e = ls[i];
          for (int m = 0; m < 3; ++m) t.y[m] = y[m];
          leaf_type_at(ls[i], y, t.t);
          out.push_back(t);
        }
      }
  return out;
}

static int key_dim(const EKey& k, int dim) {
  int d = 0;
  for (int m = 0; m < dim; ++m) d += k.v[2 * m + 1] > k.v[2 * m];
  return d;
}
static bool key_contains(const EKey& big, const EKey& small, int dim) {
  for (int m = 0; m < dim; ++m)
    if (!(big.v[2 * m] <= small.v[2 * m] && small.v[2 * m + 1] <= big.v[2 * m + 1])) return false;
  return true;
}
static double key_vol(const EKey& k, int dim) {
  double v = 1;
  for (int m = 0; m < dim; ++m) v *= std::max<int64_t>(k.v[2 * m + 1] - k.v[2 * m], 1);
  return v;
}

void Mesh::build_entities() {
  if (!ent.empty()) return;
  int nt = ntypes();
  sub.assign((size_t)ne * 27, -1);
  for (int e = 0; e < ne; ++e)
    for (int ti = 0; ti < nt; ++ti) {
      int t[3];
      type_of(ti, dim, t);
      EKey k = sub_key(e, t);
      auto it = ent_index.find(k);
      int id;
      if (it == ent_index.end()) {
        id = (int)ent.size();
        Entity E;
        E.key = k;
        E.dim = key_dim(k, dim);
        E.boundary = false;
        for (int m = 0; m < dim; ++m)
          if (k.v[2 * m] == k.v[2 * m + 1] && (k.v[2 * m] == 0 || k.v[2 * m] == 4 * N)) E.boundary = true;
        ent.push_back(E);
        ent_index.emplace(k, id);
      } else {
        id = it->second;
      }
      sub[(size_t)e * 27 + ti] = id;
    }
  // hanging and master: the leaves around one interior point of the entity
  for (size_t id = 0; id < ent.size(); ++id) {
    Entity& E = ent[id];
    int64_t y[3] = {0, 0, 0};
    for (int m = 0; m < dim; ++m)
      y[m] = E.key.v[2 * m + 1] > E.key.v[2 * m] ? E.key.v[2 * m] + 2 : E.key.v[2 * m];
    int ls[8];
    int cnt = leaves_at(y, ls);
    int best = -1;
    int bdim = -1;
    double bvol = -1;
    for (int i = 0; i < cnt; ++i) {
      int t[3];
      leaf_type_at(ls[i], y, t);
      int tid = sub[(size_t)ls[i] * 27 + type_index(t, dim)];
      if (tid == (int)id) continue;
      const EKey& tk = ent[tid].key;
      if (!key_contains(tk, E.key, dim)) continue;
      int dd = key_dim(tk, dim);
      double vv = key_vol(tk, dim);
      if (dd > bdim || (dd == bdim && vv > bvol)) { best = tid; bdim = dd; bvol = vv; }
    }
    E.hanging = best >= 0;
    E.master = best >= 0 ? best : (int)id;
  }
  for (auto& E : ent)
    if (E.hanging && ent[E.master].hanging) throw Error(-1, "master entity is hanging");
  // minimum-rule degrees, highest dimension first
  const int tin[3] = {1, 1, 1};
  for (int e = 0; e < ne; ++e) ent[sub[(size_t)e * 27 + type_index(tin, dim)]].deg = p[e];
  for (int kd = dim - 1; kd >= 0; --kd) {
    for (size_t id = 0; id < ent.size(); ++id) {
      Entity& E = ent[id];
      if (E.dim != kd || E.hanging) continue;
      int dmin = 1 << 30;
      for (const Touch& T : touching((int)id)) {
        dmin = std::min(dmin, p[T.e]);
        for (int ti = 0; ti < nt; ++ti) {
          int tp[3];
          type_of(ti, dim, tp);
          bool sup = true, same = true;
          for (int m = 0; m < dim; ++m) {
            if (tp[m] != T.t[m]) same = false;
            if (!(tp[m] == T.t[m] || (T.t[m] != 1 && tp[m] == 1))) sup = false;
          }
          if (!sup || same) continue;
          int oid = sub[(size_t)T.e * 27 + ti];
          if (!ent[oid].hanging) dmin = std::min(dmin, ent[oid].deg);
        }
      }
      E.deg = dmin;
    }
  }
  // conforming numbering: leaves in order, sub-entities in type order
  nconf = 0;
  for (int e = 0; e < ne; ++e)
    for (int ti = 0; ti < nt; ++ti) {
      Entity& E = ent[sub[(size_t)e * 27 + ti]];
      if (E.hanging || E.boundary || E.col0 >= 0) continue;
      E.col0 = (int)nconf;
      int64_t c = 1;
      for (int j = 0; j < E.dim; ++j) c *= (E.deg - 1);
      nconf += c;
    }
}

}  // namespace hpdg
