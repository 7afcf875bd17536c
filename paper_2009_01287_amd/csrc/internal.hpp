// Internal host-side structures of the hp-DG library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

namespace hpdg {

constexpr int kMaxP = 8;     // highest polynomial degree
constexpr int kMaxN = kMaxP + 1;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ----------------------------------------------------------------- 1D basis
// Gauss-Lobatto nodal basis of degree p on [0,1] and exact 1D matrices.
struct Basis1D {
  int p;
  std::vector<double> x;      // GL nodes, p+1
  std::vector<double> M, K;   // (p+1)^2 row-major, exact mass / stiffness
  std::vector<double> Minv;   // inverse of M
  std::vector<double> D0, D1; // l_i'(0), l_i'(1)
};
const Basis1D& basis(int p);
// q-point Gauss-Legendre rule on [0,1]
void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w);
void lagrange_eval(const std::vector<double>& nodes, double t, double* out);
void lagrange_deriv(const std::vector<double>& nodes, double t, double* out);

// -------------------------------------------------------------------- mesh
struct Face {
  int m;          // normal dimension
  int em;         // element on the lower side (minus), or the element itself
  int ep;         // element on the upper side (plus), -1 on the boundary
  int side;       // boundary faces: which side of em (0 lower, 1 upper)
  int64_t lo[3];  // face box in finest units (lo[m] == hi[m])
  int64_t hi[3];
};

struct EKey {  // entity geometry in quarter units: per dim (lo4, hi4)
  int64_t v[6];
  bool operator==(const EKey& o) const { return std::memcmp(v, o.v, sizeof(v)) == 0; }
};
struct EKeyHash {
  size_t operator()(const EKey& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 6; ++i) { h ^= (uint64_t)k.v[i] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2); }
    return (size_t)h;
  }
};

struct Entity {
  EKey key;
  int dim = 0;
  bool hanging = false;
  bool boundary = false;
  int master = -1;   // non-hanging container (self when not hanging)
  int deg = 0;       // minimum-rule degree
  int col0 = -1;     // first conforming column of its interior nodes
};

struct Touch { int e; int64_t y[3]; int t[3]; };

struct Mesh {
  int dim = 2, n_base = 1, L = 0;
  int64_t N = 1;                 // finest cells per unit length
  int ne = 0;
  std::vector<int> level, p;
  std::vector<int64_t> lo;       // ne*3, finest units
  std::vector<int64_t> sz;       // finest units
  std::vector<double> k, h;
  std::vector<int64_t> off;      // DOF offsets, ne+1
  int64_t ndof = 0;
  std::unordered_map<EKey, int, EKeyHash> cells;   // (level, anchor) -> leaf
  std::vector<Face> faces;
  std::vector<int> ef_ptr, ef_idx;   // faces of element e: ef_idx[ef_ptr[e] .. ef_ptr[e+1])
  int max_dlevel = 0;            // largest level jump across a face
  // entities (built on demand for the preconditioner)
  std::vector<Entity> ent;
  std::vector<int> sub;          // ne * 27 entity ids of each leaf's sub-entities
  std::unordered_map<EKey, int, EKeyHash> ent_index;
  int64_t nconf = 0;

  int locate(const int64_t y4[3]) const;
  int leaves_at(const int64_t y4[3], int* out) const;   // up to 8
  void build_faces();
  void build_entities();
  EKey sub_key(int e, const int t[3]) const;
  void leaf_type_at(int e, const int64_t y4[3], int t[3]) const;
  std::vector<Touch> touching(int ent_id) const;
  int resolve(int ent_id) const { return ent[ent_id].hanging ? ent[ent_id].master : ent_id; }
  int ntypes() const { return dim == 2 ? 9 : 27; }
};

Mesh* make_mesh(int dim, int n_base, int64_t n, const int32_t* level, const int32_t* anchor,
                const int32_t* degree, const double* kcoef);

// ------------------------------------------------------ host threading
// Host threads for the setup's row-parallel products (set per calling
// thread; 1 = serial). Results do not depend on it.
void set_setup_threads(int n);
int setup_threads();
// f(begin, end) over consecutive chunks of [0, n), one per thread
void parallel_chunks(int64_t n, const std::function<void(int64_t, int64_t, int)>& f, int64_t min_chunk = 256);

// --------------------------------------------------------------- CSR (host)
struct CSR {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<double> val;
};
CSR csr_transpose(const CSR& A);
CSR csr_matmul(const CSR& A, const CSR& B);
CSR csr_from_triplets(int64_t nr, int64_t nc, std::vector<int64_t>& r, std::vector<int32_t>& c,
                      std::vector<double>& v);

// ---------------------------------------------------- operator description
struct OpOpts {
  int form = 0;          // 0 SIPG, 1 BR2
  int penalty_rule = 0;  // 0: (p+1)^2, 1: p^2
  double eta = 1.0;
  int remark_relax = 0;
  int jb_only = 0;
  int max_block = 0;     // >0: components larger than this use point Jacobi
};

double penalty_or_br2(const Mesh& M, const OpOpts& o, const Face& f, double eta_br2);
double br2_eta(const Mesh& M, const OpOpts& o);

// host-side operator pieces
std::vector<double> dg_diagonal(const Mesh& M, const OpOpts& o);
// dense A[dofs, dofs] (row-major, len(dofs)^2), dofs sorted ascending
std::vector<double> dg_submatrix(const Mesh& M, const OpOpts& o, const std::vector<int64_t>& dofs,
                                 double eta_br2);

// conforming prolongation (CSR ndof x nconf)
CSR prolongation(Mesh& M);
// labels: 0 interior, 1 V_J, 2 N
std::vector<int8_t> dof_labels(Mesh& M, int remark_relax);
std::vector<std::vector<int64_t>> edge_spaces(const Mesh& M, const std::vector<int8_t>& lab);
// 3D: one space per master face (may overlap)
std::vector<std::vector<int64_t>> face_spaces(const Mesh& M, const std::vector<int8_t>& lab);
// LOR block-diagonal matrix applied: returns A~ P (CSR ndof x nconf)
CSR lor_times(const Mesh& M, const CSR& P);

// ------------------------------------------------------------------- AMG
struct AMGLevel {
  CSR A, P, R;            // R = P^T
  std::vector<double> l1; // l1 row sums
};
struct AMGHier {
  std::vector<AMGLevel> lv;
  std::vector<double> coarse_inv;   // dense inverse of the coarsest matrix
  int64_t nc = 0;
  std::vector<std::vector<int64_t>> aggs;
};
AMGHier amg_setup(const CSR& A, int max_levels = 12, int64_t min_rows = 256, double max_ratio = 0.4);
void aggregate(const CSR& A, std::vector<int64_t>& agg, int64_t& na, double theta);

}  // namespace hpdg
