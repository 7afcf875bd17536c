// Sparse matrix utilities and the smoothed-aggregation AMG setup used for the
// conforming low-order-refined matrix A~_C (Sec. 3.4: any uniform
// preconditioner for A~_C may be used; the paper applies one BoomerAMG
// V-cycle, whose settings it does not state).
//
// Project specification:
//   strength  j in S_i iff j != i and |a_ij| >= 0.04 sqrt(a_ii a_jj)
//   phase 1   in row order, a free row whose strong neighbours are all free
//             forms the aggregate {i} + S_i
//   phase 2   a free row joins the phase-1 aggregate of its strongest
//             phase-1-aggregated neighbour (|a_ij| within a relative 1e-10 of
//             the maximum count as ties; ties go to the lowest aggregate)
//   phase 3   a still free row forms {i} + its free strong neighbours
//   P_l = (I - w D_F^{-1} A_F) P^, P^ the 0/1 aggregate indicator, A_F the
//   filtered matrix (weak off-diagonals dropped and added to the diagonal;
//   rows whose filtered diagonal is at most 1e-8 a_ii are not smoothed),
//   w = (4/3)/rho, rho = max_i sum_j |a^F_ij| / a^F_ii; A_{l+1} = P_l^T A_l P_l
//   a level keeping > 0.4 of its rows is retried with theta = 0.02, 0.01,
//   0.005 and 0 (every connection strong);
//   stop at <= 256 rows, 12 levels, or a level that still stalls;
//   the coarsest level is solved exactly (dense Cholesky, stored inverse).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include <thread>

#include "internal.hpp"

namespace hpdg {

CSR csr_transpose(const CSR& A) {
  CSR T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign(A.ncols + 1, 0);
  for (int32_t j : A.idx) T.ptr[j + 1]++;
  for (int64_t i = 0; i < A.ncols; ++i) T.ptr[i + 1] += T.ptr[i];
  T.idx.resize(A.idx.size());
  T.val.resize(A.val.size());
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      int64_t w = pos[A.idx[q]]++;
      T.idx[w] = (int32_t)i;
      T.val[w] = A.val[q];
    }
  return T;
}

static thread_local int g_threads = 1;
void set_setup_threads(int n) { g_threads = std::max(1, n); }
int setup_threads() { return g_threads; }

void parallel_chunks(int64_t n, const std::function<void(int64_t, int64_t, int)>& f, int64_t min_chunk) {
  int T = (int)std::min<int64_t>(g_threads, std::max<int64_t>(1, n / std::max<int64_t>(1, min_chunk)));
  if (T <= 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) {
    const int64_t b = n * t / T, e = n * (t + 1) / T;
    th.emplace_back([&f, b, e, t]() { f(b, e, t); });
  }
  for (auto& x : th) x.join();
}

// Rows of a product or other row-wise result computed in chunks by several
// threads and joined in row order.
struct RowPieces {
  std::vector<std::vector<int64_t>> len;
  std::vector<std::vector<int32_t>> idx;
  std::vector<std::vector<double>> val;
  explicit RowPieces(int T) : len(T), idx(T), val(T) {}
  CSR join(int64_t nrows, int64_t ncols) {
    CSR C;
    C.nrows = nrows;
    C.ncols = ncols;
    C.ptr.assign(1, 0);
    size_t tot = 0;
    for (auto& v : idx) tot += v.size();
    C.idx.reserve(tot);
    C.val.reserve(tot);
    for (size_t t = 0; t < len.size(); ++t) {
      for (int64_t l : len[t]) C.ptr.push_back(C.ptr.back() + l);
      C.idx.insert(C.idx.end(), idx[t].begin(), idx[t].end());
      C.val.insert(C.val.end(), val[t].begin(), val[t].end());
    }
    return C;
  }
};

CSR csr_matmul(const CSR& A, const CSR& B) {
  const int T = std::max(1, setup_threads());
  RowPieces pc(T);
  parallel_chunks(A.nrows, [&](int64_t b, int64_t e, int t) {
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<char> used(B.ncols, 0);
    std::vector<int32_t> cols;
    for (int64_t i = b; i < e; ++i) {
      cols.clear();
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
        int32_t k = A.idx[q];
        double a = A.val[q];
        for (int64_t r = B.ptr[k]; r < B.ptr[k + 1]; ++r) {
          int32_t j = B.idx[r];
          if (!used[j]) { used[j] = 1; acc[j] = 0.0; cols.push_back(j); }
          acc[j] += a * B.val[r];
        }
      }
      std::sort(cols.begin(), cols.end());
      int64_t l = 0;
      for (int32_t j : cols) {
        used[j] = 0;
        if (acc[j] == 0.0) continue;
        pc.idx[t].push_back(j);
        pc.val[t].push_back(acc[j]);
        ++l;
      }
      pc.len[t].push_back(l);
    }
  });
  return pc.join(A.nrows, B.ncols);
}

CSR csr_from_triplets(int64_t nr, int64_t nc, std::vector<int64_t>& r, std::vector<int32_t>& c,
                      std::vector<double>& v) {
  std::vector<size_t> ord(r.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return r[a] != r[b] ? r[a] < r[b] : c[a] < c[b]; });
  CSR A;
  A.nrows = nr;
  A.ncols = nc;
  A.ptr.assign(nr + 1, 0);
  int64_t lr = -1;
  int32_t lc = -1;
  for (size_t t : ord) {
    if (r[t] == lr && c[t] == lc) { A.val.back() += v[t]; continue; }
    A.idx.push_back(c[t]);
    A.val.push_back(v[t]);
    A.ptr[r[t] + 1]++;
    lr = r[t];
    lc = c[t];
  }
  for (int64_t i = 0; i < nr; ++i) A.ptr[i + 1] += A.ptr[i];
  return A;
}

static std::vector<double> csr_diag(const CSR& A) {
  std::vector<double> d(A.nrows, 0.0);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (A.idx[q] == i) d[i] += A.val[q];
  return d;
}

void aggregate(const CSR& A, std::vector<int64_t>& agg, int64_t& na, double theta) {
  const double tie = 1e-10;
  int64_t n = A.nrows;
  std::vector<double> dg = csr_diag(A);
  auto strong = [&](int64_t i, int64_t q) {
    int32_t j = A.idx[q];
    return j != i && std::fabs(A.val[q]) >= theta * std::sqrt(dg[i] * dg[j]);
  };
  agg.assign(n, -1);
  na = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool ok = true;
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1] && ok; ++q)
      if (strong(i, q) && agg[A.idx[q]] >= 0) ok = false;
    if (!ok) continue;
    agg[i] = na;
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (strong(i, q)) agg[A.idx[q]] = na;
    ++na;
  }
  std::vector<int64_t> p1 = agg;
  for (int64_t i = 0; i < n; ++i) {
    if (p1[i] >= 0) continue;
    double amax = -1.0;
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (strong(i, q) && p1[A.idx[q]] >= 0) amax = std::max(amax, std::fabs(A.val[q]));
    if (amax < 0) continue;
    int64_t best = -1;
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (strong(i, q) && p1[A.idx[q]] >= 0 && std::fabs(A.val[q]) >= amax * (1.0 - tie)) {
        int64_t g = p1[A.idx[q]];
        if (best < 0 || g < best) best = g;
      }
    agg[i] = best;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (strong(i, q) && agg[A.idx[q]] < 0) agg[A.idx[q]] = na;
    ++na;
  }
}

static void dense_cholesky_inverse(const CSR& A, std::vector<double>& inv) {
  int64_t n = A.nrows;
  std::vector<double> L(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) L[i * n + A.idx[q]] += A.val[q];
  for (int64_t j = 0; j < n; ++j) {
    double s = L[j * n + j];
    for (int64_t k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0)) throw Error(-4, "coarsest AMG matrix is not positive definite");
    double dj = std::sqrt(s);
    L[j * n + j] = dj;
    for (int64_t i = j + 1; i < n; ++i) {
      double t = L[i * n + j];
      for (int64_t k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / dj;
    }
    for (int64_t i = 0; i < j; ++i) L[i * n + j] = 0.0;
  }
  // inverse = L^{-T} L^{-1}: solve for each unit vector
  inv.assign(n * n, 0.0);
  std::vector<double> y(n);
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      double t = i == c ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; ++k) t -= L[i * n + k] * y[k];
      y[i] = t / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int64_t k = i + 1; k < n; ++k) t -= L[k * n + i] * y[k];
      y[i] = t / L[i * n + i];
    }
    for (int64_t i = 0; i < n; ++i) inv[i * n + c] = y[i];
  }
}

AMGHier amg_setup(const CSR& A0, int max_levels, int64_t min_rows, double max_ratio) {
  AMGHier H;
  H.lv.push_back(AMGLevel());
  H.lv.back().A = A0;
  while (true) {
    const CSR& A = H.lv.back().A;
    int64_t n = A.nrows;
    if (n <= min_rows || (int)H.lv.size() >= max_levels) break;
    std::vector<int64_t> agg;
    int64_t na = 0;
    const double thetas[5] = {0.04, 0.02, 0.01, 0.005, 0.0};
    double theta = thetas[0];
    for (int tr = 0; tr < 5; ++tr) {
      theta = thetas[tr];
      aggregate(A, agg, na, theta);
      if ((double)na <= max_ratio * (double)n) break;
    }
    if ((double)na > max_ratio * (double)n) break;
    std::vector<double> d = csr_diag(A);
    // filtered matrix: strong entries kept, weak ones lumped on the diagonal
    std::vector<char> keep(A.idx.size(), 0);
    std::vector<double> dF(n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      double lump = 0.0;
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
        int32_t j = A.idx[q];
        if (j == i || std::fabs(A.val[q]) >= theta * std::sqrt(d[i] * d[j])) keep[q] = 1;
        else lump += A.val[q];
      }
      dF[i] = d[i] + lump;
      // a zero row sum lumps to a structural zero: such rows are not smoothed
      if (!(dF[i] > 1e-8 * d[i])) dF[i] = 0.0;
    }
    double rho = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      if (!(dF[i] > 0)) continue;
      double s = std::fabs(dF[i]);
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
        if (keep[q] && A.idx[q] != i) s += std::fabs(A.val[q]);
      rho = std::max(rho, s / dF[i]);
    }
    double w = (4.0 / 3.0) / rho;
    // P = P^ - w D_F^{-1} A_F P^ ; (A_F P^)_{i,g} = sum_{j in agg g} a^F_ij
    CSR P;
    P.nrows = n;
    P.ncols = na;
    P.ptr.assign(1, 0);
    std::vector<double> acc(na, 0.0);
    std::vector<char> used(na, 0);
    std::vector<int32_t> cols;
    for (int64_t i = 0; i < n; ++i) {
      cols.clear();
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
        if (!keep[q]) continue;
        int32_t g = (int32_t)agg[A.idx[q]];
        if (!used[g]) { used[g] = 1; acc[g] = 0.0; cols.push_back(g); }
        acc[g] += A.idx[q] == i ? dF[i] : A.val[q];
      }
      int32_t gi = (int32_t)agg[i];
      double sc = dF[i] > 0 ? -w / dF[i] : 0.0;
      for (int32_t g : cols) acc[g] = sc * acc[g];
      if (!used[gi]) { used[gi] = 1; acc[gi] = 0.0; cols.push_back(gi); }
      acc[gi] += 1.0;
      std::sort(cols.begin(), cols.end());
      for (int32_t g : cols) {
        used[g] = 0;
        if (acc[g] == 0.0) continue;
        P.idx.push_back(g);
        P.val.push_back(acc[g]);
      }
      P.ptr.push_back((int64_t)P.idx.size());
    }
    CSR R = csr_transpose(P);
    CSR Ac = csr_matmul(R, csr_matmul(A, P));
    if (std::getenv("HPDG_VERBOSE"))
      std::fprintf(stderr, "hpdg amg: level %zu rows %lld nnz %lld theta %.3g -> %lld aggregates, nnz(P) %lld, nnz(A_c) %lld\n",
                   H.lv.size() - 1, (long long)n, (long long)A.idx.size(), theta, (long long)na,
                   (long long)P.idx.size(), (long long)Ac.idx.size());
    H.lv.back().P = std::move(P);
    H.lv.back().R = std::move(R);
    H.aggs.push_back(std::move(agg));
    AMGLevel next;
    next.A = std::move(Ac);
    H.lv.push_back(std::move(next));
  }
  for (auto& L : H.lv) {
    L.l1.assign(L.A.nrows, 0.0);
    for (int64_t i = 0; i < L.A.nrows; ++i)
      for (int64_t q = L.A.ptr[i]; q < L.A.ptr[i + 1]; ++q) L.l1[i] += std::fabs(L.A.val[q]);
  }
  H.nc = H.lv.back().A.nrows;
  if (H.nc > 4096) throw Error(-6, "AMG coarsening stalled with " + std::to_string(H.nc) + " rows on the coarsest level");
  if (H.nc > 0) dense_cholesky_inverse(H.lv.back().A, H.coarse_inv);
  return H;
}

}  // namespace hpdg
