// C ABI of the hp-DG solver: setup, operator applications, PCG (see
// include/hpdg.h for the contract of every entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <array>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/hpdg.h"
#include "internal.hpp"
#include "kernels.hip"

using namespace hpdg;

static thread_local std::string g_err;

extern "C" const char* hpdg_last_error(void) { return g_err.c_str(); }

static hpdg_status fail(int code, const std::string& msg) {
  g_err = msg;
  return (hpdg_status)code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t _e = (x);                                                               \
    if (_e != hipSuccess) throw Error(HPDG_E_HIP, std::string(#x) + ": " + hipGetErrorString(_e)); \
  } while (0)

struct hpdg_mesh {
  std::unique_ptr<Mesh> M;
  int64_t anchor_n;
  std::vector<int32_t> level, anchor, degree;
  std::vector<double> kcoef;
  int dim, n_base;
};

// device bytes allocated by this thread; in a counting pass (g_dry) buffers
// record their sizes and nothing is allocated or copied
static thread_local int64_t g_dev_bytes = 0;
static thread_local bool g_dry = false;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      if (p) (void)hipFree(p);
      p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t b) {
    if (p) { (void)hipFree(p); p = nullptr; }
    bytes = b;
    if (b == 0) return;
    if (g_dry) { g_dev_bytes += (int64_t)b; return; }
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) g_dev_bytes += (int64_t)b;
    if (e != hipSuccess)
      throw Error(HPDG_E_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
  }
  template <typename T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty() && !g_dry) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  template <typename T>
  T* as() const { return (T*)p; }
};

struct DevCSR {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  int lpr = 1;                 // lanes per short row
  int nlong = 0;               // rows longer than longrow, one wavefront each
  int longrow = 32;
  // several RHS with nrhs a multiple of 64: a thread per (row, RHS) instead
  // of a wavefront per (row, 64 RHS) (HPDG_SPMM_THREAD=1 at upload; same results)
  bool spmm_thread = false;
  DevBuf ptr, idx, val, rows;  // rows: long rows first, then short rows
};
constexpr int kLongRow = 128;   // entries (32 four-entry chunks)

void bin_rows(const CSR& A, DevCSR& D, int longrow, int lpr);

// Device CSR: every row padded to a multiple of 4 entries (value 0, column
// of the row's last entry), so that the one-RHS product reads 4-entry
// chunks with vector loads; kernels that walk a row entry by entry add the
// padding's zero products and get the same sums. pad = false keeps the rows
// as they are (a matrix only such kernels read).
template <typename T>
void upload_csr(const CSR& A, DevCSR& D, bool pad = true) {
  const int64_t n = A.nrows;
  {
    const char* v = std::getenv("HPDG_SPMM_THREAD");
    D.spmm_thread = v && std::atoi(v) != 0;
  }
  const int64_t rm = pad ? 3 : 0;
  std::vector<int32_t> p32((size_t)n + 1);
  int64_t tot = 0;
  for (int64_t i = 0; i < n; ++i) {
    p32[i] = (int32_t)tot;
    tot += (A.ptr[i + 1] - A.ptr[i] + rm) & ~rm;
    if (tot > (int64_t)INT32_MAX) throw Error(HPDG_E_UNSUPPORTED, "matrix too large");
  }
  p32[n] = (int32_t)tot;
  std::vector<int32_t> idx((size_t)tot, 0);
  std::vector<T> v((size_t)tot, T(0));
  for (int64_t i = 0; i < n; ++i) {
    int64_t o = p32[i];
    for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q, ++o) {
      idx[o] = A.idx[q];
      v[o] = (T)A.val[q];
    }
    const int32_t last = A.ptr[i + 1] > A.ptr[i] ? A.idx[A.ptr[i + 1] - 1] : 0;
    for (; o < p32[i + 1]; ++o) idx[o] = last;
  }
  D.nrows = (int)n;
  D.ncols = (int)A.ncols;
  D.nnz = (int64_t)A.idx.size();
  D.ptr.upload(p32);
  D.idx.upload(idx);
  D.val.upload(v);
  bin_rows(A, D, kLongRow, 0);
}

// Row binning of a CSR matrix for the one-RHS kernels: rows longer than
// `longrow` entries get one wavefront each (listed first), the others `lpr`
// lanes (0: from the average number of 4-entry chunks of the short rows).
void bin_rows(const CSR& A, DevCSR& D, int longrow, int lpr) {
  std::vector<int32_t> lr, sr;
  int64_t snnz = 0;
  for (int64_t i = 0; i < A.nrows; ++i) {
    int64_t len = A.ptr[i + 1] - A.ptr[i];
    if (len > longrow) lr.push_back((int32_t)i);
    else { sr.push_back((int32_t)i); snnz += len; }
  }
  D.nlong = (int)lr.size();
  D.longrow = longrow;
  lr.insert(lr.end(), sr.begin(), sr.end());
  D.rows.upload(lr);
  double avg = sr.empty() ? 0.0 : 0.25 * (double)snnz / (double)sr.size();
  D.lpr = lpr > 0 ? lpr : avg > 12 ? 16 : avg > 6 ? 8 : avg > 2.5 ? 4 : avg > 1.5 ? 2 : 1;
}

struct PrecHost {
  std::vector<double> diag, dinvJ;
  std::vector<int8_t> lab;
  std::vector<std::vector<int64_t>> blocks;
  CSR P, PT, AC;
  AMGHier amg;
};

// pinned host area the device writes the CG flags and norms into
struct PinArea {
  int act[256];
  int iact[256], iters[256], err[256];
  double tol2[256], bb[256], rr[256], trr[256];
};

// state of one PCG solve that advances in chunks of iterations
struct PcgRun {
  int phase = 0;               // 0 idle, 1 iterating, 2 finishing, 3 finished
  const double* b = nullptr;
  double* x = nullptr;
  int nrhs = 1, maxit = 0, enq = 0, checked = 0;
  hipStream_t s = nullptr;
  std::chrono::steady_clock::time_point t0;
  int code = 0;
  std::string msg;
  std::vector<hpdg_solve_info> info;
};

constexpr int64_t kHistCap = 2048;   // Lanczos coefficients kept per solve

struct LevelDev {
  DevCSR A, P, R;
  DevCSR M, U;           // fused cycle: R (I - A D) and [2D - D A D, P - D A P]
  CSR hM, hU;            // host copies of M and U (row binning by the tuner)
  int fused = 0;
  int has_fused = 0;
  DevBuf tail;           // T, n x n: the whole cycle from this level down (see set_tail)
  int use_tail = 0;
  DevBuf l1inv;          // T
  DevBuf b, x, r, t;     // T, nrows * max_nrhs
};

// Work vectors of one application of B in the preconditioner's precision:
// the copies of r and z, and per AMG level the right-hand side b, the
// iterate x, the residual r and the temporary t of the V-cycle. They come
// from the operator's buffers, or from the static scratch array of
// hpdg_apply_B_noalloc.
constexpr int kMaxLevels = 16;
struct BWork {
  void* rT = nullptr;
  void* zT = nullptr;
  void* b[kMaxLevels] = {};
  void* x[kMaxLevels] = {};
  void* r[kMaxLevels] = {};
  void* t[kMaxLevels] = {};
};

}  // namespace

constexpr int64_t kPreSplitNnz = 4 << 20;   // pre-smoother in two launches above this many nonzeros

struct hpdg_operator {
  int dim = 2, ne = 0, max_nrhs = 1, form = 0, prec32 = 0, host_only = 0;
  int64_t ndof = 0, nconf = 0;
  hpdg_operator_opts opts{};
  // element data
  DevBuf off, pdeg, hh, kk, sptr, recs, tab, ftab;
  TableLayout TL{};
  std::vector<std::vector<int32_t>> bucket;  // host: elements per degree
  std::vector<DevBuf> dbucket;               // device copies (index p)
  // preconditioner (type T = float or double per prec32)
  DevBuf dinvJ;
  DevBuf blk_rowb, blk_rowl, blk_ptr, blk_off, blk_dof, blk_inv;
  int64_t blk_rows = 0, nblocks = 0;
  // overlapping V_e (3D face spaces): the block solves write slot ndof + row
  // (blk_out) and each N-DOF sums its slots (g_dof, g_ptr, g_slot)
  int blk_overlap = 0;
  DevBuf blk_out, g_dof, g_ptr, g_slot;
  int64_t g_n = 0;
  int max_blk = 0;           // largest V_e block
  int lprb = 16;             // lanes per V_e block row in the B front (one RHS)
  int blk_wg = 1;            // one RHS: V_e solves by k_block_rows (a workgroup per block, r staged in
                             // LDS) instead of the row-parallel part of the B front
  DevBuf blk_order;          // blocks by decreasing size (k_block_rows)
  int no_mfma = 0;           // HPDG_NO_MFMA=1: V_e block solves for many RHS without the matrix cores
  int no_fused_multi = 0;    // HPDG_NO_FUSED_MULTI=1: fused V-cycle levels for one RHS only
  DevCSR P, PT;
  std::vector<LevelDev> lv;
  DevBuf coarse;
  int ncoarse = 0;
  DevBuf rT, zT, rc;       // T work vectors (DG and conforming sizes)
  // CG work (double)
  DevBuf r, z, pv, Ap, part, scal, iscal, ahist, bhist;
  int64_t hist_cap = 0;      // Lanczos coefficients kept per RHS
  int64_t hist_rows = 0;     // rows of them copied to hist_pin by the last solve
  int64_t ftab_bytes = 0;
  int64_t dev_bytes = 0;     // device memory held by this operator once uploaded
  double t_setup = 0.0;      // host wall time of setup (and upload)
  int uploaded = 0;
  int no_prec = 0;           // operator only: apply_B and PCG unsupported
  int use_graph = 0;         // PCG chunks replayed from captured HIP graphs
  int epb = 1;               // elements per workgroup of the 2D element kernel
  int nm3 = 9;               // LDS size class of the 3D element kernel: largest n = p + 1 (7 or 9)
  DevBuf elem_perm;          // 3D elements by decreasing cost within each XCD's share
  // 2D elements of degree <= c and > c in mesh order, c = 5..8 (index c - 5):
  // the lane-per-right-hand-side kernel and the grouped kernel of the
  // several-RHS apply
  // index 4: every element, each XCD's eighth of the mesh order sorted by
  // decreasing estimated cost (the costly elements start first)
  DevBuf e2r_lo[5], e2r_hi[5];
  int n_e2r_lo[5] = {0, 0, 0, 0, 0}, n_e2r_hi[5] = {0, 0, 0, 0, 0};
  // 3D, one RHS: the operator in three passes (k_e3_vol, k_e3_face,
  // k_e3_lift) with the side buffer and the per-record face contributions
  int split3 = 1;
  int e3xcd = 1;             // face and lift passes in XCD-aware order (HPDG_E3_FACE_XCD=0: plain)
  int e3stage = 1;           // face pass: 1D face matrices staged in LDS (1) or read through the caches (0)
  DevBuf sboff, faux, sbuf, gbuf;
  int use_perm = 1;          // 3D element kernel dispatched in that order (autotuned)
  int cg_separate = 0;       // one RHS: CG final reductions as kernels of their own
  int64_t presplit_nnz = kPreSplitNnz;   // pre-smoother in two launches above this
  // host matrices of the fused levels and dense tails, built once and kept
  // across uploads (the counting pass and the upload share them)
  struct HostCycle {
    bool fused = false, tail = false;
    CSR M, U;
    std::vector<double> T;
  };
  std::vector<HostCycle> hcyc;
  int fchunk = 16;           // face records per pass of the 2D element kernel
  int rhs_group = 1;         // right-hand sides per item of the 2D element kernel; 0: a lane per
                             // right-hand side (k_elem2d_rhs) for degrees <= 5 when nrhs > 1
  int rhs_group_hi = 4;      // with rhs_group 0: the group size of the degrees above e2r_split
  int e2r_split = 5;         // with rhs_group 0: the highest degree on the lane form (5..8), the
                             // others grouped; 9: all on the lane form in two launches (<= 5, >= 6);
                             // 10: all in one launch, by decreasing cost within each XCD's share
  struct GraphEntry {
    int k, nrhs;
    double* x;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;   // private stream the chunks are captured on
  PinArea* pin = nullptr;    // pinned host mirror of the CG flags and norms
  double* hist_pin = nullptr;
  hipEvent_t ev = nullptr;   // completion of the last enqueued PCG chunk
  // one RHS: the V_e block solves on a second stream, concurrent with the
  // V-cycle (both only read r; they write disjoint parts of B's work
  // vectors), joined before z = z_B + P e
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int b_fork = 0;
  int b_fork_env = -1;       // HPDG_B_FORK, when set
  int fork_level = 0;        // the block solves start after this V-cycle level's down-leg, -1: before the
                             // B front (autotuned)
  PcgRun run;
  ~hpdg_operator() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (aux) (void)hipStreamDestroy(aux);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (pin) (void)hipHostFree(pin);
    if (hist_pin) (void)hipHostFree(hist_pin);
    if (ev) (void)hipEventDestroy(ev);
  }
  // host copies of the element data for the upload
  struct {
    std::vector<int64_t> off;
    std::vector<int8_t> pd;
    std::vector<double> h, k, ftab, binv;
    std::vector<int32_t> sptr;
    std::vector<FaceRec> recs;
    int max_dlevel = 0;
  } up;
  PrecHost host;           // kept for export
  std::vector<double> coords;
};

// ---------------------------------------------------------------- helpers
static inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }
// blocks of the dot-product kernels (grid-stride loops; a multiple of nrhs
// threads per block): at most 1024, about 1024 elements per block
static inline int dot_grid(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 1023) / 1024)); }

extern "C" hpdg_status hpdg_setup_mesh(int dim, int n_base, int64_t n_elem, const int32_t* level,
                                       const int32_t* anchor, const int32_t* degree, const double* kcoef,
                                       hpdg_mesh** out) {
  if (!out || !level || !anchor || !degree || !kcoef) return fail(HPDG_E_INVALID, "null argument");
  *out = nullptr;
  try {
    auto* h = new hpdg_mesh();
    h->M.reset(make_mesh(dim, n_base, n_elem, level, anchor, degree, kcoef));
    h->dim = dim;
    h->n_base = n_base;
    h->level.assign(level, level + n_elem);
    h->anchor.assign(anchor, anchor + n_elem * dim);
    h->degree.assign(degree, degree + n_elem);
    h->kcoef.assign(kcoef, kcoef + n_elem);
    *out = h;
    return HPDG_OK;
  } catch (Error& e) {
    return fail(e.code, e.what());
  } catch (std::bad_alloc&) {
    return fail(HPDG_E_NOMEM, "host allocation failed");
  }
}

extern "C" hpdg_status hpdg_mesh_info(const hpdg_mesh* m, int64_t* ndof, int64_t* nface, int* jump) {
  if (!m) return fail(HPDG_E_INVALID, "null mesh");
  if (ndof) *ndof = m->M->ndof;
  if (nface) *nface = (int64_t)m->M->faces.size();
  if (jump) *jump = m->M->max_dlevel;
  return HPDG_OK;
}

extern "C" void hpdg_mesh_destroy(hpdg_mesh* m) { delete m; }

// code of the sub-interval [a, b] (finest units) inside [lo, lo+sz]
static uint8_t sub_code(int64_t a, int64_t b, int64_t lo, int64_t sz) {
  int64_t len = b - a;
  int delta = 0;
  while ((sz >> delta) > len) ++delta;
  int64_t idx = (a - lo) / len;
  return (uint8_t)((1 << delta) + idx);
}

static void build_tables(hpdg_operator* op, int max_delta) {
  TableLayout& L = op->TL;
  if (max_delta > 7) throw Error(HPDG_E_UNSUPPORTED, "level jump across a face larger than 7");
  std::vector<double> T;
  L.dside = (int64_t)T.size();
  T.resize(T.size() + 9 * 2 * 9, 0.0);
  for (int p = 1; p <= kMaxP; ++p)
    for (int i = 0; i <= p; ++i) {
      T[L.dside + (p * 2 + 0) * 9 + i] = basis(p).D0[i];
      T[L.dside + (p * 2 + 1) * 9 + i] = basis(p).D1[i];
    }
  L.minv = (int64_t)T.size();
  T.resize(T.size() + 9 * 81, 0.0);
  for (int p = 1; p <= kMaxP; ++p)
    for (size_t i = 0; i < basis(p).Minv.size(); ++i) T[L.minv + p * 81 + i] = basis(p).Minv[i];
  L.mk = (int64_t)T.size();
  T.resize(T.size() + 9 * 2 * 81, 0.0);
  for (int p = 1; p <= kMaxP; ++p)
    for (size_t i = 0; i < basis(p).M.size(); ++i) {
      T[L.mk + (p * 2 + 0) * 81 + i] = basis(p).M[i];
      T[L.mk + (p * 2 + 1) * 81 + i] = basis(p).K[i];
    }
  L.total = (int64_t)T.size();
  op->tab.upload(T);
  if (g_dry) return;
  // constant-memory M, K for the volume kernels: the same for every operator,
  // uploaded once per device
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, 0);
  if (!done[dev]) {
    std::vector<double> mk(9 * 2 * 81, 0.0);
    for (int p = 1; p <= kMaxP; ++p)
      for (size_t i = 0; i < basis(p).M.size(); ++i) {
        mk[(p * 2 + 0) * 81 + i] = basis(p).M[i];
        mk[(p * 2 + 1) * 81 + i] = basis(p).K[i];
      }
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_MK), mk.data(), mk.size() * sizeof(double)));
    HIPCHK(hipDeviceSynchronize());
    done[dev] = 1;
  }
}

// sum_k a[k] b[k] in four interleaved partial sums (vectorisable; fixed order)
static inline double dot4(const double* a, const double* b, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    s0 += a[k] * b[k];
    s1 += a[k + 1] * b[k + 1];
    s2 += a[k + 2] * b[k + 2];
    s3 += a[k + 3] * b[k + 3];
  }
  for (; k < n; ++k) s0 += a[k] * b[k];
  return (s0 + s1) + (s2 + s3);
}

// inverse of an SPD matrix (row-major, in place) by Cholesky A = L L^T (row
// by row, each entry one dot product of two rows), W = L^{-1},
// A^{-1} = W^T W; throws if A is not positive definite
static void spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(A);
  // rows in groups of four: each finished row j below the group is read once
  // for the four rows' entries in column j (same sums as row by row)
  for (int i0 = 0; i0 < n; i0 += 4) {
    const int i1 = std::min(n, i0 + 4);
    for (int j = 0; j < i0; ++j) {
      const double* lj = &L[(size_t)j * n];
      for (int i = i0; i < i1; ++i) {
        double* li = &L[(size_t)i * n];
        li[j] = (li[j] - dot4(li, lj, j)) / lj[j];
      }
    }
    for (int i = i0; i < i1; ++i) {
      double* li = &L[(size_t)i * n];
      for (int j = i0; j < i; ++j) {
        const double* lj = &L[(size_t)j * n];
        li[j] = (li[j] - dot4(li, lj, j)) / lj[j];
      }
      const double s = li[i] - dot4(li, li, i);
      if (!(s > 0)) throw Error(HPDG_E_NOT_SPD, "V_e block is not positive definite");
      li[i] = std::sqrt(s);
    }
  }
  // W lower triangular, row by row: W[i][j] = (delta_ij - sum_{j<=k<i} L[i][k] W[k][j]) / L[i][i]
  std::vector<double> W((size_t)n * n, 0.0);
  for (int i0 = 0; i0 < n; i0 += 4) {
    const int i1 = std::min(n, i0 + 4);
    // rows of W below the group are final: each is read once for the group
    for (int k = 0; k < i0; ++k) {
      const double* wk = &W[(size_t)k * n];
      for (int i = i0; i < i1; ++i) {
        const double lik = L[(size_t)i * n + k];
        double* wi = &W[(size_t)i * n];
        for (int j = 0; j <= k; ++j) wi[j] -= lik * wk[j];
      }
    }
    for (int i = i0; i < i1; ++i) {
      const double inv = 1.0 / L[(size_t)i * n + i];
      double* wi = &W[(size_t)i * n];
      for (int k = i0; k < i; ++k) {
        const double lik = L[(size_t)i * n + k];
        const double* wk = &W[(size_t)k * n];
        for (int j = 0; j <= k; ++j) wi[j] -= lik * wk[j];
      }
      for (int j = 0; j < i; ++j) wi[j] *= inv;
      wi[i] = inv;
    }
  }
  // A^{-1}[i][k] = sum_{m >= max(i,k)} W[m][i] W[m][k]: rows of A in groups
  // of four, each row of W read once per group
  std::fill(A.begin(), A.end(), 0.0);
  for (int i0 = 0; i0 < n; i0 += 4) {
    const int i1 = std::min(n, i0 + 4);
    for (int m = i0; m < n; ++m) {
      const double* wm = &W[(size_t)m * n];
      for (int i = i0; i < i1 && i <= m; ++i) {
        const double a = wm[i];
        double* ai = &A[(size_t)i * n];
        for (int k = 0; k <= i; ++k) ai[k] += a * wm[k];
      }
    }
  }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < i; ++k) A[(size_t)k * n + i] = A[(size_t)i * n + k];
}

constexpr int64_t kFuseNnz = 4 << 20;   // levels the fused cycle is tried on (nonzeros of A)
constexpr int kTailMax = 2048;          // largest level the dense tail is tried on (rows)
constexpr int kAutoTail = 512;          // largest level auto_cycle gives the dense tail (rows)
constexpr int64_t kAutoFuse = 256 << 10; // largest level auto_cycle fuses (nonzeros of A): small,
                                         // launch-bound levels whose products are cheap to form
template <typename T>
static void set_tail(hpdg_operator* op, size_t l, bool on);

// host matrices of a fused V-cycle level, with D = diag(1/l1):
//   M = R (I - A D)                       (down-leg: b_c = M b)
//   U = [2D - D A D | P - D A P]          (up-leg: x = U [b; x_c])
// The up-leg is the V(1,1) post-steps t = D b + P x_c, x = t + D (b - A t)
// written as one product over the concatenated vector [b; x_c].
static void fused_mats(const AMGLevel& L, CSR& M, CSR& U) {
  CSR RA = csr_matmul(L.R, L.A);
  std::vector<int64_t> r;
  std::vector<int32_t> cc;
  std::vector<double> v;
  for (int64_t i = 0; i < L.R.nrows; ++i) {
    for (int64_t q = L.R.ptr[i]; q < L.R.ptr[i + 1]; ++q) {
      r.push_back(i);
      cc.push_back(L.R.idx[q]);
      v.push_back(L.R.val[q]);
    }
    for (int64_t q = RA.ptr[i]; q < RA.ptr[i + 1]; ++q) {
      r.push_back(i);
      cc.push_back(RA.idx[q]);
      v.push_back(-RA.val[q] / L.l1[RA.idx[q]]);
    }
  }
  M = csr_from_triplets(L.R.nrows, L.R.ncols, r, cc, v);
  const CSR AP = csr_matmul(L.A, L.P);
  const int64_t n = L.A.nrows;
  U = CSR();
  U.nrows = n;
  U.ncols = n + L.P.ncols;
  U.ptr.assign(n + 1, 0);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < n; ++i) {
    const double di = 1.0 / L.l1[i];
    row.clear();
    row.push_back({(int32_t)i, 2.0 * di});
    for (int64_t q = L.A.ptr[i]; q < L.A.ptr[i + 1]; ++q) {
      const int32_t j = L.A.idx[q];
      row.push_back({j, -di * L.A.val[q] / L.l1[j]});
    }
    for (int64_t q = L.P.ptr[i]; q < L.P.ptr[i + 1]; ++q) row.push_back({(int32_t)(n + L.P.idx[q]), L.P.val[q]});
    for (int64_t q = AP.ptr[i]; q < AP.ptr[i + 1]; ++q) row.push_back({(int32_t)(n + AP.idx[q]), -di * AP.val[q]});
    std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t t = 0; t < row.size(); ++t) {
      if (t > 0 && row[t].first == row[t - 1].first) { U.val.back() += row[t].second; continue; }
      U.idx.push_back(row[t].first);
      U.val.push_back(row[t].second);
    }
    U.ptr[i + 1] = (int64_t)U.idx.size();
  }
}

template <typename T>
static void set_fused(hpdg_operator* op, size_t l, bool on) {
  LevelDev& D = op->lv[l];
  if (on && !D.has_fused) {
    if (op->hcyc.size() < op->lv.size()) op->hcyc.resize(op->lv.size());
    auto& hc = op->hcyc[l];
    if (!hc.fused) {
      fused_mats(op->host.amg.lv[l], hc.M, hc.U);
      hc.fused = true;
    }
    D.hM = hc.M;
    D.hU = hc.U;
    upload_csr<T>(D.hM, D.M);
    upload_csr<T>(D.hU, D.U);
    D.has_fused = 1;
  }
  if (!on && D.has_fused) {
    D.M = DevCSR();
    D.U = DevCSR();
    D.hM = CSR();
    D.hU = CSR();
    D.has_fused = 0;
  }
  D.fused = on ? 1 : 0;
}

// rows of B's z work vector: the DG vector, plus one slot per block row when
// the V_e overlap
static int64_t zt_rows(const hpdg_operator* op) { return op->ndof + (op->blk_overlap ? op->blk_rows : 0); }

// the stored inverses (host: blocks packed m x m one after another) in the
// device layout, rows padded to blk_ld(m) entries
template <typename T>
static std::vector<T> padded_blocks(const std::vector<std::vector<int64_t>>& blocks, const std::vector<double>& binv) {
  size_t tot = 0;
  for (auto& B : blocks) tot += B.size() * (size_t)blk_ld((int)B.size());
  std::vector<T> out(tot, T(0));
  size_t so = 0, d = 0;
  for (auto& B : blocks) {
    const int m = (int)B.size(), ld = blk_ld(m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) out[d + (size_t)i * ld + j] = (T)binv[so + (size_t)i * m + j];
    so += (size_t)m * m;
    d += (size_t)m * ld;
  }
  return out;
}

template <typename T>
static void upload_prec(hpdg_operator* op) {
  PrecHost& H = op->host;
  std::vector<T> dj(H.dinvJ.begin(), H.dinvJ.end());
  op->dinvJ.upload(dj);
  // blocks
  std::vector<int32_t> rowb, rowl, bdof;
  std::vector<int64_t> bptr{0}, boff{0};
  std::vector<T> binv;
  for (size_t b = 0; b < H.blocks.size(); ++b) {
    const auto& B = H.blocks[b];
    int m = (int)B.size();
    for (int i = 0; i < m; ++i) bdof.push_back((int32_t)B[i]);
    bptr.push_back(bptr.back() + m);
    boff.push_back(boff.back() + (int64_t)m * blk_ld(m));
  }
  // the row list of the row-parallel block solves: largest blocks first (their
  // rows take longest), the rows of a block together
  std::vector<int32_t> border(H.blocks.size());
  std::iota(border.begin(), border.end(), 0);
  std::stable_sort(border.begin(), border.end(),
                   [&](int32_t a, int32_t b) { return H.blocks[a].size() > H.blocks[b].size(); });
  for (int32_t b : border)
    for (int i = 0; i < (int)H.blocks[b].size(); ++i) { rowb.push_back(b); rowl.push_back(i); }
  op->blk_rows = (int64_t)rowb.size();
  op->nblocks = (int64_t)H.blocks.size();
  op->max_blk = 0;
  for (auto& B : H.blocks) op->max_blk = std::max(op->max_blk, (int)B.size());
  op->blk_rowb.upload(rowb);
  op->blk_rowl.upload(rowl);
  op->blk_order.upload(border);
  op->blk_ptr.upload(bptr);
  op->blk_off.upload(boff);
  op->blk_dof.upload(bdof);
  // overlapping spaces: output slots past the DG vector and, per N-DOF, the
  // slots to sum (in block order)
  {
    std::vector<int32_t> cnt(op->ndof, 0);
    bool overlap = false;
    for (int32_t g : bdof) overlap |= ++cnt[g] > 1;
    op->blk_overlap = overlap ? 1 : 0;
    op->blk_out = DevBuf();
    op->g_dof = DevBuf();
    op->g_ptr = DevBuf();
    op->g_slot = DevBuf();
    op->g_n = 0;
    if (overlap) {
      if (op->ndof + (int64_t)bdof.size() > (int64_t)INT32_MAX)
        throw Error(HPDG_E_UNSUPPORTED, "DOFs plus block rows exceed 2^31");
      std::vector<int32_t> out(bdof.size());
      for (size_t q = 0; q < bdof.size(); ++q) out[q] = (int32_t)(op->ndof + (int64_t)q);
      std::vector<int32_t> gdof, gptr{0}, gslot;
      std::vector<int32_t> first(op->ndof + 1, 0);
      for (int64_t g = 0; g < op->ndof; ++g) first[g + 1] = first[g] + cnt[g];
      std::vector<int32_t> fill(first.begin(), first.end() - 1), slots(bdof.size());
      for (size_t q = 0; q < bdof.size(); ++q) slots[fill[bdof[q]]++] = out[q];   // block order
      for (int64_t g = 0; g < op->ndof; ++g) {
        if (cnt[g] == 0) continue;
        gdof.push_back((int32_t)g);
        for (int32_t q = first[g]; q < first[g + 1]; ++q) gslot.push_back(slots[q]);
        gptr.push_back((int32_t)gslot.size());
      }
      op->blk_out.upload(out);
      op->g_dof.upload(gdof);
      op->g_ptr.upload(gptr);
      op->g_slot.upload(gslot);
      op->g_n = (int64_t)gdof.size();
    }
  }
  // block inverses were computed in FP64 (binv64) during setup
  op->blk_inv.alloc(0);
  upload_csr<T>(H.P, op->P, false);   // read row by row (k_prolong_out): no padding
  upload_csr<T>(H.PT, op->PT);
  if (H.amg.lv.size() > (size_t)kMaxLevels) throw Error(HPDG_E_UNSUPPORTED, "too many AMG levels");
  op->lv.clear();
  op->lv.resize(H.amg.lv.size());
  for (size_t l = 0; l < H.amg.lv.size(); ++l) {
    const AMGLevel& L = H.amg.lv[l];
    LevelDev& D = op->lv[l];
    upload_csr<T>(L.A, D.A);
    if (l + 1 < H.amg.lv.size()) {
      upload_csr<T>(L.P, D.P);
      upload_csr<T>(L.R, D.R);
    }
    std::vector<T> li(L.l1.size());
    for (size_t i = 0; i < li.size(); ++i) li[i] = (T)(1.0 / L.l1[i]);
    D.l1inv.upload(li);
    size_t nb = (size_t)L.A.nrows * op->max_nrhs * sizeof(T);
    D.b.alloc(nb);
    D.x.alloc(nb);
    D.r.alloc(nb);
    D.t.alloc(nb);
  }
  std::vector<T> ci(H.amg.coarse_inv.begin(), H.amg.coarse_inv.end());
  op->coarse.upload(ci);
  op->ncoarse = (int)H.amg.nc;
  if (std::getenv("HPDG_FUSE_LEVELS") && !g_dry)
    for (size_t l = 0; l + 1 < op->lv.size(); ++l)
      if (op->lv[l].A.nnz <= kFuseNnz) set_fused<T>(op, l, true);
  // HPDG_DENSE_TAIL=1: the dense tail on the level above the coarsest
  if (std::getenv("HPDG_DENSE_TAIL") && !g_dry && op->lv.size() >= 2 && op->ncoarse > 0 &&
      op->lv[op->lv.size() - 2].A.nrows <= kTailMax)
    set_tail<T>(op, op->lv.size() - 2, true);
  // auto_cycle: fused levels and a small dense tail without timing (also in
  // the counting pass, so their bytes are counted; the levels are rebuilt at
  // every upload)
  if (op->opts.auto_cycle && op->lv.size() >= 2) {
    const size_t nl = op->lv.size();
    if (op->ncoarse > 0 && op->lv[nl - 2].A.nrows <= kAutoTail) set_tail<T>(op, nl - 2, true);
    for (size_t l = 0; l + 1 < nl; ++l)
      if (!op->lv[l].use_tail && op->lv[l].A.nnz <= kAutoFuse) set_fused<T>(op, l, true);
  }
  op->rT.alloc((size_t)op->ndof * op->max_nrhs * sizeof(T));
  op->zT.alloc((size_t)zt_rows(op) * op->max_nrhs * sizeof(T));
}

// second region of the share buffer (one RHS), after the largest first region
static int64_t part_off2(const hpdg_operator* op) {
  return std::max<int64_t>(op->ne, (op->ndof + 255) / 256) + 64;
}

// the second stream and its two events, created on first use
static void ensure_aux(hpdg_operator* op) {
  if (!op->aux) HIPCHK(hipStreamCreateWithFlags(&op->aux, hipStreamNonBlocking));
  if (!op->ev_fork) HIPCHK(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming));
  if (!op->ev_join) HIPCHK(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming));
}

// All device buffers of an operator from its host data. In a counting pass
// (g_dry) only the sizes are recorded. Copies are synchronous; the call ends
// with a synchronisation of `s`.
static void upload_device(hpdg_operator* op, hipStream_t s) {
  auto& U = op->up;
  const int64_t b0 = g_dev_bytes;
  op->off.upload(U.off);
  op->pdeg.upload(U.pd);
  {
    int pm = 0;
    for (int8_t v : U.pd) pm = std::max(pm, (int)v);
    op->nm3 = pm <= 6 ? 7 : 9;   // degree <= 6: LDS for 7 nodes per direction
  }
  op->hh.upload(U.h);
  op->kk.upload(U.k);
  op->sptr.upload(U.sptr);
  if (op->dim == 3) {
    // cost estimate: (p+1)^4 for the volume, (p+1)^3 per face record
    const int64_t ne = (int64_t)U.pd.size();
    std::vector<int64_t> cost(ne);
    for (int64_t e = 0; e < ne; ++e) {
      const int64_t n = U.pd[e] + 1;
      cost[e] = n * n * n * n + (int64_t)(U.sptr[e * 6 + 6] - U.sptr[e * 6]) * n * n * n;
    }
    // the element kernel gives each XCD a contiguous eighth of the element
    // positions and starts its workgroups in order: within each eighth the
    // elements (a contiguous piece of the mesh) are put in decreasing cost,
    // so the heavy ones start first and the last to start are short
    std::vector<int32_t> perm(ne);
    std::iota(perm.begin(), perm.end(), 0);
    const int64_t chunk = (ne + 7) / 8;
    for (int64_t c0 = 0; c0 < ne; c0 += chunk)
      std::stable_sort(perm.begin() + c0, perm.begin() + std::min(ne, c0 + chunk),
                       [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    op->elem_perm.upload(perm);
  }
  op->recs.upload(U.recs);
  op->ftab.upload(U.ftab);
  if (op->dim == 3) {
    // side-buffer offsets (12 n^2 per element) and the per-record FaceAux
    const int64_t ne = (int64_t)U.pd.size();
    std::vector<int64_t> sbo(ne + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
      const int64_t n = U.pd[e] + 1;
      sbo[e + 1] = sbo[e] + 12 * n * n;
    }
    std::vector<FaceAux> ax(U.recs.size());
    int64_t go = 0;
    for (int64_t e = 0; e < ne; ++e) {
      const int64_t n = U.pd[e] + 1;
      for (int32_t q = U.sptr[e * 6]; q < U.sptr[e * 6 + 6]; ++q) {
        const FaceRec& r = U.recs[q];
        FaceAux& a = ax[q];
        a.h = U.h[e];
        a.k = U.k[e];
        a.p = U.pd[e];
        a.pad = 0;
        a.sb_own = sbo[e] + (2 * r.m + r.side) * 2 * n * n;
        if (r.nbr >= 0) {
          const int64_t nn = U.pd[r.nbr] + 1;
          a.sb_nbr = sbo[r.nbr] + (2 * r.m + 1 - r.side) * 2 * nn * nn;
        } else {
          a.sb_nbr = -1;
        }
        a.goff = go;
        go += 2 * n * n;
      }
    }
    const int64_t sb_total = sbo[ne];
    sbo.pop_back();
    op->sboff.upload(sbo);
    op->faux.upload(ax);
    op->sbuf.alloc((size_t)sb_total * sizeof(double));
    op->gbuf.alloc((size_t)go * sizeof(double));
  }
  build_tables(op, U.max_dlevel);
  op->dbucket.clear();
  op->dbucket.resize(kMaxP + 1);
  for (int p = 1; p <= kMaxP; ++p) op->dbucket[p].upload(op->bucket[p]);
  if (op->dim == 2) {
    std::vector<int8_t> degh((size_t)op->ne, 0);
    for (int p = 1; p <= kMaxP; ++p)
      for (int32_t e : op->bucket[p]) degh[e] = (int8_t)p;
    for (int c = 5; c <= 8; ++c) {
      std::vector<int32_t> lo, hi;
      for (int p = 1; p <= kMaxP; ++p)
        for (int32_t e : op->bucket[p]) (p <= c ? lo : hi).push_back(e);
      std::sort(lo.begin(), lo.end());
      std::sort(hi.begin(), hi.end());
      op->n_e2r_lo[c - 5] = (int)lo.size();
      op->n_e2r_hi[c - 5] = (int)hi.size();
      op->e2r_lo[c - 5].upload(lo);
      op->e2r_hi[c - 5].upload(hi);
      if (c == 8) {
        // the XCD-aware order gives XCD x the list positions [x per, (x+1) per)
        // for 64 RHS (per = ceil(n / 8)), started in list order
        // estimated cost: the volume's 4 n^3 and about 3 n^2 per face record
        const int n = (int)lo.size(), per = (n + 7) / 8;
        auto est = [&](int32_t e) {
          const int64_t q = degh[e] + 1, nrec = U.sptr[4 * (size_t)e + 4] - U.sptr[4 * (size_t)e];
          return 4 * q * q * q + 3 * nrec * q * q;
        };
        std::vector<int32_t> cost = lo;
        for (int x = 0; x < 8; ++x) {
          auto b0 = cost.begin() + std::min(n, x * per), b1 = cost.begin() + std::min(n, (x + 1) * per);
          std::stable_sort(b0, b1, [&](int32_t a, int32_t b) { return est(a) > est(b); });
        }
        op->n_e2r_lo[4] = n;
        op->e2r_lo[4].upload(cost);
      }
    }
  }
  if (op->no_prec) {
  } else if (op->prec32) {
    upload_prec<float>(op);
    op->blk_inv.upload(padded_blocks<float>(op->host.blocks, U.binv));
  } else {
    upload_prec<double>(op);
    op->blk_inv.upload(padded_blocks<double>(op->host.blocks, U.binv));
  }
  const int64_t hs = op->max_nrhs;
  size_t nv = (size_t)op->ndof * hs * sizeof(double);
  op->r.alloc(nv);
  op->z.alloc(nv);
  op->pv.alloc(nv);
  op->Ap.alloc(nv);
  // dot-product shares: 1024 blocks per RHS, or one per element / per 256 DOFs
  op->part.alloc((size_t)std::max<int64_t>(1024 * hs, 3 * part_off2(op)) * sizeof(double));
  op->scal.alloc((size_t)16 * 256 * sizeof(double));
  op->iscal.alloc((size_t)4 * 256 * sizeof(int));
  op->hist_cap = kHistCap;
  op->ahist.alloc((size_t)kHistCap * hs * sizeof(double));
  op->bhist.alloc((size_t)kHistCap * hs * sizeof(double));
  if (g_dry) return;
  HIPCHK(hipMemsetAsync(op->iscal.p, 0, 4 * 256 * sizeof(int), s));
  if (!op->pin) HIPCHK(hipHostMalloc((void**)&op->pin, sizeof(PinArea), hipHostMallocDefault));
  if (!op->hist_pin)
    HIPCHK(hipHostMalloc((void**)&op->hist_pin, (size_t)2 * kHistCap * hs * sizeof(double), hipHostMallocDefault));
  if (!op->ev) HIPCHK(hipEventCreateWithFlags(&op->ev, hipEventDisableTiming));
  // default: blocks on the second stream when their stored inverses reach
  // 32 MB (the autotuner times both)
  op->b_fork = op->b_fork_env >= 0 ? op->b_fork_env : op->blk_inv.bytes >= ((size_t)32 << 20) ? 1 : 0;
  if (op->b_fork) ensure_aux(op);
  HIPCHK(hipStreamSynchronize(s));
  op->dev_bytes = g_dev_bytes - b0;
  op->uploaded = 1;
  op->host_only = 0;
}

// device bytes the operator holds once uploaded (a counting pass if it is not)
static int64_t device_bytes(hpdg_operator* op) {
  if (op->uploaded) return op->dev_bytes;
  const int64_t b0 = g_dev_bytes;
  g_dry = true;
  try {
    upload_device(op, nullptr);
  } catch (...) {
    g_dry = false;
    g_dev_bytes = b0;
    throw;
  }
  g_dry = false;
  int64_t need = g_dev_bytes - b0;
  g_dev_bytes = b0;
  return need;
}

extern "C" hpdg_status hpdg_operator_upload(hpdg_operator* op, void* stream) {
  if (!op) return fail(HPDG_E_INVALID, "null operator");
  if (op->uploaded) return HPDG_OK;
  try {
    const auto t0 = std::chrono::steady_clock::now();
    upload_device(op, (hipStream_t)stream);
    op->t_setup += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return HPDG_OK;
  } catch (Error& e) {
    return fail(e.code, e.what());
  } catch (std::bad_alloc&) {
    return fail(HPDG_E_NOMEM, "host allocation failed");
  }
}

extern "C" hpdg_status hpdg_operator_device_bytes(hpdg_operator* op, int64_t* bytes) {
  if (!op || !bytes) return fail(HPDG_E_INVALID, "null argument");
  try {
    *bytes = device_bytes(op);
    return HPDG_OK;
  } catch (Error& e) {
    return fail(e.code, e.what());
  }
}

extern "C" hpdg_status hpdg_setup_operator(const hpdg_mesh* mh, const hpdg_operator_opts* o, void* stream,
                                          hpdg_operator** out) {
  if (!mh || !o || !out) return fail(HPDG_E_INVALID, "null argument");
  *out = nullptr;
  if (o->form != 0 && o->form != 1) return fail(HPDG_E_INVALID, "form must be 0 (SIPG) or 1 (BR2)");
  if (o->form == 0 && !(o->eta > 0)) return fail(HPDG_E_INVALID, "SIPG needs eta > 0");
  if (o->max_nrhs < 1 || o->max_nrhs > 256 || (256 % o->max_nrhs) != 0)
    return fail(HPDG_E_INVALID, "max_nrhs must divide 256");
  if (o->penalty_rule != 0 && o->penalty_rule != 1) return fail(HPDG_E_INVALID, "penalty_rule must be 0 or 1");
  const auto t_setup0 = std::chrono::steady_clock::now();
  auto op = std::make_unique<hpdg_operator>();
  {
    int nt = o->setup_threads;
    if (nt <= 0) nt = (int)std::max(1u, std::thread::hardware_concurrency());
    set_setup_threads(std::min(nt, 64));
  }
  try {
    // a private copy of the mesh: entity tables are built lazily
    std::unique_ptr<Mesh> Mp(make_mesh(mh->dim, mh->n_base, (int64_t)mh->level.size(), mh->level.data(),
                                       mh->anchor.data(), mh->degree.data(), mh->kcoef.data()));
    Mesh& M = *Mp;
    if (M.ndof > (int64_t)INT32_MAX / 2) throw Error(HPDG_E_UNSUPPORTED, "too many DOFs");
    op->opts = *o;
    op->dim = M.dim;
    op->ne = M.ne;
    op->ndof = M.ndof;
    op->max_nrhs = o->max_nrhs;
    op->form = o->form;
    op->prec32 = o->prec_fp32 ? 1 : 0;
    OpOpts oo;
    oo.form = o->form;
    oo.penalty_rule = o->penalty_rule;
    oo.eta = o->eta;
    oo.remark_relax = o->remark_relax;
    oo.jb_only = o->jb_only;
    oo.max_block = o->max_block;
    double eta2 = o->form == 1 ? br2_eta(M, oo) : 0.0;
    int d = M.dim;
    // ---- element data and face records
    std::vector<int8_t> pd(M.p.begin(), M.p.end());
    op->up.off = M.off;
    op->up.pd = pd;
    op->up.h = M.h;
    op->up.k = M.k;
    op->up.max_dlevel = M.max_dlevel;
    std::vector<std::vector<FaceRec>> per(M.ne * 2 * d);
    // 1D face-mass matrices F[j][j'] = sum_g w_g l^a_j(x^a_g) l^b_j'(x^b_g) of the
    // face's sub-intervals in each side (unit length), deduplicated by type
    std::map<std::array<int, 5>, int32_t> fmap;
    std::vector<double> ftab;
    auto sub_vals = [&](int p, int code, int q, std::vector<double>& out) {
      std::vector<double> gx, gw;
      gauss_rule(q, gx, gw);
      int delta = 0;
      while ((2 << delta) <= code) ++delta;
      double len = 1.0 / (double)(1 << delta), a = (code - (1 << delta)) * len;
      out.assign(q * (p + 1), 0.0);
      for (int g = 0; g < q; ++g) lagrange_eval(basis(p).x, a + len * gx[g], &out[g * (p + 1)]);
      return gw;
    };
    // exact integrals: the matrices depend on the degrees and codes only
    auto face_mat = [&](int p, int oc, int po, int nc) -> int32_t {
      std::array<int, 5> key{p, oc, po, nc, 0};
      auto it = fmap.find(key);
      if (it != fmap.end()) return it->second;
      int32_t at = (int32_t)ftab.size();
      int q = std::max(p, po) + 1;
      std::vector<double> Io, In;
      std::vector<double> gw = sub_vals(p, oc, q, Io);
      sub_vals(po, nc, q, In);
      int n = p + 1, no = po + 1;
      for (int j = 0; j < n; ++j)
        for (int jj = 0; jj < no; ++jj) {
          double s = 0;
          for (int g = 0; g < q; ++g) s += gw[g] * Io[g * n + j] * In[g * no + jj];
          ftab.push_back(s);
        }
      fmap.emplace(key, at);
      return at;
    };
    // BR2 liftings (3D): a face-mass matrix times the inverse 1D mass matrix
    // of its column side, L = A Minv (rows p_row+1, columns p_col+1)
    auto lift_mat = [&](int32_t a_off, int prow, int pcol, int kind, int k0, int k1, int k2, int k3) -> int32_t {
      std::array<int, 5> key{k0, k1, k2, k3, kind};
      auto it = fmap.find(key);
      if (it != fmap.end()) return it->second;
      int32_t at = (int32_t)ftab.size();
      const int nr = prow + 1, nc = pcol + 1;
      const std::vector<double>& Mi = basis(pcol).Minv;
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) {
          double s = 0;
          for (int l = 0; l < nc; ++l) s += ftab[a_off + i * nc + l] * Mi[l * nc + j];
          ftab.push_back(s);
        }
      fmap.emplace(key, at);
      return at;
    };
    for (const Face& f : M.faces) {
      double sig = penalty_or_br2(M, oo, f, eta2);
      int tdim[2] = {0, 0}, nt = 0;
      for (int t = 0; t < d; ++t)
        if (t != f.m) tdim[nt++] = t;
      int qv = std::max(M.p[f.em], f.ep >= 0 ? M.p[f.ep] : 0) + 1;
      auto make = [&](int e, int side, int nb) {
        FaceRec r;
        std::memset(&r, 0, sizeof(r));
        r.nbr = nb;
        r.side = (int8_t)side;
        r.m = (int8_t)f.m;
        r.q = (int8_t)qv;
        for (int j = 0; j < nt; ++j) {
          int t = tdim[j];
          r.oc[j] = sub_code(f.lo[t], f.hi[t], M.lo[3 * e + t], M.sz[e]);
          if (nb >= 0) r.nc[j] = sub_code(f.lo[t], f.hi[t], M.lo[3 * nb + t], M.sz[nb]);
        }
        r.flen = (double)(f.hi[tdim[0]] - f.lo[tdim[0]]) / (double)M.N;
        r.sig = sig;
        r.pn = (int8_t)(nb >= 0 ? M.p[nb] : 0);
        r.nbase = nb >= 0 ? (int32_t)M.off[nb] : 0;
        r.kho = nb >= 0 ? M.k[nb] / M.h[nb] : 0.0;
        r.hn = nb >= 0 ? M.h[nb] : 1.0;
        for (int j = 0; j < nt; ++j) {
          r.foo[j] = face_mat(M.p[e], r.oc[j], M.p[e], r.oc[j]);
          if (nb >= 0) {
            r.fon[j] = face_mat(M.p[e], r.oc[j], M.p[nb], r.nc[j]);
            r.fnn[j] = face_mat(M.p[nb], r.nc[j], M.p[nb], r.nc[j]);
          }
          if (o->form == 1 && d == 3) {
            r.loo[j] = lift_mat(r.foo[j], M.p[e], M.p[e], 1, M.p[e], r.oc[j], M.p[e], r.oc[j]);
            if (nb >= 0) r.lon[j] = lift_mat(r.fon[j], M.p[e], M.p[nb], 2, M.p[e], r.oc[j], M.p[nb], r.nc[j]);
          }
        }
        per[(size_t)e * 2 * d + 2 * f.m + side].push_back(r);
      };
      if (f.ep >= 0) {
        make(f.em, 1, f.ep);
        make(f.ep, 0, f.em);
      } else {
        make(f.em, f.side, -1);
      }
    }
    std::vector<int32_t> sptr{0};
    std::vector<FaceRec> recs;
    for (auto& v : per) {
      for (auto& r : v) recs.push_back(r);
      sptr.push_back((int32_t)recs.size());
    }
    op->host_only = o->host_only ? 1 : 0;
    op->bucket.assign(kMaxP + 1, {});
    for (int e = 0; e < M.ne; ++e) op->bucket[M.p[e]].push_back(e);
    if (ftab.size() > (size_t)INT32_MAX) throw Error(HPDG_E_UNSUPPORTED, "face table too large");
    op->ftab_bytes = (int64_t)(ftab.size() * sizeof(double));
    op->up.sptr.swap(sptr);
    op->up.recs.swap(recs);
    op->up.ftab.swap(ftab);
    // ---- preconditioner (host)
    const bool verbose = std::getenv("HPDG_VERBOSE") != nullptr;
    auto tlast = std::chrono::steady_clock::now();
    auto phase = [&](const char* name) {
      auto now = std::chrono::steady_clock::now();
      if (verbose) std::fprintf(stderr, "hpdg setup: %-12s %8.3f s\n", name, std::chrono::duration<double>(now - tlast).count());
      tlast = now;
    };
    phase("faces");
    op->no_prec = o->no_prec ? 1 : 0;
    op->use_graph = o->graph ? 1 : 0;
    if (const char* v = std::getenv("HPDG_ELEM2D_EPB")) op->epb = std::atoi(v) == 2 ? 2 : 1;
    if (const char* v = std::getenv("HPDG_ELEM2D_FCHUNK")) op->fchunk = std::atoi(v) == 8 ? 8 : std::atoi(v) == 32 ? 32 : 16;
    if (const char* v = std::getenv("HPDG_ELEM2D_RHSGROUP")) op->rhs_group = std::max(0, std::atoi(v));
    if (const char* v = std::getenv("HPDG_ELEM2D_RHSGROUP_HI")) op->rhs_group_hi = std::max(1, std::atoi(v));
    if (const char* v = std::getenv("HPDG_ELEM2D_LANE_DEG")) op->e2r_split = std::min(10, std::max(5, std::atoi(v)));
    if (const char* v = std::getenv("HPDG_NO_MFMA")) op->no_mfma = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_NO_FUSED_MULTI")) op->no_fused_multi = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_ELEM3D_COST_ORDER")) op->use_perm = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_ELEM3D_SPLIT")) op->split3 = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_E3_FACE_XCD")) op->e3xcd = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_BLOCK_WG")) op->blk_wg = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_B_FORK")) op->b_fork_env = std::atoi(v) != 0 ? 1 : 0;
    if (const char* v = std::getenv("HPDG_FORK_LEVEL")) op->fork_level = std::max(-1, std::atoi(v));
    if (const char* v = std::getenv("HPDG_BLOCK_LANES")) {
      const int l = std::atoi(v);
      op->lprb = (l == 1 || l == 2 || l == 4 || l == 8 || l == 32) ? l : 16;
    }
    if (const char* v = std::getenv("HPDG_ELEM3D_STAGE")) op->e3stage = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_CG_SEPARATE_FINALS")) op->cg_separate = std::atoi(v) != 0;
    if (const char* v = std::getenv("HPDG_PRESPLIT_NNZ")) op->presplit_nnz = std::max<int64_t>(-1, std::atoll(v));
    if (!op->no_prec) {
      PrecHost& H = op->host;
      H.diag = dg_diagonal(M, oo);
      phase("diagonal");
      H.lab = dof_labels(M, o->remark_relax);
      phase("labels");
      if (o->jb_only)
        for (auto& l : H.lab)
          if (l == 2) l = 1;
      H.blocks = M.dim == 2 ? edge_spaces(M, H.lab) : face_spaces(M, H.lab);
      if (o->max_block > 0) {
        // a space larger than max_block gets no block solve; N-DOFs left in
        // no block are handled by point Jacobi
        std::vector<std::vector<int64_t>> keep;
        std::vector<char> covered(M.ndof, 0);
        for (auto& b : H.blocks)
          if ((int)b.size() <= o->max_block) {
            for (int64_t g : b) covered[g] = 1;
            keep.push_back(std::move(b));
          }
        for (int64_t g = 0; g < M.ndof; ++g)
          if (H.lab[g] == 2 && !covered[g]) H.lab[g] = 1;
        H.blocks.swap(keep);
      }
      // inverse diagonal on V_J, +0 on interior DOFs, -0 on V_e DOFs (marks
      // the DOFs that the block solves write)
      H.dinvJ.assign(M.ndof, 0.0);
      for (int64_t g = 0; g < M.ndof; ++g) {
        if (H.lab[g] == 1) H.dinvJ[g] = 1.0 / H.diag[g];
        else if (H.lab[g] == 2) H.dinvJ[g] = -0.0;
      }
      phase("edge spaces");
      // the blocks are independent: assembled and inverted on the setup
      // threads, each into its own slice of binv (results do not depend on
      // the thread count)
      std::vector<double>& binv = op->up.binv;
      std::vector<int64_t> boff(H.blocks.size() + 1, 0);
      for (size_t b = 0; b < H.blocks.size(); ++b)
        boff[b + 1] = boff[b] + (int64_t)H.blocks[b].size() * (int64_t)H.blocks[b].size();
      binv.assign((size_t)boff.back(), 0.0);
      {
        const int64_t nbk = (int64_t)H.blocks.size();
        std::atomic<int64_t> next{0};
        std::mutex emu;
        int ecode = 0;
        std::string emsg;
        std::atomic<int64_t> ns_asm{0}, ns_inv{0};   // summed over threads (verbose timing)
        parallel_chunks(std::min<int64_t>(setup_threads(), std::max<int64_t>(1, nbk)),
                        [&](int64_t, int64_t, int) {
                          for (;;) {
                            const int64_t b = next.fetch_add(1);
                            if (b >= nbk) break;
                            try {
                              const auto c0 = std::chrono::steady_clock::now();
                              std::vector<double> S = dg_submatrix(M, oo, H.blocks[b], eta2);
                              const auto c1 = std::chrono::steady_clock::now();
                              spd_inverse(S, (int)H.blocks[b].size());
                              const auto c2 = std::chrono::steady_clock::now();
                              if (verbose) {
                                ns_asm += std::chrono::duration_cast<std::chrono::nanoseconds>(c1 - c0).count();
                                ns_inv += std::chrono::duration_cast<std::chrono::nanoseconds>(c2 - c1).count();
                              }
                              std::copy(S.begin(), S.end(), binv.begin() + boff[b]);
                            } catch (Error& e) {
                              std::lock_guard<std::mutex> lk(emu);
                              if (!ecode) { ecode = e.code; emsg = e.what(); }
                              next.store(nbk);
                            } catch (std::bad_alloc&) {
                              std::lock_guard<std::mutex> lk(emu);
                              if (!ecode) { ecode = HPDG_E_NOMEM; emsg = "host allocation failed"; }
                              next.store(nbk);
                            }
                          }
                        },
                        1);
        if (ecode) throw Error(ecode, emsg);
        if (verbose)
          std::fprintf(stderr, "hpdg setup:   block assembly %.3f s, inverses %.3f s (summed over threads)\n",
                       1e-9 * (double)ns_asm.load(), 1e-9 * (double)ns_inv.load());
      }
      phase("blocks");
      H.P = prolongation(M);
      phase("prolongation");
      op->nconf = M.nconf;
      H.PT = csr_transpose(H.P);
      CSR AP = lor_times(M, H.P);
      phase("lor A P");
      H.AC = csr_matmul(H.PT, AP);
      phase("lor P'(AP)");
      H.amg = amg_setup(H.AC);
      phase("amg");
    }
    // node coordinates (export)
    op->coords.assign(M.ndof * d, 0.0);
    for (int e = 0; e < M.ne; ++e) {
      const Basis1D& B = basis(M.p[e]);
      int n = M.p[e] + 1;
      for (int64_t r = 0; r < M.off[e + 1] - M.off[e]; ++r) {
        int64_t rr = r;
        for (int m = 0; m < d; ++m) {
          int i = (int)(rr % n);
          rr /= n;
          op->coords[(M.off[e] + r) * d + m] = ((double)M.lo[3 * e + m] + (double)M.sz[e] * B.x[i]) / (double)M.N;
        }
      }
    }
    if (!op->host_only) upload_device(op.get(), (hipStream_t)stream);
    op->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_setup0).count();
    *out = op.release();
    return HPDG_OK;
  } catch (Error& e) {
    return fail(e.code, e.what());
  } catch (std::bad_alloc&) {
    return fail(HPDG_E_NOMEM, "host allocation failed");
  }
}

extern "C" void hpdg_operator_destroy(hpdg_operator* op) { delete op; }

// ------------------------------------------------------------- launchers
template <int DIM, int P>
static void launch_mass_p(hpdg_operator* op, int nrhs, const double* x, double* y, hipStream_t s) {
  using S = VolShape<DIM, P>;
  int nel = (int)op->bucket[P].size();
  if (nel == 0) return;
  int nitems = nel * nrhs;
  unsigned grid = (unsigned)((nitems + S::E - 1) / S::E);
  hipLaunchKernelGGL((k_mass<DIM, P>), dim3(grid), dim3(S::BS), 0, s, op->dbucket[P].as<int32_t>(), nitems, nrhs,
                     op->off.as<int64_t>(), op->hh.as<double>(), x, y);
}

// y = M x (element mass matrices), one launch per degree present
template <int DIM>
static void launch_mass(hpdg_operator* op, int nrhs, const double* x, double* y, hipStream_t s) {
  launch_mass_p<DIM, 1>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 2>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 3>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 4>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 5>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 6>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 7>(op, nrhs, x, y, s);
  launch_mass_p<DIM, 8>(op, nrhs, x, y, s);
}

// y = A x. With pdot (one RHS) the kernel that supports it also writes
// per-element shares of x'y there and the call returns their count; 0 when
// the caller has to form x'y itself.
static int apply_A_dev(hpdg_operator* op, const double* x, double* y, int nrhs, hipStream_t s,
                       double* pdot = nullptr) {
  if (nrhs != 1) pdot = nullptr;
  const int64_t items = (int64_t)op->ne * nrhs;   // (element, RHS) pairs
  if (op->dim == 2) {
    // the element kernel with groups of rg right-hand sides per item over the
    // elements of elist (all when null)
    auto grouped = [&](int nel, const int32_t* elist, int rg) {
      const int64_t items2 = (int64_t)nel * ((nrhs + rg - 1) / rg);   // (element, RHS group) pairs
      auto launch = [&](auto epb_c, auto fc_c) {
        constexpr int EPB = decltype(epb_c)::value, FC = decltype(fc_c)::value;
        // grid a multiple of 8 workgroups of EPB items (XCD-aware order)
        const unsigned grid = 8u * (unsigned)((items2 + 8 * EPB - 1) / (8 * EPB));
        auto kern = rg > 1 ? k_elem2d<EPB, FC, true> : k_elem2d<EPB, FC, false>;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * EPB), 0, s, nel, elist, nrhs, rg, op->form,
                           op->off.as<int64_t>(), op->pdeg.as<int8_t>(), op->hh.as<double>(), op->kk.as<double>(),
                           op->sptr.as<int32_t>(), op->recs.as<FaceRec>(), op->ftab.as<double>(),
                           op->tab.as<double>(), op->TL, x, y, pdot);
      };
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      auto with_fc = [&](auto epb_c) {
        switch (op->fchunk) {
          case 8: launch(epb_c, std::integral_constant<int, 8>()); break;
          case 32: launch(epb_c, std::integral_constant<int, 32>()); break;
          default: launch(epb_c, std::integral_constant<int, 16>()); break;
        }
      };
      if (op->epb == 2) with_fc(I2());
      else with_fc(I1());
    };
    if (nrhs > 1 && op->rhs_group == 0) {
      // degrees up to e2r_split with a lane per right-hand side (one
      // wavefront per element and 64 RHS), the others grouped: at high
      // degree a wavefront of the lane form holds many values per lane and
      // runs long, which the last wavefronts of the launch wait for
      const int split = std::min(10, std::max(5, op->e2r_split));
      const int c = std::min(8, split) - 5;
      const int ng = (nrhs + 63) / 64;
      // the lane kernel over a list: up to degree 5 with two wavefronts per
      // SIMD (face loads not overlapped), higher with one (overlapped)
      auto lanes = [&](int nl, const int32_t* list, bool low) {
        if (nl <= 0) return;
        const unsigned grid = 8u * (unsigned)(((int64_t)nl * ng + 7) / 8);   // XCD-aware: multiple of 8
        hipLaunchKernelGGL((low ? k_elem2d_rhs<6, false> : k_elem2d_rhs<9, true>), dim3(grid), dim3(64), 0, s, nl,
                           list, nrhs, op->form, op->off.as<int64_t>(), op->pdeg.as<int8_t>(), op->hh.as<double>(),
                           op->kk.as<double>(), op->sptr.as<int32_t>(), op->recs.as<FaceRec>(),
                           op->ftab.as<double>(), op->tab.as<double>(), op->TL, x, y);
      };
      if (split == 10) {
        lanes(op->n_e2r_lo[4], op->e2r_lo[4].as<int32_t>(), false);
        return 0;
      }
      if (split == 9) {
        lanes(op->n_e2r_hi[0], op->e2r_hi[0].as<int32_t>(), false);
        lanes(op->n_e2r_lo[0], op->e2r_lo[0].as<int32_t>(), true);
        return 0;
      }
      lanes(op->n_e2r_lo[c], op->e2r_lo[c].as<int32_t>(), c == 0);
      if (op->n_e2r_hi[c] > 0)
        grouped(op->n_e2r_hi[c], op->e2r_hi[c].as<int32_t>(), std::max(1, std::min(nrhs, op->rhs_group_hi)));
      return 0;
    }
    grouped(op->ne, nullptr, std::max(1, std::min(nrhs, op->rhs_group)));
    return pdot ? op->ne : 0;
  } else if (nrhs == 1 && op->split3) {
    // three passes: volume and side traces, face records, lift
    const unsigned grid = 8u * (unsigned)((op->ne + 7) / 8);   // XCD-aware order: a multiple of 8
    const int32_t* perm = op->use_perm ? op->elem_perm.as<int32_t>() : nullptr;
    const int nrec = (int)(op->recs.bytes / sizeof(FaceRec));
    // face pass: four records per workgroup; XCD-aware order needs a multiple of 8
    const unsigned fgrid = op->e3xcd ? 8u * (unsigned)(((nrec + 3) / 4 + 7) / 8) : (unsigned)((nrec + 3) / 4);
    if (op->nm3 == 7) {
      hipLaunchKernelGGL(k_e3_vol<7>, dim3(grid), dim3(256), 0, s, op->ne, op->off.as<int64_t>(),
                         op->pdeg.as<int8_t>(), op->hh.as<double>(), op->kk.as<double>(), op->sboff.as<int64_t>(),
                         op->tab.as<double>(), op->TL, x, y, op->sbuf.as<double>(), perm);
      hipLaunchKernelGGL((op->e3stage ? k_e3_face<7, true> : k_e3_face<7, false>), dim3(fgrid), dim3(256), 0, s, nrec, op->e3xcd, op->form,
                         op->recs.as<FaceRec>(), op->faux.as<FaceAux>(), op->ftab.as<double>(), op->tab.as<double>(),
                         op->TL, op->sbuf.as<double>(), op->gbuf.as<double>());
    } else {
      hipLaunchKernelGGL(k_e3_vol<9>, dim3(grid), dim3(256), 0, s, op->ne, op->off.as<int64_t>(),
                         op->pdeg.as<int8_t>(), op->hh.as<double>(), op->kk.as<double>(), op->sboff.as<int64_t>(),
                         op->tab.as<double>(), op->TL, x, y, op->sbuf.as<double>(), perm);
      hipLaunchKernelGGL((op->e3stage ? k_e3_face<9, true> : k_e3_face<9, false>), dim3(fgrid), dim3(256), 0, s, nrec, op->e3xcd, op->form,
                         op->recs.as<FaceRec>(), op->faux.as<FaceAux>(), op->ftab.as<double>(), op->tab.as<double>(),
                         op->TL, op->sbuf.as<double>(), op->gbuf.as<double>());
    }
    hipLaunchKernelGGL(k_e3_lift, dim3(op->e3xcd ? grid : (unsigned)op->ne), dim3(256), 0, s, op->ne, op->e3xcd,
                       op->off.as<int64_t>(),
                       op->pdeg.as<int8_t>(), op->hh.as<double>(), op->sptr.as<int32_t>(), op->recs.as<FaceRec>(),
                       op->faux.as<FaceAux>(), op->tab.as<double>(), op->TL, op->gbuf.as<double>(), x, y, pdot);
    return pdot ? op->ne : 0;
  } else {
    const unsigned grid = 8u * (unsigned)((items + 7) / 8);   // k_elem3d needs a multiple of 8
    auto kern = op->nm3 == 7 ? k_elem3d<7> : k_elem3d<9>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, op->ne, nrhs, op->form, op->off.as<int64_t>(),
                       op->pdeg.as<int8_t>(), op->hh.as<double>(), op->kk.as<double>(), op->sptr.as<int32_t>(),
                       op->recs.as<FaceRec>(), op->ftab.as<double>(), op->tab.as<double>(), op->TL, x, y, pdot,
                       op->use_perm ? op->elem_perm.as<int32_t>() : nullptr);
    return pdot ? op->ne : 0;
  }
  return 0;
}

template <typename T, int MODE, int LPR>
static void spmv_launch(const DevCSR& A, const T* x, const T* b, const T* d, T* xo, T* y, hipStream_t s) {
  int nshort = A.nrows - A.nlong;
  int nlb = (A.nlong + 3) / 4;
  unsigned grid = (unsigned)(nlb + nblk((int64_t)nshort * LPR));
  // MODE 5: the first nrows columns read x, the others b
  hipLaunchKernelGGL((k_spmv<T, MODE, LPR>), dim3(grid), dim3(256), 0, s, A.nlong, nlb, nshort, A.nrows,
                     A.rows.as<int32_t>(), A.ptr.as<int32_t>(), A.idx.as<int32_t>(), A.val.as<T>(), x, b, d, xo, y);
}

template <typename T, int MODE>
static void spmv(const DevCSR& A, int nrhs, const T* x, const T* b, const T* d, T* xo, T* y, hipStream_t s) {
  if (A.nrows == 0) return;
  if (nrhs == 1) {
    switch (A.lpr) {
      case 1: spmv_launch<T, MODE, 1>(A, x, b, d, xo, y, s); break;
      case 2: spmv_launch<T, MODE, 2>(A, x, b, d, xo, y, s); break;
      case 4: spmv_launch<T, MODE, 4>(A, x, b, d, xo, y, s); break;
      case 8: spmv_launch<T, MODE, 8>(A, x, b, d, xo, y, s); break;
      default: spmv_launch<T, MODE, 16>(A, x, b, d, xo, y, s); break;
    }
  } else {
    // MODE 5: the first nrows columns read x, the others b
    int64_t nt = (int64_t)A.nrows * nrhs;
    if (nrhs % 64 == 0 && !A.spmm_thread)
      hipLaunchKernelGGL((k_spmm64<T, MODE, 16>), dim3(nblk(nt)), dim3(256), 0, s, A.nrows, nrhs, A.nrows,
                         A.ptr.as<int32_t>(), A.idx.as<int32_t>(), A.val.as<T>(), x, b, d, xo, y);
    else
      hipLaunchKernelGGL((k_spmm<T, MODE>), dim3(nblk(nt)), dim3(256), 0, s, A.nrows, nrhs, A.nrows,
                         A.ptr.as<int32_t>(), A.idx.as<int32_t>(), A.val.as<T>(), x, b, d, xo, y);
  }
}

template <typename T>
static void vcycle(hpdg_operator* op, const BWork& W, size_t l, int nrhs, hipStream_t s,
                   const std::function<void()>* at_coarse = nullptr);

// Dense tail of the V-cycle: on the level just above the coarsest, one
// V(1,1) cycle is a fixed linear map of that level's right-hand side,
//   x = G b + W C M b,  with U = [G | W] and M the fused up- and down-leg
// matrices and C the dense coarsest inverse. For a small level the map is
// stored as a dense n x n matrix and the cycle is one dense product (same
// operator, other rounding). The autotuner turns it on where it is faster.

template <typename T>
static void set_tail(hpdg_operator* op, size_t l, bool on) {
  LevelDev& D = op->lv[l];
  if (!on) {
    D.tail = DevBuf();
    D.use_tail = 0;
    return;
  }
  if (D.use_tail) return;
  if (op->hcyc.size() < op->lv.size()) op->hcyc.resize(op->lv.size());
  auto& hc = op->hcyc[l];
  if (hc.tail) {
    std::vector<T> tv(hc.T.begin(), hc.T.end());
    D.tail.upload(tv);
    D.use_tail = 1;
    return;
  }
  const AMGLevel& L = op->host.amg.lv[l];
  const int64_t n = L.A.nrows, nc = op->ncoarse;
  const std::vector<double>& Cinv = op->host.amg.coarse_inv;
  if (!hc.fused) {
    fused_mats(L, hc.M, hc.U);
    hc.fused = true;
  }
  const CSR& M = hc.M;
  const CSR& U = hc.U;
  // CM = C M  (nc x n, dense)
  std::vector<double> CM((size_t)nc * n, 0.0);
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t k = 0; k < nc; ++k) {
      const double c = Cinv[(size_t)i * nc + k];
      if (c == 0.0) continue;
      for (int64_t q = M.ptr[k]; q < M.ptr[k + 1]; ++q) CM[(size_t)i * n + M.idx[q]] += c * M.val[q];
    }
  // tail = G + W (C M)
  std::vector<double> Tl((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    double* ti = &Tl[(size_t)i * n];
    for (int64_t q = U.ptr[i]; q < U.ptr[i + 1]; ++q) {
      const int64_t j = U.idx[q];
      if (j < n) ti[j] += U.val[q];
      else {
        const double w = U.val[q];
        const double* cm = &CM[(size_t)(j - n) * n];
        for (int64_t t = 0; t < n; ++t) ti[t] += w * cm[t];
      }
    }
  }
  std::vector<T> tv(Tl.begin(), Tl.end());
  D.tail.upload(tv);
  D.use_tail = 1;
  hc.T.swap(Tl);
  hc.tail = true;
}

// fused level (one RHS): two launches instead of four, same V(1,1) steps
template <typename T>
static void vcycle_fused(hpdg_operator* op, const BWork& W, size_t l, int nrhs, hipStream_t s) {
  LevelDev& L = op->lv[l];
  T *b = (T*)W.b[l], *x = (T*)W.x[l], *bc = (T*)W.b[l + 1], *xc = (T*)W.x[l + 1];
  spmv<T, 0>(L.M, nrhs, b, nullptr, nullptr, nullptr, bc, s);
  vcycle<T>(op, W, l + 1, nrhs, s);
  spmv<T, 5>(L.U, nrhs, b, xc, nullptr, nullptr, x, s);
}

// x = C b for a dense n x n matrix and nrhs > 1 interleaved right-hand sides:
// on the matrix cores when nrhs is a multiple of 16, else a workgroup per row
template <typename T>
static void dense_many(hpdg_operator* op, int n, int nrhs, const T* C, const T* b, T* x, hipStream_t s) {
  if (nrhs % 16 == 0 && !op->no_mfma)
    hipLaunchKernelGGL(k_dense_mfma<T>, dim3((unsigned)((n + 15) / 16), (unsigned)(nrhs / 16)), dim3(256), 0, s, n,
                       nrhs, C, b, x);
  else
    hipLaunchKernelGGL(k_dense_gemm<T>, dim3(n), dim3(256), 0, s, n, nrhs, C, b, x);
}

// at_coarse (if set) is called once, after the down-leg of level
// op->fork_level is enqueued (at the start of the first level below it that
// has no down-leg of its own: fused, dense tail or coarsest)
template <typename T>
static void vcycle(hpdg_operator* op, const BWork& W, size_t l, int nrhs, hipStream_t s,
                   const std::function<void()>* at_coarse) {
  T *b = (T*)W.b[l], *x = (T*)W.x[l];
  if (at_coarse && (op->lv[l].use_tail || (l + 1 < op->lv.size() && op->lv[l].fused && (nrhs == 1 || !op->no_fused_multi)) ||
                    l + 1 == op->lv.size()))
    (*at_coarse)();
  if (op->lv[l].use_tail) {
    LevelDev& L = op->lv[l];
    const int n = L.A.nrows;
    if (nrhs == 1)
      hipLaunchKernelGGL(k_dense_gemv1<T>, dim3((n + 3) / 4), dim3(256), 0, s, n, L.tail.as<T>(), b, x);
    else
      dense_many<T>(op, n, nrhs, L.tail.as<T>(), b, x, s);
    return;
  }
  if (l + 1 < op->lv.size() && op->lv[l].fused && (nrhs == 1 || !op->no_fused_multi)) {
    vcycle_fused<T>(op, W, l, nrhs, s);
    return;
  }
  LevelDev& L = op->lv[l];
  int n = L.A.nrows;
  if (l + 1 == op->lv.size()) {
    int nt = op->ncoarse * nrhs;
    if (nt == 0) return;
    if (nrhs == 1)
      hipLaunchKernelGGL(k_dense_gemv1<T>, dim3((op->ncoarse + 3) / 4), dim3(256), 0, s, op->ncoarse,
                         op->coarse.as<T>(), b, x);
    else
      dense_many<T>(op, op->ncoarse, nrhs, op->coarse.as<T>(), b, x, s);
    return;
  }
  T *r = (T*)W.r[l], *t = (T*)W.t[l], *bc = (T*)W.b[l + 1], *xc = (T*)W.x[l + 1];
  // pre-smoothing from zero and residual: x = D b, r = b - A D b; on large
  // levels x is formed first, so that the product gathers one vector
  // instead of two (the same values: x is rounded as in the fused form)
  if (nrhs == 1 && L.A.nnz > op->presplit_nnz) {
    hipLaunchKernelGGL(k_dscale<T>, dim3(nblk(n)), dim3(256), 0, s, n, L.l1inv.as<T>(), b, x);
    spmv<T, 1>(L.A, 1, x, b, nullptr, nullptr, r, s);
  } else {
    spmv<T, 3>(L.A, nrhs, b, nullptr, L.l1inv.as<T>(), x, r, s);
  }
  // restriction b_c = P^T r
  spmv<T, 0>(L.R, nrhs, r, nullptr, nullptr, nullptr, bc, s);
  const bool here = at_coarse && (int)l >= op->fork_level;
  if (here) (*at_coarse)();
  vcycle<T>(op, W, l + 1, nrhs, s, here ? nullptr : at_coarse);
  // t = x + P x_c ; x = t + D (b - A t)
  spmv<T, 2>(L.P, nrhs, xc, x, nullptr, nullptr, t, s);
  spmv<T, 4>(L.A, nrhs, t, b, L.l1inv.as<T>(), nullptr, x, s);
}

// the operator's own work vectors for B
static BWork op_work(hpdg_operator* op) {
  BWork W;
  W.rT = op->rT.p;
  W.zT = op->zT.p;
  for (size_t l = 0; l < op->lv.size(); ++l) {
    W.b[l] = op->lv[l].b.p;
    W.x[l] = op->lv[l].x.p;
    W.r[l] = op->lv[l].r.p;
    W.t[l] = op->lv[l].t.p;
  }
  return W;
}

// ------------------------------------------------------------ autotuner
// Times y = A x for one sparse matrix of the one-RHS path under every row
// binning (long-row threshold x lanes per short row) and keeps the fastest.
template <typename T>
static bool launch_front(hpdg_operator* op, const T* rt, T* zb, T* bc0, hipStream_t s, bool fork = false);
// where the block solves write: the DOF itself, or its slot when the V_e overlap
static const int32_t* blk_out(const hpdg_operator* op) {
  return op->blk_overlap ? op->blk_out.as<int32_t>() : op->blk_dof.as<int32_t>();
}

// a candidate replaces the default only when this much faster (timing noise)
constexpr double kTuneMargin = 0.95;
constexpr int64_t kCgFoldReads = 8 << 20;

template <typename T>
static void tune_csr(const CSR& H, DevCSR& D, const T* x, T* y, hipStream_t s, int64_t* rep,
                     std::function<void()> run = nullptr) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto once = [&]() {
    if (run) run();
    else spmv<T, 0>(D, 1, x, nullptr, nullptr, nullptr, y, s);
  };
  auto time_it = [&]() {
    for (int w = 0; w < 3; ++w) once();
    HIPCHK(hipEventRecord(e0, s));
    const int reps = 10;
    for (int w = 0; w < reps; ++w) once();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms * 1e6 / reps;
  };
  const int def_long = D.longrow, def_lpr = D.lpr;
  const double t_def = time_it();
  double best = t_def * kTuneMargin;
  int bl = def_long, bp = def_lpr;
  for (int longrow : {64, 128, 256, 512, 1 << 30})
    for (int lpr : {1, 2, 4, 8, 16}) {
      bin_rows(H, D, longrow, lpr);
      const double t = time_it();
      if (t < best) { best = t; bl = longrow; bp = lpr; }
    }
  if (bl == def_long && bp == def_lpr) best = t_def;
  bin_rows(H, D, bl, bp);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  rep[0] = D.nrows; rep[1] = D.nnz; rep[2] = bl; rep[3] = bp;
  rep[4] = (int64_t)t_def; rep[5] = (int64_t)best;
}

static int apply_A_dev(hpdg_operator* op, const double* x, double* y, int nrhs, hipStream_t s, double* pdot);

// elements per workgroup of the 2D element kernel (results do not depend on it)
static void tune_elem(hpdg_operator* op, hipStream_t s, int64_t* rep) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double* x = op->pv.as<double>();
  double* y = op->Ap.as<double>();
  HIPCHK(hipMemsetAsync(x, 0, op->pv.bytes, s));
  auto time_it = [&]() {
    for (int w = 0; w < 3; ++w) apply_A_dev(op, x, y, 1, s, nullptr);
    HIPCHK(hipEventRecord(e0, s));
    const int reps = 20;
    for (int w = 0; w < reps; ++w) apply_A_dev(op, x, y, 1, s, nullptr);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms * 1e6 / reps;
  };
  const int def_epb = op->epb, def_fc = op->fchunk;
  const double t_def = time_it();
  double best = t_def * kTuneMargin;
  int be = def_epb, bf = def_fc;
  for (int epb : {1, 2})
    for (int fc : {8, 16, 32}) {
      op->epb = epb;
      op->fchunk = fc;
      const double t = time_it();
      if (t < best) { best = t; be = epb; bf = fc; }
    }
  if (be == def_epb && bf == def_fc) best = t_def;
  op->epb = be;
  op->fchunk = bf;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  rep[0] = op->ndof; rep[1] = op->ne; rep[2] = bf; rep[3] = be;
  rep[4] = (int64_t)t_def; rep[5] = (int64_t)best;
}

// element order of the 3D element kernel: mesh order, or by decreasing
// estimated cost within each XCD's share (results do not depend on it)
static void tune_elem_order(hpdg_operator* op, hipStream_t s, int64_t* rep) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double* x = op->pv.as<double>();
  double* y = op->Ap.as<double>();
  HIPCHK(hipMemsetAsync(x, 0, op->pv.bytes, s));
  auto time_it = [&]() {
    for (int w = 0; w < 2; ++w) apply_A_dev(op, x, y, 1, s, nullptr);
    HIPCHK(hipEventRecord(e0, s));
    const int reps = 6;
    for (int w = 0; w < reps; ++w) apply_A_dev(op, x, y, 1, s, nullptr);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms * 1e6 / reps;
  };
  op->use_perm = 0;
  const double t0 = time_it();
  op->use_perm = 1;
  const double t1 = time_it();
  const bool keep = t1 < kTuneMargin * t0;
  op->use_perm = keep ? 1 : 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  rep[0] = op->ndof; rep[1] = op->ne; rep[2] = (int64_t)t1; rep[3] = keep ? 1 : 0;
  rep[4] = (int64_t)t0; rep[5] = (int64_t)(keep ? t1 : t0);
}

// right-hand sides per item of the 2D element kernel at the operator's
// largest nrhs (results do not depend on it)
static void tune_rhs_group(hpdg_operator* op, hipStream_t s, int64_t* rep) {
  const int nr = op->max_nrhs;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double* x = op->pv.as<double>();
  double* y = op->Ap.as<double>();
  HIPCHK(hipMemsetAsync(x, 0, op->pv.bytes, s));
  auto time_it = [&]() {
    for (int w = 0; w < 2; ++w) apply_A_dev(op, x, y, nr, s, nullptr);
    HIPCHK(hipEventRecord(e0, s));
    const int reps = 5;
    for (int w = 0; w < reps; ++w) apply_A_dev(op, x, y, nr, s, nullptr);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms * 1e6 / reps;
  };
  const int def = op->rhs_group, def_hi = op->rhs_group_hi, def_c = op->e2r_split;
  const double t_def = time_it();
  double best = t_def * kTuneMargin;
  int bg = def, bh = def_hi, bc = def_c;
  // groups for every degree, then (0) the lane form for degrees <= 5 with the
  // best group size for the others
  double tg = 0.0;
  int gg = 0;
  for (int g : {1, 2, 4, 8, 16, 32, 64}) {
    if (g > nr) break;
    op->rhs_group = g;
    const double t = time_it();
    if (gg == 0 || t < tg) { tg = t; gg = g; }
    if (t < best) { best = t; bg = g; }
  }
  if (nr > 1 && gg > 0) {
    op->rhs_group = 0;
    op->rhs_group_hi = gg;
    for (int c = 5; c <= 10; ++c) {
      op->e2r_split = c;
      const double t = time_it();
      if (t < best) { best = t; bg = 0; bh = gg; bc = c; }
    }
  }
  if (bg == def && bh == def_hi && bc == def_c) best = t_def;
  op->rhs_group = bg;
  op->rhs_group_hi = bh;
  op->e2r_split = bc;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  rep[0] = op->ndof; rep[1] = op->ne; rep[2] = bg == 0 ? bc : nr; rep[3] = bg;
  rep[4] = (int64_t)t_def; rep[5] = (int64_t)best;
}

template <typename T>
static int apply_B_dev(hpdg_operator* op, const BWork& W, const double* r, double* z, int nrhs, hipStream_t s,
                       double* pdot = nullptr, bool r_cast = false, bool allow_fork = true);

template <typename T>
static int tune_all(hpdg_operator* op, hipStream_t s, int64_t* report, int cap) {
  PrecHost& H = op->host;
  int k = 0;
  auto slot = [&](int kind, int level) -> int64_t* {
    static thread_local int64_t dummy[8];
    if (k >= cap) return dummy;
    int64_t* r = report + 8 * k++;
    r[0] = kind;
    r[1] = level;
    return r + 2;
  };
  if (op->dim == 2) {
    tune_elem(op, s, slot(4, 0));
    if (op->max_nrhs > 1) tune_rhs_group(op, s, slot(6, 0));
  }
  if (op->dim == 3) tune_elem_order(op, s, slot(10, 0));
  HIPCHK(hipMemsetAsync(op->rT.p, 0, op->rT.bytes, s));
  for (auto& L : op->lv) {
    HIPCHK(hipMemsetAsync(L.b.p, 0, L.b.bytes, s));
    HIPCHK(hipMemsetAsync(L.x.p, 0, L.x.bytes, s));
    HIPCHK(hipMemsetAsync(L.r.p, 0, L.r.bytes, s));
  }
  // P^T runs inside the B front kernel: time that kernel
  T* zb = op->zT.as<T>();
  tune_csr<T>(H.PT, op->PT, op->rT.as<T>(), op->lv[0].b.as<T>(), s, slot(3, 0),
              [&]() { launch_front<T>(op, op->rT.as<T>(), zb, op->lv[0].b.as<T>(), s); });
  // then the lanes per V_e block row of the same kernel
  if (op->blk_rows > 0) {
    hipEvent_t f0, f1;
    HIPCHK(hipEventCreate(&f0));
    HIPCHK(hipEventCreate(&f1));
    auto time_front = [&]() {
      for (int w = 0; w < 3; ++w) launch_front<T>(op, op->rT.as<T>(), zb, op->lv[0].b.as<T>(), s);
      HIPCHK(hipEventRecord(f0, s));
      for (int w = 0; w < 10; ++w) launch_front<T>(op, op->rT.as<T>(), zb, op->lv[0].b.as<T>(), s);
      HIPCHK(hipEventRecord(f1, s));
      HIPCHK(hipEventSynchronize(f1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, f0, f1));
      return (double)ms * 1e6 / 10;
    };
    // lanes per row, for the rows of all blocks in the front kernel and for
    // a workgroup per block (k_block_rows)
    const int def = op->lprb, def_wg = op->blk_wg;
    const double t_def = time_front();
    double best = t_def * kTuneMargin;
    int bb = def, bw = def_wg;
    for (int wgm : {1, 0})
      for (int lb : {1, 2, 4, 8, 16, 32}) {
        if (lb == def && wgm == def_wg) continue;
        op->lprb = lb;
        op->blk_wg = wgm;
        const double t = time_front();
        if (t < best) { best = t; bb = lb; bw = wgm; }
      }
    if (bb == def && bw == def_wg) best = t_def;
    op->lprb = bb;
    op->blk_wg = bw;
    (void)hipEventDestroy(f0);
    (void)hipEventDestroy(f1);
    int64_t* r = slot(7, 0);
    r[0] = op->blk_rows; r[1] = op->nblocks; r[2] = bw; r[3] = bb;
    r[4] = (int64_t)t_def; r[5] = (int64_t)best;
  }
  for (size_t l = 0; l < op->lv.size(); ++l) {
    LevelDev& L = op->lv[l];
    tune_csr<T>(H.amg.lv[l].A, L.A, L.b.as<T>(), L.r.as<T>(), s, slot(0, (int)l));
    if (l + 1 < op->lv.size()) {
      LevelDev& C = op->lv[l + 1];
      tune_csr<T>(H.amg.lv[l].R, L.R, L.r.as<T>(), C.b.as<T>(), s, slot(1, (int)l));
      tune_csr<T>(H.amg.lv[l].P, L.P, C.x.as<T>(), L.t.as<T>(), s, slot(2, (int)l));
    }
  }
  // fused V-cycle levels, coarsest first (the cycle below a level is settled
  // when it is timed)
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int l = (int)op->lv.size() - 2; l >= 0; --l) {
    auto time_cycle = [&]() {
      for (int w = 0; w < 3; ++w) vcycle<T>(op, op_work(op), l, 1, s);
      HIPCHK(hipEventRecord(e0, s));
      for (int w = 0; w < 10; ++w) vcycle<T>(op, op_work(op), l, 1, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      return (double)ms * 1e6 / 10;
    };
    if (l == (int)op->lv.size() - 2) set_tail<T>(op, l, false);
    if (op->lv[l].A.nnz > kFuseNnz) continue;
    set_fused<T>(op, l, false);
    const double t0 = time_cycle();
    set_fused<T>(op, l, true);
    // row binning of the two fused products, each timed alone; then the
    // fused cycle, which keeps the default binning unless the tuned one is
    // faster there too (a product timed alone runs from a hot cache)
    LevelDev& F = op->lv[l];
    LevelDev& FC = op->lv[l + 1];
    const double t_fd = time_cycle();
    int64_t um[6], uu[6];
    tune_csr<T>(F.hM, F.M, F.b.as<T>(), FC.b.as<T>(), s, um);
    tune_csr<T>(F.hU, F.U, F.b.as<T>(), F.x.as<T>(), s, uu,
                [&]() { spmv<T, 5>(F.U, 1, F.b.as<T>(), FC.x.as<T>(), nullptr, nullptr, F.x.as<T>(), s); });
    double t1 = time_cycle();
    if (!(t1 < t_fd)) {
      bin_rows(F.hM, F.M, kLongRow, 0);
      bin_rows(F.hU, F.U, kLongRow, 0);
      uu[3] = F.U.lpr;
      t1 = t_fd;
    }
    const bool keep = t1 < kTuneMargin * t0;
    if (!keep) set_fused<T>(op, l, false);
    int64_t* r = slot(5, l);
    r[0] = op->lv[l].A.nrows;
    r[1] = op->lv[l].A.nnz;
    r[2] = keep ? uu[3] : 0;
    r[3] = keep ? 1 : 0;
    r[4] = (int64_t)t0;
    r[5] = (int64_t)(keep ? t1 : t0);
    // the dense tail on the level above the coarsest, against the best above
    if (l == (int)op->lv.size() - 2 && op->lv[l].A.nrows <= kTailMax && op->ncoarse > 0) {
      const double tb = keep ? t1 : t0;
      set_tail<T>(op, l, true);
      const double tt = time_cycle();
      const bool kt = tt < kTuneMargin * tb;
      if (!kt) set_tail<T>(op, l, false);
      else if (keep) set_fused<T>(op, l, false);   // the tail replaces the fused level
      int64_t* q = slot(8, l);
      q[0] = op->lv[l].A.nrows;
      q[1] = (int64_t)op->lv[l].A.nrows * op->lv[l].A.nrows;
      q[2] = 0;
      q[3] = kt ? 1 : 0;
      q[4] = (int64_t)tb;
      q[5] = (int64_t)(kt ? tt : tb);
    }
  }
  // the V_e block solves on the second stream, concurrent with the V-cycle,
  // against one stream: whole applications of B
  if (op->nblocks > 0 && op->blk_wg && op->b_fork_env < 0) {
    ensure_aux(op);
    const BWork W = op_work(op);
    double* rin = op->pv.as<double>();
    double* zout = op->Ap.as<double>();
    HIPCHK(hipMemsetAsync(rin, 0, (size_t)op->ndof * sizeof(double), s));
    auto time_b = [&]() {
      for (int w = 0; w < 3; ++w) apply_B_dev<T>(op, W, rin, zout, 1, s);
      HIPCHK(hipEventRecord(e0, s));
      const int reps = 10;
      for (int w = 0; w < reps; ++w) apply_B_dev<T>(op, W, rin, zout, 1, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      return (double)ms * 1e6 / reps;
    };
    const int def = op->b_fork, def_lv = op->fork_level;
    const double t_def = time_b();
    double best = t_def * kTuneMargin;
    int bf = def, bl = def_lv;
    const int nlv = std::min<int>(3, (int)op->lv.size());
    for (int f : {0, 1})
      for (int lv = f ? -1 : 0; lv < (f ? nlv : 1); ++lv) {
        if (f == def && (f == 0 || lv == def_lv)) continue;
        op->b_fork = f;
        op->fork_level = lv;
        const double t = time_b();
        if (t < best) { best = t; bf = f; bl = lv; }
      }
    if (bf == def && (bf == 0 || bl == def_lv)) best = t_def;
    op->b_fork = bf;
    op->fork_level = bl;
    int64_t* r = slot(11, 0);
    r[0] = op->ndof;
    r[1] = op->nblocks;
    r[2] = op->fork_level;
    r[3] = op->b_fork;
    r[4] = (int64_t)t_def;
    r[5] = (int64_t)best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipStreamSynchronize(s));
  return k;
}

extern "C" hpdg_status hpdg_operator_tune(hpdg_operator* op, void* stream, int64_t* report, int cap, int* n) {
  if (!op || (cap > 0 && !report) || cap < 0) return fail(HPDG_E_INVALID, "bad argument");
  if (!op->uploaded) return fail(HPDG_E_UNSUPPORTED, "operator is not on the device");
  if (op->run.phase == 1 || op->run.phase == 2) return fail(HPDG_E_INVALID, "operator has a solve in flight");
  try {
    for (auto& g : op->graphs) (void)hipGraphExecDestroy(g.exec);   // captured with the old binning
    op->graphs.clear();
    hipStream_t s = (hipStream_t)stream;
    int k = 0;
    if (op->no_prec) {
      static thread_local int64_t dummy[8];
      int64_t* r = cap > 0 ? report : dummy;
      r[0] = 4;
      r[1] = 0;
      if (op->dim == 2) {
        tune_elem(op, s, r + 2);
        k = 1;
        if (op->max_nrhs > 1) {
          int64_t* r2 = cap > 1 ? report + 8 : dummy;
          r2[0] = 6;
          r2[1] = 0;
          tune_rhs_group(op, s, r2 + 2);
          k = 2;
        }
      }
    } else {
      k = op->prec32 ? tune_all<float>(op, s, report, cap) : tune_all<double>(op, s, report, cap);
    }
    if (n) *n = std::min(k, cap);
    return HPDG_OK;
  } catch (Error& e) {
    return fail(e.code, e.what());
  }
}

// front of B with one RHS: point Jacobi, V_e block solves and r_c = P^T r in
// one launch (k_front)
// V_e block solves for one RHS as a workgroup per block (k_block_rows)
template <typename T>
static void launch_block_rows(hpdg_operator* op, const T* rt, T* zb, hipStream_t s) {
  const size_t shm = (size_t)blk_ld(op->max_blk) * sizeof(T);
  auto lb = [&](auto lpr) {
    constexpr int L = decltype(lpr)::value;
    hipLaunchKernelGGL((k_block_rows<T, L>), dim3((unsigned)op->nblocks), dim3(256), shm, s, (int)op->nblocks,
                       op->blk_order.as<int32_t>(), op->blk_ptr.as<int64_t>(), op->blk_off.as<int64_t>(),
                       op->blk_dof.as<int32_t>(), blk_out(op), op->blk_inv.as<T>(), rt, zb);
  };
  switch (op->lprb) {
    case 1: lb(std::integral_constant<int, 1>()); break;
    case 2: lb(std::integral_constant<int, 2>()); break;
    case 4: lb(std::integral_constant<int, 4>()); break;
    case 8: lb(std::integral_constant<int, 8>()); break;
    case 32: lb(std::integral_constant<int, 32>()); break;
    default: lb(std::integral_constant<int, 16>()); break;
  }
}

// With fork (and the workgroup-per-block form) the block solves are left to
// the caller, which runs them on the operator's second stream; returns
// whether it must.
template <typename T>
static bool launch_front(hpdg_operator* op, const T* rt, T* zb, T* bc0, hipStream_t s, bool fork) {
  const DevCSR& A = op->PT;
  const int nb_diag = (int)nblk(op->ndof);
  const int nlb = (A.nlong + 3) / 4;
  const int nshort = A.nrows - A.nlong;
  const bool wg = op->blk_wg && op->nblocks > 0 && (size_t)blk_ld(op->max_blk) * sizeof(T) <= 64 * 1024;
  const int64_t brows = wg ? 0 : op->blk_rows;   // block solves in k_block_rows instead
  auto launch = [&](auto lprb, auto lprp) {
    constexpr int LB = decltype(lprb)::value, LP = decltype(lprp)::value;
    const int nb_blk = (int)nblk(brows * LB);
    unsigned grid = (unsigned)(nb_diag + nb_blk + nlb + (int)nblk((int64_t)nshort * LP));
    hipLaunchKernelGGL((k_front<T, LB, LP>), dim3(grid), dim3(256), 0, s, op->ndof, nb_diag, op->dinvJ.as<T>(),
                       brows, nb_blk, op->blk_rowb.as<int32_t>(), op->blk_rowl.as<int32_t>(),
                       op->blk_ptr.as<int64_t>(), op->blk_off.as<int64_t>(), op->blk_dof.as<int32_t>(),
                       blk_out(op), op->blk_inv.as<T>(), A.nlong, nlb, nshort, A.rows.as<int32_t>(), A.ptr.as<int32_t>(),
                       A.idx.as<int32_t>(), A.val.as<T>(), rt, zb, bc0);
  };
  auto with_lprp = [&](auto lprb) {
    switch (A.lpr) {
      case 1: launch(lprb, std::integral_constant<int, 1>()); break;
      case 2: launch(lprb, std::integral_constant<int, 2>()); break;
      case 4: launch(lprb, std::integral_constant<int, 4>()); break;
      case 8: launch(lprb, std::integral_constant<int, 8>()); break;
      default: launch(lprb, std::integral_constant<int, 16>()); break;
    }
  };
  switch (op->lprb) {
    case 1: with_lprp(std::integral_constant<int, 1>()); break;
    case 2: with_lprp(std::integral_constant<int, 2>()); break;
    case 4: with_lprp(std::integral_constant<int, 4>()); break;
    case 8: with_lprp(std::integral_constant<int, 8>()); break;
    case 32: with_lprp(std::integral_constant<int, 32>()); break;
    default: with_lprp(std::integral_constant<int, 16>()); break;
  }
  fork = fork && wg && op->aux;
  if (wg && !fork) launch_block_rows<T>(op, rt, zb, s);
  return fork;
}

// z = B r with the work vectors W. With pdot (one RHS) the last kernel also
// writes per-block shares of r'z there; returns their count (0 without pdot).
// allow_fork: the block solves may use the operator's second stream (not for
// callers that may overlap another call on the same operator)
template <typename T>
static int apply_B_dev(hpdg_operator* op, const BWork& W, const double* r, double* z, int nrhs, hipStream_t s,
                       double* pdot, bool r_cast, bool allow_fork) {
  int64_t n = op->ndof * nrhs;
  const T* rt;
  T* zb = (T*)W.zT;
  T* rT = (T*)W.rT;
  const bool lowp = !std::is_same<T, double>::value;
  if (!lowp) rt = (const T*)r;
  else if (nrhs == 1 && r_cast) {
    rt = rT;   // written by the CG update together with r
  } else if (nrhs == 1) {
    hipLaunchKernelGGL((k_cast<double, T>), dim3(nblk(n)), dim3(256), 0, s, n, r, rT);
    rt = rT;
  } else {
    // the cast and the point Jacobi part in one pass
    hipLaunchKernelGGL(k_cast_diag_scale<T>, dim3(nblk(n)), dim3(256), 0, s, n, nrhs, op->dinvJ.as<T>(), r, rT,
                       zb);
    rt = rT;
  }
  T* b0 = (T*)W.b[0];
  auto gather = [&](hipStream_t g) {
    if (op->blk_overlap)
      hipLaunchKernelGGL(k_block_gather<T>, dim3(nblk(op->g_n * nrhs)), dim3(256), 0, g, (int)op->g_n, nrhs,
                         op->g_dof.as<int32_t>(), op->g_ptr.as<int32_t>(), op->g_slot.as<int32_t>(), zb);
  };
  // forked: the block solves (they read only r and write only their own
  // entries of z_B) run on the second stream, started once level
  // op->fork_level's down-leg of the V-cycle is enqueued (or before the B
  // front for level -1), so that they overlap latency-bound kernels, and
  // are joined before z = z_B + P e
  std::function<void()> fork_blocks = [&]() {
    HIPCHK(hipEventRecord(op->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(op->aux, op->ev_fork, 0));
    launch_block_rows<T>(op, rt, zb, op->aux);
    gather(op->aux);
    HIPCHK(hipEventRecord(op->ev_join, op->aux));
  };
  bool forked = false, early = false;
  if (nrhs == 1) {
    const bool want = allow_fork && op->b_fork && op->aux && op->blk_wg && op->nblocks > 0 &&
                      (size_t)blk_ld(op->max_blk) * sizeof(T) <= 64 * 1024;
    if (want && op->fork_level < 0) {
      fork_blocks();
      early = true;
    }
    forked = launch_front<T>(op, rt, zb, b0, s, want);
  } else {
    if (!lowp)
      hipLaunchKernelGGL(k_diag_scale<T>, dim3(nblk(n)), dim3(256), 0, s, n, nrhs, op->dinvJ.as<T>(), rt, zb);
    if (op->blk_rows > 0) {
      int64_t nt = op->blk_rows * nrhs;
      const size_t shm = (size_t)op->max_blk * nrhs * sizeof(T);
      if (nrhs % 16 == 0 && (size_t)op->max_blk * sizeof(int32_t) <= 48 * 1024 && !op->no_mfma)
        hipLaunchKernelGGL(k_block_mfma<T>, dim3((unsigned)op->nblocks), dim3(256),
                           (size_t)op->max_blk * sizeof(int32_t), s, (int)op->nblocks, nrhs,
                           op->blk_ptr.as<int64_t>(), op->blk_off.as<int64_t>(), op->blk_dof.as<int32_t>(),
                           blk_out(op), op->blk_inv.as<T>(), rt, zb);
      else if (shm <= 48 * 1024)
        hipLaunchKernelGGL(k_block_gemm<T>, dim3((unsigned)op->nblocks), dim3(256), shm, s, (int)op->nblocks, nrhs,
                           op->blk_ptr.as<int64_t>(), op->blk_off.as<int64_t>(), op->blk_dof.as<int32_t>(),
                           blk_out(op), op->blk_inv.as<T>(), rt, zb);
      else
        hipLaunchKernelGGL(k_block_gemv<T>, dim3(nblk(nt)), dim3(256), 0, s, op->blk_rows, nrhs,
                           op->blk_rowb.as<int32_t>(), op->blk_rowl.as<int32_t>(), op->blk_ptr.as<int64_t>(),
                           op->blk_off.as<int64_t>(), op->blk_dof.as<int32_t>(), blk_out(op), op->blk_inv.as<T>(),
                           rt, zb);
    }
    spmv<T, 0>(op->PT, nrhs, rt, nullptr, nullptr, nullptr, b0, s);
  }
  if (!forked) gather(s);
  vcycle<T>(op, W, 0, nrhs, s, forked && !early ? &fork_blocks : nullptr);
  if (forked) HIPCHK(hipStreamWaitEvent(s, op->ev_join, 0));
  int64_t nt = op->ndof * nrhs;
  if (nrhs != 1) pdot = nullptr;
  hipLaunchKernelGGL(k_prolong_out<T>, dim3(nblk(nt)), dim3(256), 0, s, (int)op->ndof, nrhs,
                     op->P.ptr.as<int32_t>(), op->P.idx.as<int32_t>(), op->P.val.as<T>(), (T*)W.x[0], zb, z, r,
                     pdot);
  return pdot ? (int)nblk(nt) : 0;
}

static hpdg_status check_vec_args(hpdg_operator* op, const void* a, const void* b, int nrhs) {
  if (!op) return fail(HPDG_E_INVALID, "null operator");
  if (op->host_only) return fail(HPDG_E_UNSUPPORTED, "operator was built with host_only");
  if (!a || !b) return fail(HPDG_E_INVALID, "null vector");
  if (a == b) return fail(HPDG_E_INVALID, "input and output must not alias");
  if (nrhs < 1 || nrhs > op->max_nrhs || 256 % nrhs != 0) return fail(HPDG_E_INVALID, "bad nrhs");
  if ((int64_t)op->ne * nrhs > (int64_t)INT32_MAX || op->ndof * nrhs > (int64_t)INT32_MAX)
    return fail(HPDG_E_UNSUPPORTED, "elements x right-hand sides or DOFs x right-hand sides exceed 2^31");
  return HPDG_OK;
}

extern "C" hpdg_status hpdg_apply_A(hpdg_operator* op, const double* x, double* y, int nrhs, void* stream) {
  hpdg_status st = check_vec_args(op, x, y, nrhs);
  if (st != HPDG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  apply_A_dev(op, x, y, nrhs, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HPDG_E_HIP, hipGetErrorString(e));
  return HPDG_OK;
}

extern "C" hpdg_status hpdg_apply_B(hpdg_operator* op, const double* r, double* z, int nrhs, void* stream) {
  hpdg_status st = check_vec_args(op, r, z, nrhs);
  if (st != HPDG_OK) return st;
  if (op->no_prec) return fail(HPDG_E_UNSUPPORTED, "operator was built with no_prec");
  if (op->run.phase == 1 || op->run.phase == 2)
    return fail(HPDG_E_INVALID, "operator has a solve in flight (its work vectors are in use)");
  hipStream_t s = (hipStream_t)stream;
  const BWork W = op_work(op);
  if (op->prec32) apply_B_dev<float>(op, W, r, z, nrhs, s);
  else apply_B_dev<double>(op, W, r, z, nrhs, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HPDG_E_HIP, hipGetErrorString(e));
  return HPDG_OK;
}

// ------------------------------------------- B without device allocation
// The work vectors of hpdg_apply_B_noalloc live in this array: one copy per
// GPU, held until the process ends. Host code never passes the array's name
// to a kernel or a copy; it uses the device address that hipGetSymbolAddress
// returns for the current device (kept per device after the first call).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static hpdg_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HPDG_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HPDG_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HPDG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HPDG_OK;
}

// carves the work vectors of B for nrhs right-hand sides out of the scratch
// array at base (256-byte aligned pieces); returns the bytes needed
static size_t scratch_work(const hpdg_operator* op, int nrhs, char* base, BWork& W) {
  const size_t es = op->prec32 ? sizeof(float) : sizeof(double);
  size_t at = 0;
  auto take = [&](int64_t elems) -> void* {
    void* p = base ? base + at : nullptr;
    at += ((size_t)elems * es + 255) / 256 * 256;
    return p;
  };
  const int64_t nv = op->ndof * nrhs;
  W.rT = op->prec32 ? take(nv) : nullptr;   // FP64 B reads r itself
  W.zT = take(zt_rows(op) * nrhs);
  for (size_t l = 0; l < op->lv.size(); ++l) {
    const int64_t nl = (int64_t)op->lv[l].A.nrows * nrhs;
    W.b[l] = take(nl);
    W.x[l] = take(nl);
    W.r[l] = take(nl);
    W.t[l] = take(nl);
  }
  return at;
}

extern "C" hpdg_status hpdg_apply_B_noalloc(hpdg_operator* op, const double* r, double* z, int nrhs,
                                            void* stream) {
  hpdg_status st = check_vec_args(op, r, z, nrhs);
  if (st != HPDG_OK) return st;
  if (op->no_prec) return fail(HPDG_E_UNSUPPORTED, "operator was built with no_prec");
  BWork W;
  const size_t need = scratch_work(op, nrhs, nullptr, W);
  if (need > kScratchBytes)
    return fail(HPDG_E_INVALID, "hpdg_apply_B_noalloc: the work vectors need " + std::to_string(need) +
                                    " bytes, more than the " + std::to_string(kScratchBytes) +
                                    "-byte scratch array (use hpdg_apply_B)");
  void* base = nullptr;
  st = scratch_address(&base);
  if (st != HPDG_OK) return st;
  scratch_work(op, nrhs, (char*)base, W);
  hipStream_t s = (hipStream_t)stream;
  if (op->prec32) apply_B_dev<float>(op, W, r, z, nrhs, s, nullptr, false, false);
  else apply_B_dev<double>(op, W, r, z, nrhs, s, nullptr, false, false);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HPDG_E_HIP, hipGetErrorString(e));
  return HPDG_OK;
}

extern "C" hpdg_status hpdg_rhs(hpdg_operator* op, const double* f, double* b, int nrhs, void* stream) {
  hpdg_status st = check_vec_args(op, f, b, nrhs);
  if (st != HPDG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (op->dim == 2) launch_mass<2>(op, nrhs, f, b, s);
  else launch_mass<3>(op, nrhs, f, b, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HPDG_E_HIP, hipGetErrorString(e));
  return HPDG_OK;
}


// extreme eigenvalues of the symmetric tridiagonal Lanczos matrix by bisection
static void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lmin, double& lmax) {
  int n = (int)a.size();
  if (n == 0) { lmin = lmax = NAN; return; }
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < n ? std::fabs(b[i]) : 0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
      double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = a[i] - x - (i > 0 ? bb / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  auto kth = [&](int k) {
    double l = lo, h = hi;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (l + h);
      if (count_below(mid) > k) h = mid;
      else l = mid;
    }
    return 0.5 * (l + h);
  };
  lmin = kth(0);
  lmax = kth(n - 1);
}

// dot product with a scalar epilogue: per-block partials, then one block
// that sums them in a fixed order and updates the CG scalars
static void dot_ep(hpdg_operator* op, const double* a, const double* b, int nrhs, int mode, const CGScal& S,
                   hipStream_t s) {
  int64_t n = op->ndof * nrhs;
  const int nb = dot_grid(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, s, n, nrhs, a, b, op->part.as<double>());
  if (nrhs == 1)
    hipLaunchKernelGGL(k_dot_final_ep, dim3(1), dim3(256), 0, s, nb, nrhs, op->part.as<double>(), mode, S);
  else
    hipLaunchKernelGGL(k_dot_final_rhs, dim3(nrhs), dim3(256), 0, s, nb, nrhs, op->part.as<double>(), mode, S);
}

static CGScal cg_scal(hpdg_operator* op) {
  double* D = op->scal.as<double>();
  int* I = op->iscal.as<int>();
  CGScal S;
  S.rz = D; S.pAp = D + 256; S.rr = D + 512; S.bb = D + 768; S.alpha = D + 1024; S.beta = D + 1280;
  S.tol2 = D + 1536;
  S.rzn = D + 1792;
  S.act = I; S.iters = I + 256; S.err = I + 512;
  S.ahist = op->ahist.as<double>();
  S.bhist = op->bhist.as<double>();
  S.maxit = (int)op->hist_cap;
  S.hs = op->max_nrhs;
  return S;
}

// r_cast: the FP32 copy of in is already in rT (one RHS)
static int apply_B_any(hpdg_operator* op, const double* in, double* outv, int nrhs, hipStream_t s,
                       double* pdot = nullptr, bool r_cast = false) {
  const BWork W = op_work(op);
  if (op->prec32) return apply_B_dev<float>(op, W, in, outv, nrhs, s, pdot, r_cast);
  return apply_B_dev<double>(op, W, in, outv, nrhs, s, pdot);
}

// final stage of a dot product whose per-block shares are already in part
static void dot_final(hpdg_operator* op, int nparts, int mode, const CGScal& S, hipStream_t s) {
  if (mode == EP_PAP)
    hipLaunchKernelGGL(k_dot_final_pap, dim3(1), dim3(256), 0, s, nparts, op->part.as<double>(), S);
  else
    hipLaunchKernelGGL(k_dot_final_ep, dim3(1), dim3(256), 0, s, nparts, 1, op->part.as<double>(), mode, S);
}


// k PCG iterations (Alg. PCG: alpha from r'z / p'Ap, residual update, B
// application, beta, new direction), then the activity flags to the pinned
// area and the completion event
static void pcg_iters(hpdg_operator* op, int k, hipStream_t s);

// the HIP graph of k iterations for the current solve's x (captured once on a
// private stream, then replayed on the solve's stream)
static hipGraphExec_t chunk_graph(hpdg_operator* op, int k) {
  PcgRun& R = op->run;
  for (auto& g : op->graphs)
    if (g.k == k && g.nrhs == R.nrhs && g.x == R.x) return g.exec;
  if (!op->cap_stream) HIPCHK(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking));
  if (op->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(op->graphs.front().exec);
    op->graphs.erase(op->graphs.begin());
  }
  hipGraph_t g = nullptr;
  // relaxed: other host threads may allocate and copy while this one captures
  HIPCHK(hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeRelaxed));
  try {
    pcg_iters(op, k, op->cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(op->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHK(hipStreamEndCapture(op->cap_stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw Error(HPDG_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  op->graphs.push_back({k, R.nrhs, R.x, ex});
  return ex;
}

static void pcg_chunk(hpdg_operator* op, int k) {
  PcgRun& R = op->run;
  const int nrhs = R.nrhs;
  hipStream_t s = R.s;
  CGScal S = cg_scal(op);
  if (k > 0 && op->use_graph) HIPCHK(hipGraphLaunch(chunk_graph(op, k), s));
  else if (k > 0) pcg_iters(op, k, s);
  R.enq += k;
  HIPCHK(hipMemcpyAsync(op->pin->act, S.act, nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(op->ev, s));
}

static void pcg_iters(hpdg_operator* op, int k, hipStream_t s) {
  PcgRun& R = op->run;
  const int nrhs = R.nrhs;
  const int64_t n = op->ndof * nrhs;
  CGScal S = cg_scal(op);
  double *r = op->r.as<double>(), *z = op->z.as<double>(), *p = op->pv.as<double>(), *Ap = op->Ap.as<double>();
  double* part = op->part.as<double>();
  // one RHS, FP32 B: the update writes B's single-precision copy of r
  float* rt32 = (nrhs == 1 && op->prec32 && !op->no_prec) ? op->rT.as<float>() : nullptr;
  for (int i = 0; i < k; ++i) {
    // every block of the folded kernels re-reads all shares: kept for
    // systems where that stays small (up to 8M share reads per kernel)
    const int64_t nbk = (int64_t)nblk(n);
    const bool fold = !op->cg_separate && nbk * std::max<int64_t>(op->ne, 2 * nbk) <= kCgFoldReads;
    if (nrhs == 1 && !fold) {
      // the same with the final reductions as one-block kernels of their own
      const int na = apply_A_dev(op, p, Ap, 1, s, part);
      if (na) dot_final(op, na, EP_PAP, S, s);
      else dot_ep(op, p, Ap, 1, EP_PAP, S, s);
      hipLaunchKernelGGL(k_cg_update_rr, dim3(nblk(n)), dim3(256), 0, s, n, S.alpha, p, Ap, R.x, r, part, rt32);
      double* part2 = part + part_off2(op);
      const int nb = apply_B_any(op, r, z, 1, s, part2, rt32 != nullptr);
      hipLaunchKernelGGL(k_dot_final_rr_rz, dim3(1), dim3(256), 0, s, (int)nblk(n), part, nb, part2, S);
      hipLaunchKernelGGL(k_cg_dir2, dim3(nblk(n)), dim3(256), 0, s, n, 1, S.beta, S.act, z, p);
      continue;
    }
    if (nrhs == 1) {
      // the producers of Ap, r and z write their shares of p'Ap (first
      // region), r'r (third) and r'z (second, by the last kernel of B); the
      // final reductions run inside the update and direction kernels
      int na = apply_A_dev(op, p, Ap, 1, s, part);
      if (!na) {
        na = dot_grid(n);
        hipLaunchKernelGGL(k_dot_partial, dim3(na), dim3(256), 0, s, n, 1, p, Ap, part);
      }
      double* part2 = part + part_off2(op);
      double* part3 = part + 2 * part_off2(op);
      hipLaunchKernelGGL(k_cg_update_pap, dim3(nblk(n)), dim3(256), 0, s, n, na, part, S, p, Ap, R.x, r, part3,
                         rt32);
      const int nb = apply_B_any(op, r, z, 1, s, part2, rt32 != nullptr);
      hipLaunchKernelGGL(k_cg_dir_rr_rz, dim3(nblk(n)), dim3(256), 0, s, n, (int)nblk(n), part3, nb, part2, S,
                         z, p);
      continue;
    }
    apply_A_dev(op, p, Ap, nrhs, s, nullptr);
    dot_ep(op, p, Ap, nrhs, EP_PAP, S, s);
    // the update writes the per-RHS shares of r'r (on the grid of the dot
    // kernels, so they are bitwise those of a separate pass)
    const int g = dot_grid(n);
    hipLaunchKernelGGL(k_cg_update2, dim3(g), dim3(256), 0, s, n, nrhs, S.alpha, p, Ap, R.x, r, part);
    hipLaunchKernelGGL(k_dot_final_rhs, dim3(nrhs), dim3(256), 0, s, g, nrhs, part, EP_RR, S);
    apply_B_any(op, r, z, nrhs, s);
    dot_ep(op, r, z, nrhs, EP_RZ, S, s);
    hipLaunchKernelGGL(k_cg_dir2, dim3(nblk(n)), dim3(256), 0, s, n, nrhs, S.beta, S.act, z, p);
  }
  HIPCHK(hipGetLastError());
}

// r = b - A x, z = B r, p = z and the initial norms; no iteration yet
static void pcg_begin(hpdg_operator* op, const double* b, double* x, int nrhs, double rtol, int maxit,
                      hipStream_t s) {
  PcgRun& R = op->run;
  R = PcgRun();
  R.phase = 1;
  R.b = b;
  R.x = x;
  R.nrhs = nrhs;
  R.maxit = maxit;
  R.s = s;
  R.t0 = std::chrono::steady_clock::now();
  const int64_t n = op->ndof * nrhs;
  CGScal S = cg_scal(op);
  double *r = op->r.as<double>(), *z = op->z.as<double>(), *p = op->pv.as<double>(), *Ap = op->Ap.as<double>();
  for (int c = 0; c < nrhs; ++c) op->pin->tol2[c] = rtol * rtol;
  HIPCHK(hipMemcpyAsync(S.tol2, op->pin->tol2, nrhs * sizeof(double), hipMemcpyHostToDevice, s));
  apply_A_dev(op, x, Ap, nrhs, s);
  hipLaunchKernelGGL(k_sub, dim3(nblk(n)), dim3(256), 0, s, n, b, Ap, r);
  dot_ep(op, b, b, nrhs, EP_BB, S, s);
  dot_ep(op, r, r, nrhs, EP_RR0, S, s);
  apply_B_any(op, r, z, nrhs, s);
  HIPCHK(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  dot_ep(op, r, z, nrhs, EP_RZ0, S, s);
  HIPCHK(hipMemcpyAsync(op->pin->bb, S.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  pcg_chunk(op, 0);
}

// true residual b - A x in FP64 and the per-RHS results to the pinned area
static void pcg_finish_enqueue(hpdg_operator* op) {
  PcgRun& R = op->run;
  const int nrhs = R.nrhs;
  const int64_t n = op->ndof * nrhs;
  hipStream_t s = R.s;
  CGScal S = cg_scal(op);
  double *r = op->r.as<double>(), *Ap = op->Ap.as<double>();
  PinArea* P = op->pin;
  HIPCHK(hipMemcpyAsync(P->rr, S.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  apply_A_dev(op, R.x, Ap, nrhs, s);
  hipLaunchKernelGGL(k_sub, dim3(nblk(n)), dim3(256), 0, s, n, R.b, Ap, r);
  dot_ep(op, r, r, nrhs, EP_TRUE, S, s);
  HIPCHK(hipMemcpyAsync(P->iact, S.act, nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(P->iters, S.iters, nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(P->err, S.err, nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(P->trr, S.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  const int64_t hs = op->max_nrhs;
  const int64_t rows = std::min<int64_t>(R.enq, op->hist_cap);
  op->hist_rows = rows;
  if (rows > 0) {
    HIPCHK(hipMemcpyAsync(op->hist_pin, S.ahist, (size_t)(rows * hs) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(op->hist_pin + op->hist_cap * hs, S.bhist, (size_t)(rows * hs) * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipEventRecord(op->ev, s));
}

// per-RHS results and Lanczos extremes from the pinned area
static void pcg_collect(hpdg_operator* op) {
  PcgRun& R = op->run;
  const PinArea* P = op->pin;
  const int64_t hs = op->max_nrhs;
  const double* ha = op->hist_pin;
  const double* hb = op->hist_pin + op->hist_cap * hs;
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t0).count();
  bool all_conv = true, breakdown = false;
  R.info.assign(R.nrhs, hpdg_solve_info{});
  for (int c = 0; c < R.nrhs; ++c) {
    double bn = std::sqrt(P->bb[c]);
    bool conv = !P->iact[c] && !P->err[c];
    breakdown |= P->err[c] != 0;
    all_conv &= conv;
    hpdg_solve_info& In = R.info[c];
    In.iters = P->iters[c];
    In.converged = conv;
    In.rel_res = bn > 0 ? std::sqrt(P->rr[c]) / bn : 0.0;
    In.true_rel_res = bn > 0 ? std::sqrt(P->trr[c]) / bn : 0.0;
    int kk = (int)std::min<int64_t>(P->iters[c], op->hist_cap);
    std::vector<double> da(kk), db(kk > 0 ? kk - 1 : 0);
    for (int q = 0; q < kk; ++q) {
      double aq = ha[(size_t)q * hs + c];
      da[q] = 1.0 / aq + (q > 0 ? hb[(size_t)(q - 1) * hs + c] / ha[(size_t)(q - 1) * hs + c] : 0.0);
      if (q + 1 < kk) db[q] = std::sqrt(hb[(size_t)q * hs + c]) / aq;
    }
    tridiag_extremes(da, db, In.lambda_min, In.lambda_max);
    In.cond_est = In.lambda_max / In.lambda_min;
    In.t_solve_s = secs;
    In.t_setup_s = op->t_setup;
  }
  if (breakdown) { R.code = HPDG_E_NOT_SPD; R.msg = "CG breakdown: p'Ap <= 0 or r'z <= 0"; }
  else if (!all_conv) { R.code = HPDG_E_NOT_CONVERGED; R.msg = "maximum number of iterations reached"; }
  else R.code = HPDG_OK;
}

// one step of the state machine once the last enqueued chunk has completed:
// check the flags, then enqueue the next chunk, the final residual, or end.
// The flags are read after the first iteration and then every 4.
static void pcg_advance(hpdg_operator* op) {
  PcgRun& R = op->run;
  if (R.phase == 1) {
    if (!R.checked) {
      R.checked = 1;
      for (int c = 0; c < R.nrhs; ++c)
        if (!std::isfinite(op->pin->bb[c])) {
          R.code = HPDG_E_INVALID;
          R.msg = "non-finite right-hand side";
          R.phase = 3;
          return;
        }
    }
    bool any = false;
    for (int c = 0; c < R.nrhs; ++c) any |= op->pin->act[c] != 0;
    if (!any || R.enq >= R.maxit) {
      pcg_finish_enqueue(op);
      R.phase = 2;
      return;
    }
    int k = R.enq == 0 ? 1 : R.enq < 4 ? 4 - R.enq : 4;
    pcg_chunk(op, std::min(k, R.maxit - R.enq));
  } else if (R.phase == 2) {
    pcg_collect(op);
    R.phase = 3;
  }
}

static hpdg_status check_pcg_args(hpdg_operator* op, const double* b, double* x, int nrhs, double rtol, int maxit) {
  hpdg_status st = check_vec_args(op, b, x, nrhs);
  if (st != HPDG_OK) return st;
  if (op->no_prec) return fail(HPDG_E_UNSUPPORTED, "operator was built with no_prec");
  if (!(rtol > 0) || maxit < 0) return fail(HPDG_E_INVALID, "bad rtol or maxit");
  if (op->run.phase == 1 || op->run.phase == 2) return fail(HPDG_E_INVALID, "operator has a solve in flight");
  return HPDG_OK;
}

extern "C" hpdg_status hpdg_pcg_solve(hpdg_operator* op, const double* b, double* x, int nrhs, double rtol,
                                      int maxit, void* stream, hpdg_solve_info* info) {
  hpdg_status st = check_pcg_args(op, b, x, nrhs, rtol, maxit);
  if (st != HPDG_OK) return st;
  try {
    pcg_begin(op, b, x, nrhs, rtol, maxit, (hipStream_t)stream);
    while (op->run.phase != 3) {
      HIPCHK(hipEventSynchronize(op->ev));
      pcg_advance(op);
    }
  } catch (Error& e) {
    op->run.phase = 0;
    return fail(e.code, e.what());
  }
  PcgRun& R = op->run;
  if (info && !R.info.empty())
    for (int c = 0; c < nrhs; ++c) info[c] = R.info[c];
  if (R.code != HPDG_OK) return fail(R.code, R.msg);
  return HPDG_OK;
}

// ------------------------------------------------------- batch executor
struct hpdg_batch {
  struct Slot {
    hpdg_operator* op = nullptr;
    int64_t tag = 0;
  };
  struct Done {
    int64_t tag;
    int code;
    hpdg_solve_info info;
  };
  std::vector<hipStream_t> streams;
  std::vector<Slot> slots;
  int n_active = 0;
  std::deque<Done> done;
  ~hpdg_batch() {
    for (hipStream_t s : streams) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

extern "C" hpdg_status hpdg_batch_create(int max_active, hpdg_batch** out) {
  if (!out) return fail(HPDG_E_INVALID, "null argument");
  *out = nullptr;
  if (max_active < 1 || max_active > 64) return fail(HPDG_E_INVALID, "max_active must be in 1..64");
  auto bt = std::make_unique<hpdg_batch>();
  try {
    for (int i = 0; i < max_active; ++i) {
      hipStream_t s;
      HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      bt->streams.push_back(s);
    }
  } catch (Error& e) {
    return fail(e.code, e.what());
  }
  bt->slots.resize(max_active);
  *out = bt.release();
  return HPDG_OK;
}

extern "C" void hpdg_batch_destroy(hpdg_batch* bt) { delete bt; }

extern "C" hpdg_status hpdg_batch_admit(hpdg_batch* bt, hpdg_operator* op, const double* b, double* x, double rtol,
                                        int maxit, int64_t tag) {
  if (!bt) return fail(HPDG_E_INVALID, "null batch");
  if (op && !op->uploaded) return fail(HPDG_E_UNSUPPORTED, "operator is not on the device (hpdg_operator_upload)");
  hpdg_status st = check_pcg_args(op, b, x, 1, rtol, maxit);
  if (st != HPDG_OK) return st;
  for (auto& sl : bt->slots)
    if (sl.op == op) return fail(HPDG_E_INVALID, "operator already admitted");
  int k = -1;
  for (size_t i = 0; i < bt->slots.size(); ++i)
    if (!bt->slots[i].op) { k = (int)i; break; }
  if (k < 0) return fail(HPDG_E_BUSY, "no free slot");
  try {
    pcg_begin(op, b, x, 1, rtol, maxit, bt->streams[k]);
  } catch (Error& e) {
    op->run.phase = 0;
    return fail(e.code, e.what());
  }
  bt->slots[k].op = op;
  bt->slots[k].tag = tag;
  ++bt->n_active;
  return HPDG_OK;
}

extern "C" hpdg_status hpdg_batch_step(hpdg_batch* bt, int wait_us, int* n_active, int* n_done) {
  if (!bt) return fail(HPDG_E_INVALID, "null batch");
  auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(std::max(wait_us, 0));
  for (;;) {
    int progress = 0;
    for (auto& sl : bt->slots) {
      if (!sl.op) continue;
      hpdg_operator* op = sl.op;
      hipError_t e = hipEventQuery(op->ev);
      if (e == hipErrorNotReady) continue;
      ++progress;
      if (e != hipSuccess) {
        op->run.code = HPDG_E_HIP;
        op->run.msg = hipGetErrorString(e);
        op->run.phase = 3;
      } else {
        try {
          pcg_advance(op);
        } catch (Error& err) {
          op->run.code = err.code;
          op->run.msg = err.what();
          op->run.phase = 3;
        }
      }
      if (op->run.phase == 3) {
        hpdg_batch::Done d{sl.tag, op->run.code, hpdg_solve_info{}};
        if (!op->run.info.empty()) d.info = op->run.info[0];
        bt->done.push_back(d);
        sl.op = nullptr;
        --bt->n_active;
      }
    }
    if (progress || bt->n_active == 0 || std::chrono::steady_clock::now() >= deadline) break;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (n_active) *n_active = bt->n_active;
  if (n_done) *n_done = (int)bt->done.size();
  return HPDG_OK;
}

extern "C" hpdg_status hpdg_batch_poll(hpdg_batch* bt, int cap, int64_t* tags, int* codes, hpdg_solve_info* info,
                                       int* n) {
  if (!bt || !n || cap < 0 || (cap > 0 && (!tags || !codes))) return fail(HPDG_E_INVALID, "bad argument");
  int k = 0;
  while (k < cap && !bt->done.empty()) {
    const auto& d = bt->done.front();
    tags[k] = d.tag;
    codes[k] = d.code;
    if (info) info[k] = d.info;
    bt->done.pop_front();
    ++k;
  }
  *n = k;
  return HPDG_OK;
}

template <typename V>
static hpdg_status put(const V* src, size_t n, void* buf, size_t* bytes) {
  size_t need = n * sizeof(V);
  size_t cap = *bytes;
  *bytes = need;
  if (!buf) return HPDG_OK;
  if (cap < need) return fail(HPDG_E_INVALID, "export buffer too small");
  std::memcpy(buf, src, need);
  return HPDG_OK;
}

static std::vector<char> pack_csr(const CSR& A) {
  std::vector<char> out;
  int64_t hdr[3] = {A.nrows, A.ncols, (int64_t)A.idx.size()};
  auto app = [&](const void* p, size_t b) { const char* c = (const char*)p; out.insert(out.end(), c, c + b); };
  app(hdr, sizeof(hdr));
  app(A.ptr.data(), A.ptr.size() * 8);
  app(A.idx.data(), A.idx.size() * 4);
  app(A.val.data(), A.val.size() * 8);
  return out;
}

extern "C" hpdg_status hpdg_export(const hpdg_operator* op, int what, void* buf, size_t* bytes) {
  if (!op || !bytes) return fail(HPDG_E_INVALID, "null argument");
  const PrecHost& H = op->host;
  switch (what) {
    case 0: return put(H.diag.data(), H.diag.size(), buf, bytes);
    case 1: return put(H.lab.data(), H.lab.size(), buf, bytes);
    case 2: { auto v = pack_csr(H.P); return put(v.data(), v.size(), buf, bytes); }
    case 3: { auto v = pack_csr(H.AC); return put(v.data(), v.size(), buf, bytes); }
    case 4: {
      std::vector<int64_t> v{(int64_t)H.blocks.size(), 0};
      for (auto& b : H.blocks) v.push_back(v.back() + (int64_t)b.size());
      for (auto& b : H.blocks) v.insert(v.end(), b.begin(), b.end());
      return put(v.data(), v.size(), buf, bytes);
    }
    case 5: return put(op->coords.data(), op->coords.size(), buf, bytes);
    case 6: {
      std::vector<int64_t> v{(int64_t)H.amg.lv.size()};
      for (auto& L : H.amg.lv) v.push_back(L.A.nrows);
      for (auto& L : H.amg.lv) v.push_back((int64_t)L.A.idx.size());
      for (auto& L : H.amg.lv) v.push_back((int64_t)L.P.idx.size());
      return put(v.data(), v.size(), buf, bytes);
    }
    case 7: {
      int64_t mx = 0, ent = 0;
      for (auto& b : H.blocks) { mx = std::max<int64_t>(mx, b.size()); ent += (int64_t)b.size() * b.size(); }
      std::vector<int64_t> v{op->ndof, op->nconf, (int64_t)H.blocks.size(), mx, ent, (int64_t)H.amg.lv.size(),
                             (int64_t)H.AC.idx.size(), (int64_t)H.P.idx.size(), op->ftab_bytes, op->dev_bytes};
      return put(v.data(), v.size(), buf, bytes);
    }
    case 8: return put(op->up.binv.data(), op->up.binv.size(), buf, bytes);
    case 9: {
      // CG coefficients of the last finished solve: rows, stride (max_nrhs),
      // then alpha[rows * stride] and beta[rows * stride]
      if (op->run.phase != 3 || !op->hist_pin) return fail(HPDG_E_INVALID, "no finished solve");
      const int64_t hs = op->max_nrhs, rows = op->hist_rows;
      std::vector<double> v(2 + 2 * rows * hs);
      v[0] = (double)rows;
      v[1] = (double)hs;
      std::copy(op->hist_pin, op->hist_pin + rows * hs, v.begin() + 2);
      std::copy(op->hist_pin + op->hist_cap * hs, op->hist_pin + op->hist_cap * hs + rows * hs, v.begin() + 2 + rows * hs);
      return put(v.data(), v.size(), buf, bytes);
    }
    default:
      if (what >= 100 && what < 100 + (int)H.amg.lv.size()) {
        auto v = pack_csr(H.amg.lv[what - 100].A);
        return put(v.data(), v.size(), buf, bytes);
      }
      if (what >= 200 && what + 1 < 200 + (int)H.amg.lv.size()) {
        auto v = pack_csr(H.amg.lv[what - 200].P);
        return put(v.data(), v.size(), buf, bytes);
      }
      if (what >= 300 && what < 300 + (int)H.amg.aggs.size())
        return put(H.amg.aggs[what - 300].data(), H.amg.aggs[what - 300].size(), buf, bytes);
      return fail(HPDG_E_INVALID, "unknown export item");
  }
}
