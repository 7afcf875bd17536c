// HIP kernels for gfx950 (MI355X): DG operator, preconditioner pieces and
// CG vector operations.
//
//   k_elem2d, k_elem3d  the DG operator (Sec. 2; BR2 Sec. 4.4): volume term by
//                  sum factorisation and every face term of one element in
//                  one workgroup, faces through exact 1D face-mass matrices
//                  (conforming, mismatched-degree and nonconforming sub-faces
//                  alike); one item per (element, right-hand side).
//   k_e3_vol, k_e3_face, k_e3_lift  the 3D operator for one right-hand side
//                  in three passes (volume and side traces, one face record
//                  per wavefront, side sums lifted per element).
//   k_elem2d_rhs   the 2D operator for several right-hand sides with a lane
//                  per right-hand side (one wavefront per element and 64 RHS).
//   k_mass<DIM,P>  element mass matrices by degree bucket (the load vector).
//   k_front        B's point Jacobi, V_e block solves and P^T in one launch.
//   k_spmv, k_spmm, k_spmm64  CSR products for P, P^T and the AMG levels
//                  (one RHS; several: a thread per row and RHS, or a
//                  wavefront per row and 64 RHS), with fused smoother /
//                  residual / prolongation-add forms and the two-vector
//                  product of a fused V-cycle level's up-leg.
//   k_block_mfma, k_block_gemm, k_block_gemv, k_diag_scale  multi-RHS pieces
//                  of B (V_e block solves on the matrix cores for nrhs a
//                  multiple of 16).
//   k_dense_gemv1, k_dense_mfma, k_dense_gemm  dense products of the V-cycle
//                  (coarsest solve, dense tail) for one and for many RHS.
//   k_dot_*, k_cg_*     deterministic two-stage reductions (fixed order) with
//                  the CG scalar updates on the device, and the vector updates.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hpdg {

__constant__ double c_MK[9][2][81];

// ----------------------------------------------------------------- volume
template <int DIM, int P>
struct VolShape {
  static constexpr int n = P + 1;
  static constexpr int nn = DIM == 2 ? n * n : n * n * n;
  static constexpr int E = nn >= 256 ? 1 : 256 / nn;
  static constexpr int BS = ((E * nn + 63) / 64) * 64;
};

// y = M x with the exact element mass matrix h^d (M^ x ... x M^), one degree
// per launch (overwrites y)
template <int DIM, int P>
__global__ __launch_bounds__((VolShape<DIM, P>::BS)) void k_mass(
    const int32_t* __restrict__ elems, int nitems, int nrhs, const int64_t* __restrict__ off,
    const double* __restrict__ hh, const double* __restrict__ x, double* __restrict__ y) {
  using S = VolShape<DIM, P>;
  constexpr int n = S::n, nn = S::nn, E = S::E;
  __shared__ double sX[E * nn];
  __shared__ double sA[E * nn];
  const int slot = threadIdx.x / nn;
  const int r = threadIdx.x - slot * nn;
  const int item = blockIdx.x * E + slot;
  const bool active = slot < E && item < nitems;
  int e = 0, rr = 0;
  int64_t base = 0;
  if (active) {
    e = elems[item / nrhs];
    rr = item - (item / nrhs) * nrhs;
    base = off[e];
  }
  const double* Mt = c_MK[P][0];
  const int i0 = r % n;
  const int i1 = (r / n) % n;
  const int i2 = DIM == 3 ? r / (n * n) : 0;
  if (slot < E) sX[slot * nn + r] = active ? x[(base + r) * nrhs + rr] : 0.0;
  __syncthreads();
  // along dim 0
  if (slot < E) {
    const double* row = &sX[slot * nn + (i2 * n + i1) * n];
    double a0 = 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) a0 += row[a] * Mt[a * n + i0];
    sA[slot * nn + r] = a0;
  }
  __syncthreads();
  double out = 0.0;
  if constexpr (DIM == 2) {
    if (slot < E) {
#pragma unroll
      for (int b = 0; b < n; ++b) out += Mt[i1 * n + b] * sA[slot * nn + b * n + i0];
    }
  } else {
    // along dim 1 (into sX, no longer needed), then dim 2
    if (slot < E) {
      double aa = 0.0;
#pragma unroll
      for (int b = 0; b < n; ++b) aa += sA[slot * nn + (i2 * n + b) * n + i0] * Mt[b * n + i1];
      sX[slot * nn + r] = aa;
    }
    __syncthreads();
    if (slot < E) {
#pragma unroll
      for (int c = 0; c < n; ++c) out += Mt[c * n + i2] * sX[slot * nn + (c * n + i1) * n + i0];
    }
  }
  if (active) {
    const double h = hh[e];
    y[(base + r) * nrhs + rr] = (DIM == 3 ? h * h * h : h * h) * out;
  }
}

// 2D element kernel: volume and face terms of one element per 64-lane block,
// all degrees in one launch, y written once.
//  volume: y_K = k (K x M + M x K) x_K, 1D contractions through LDS.
//  faces:  lanes (side, j) hold the side's trace T and normal derivative D
//          at its nodes. With the 1D face-mass matrices of the face
//          A_oo = I_o^T W I_o, A_on = I_o^T W I_n, A_nn = I_n^T W I_n
//          (W = unit-length Gauss weights, I = Lagrange values of each
//          side's basis at the face's Gauss points) the tests against phi
//          (G1) and against d phi/dn (G2) are, with jump v = A_oo To - A_on Tn:
//          SIPG  G1 += L (sigma v - sgn/2 (k A_oo Do + k_o A_on Dn)),
//                G2 += -k sgn L v / 2                       (interior)
//                G1 += L (sigma A_oo To - sgn k A_oo Do), G2 += -k sgn L A_oo To
//          BR2   sigma v -> c^2 eta k_e L [s_o A_oo Minv_o v
//                                          + s_n A_on Minv_n (A_on^T To - A_nn Tn)]
//          with L the face length, s = m00 / h^2 (Sec. 2; Sec. 4.4).
//  Faces are taken seven at a time by groups of 9 lanes; each face's
//  contributions are summed per side node in record order afterwards.
//  Memory: the element's face records (kFChunk per pass: 8, 16 or 32, a
//  tuning choice between LDS use and passes) and all
//  neighbour traces are fetched in two parallel rounds into LDS before any
//  face arithmetic, so a face costs no dependent global round trip.
// every element is one wavefront: LDS exchanges between its lanes need only a
// wave-level fence, so several elements share a workgroup without barriers
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int EPB, int kFChunk, bool GROUPED>
__global__ __launch_bounds__(64 * EPB) void k_elem2d(int ne, const int32_t* __restrict__ elist, int nrhs, int rg,
                                               int form, const int64_t* __restrict__ off,
                                               const int8_t* __restrict__ pdeg, const double* __restrict__ hh,
                                               const double* __restrict__ kk, const int32_t* __restrict__ sptr,
                                               const FaceRec* __restrict__ recs, const double* __restrict__ ftab,
                                               const double* __restrict__ tab, TableLayout TL,
                                               const double* __restrict__ x, double* __restrict__ y,
                                               double* __restrict__ pdot) {
  // per element: x, the two volume temporaries (reused after the volume for
  // the face sums), the 1D mass / stiffness of its degree, side traces, and
  // one pass of face records with their neighbour traces
  __shared__ double sXw[EPB][81], sAw[EPB][81], sBw[EPB][81], sMKw[EPB][2][81], sDsw[EPB][18];
  __shared__ double sTow[EPB][4][9], sDow[EPB][4][9];
  __shared__ double sTnw[EPB][kFChunk][9], sDnw[EPB][kFChunk][9];
  __shared__ FaceRec sRw[EPB][kFChunk];
  const int wv = EPB == 1 ? 0 : (int)(threadIdx.x >> 6);
  double* sX = sXw[wv];
  double* sA = sAw[wv];
  double* sB = sBw[wv];
  double (*sTo)[9] = sTow[wv];
  double (*sDo)[9] = sDow[wv];
  // after the volume: BR2 scratch of the 7 face groups in sA, the side sums in sB
  double (*sVg)[9] = reinterpret_cast<double (*)[9]>(sAw[wv]);        // 63 of the 81
  double (*sWg)[9] = reinterpret_cast<double (*)[9]>(sBw[wv]);
  double (*sG1)[9] = reinterpret_cast<double (*)[9]>(sBw[wv]);
  double (*sG2)[9] = reinterpret_cast<double (*)[9]>(sBw[wv] + 40);
  double (*sTn)[9] = sTnw[wv];
  double (*sDn)[9] = sDnw[wv];
  FaceRec* sR = sRw[wv];
  // XCD-aware order: workgroups go round-robin to the 8 XCDs, so block b
  // takes element group (b % 8) * per + b / 8 and each XCD walks a contiguous
  // range of the (space-filling ordered) element list; neighbours then share
  // its L2
  const int per = (int)(gridDim.x >> 3);
  // one item per (element, group of rg right-hand sides), the RHS of a group
  // taken one after another (metadata, tables and records stay hot); the
  // groups of an element are consecutive items, on one XCD
  // (without GROUPED: one right-hand side per item)
  const int rgc = GROUPED ? rg : 1;
  const int ngrp = (nrhs + rgc - 1) / rgc;
  const int item = ((int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3)) * EPB + wv;
  if (item >= ne * ngrp) return;
  // elist: the elements to apply (all when null)
  const int il = item / ngrp, r0 = (item - il * ngrp) * rgc, r1 = GROUPED ? min(nrhs, r0 + rgc) : r0 + 1;
  const int e = elist ? elist[il] : il;
  const int lane = (int)(threadIdx.x & 63);
  const int gq = lane / 9, jq = lane - 9 * (lane / 9);   // face groups of 9 lanes
  const int p = pdeg[e], n = p + 1, nn = n * n;
  const double h = hh[e], k = kk[e];
  const int64_t base = off[e];
  int sp[5];
#pragma unroll
  for (int t = 0; t < 5; ++t) sp[t] = sptr[e * 4 + t];
  const double* gMK = tab + TL.mk + p * 2 * 81;          // 1D mass and stiffness of degree p
  const double* sM = sMKw[wv][0];
  const double* sK = sMKw[wv][1];
  {
    // nn <= 81: at most two entries per lane, loads issued together
    const int i0 = min(lane, nn - 1), i1 = min(lane + 64, nn - 1);
    const double m0 = gMK[i0], k0 = gMK[81 + i0], m1 = gMK[i1], k1 = gMK[81 + i1];
    if (lane < nn) {
      sMKw[wv][0][lane] = m0;
      sMKw[wv][1][lane] = k0;
    }
    if (lane + 64 < nn) {
      sMKw[wv][0][lane + 64] = m1;
      sMKw[wv][1][lane + 64] = k1;
    }
  }
  // l_i'(0), l_i'(1) of degree p
  if (lane < 18) sDsw[wv][lane] = tab[TL.dside + p * 2 * 9 + lane];
  auto fetch_records = [&](int c0, int nF) {
    constexpr int W = (int)(sizeof(FaceRec) / 8);
    constexpr int NT = (kFChunk * W + 63) / 64;   // words per lane
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(recs + c0);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(sR);
    const int nw = nF * W;
    if (nw <= 0) return;
    unsigned long long w[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) w[u] = src[min(lane + 64 * u, nw - 1)];
#pragma unroll
    for (int u = 0; u < NT; ++u)
      if (lane + 64 * u < nw) dst[lane + 64 * u] = w[u];
  };
  // an element whose face records fit one pass (nearly all) fetches them
  // here, beside its other loads, instead of after the volume; the pass never
  // rewrites them, so they serve every right-hand side of the item
  const bool onepass = sp[4] - sp[0] <= kFChunk;
  if (onepass) fetch_records(sp[0], sp[4] - sp[0]);
  for (int rhs = r0; rhs < r1; ++rhs) {
  {
    const double x0 = x[(base + min(lane, nn - 1)) * nrhs + rhs];
    const double x1 = x[(base + min(lane + 64, nn - 1)) * nrhs + rhs];
    if (lane < nn) sX[lane] = x0;
    if (lane + 64 < nn) sX[lane + 64] = x1;
  }
  wave_sync();
  // volume, phase 1 (dimension 0)
  for (int i = lane; i < nn; i += 64) {
    const int i0 = i % n, i1 = i / n;
    double t1 = 0.0, t2 = 0.0;
    for (int a = 0; a < n; ++a) {
      double xa = sX[i1 * n + a];
      t1 += xa * sK[a * n + i0];
      t2 += xa * sM[a * n + i0];
    }
    sA[i] = t1;
    sB[i] = t2;
  }
  // own traces: lane = 9*side + j
  const int sidx = lane / 9, j = lane - 9 * (lane / 9);
  const bool grp = lane < 36;
  const int m = sidx >> 1, s = sidx & 1;
  const int stm = m == 0 ? 1 : n, stt = m == 0 ? n : 1;
  if (grp && j < n) {
    const double* Ds = sDsw[wv] + s * 9;
    double dv = 0.0;
    for (int a = 0; a < n; ++a) dv += Ds[a] * sX[a * stm + j * stt];
    sTo[sidx][j] = sX[(s ? p : 0) * stm + j * stt];
    sDo[sidx][j] = dv / h;
  }
  wave_sync();
  // volume, phase 2 (dimension 1)
  double yv[2] = {0.0, 0.0};
  for (int i = lane, c = 0; i < nn; i += 64, ++c) {
    const int i0 = i % n, i1 = i / n;
    double acc = 0.0;
    for (int b = 0; b < n; ++b) acc += sM[i1 * n + b] * sA[b * n + i0] + sK[i1 * n + b] * sB[b * n + i0];
    yv[c] = k * acc;
  }
  // faces, in passes of up to kFChunk records
  double G1 = 0.0, G2 = 0.0;
  const int sb = grp ? sp[sidx] : 0, se = grp ? sp[sidx + 1] : 0;
  for (int c0 = sp[0]; c0 < sp[4]; c0 += kFChunk) {
    const int nF = min(kFChunk, sp[4] - c0);
    // first fetch: the records of this pass (already there for one pass)
    if (!onepass) {
      fetch_records(c0, nF);
      wave_sync();
    }
    // second fetch: neighbour trace Tn and k_n/h_n-scaled normal derivative Dn per (face, node)
    for (int t = lane; t < nF * 9; t += 64) {
      const int f = t / 9, jj = t - 9 * f;
      const int nb = sR[f].nbr, po = sR[f].pn;
      if (nb >= 0 && jj <= po) {
        const int no = po + 1, so = 1 - sR[f].side, mm = sR[f].m;
        const int som = mm == 0 ? 1 : no, sot = mm == 0 ? no : 1;
        const double* Dso = tab + TL.dside + (po * 2 + so) * 9;
        const double* xn = x + (int64_t)sR[f].nbase * nrhs + rhs;
        double dv = 0.0;
#pragma unroll 4
        for (int a = 0; a < no; ++a) dv += Dso[a] * xn[(int64_t)(a * som + jj * sot) * nrhs];
        sTn[f][jj] = xn[(int64_t)((so ? po : 0) * som + jj * sot) * nrhs];
        sDn[f][jj] = sR[f].kho * dv;
      }
    }
    wave_sync();
    // faces of this pass in rounds of seven: lane group g (9 lanes, one per
    // own trace node) takes face r0 + g; its contributions to the side sums
    // go to LDS in place of the face's neighbour traces
    for (int r0 = 0; r0 < nF; r0 += 7) {
      const int f = r0 + gq;
      const bool have = gq < 7 && f < nF;
      const int fr = have ? f : 0;
      const int fm = sR[fr].m, fsd = sR[fr].side, fside = 2 * fm + fsd;
      const double fsgn = fsd ? 1.0 : -1.0;
      const double flen = sR[fr].flen, sig = sR[fr].sig;
      const bool inner = have && sR[fr].nbr >= 0;
      const int po = inner ? (int)sR[fr].pn : 0;
      const int no = inner ? po + 1 : 0;
      const double* Aoo = ftab + sR[fr].foo[0];     // face matrices (cached)
      const double* Aon = ftab + (inner ? sR[fr].fon[0] : 0);
      const double* Ann = ftab + (inner ? sR[fr].fnn[0] : 0);
      const double csym = inner ? 0.5 : 1.0;
      double g1 = 0.0, g2 = 0.0, v = 0.0;
      if (have && jq < n) {
        double dsum = 0.0;
        // (unrolled so that several face-matrix loads are in flight at once)
#pragma unroll 4
        for (int a = 0; a < n; ++a) {
          v += Aoo[jq * n + a] * sTo[fside][a];
          dsum += k * Aoo[jq * n + a] * sDo[fside][a];
        }
#pragma unroll 4
        for (int a = 0; a < no; ++a) {
          v -= Aon[jq * no + a] * sTn[fr][a];
          dsum += Aon[jq * no + a] * sDn[fr][a];
        }
        g1 = -flen * csym * fsgn * dsum;
        g2 = -csym * k * fsgn * flen * v;
        if (form == 0) g1 += flen * sig * v;
      }
      if (form == 1) {
        const double c2 = inner ? 0.25 : 1.0;
        const double L2 = c2 * sig * flen * flen;
        // own lifting: g1 += L2 s_o A_oo Minv_o v
        if (have && jq < n) sVg[gq][jq] = v;
        wave_sync();
        if (have && jq < n) {
          const double* Mi = tab + TL.minv + p * 81;
          double w = 0.0;
          #pragma unroll 4
          for (int a = 0; a < n; ++a) w += Mi[jq * n + a] * sVg[gq][a];
          sWg[gq][jq] = w;
        }
        wave_sync();
        if (have && jq < n) {
          const double* Mi = tab + TL.minv + p * 81;
          const int sk = fsd ? p : 0;
          const double so = Mi[sk * n + sk] / (h * h);
          double acc = 0.0;
          #pragma unroll 4
          for (int a = 0; a < n; ++a) acc += Aoo[jq * n + a] * sWg[gq][a];
          g1 += L2 * so * acc;
        }
        // neighbour lifting: g1 += L2 s_n A_on Minv_n (A_on^T To - A_nn Tn)
        wave_sync();
        if (inner && jq < no) {
          double vn = 0.0;
          #pragma unroll 4
          for (int a = 0; a < n; ++a) vn += Aon[a * no + jq] * sTo[fside][a];
          #pragma unroll 4
          for (int a = 0; a < no; ++a) vn -= Ann[jq * no + a] * sTn[fr][a];
          sVg[gq][jq] = vn;
        }
        wave_sync();
        if (inner && jq < no) {
          const double* Mi = tab + TL.minv + po * 81;
          double w = 0.0;
          #pragma unroll 4
          for (int a = 0; a < no; ++a) w += Mi[jq * no + a] * sVg[gq][a];
          sWg[gq][jq] = w;
        }
        wave_sync();
        if (inner && jq < n) {
          const double* Mi = tab + TL.minv + po * 81;
          const int sk = (1 - fsd) ? po : 0;
          const double hn = sR[fr].hn;
          const double sn = Mi[sk * no + sk] / (hn * hn);
          double acc = 0.0;
          #pragma unroll 4
          for (int a = 0; a < no; ++a) acc += Aon[jq * no + a] * sWg[gq][a];
          g1 += L2 * sn * acc;
        }
      }
      wave_sync();
      if (have && jq < n) {
        sTn[fr][jq] = g1;
        sDn[fr][jq] = g2;
      }
    }
    wave_sync();
    // side sums in record order (deterministic)
    {
      const int fb = max(sb, c0) - c0, fe = min(se, c0 + nF) - c0;
      if (grp && j < n)
        for (int f = fb; f < fe; ++f) {
          G1 += sTn[f][j];
          G2 += sDn[f][j];
        }
    }
    wave_sync();   // sR, sTn, sDn are rewritten by the next pass
  }
  if (grp && j < n) {
    sG1[sidx][j] = G1;
    sG2[sidx][j] = G2 / h;
  }
  wave_sync();
  const double* D0 = sDsw[wv];
  const double* D1 = sDsw[wv] + 9;
  double xy = 0.0;
  for (int i = lane, c = 0; i < nn; i += 64, ++c) {
    const int i0 = i % n, i1 = i / n;
    double v = yv[c];
    v += D0[i0] * sG2[0][i1] + D1[i0] * sG2[1][i1];
    if (i0 == 0) v += sG1[0][i1];
    if (i0 == p) v += sG1[1][i1];
    v += D0[i1] * sG2[2][i0] + D1[i1] * sG2[3][i0];
    if (i1 == 0) v += sG1[2][i0];
    if (i1 == p) v += sG1[3][i0];
    y[(base + i) * nrhs + rhs] = v;
    xy += sX[i] * v;
  }
  // this element's share of x'y (the block is one wavefront), fixed order
  if (pdot) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) xy += __shfl_xor(xy, o, 64);
    if (lane == 0) pdot[e] = xy;
  }
  if (GROUPED) wave_sync();   // the next right-hand side rewrites the LDS
  }
}

// 2D element kernel for several right-hand sides: one wavefront per (element,
// 64 right-hand sides), lane = right-hand side. Each lane applies the whole
// element operator (the terms of k_elem2d) to its own column of x. The
// element's n, and each face's neighbour n, is a compile-time constant of the
// code path taken, so the lane's values stay in registers. The 1D tables of
// the element and the matrices of each face are wave-uniform: they are copied
// into the wavefront's LDS with one batch of vector loads and read from there
// as broadcasts (LDS reads complete in order, so several stay in flight;
// scalar loads are waited for all at once); x is read and y written in rows
// of 64 consecutive values (x and y interleave the right-hand sides).

// LDS of one wavefront (doubles): the element's M, K, Minv and l_i'(0),
// l_i'(1), then the current face's A_oo, A_on, A_nn, the neighbour's Minv and
// l_i'(side)
struct E2RLds {
  double M[81], K[81], Mi[81], D[18];
  double Aoo[81], Aon[81], Ann[81], Mn[81], Dso[9];
};

// dst[0, CNT) = src[0, CNT) by the 64 lanes, loads issued together
template <int CNT>
__device__ __forceinline__ void e2r_stage(double* __restrict__ dst, const double* __restrict__ src, int lane) {
  constexpr int T = (CNT + 63) / 64;
  double v[T];
#pragma unroll
  for (int u = 0; u < T; ++u) v[u] = src[min(lane + 64 * u, CNT - 1)];
#pragma unroll
  for (int u = 0; u < T; ++u)
    if (lane + 64 * u < CNT) dst[lane + 64 * u] = v[u];
}

// the same in two halves: the loads (into v) and, later, the LDS stores
template <int CNT>
struct E2RStaged {
  static constexpr int T = (CNT + 63) / 64;
  double v[T];
  __device__ __forceinline__ void load(const double* __restrict__ src, int lane) {
#pragma unroll
    for (int u = 0; u < T; ++u) v[u] = src[min(lane + 64 * u, CNT - 1)];
  }
  __device__ __forceinline__ void store(double* __restrict__ dst, int lane) const {
#pragma unroll
    for (int u = 0; u < T; ++u)
      if (lane + 64 * u < CNT) dst[lane + 64 * u] = v[u];
  }
};

// a wave-uniform pointer the compiler cannot see through: the table reads
// behind it are issued where they are used instead of being hoisted and kept
// live across the unrolled loops (which would exhaust the registers)
template <typename T>
__device__ __forceinline__ const T* e2r_opaque(const T* p) {
  int o = 0;   // an opaque zero offset keeps the pointer's provenance
  asm volatile("" : "+s"(o));
  return p + o;
}

// One face of an element of n = N against a neighbour of n = NO (NO = 0 on
// the boundary): the face's g1 (tests against phi) and g2 (against d phi/dn,
// before the division by h) added to the side sums G1, G2 at the side's
// nodes. To, Do: own trace and normal derivative / h at those nodes.
template <int N, int NO, bool OVL>
__device__ __forceinline__ void e2r_face(const FaceRec& R, int form, double k, double h, const double (&To)[N],
                                         const double (&Do)[N], const double* __restrict__ xs, int nrhs,
                                         const double* __restrict__ ftab, const double* __restrict__ tab,
                                         const TableLayout& TL, E2RLds& L, int lane, double (&G1)[N],
                                         double (&G2)[N]) {
  constexpr int P = N - 1;
  constexpr bool inner = NO > 0;
  constexpr int NA = inner ? NO : 1;
  const double fsgn = R.side ? 1.0 : -1.0;
  const double csym = inner ? 0.5 : 1.0;
  const double flen = R.flen, sig = R.sig;
  // the face's matrices go to LDS. OVL: their loads and the neighbour's
  // values are issued together (one round trip; the neighbour's l_i'(side)
  // read as scalars so that its traces are formed before the LDS
  // hand-over), at the cost of more values in flight per lane; otherwise
  // the neighbour's values are read after the hand-over
  wave_sync();   // the previous face's LDS reads are done
  E2RStaged<N * N> sAoo;
  E2RStaged<inner ? N * NO : 1> sAon;
  E2RStaged<inner ? NO * NO : 1> sAnn, sMn;
  if constexpr (OVL) {
    sAoo.load(ftab + R.foo[0], lane);
    if constexpr (inner) {
      sAon.load(ftab + R.fon[0], lane);
      if (form == 1) {
        sAnn.load(ftab + R.fnn[0], lane);
        sMn.load(tab + TL.minv + (NO - 1) * 81, lane);
      }
    }
  }
  double Tn[NA], Dn[NA];
  // neighbour trace and k_n/h_n-scaled normal derivative at its side nodes
  auto neighbour = [&]() {
    if constexpr (inner) {
      const int so = 1 - R.side;
      const int som = R.m == 0 ? 1 : NO, sot = R.m == 0 ? NO : 1;
      const double* __restrict__ Dso = OVL ? tab + TL.dside + ((NO - 1) * 2 + so) * 9 : L.Dso;
      const double* __restrict__ xn = xs + (int64_t)R.nbase * nrhs;
      const int c0 = so ? NO - 1 : 0;
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        double dv = 0.0;
#pragma unroll
        for (int a = 0; a < NO; ++a) dv += Dso[a] * xn[(int64_t)(a * som + j * sot) * nrhs];
        Tn[j] = xn[(int64_t)(c0 * som + j * sot) * nrhs];
        Dn[j] = R.kho * dv;
      }
    }
  };
  if constexpr (OVL) {
    neighbour();
    sAoo.store(L.Aoo, lane);
    if constexpr (inner) {
      sAon.store(L.Aon, lane);
      if (form == 1) {
        sAnn.store(L.Ann, lane);
        sMn.store(L.Mn, lane);
      }
    }
  } else {
    e2r_stage<N * N>(L.Aoo, ftab + R.foo[0], lane);
    if constexpr (inner) {
      e2r_stage<N * NO>(L.Aon, ftab + R.fon[0], lane);
      e2r_stage<9>(L.Dso, tab + TL.dside + ((NO - 1) * 2 + 1 - R.side) * 9, lane);
      if (form == 1) {
        e2r_stage<NO * NO>(L.Ann, ftab + R.fnn[0], lane);
        e2r_stage<NO * NO>(L.Mn, tab + TL.minv + (NO - 1) * 81, lane);
      }
    }
  }
  wave_sync();
  if constexpr (!OVL) neighbour();
  const double* __restrict__ Aoo = L.Aoo;
  const double* __restrict__ Aon = L.Aon;
  double v[N], g1[N];
  // one opaque base per loop: no reuse of table reads across the loops,
  // free scheduling of the reads within each
  const double* __restrict__ A1 = e2r_opaque(Aoo);
  const double* __restrict__ B1 = e2r_opaque(Aon);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double vv = 0.0, ds = 0.0;
    const double* __restrict__ Ar = A1 + j * N;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      vv += Ar[a] * To[a];
      ds += k * Ar[a] * Do[a];
    }
    if constexpr (inner) {
      const double* __restrict__ Br = B1 + j * NO;
#pragma unroll
      for (int a = 0; a < NO; ++a) {
        vv -= Br[a] * Tn[a];
        ds += Br[a] * Dn[a];
      }
    }
    v[j] = vv;
    g1[j] = -flen * csym * fsgn * ds;
    G2[j] += -csym * k * fsgn * flen * vv;
    if (form == 0) g1[j] += flen * sig * vv;
  }
  if (form == 1) {
    // BR2: own lifting L2 s_o A_oo Minv_o v, neighbour lifting
    // L2 s_n A_on Minv_n (A_on^T To - A_nn Tn)
    const double L2 = (inner ? 0.25 : 1.0) * sig * flen * flen;
    const double* __restrict__ Mi = L.Mi;
    const int sk = R.side ? P : 0;
    const double so_ = Mi[sk * N + sk] / (h * h);
    double w[N];
    const double* __restrict__ M1 = e2r_opaque(Mi);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double acc = 0.0;
      const double* __restrict__ Mr = M1 + j * N;
#pragma unroll
      for (int a = 0; a < N; ++a) acc += Mr[a] * v[a];
      w[j] = acc;
    }
    const double* __restrict__ A2 = e2r_opaque(Aoo);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double acc = 0.0;
      const double* __restrict__ Ar = A2 + j * N;
#pragma unroll
      for (int a = 0; a < N; ++a) acc += Ar[a] * w[a];
      g1[j] += L2 * so_ * acc;
    }
    if constexpr (inner) {
      const double* __restrict__ Ann = L.Ann;
      const double* __restrict__ Mn = L.Mn;
      double vn[NO], wn[NO];
      const double* __restrict__ B2 = e2r_opaque(Aon);
      const double* __restrict__ C1 = e2r_opaque(Ann);
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        double acc = 0.0;
        const double* __restrict__ Bc = B2 + j;
        const double* __restrict__ Cr = C1 + j * NO;
#pragma unroll
        for (int a = 0; a < N; ++a) acc += Bc[a * NO] * To[a];
#pragma unroll
        for (int a = 0; a < NO; ++a) acc -= Cr[a] * Tn[a];
        vn[j] = acc;
      }
      const double* __restrict__ M2 = e2r_opaque(Mn);
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        double acc = 0.0;
        const double* __restrict__ Mr = M2 + j * NO;
#pragma unroll
        for (int a = 0; a < NO; ++a) acc += Mr[a] * vn[a];
        wn[j] = acc;
      }
      const int skn = R.side ? 0 : NO - 1;
      const double sn = Mn[skn * NO + skn] / (R.hn * R.hn);
      const double* __restrict__ B3 = e2r_opaque(Aon);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double acc = 0.0;
        const double* __restrict__ Br = B3 + j * NO;
#pragma unroll
        for (int a = 0; a < NO; ++a) acc += Br[a] * wn[a];
        g1[j] += L2 * sn * acc;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) G1[j] += g1[j];
}

// the sums G1, G2 (before the division by h) of side s over its face
// records, in record order
template <int N, bool OVL>
__device__ __forceinline__ void e2r_side(int e, int s, int nrhs, int form, double h, double k,
                                         const int32_t* __restrict__ sptr, const FaceRec* __restrict__ recs,
                                         const double* __restrict__ ftab, const double* __restrict__ tab,
                                         const TableLayout& TL, const double* __restrict__ xs,
                                         const double* __restrict__ xe, E2RLds& L, int lane, double (&G1)[N],
                                         double (&G2)[N]) {
  constexpr int P = N - 1;
  const int f0 = sptr[e * 4 + s], f1 = sptr[e * 4 + s + 1];
  const int m = s >> 1, sd = s & 1;
  const int stm = m == 0 ? 1 : N, stt = m == 0 ? N : 1;
  const double* __restrict__ Ds = L.D + sd * 9;   // l_i'(sd)
  const int c0 = sd ? P : 0;
  double To[N], Do[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double dv = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) dv += Ds[a] * xe[(int64_t)(a * stm + j * stt) * nrhs];
    To[j] = xe[(int64_t)(c0 * stm + j * stt) * nrhs];
    Do[j] = dv / h;
    G1[j] = 0.0;
    G2[j] = 0.0;
  }
#pragma unroll 1
  for (int f = f0; f < f1; ++f) {
    const FaceRec R = recs[f];
    const int no = R.nbr >= 0 ? (int)R.pn + 1 : 0;
    switch (no) {
      case 0: e2r_face<N, 0, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 2: e2r_face<N, 2, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 3: e2r_face<N, 3, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 4: e2r_face<N, 4, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 5: e2r_face<N, 5, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 6: e2r_face<N, 6, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 7: e2r_face<N, 7, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      case 8: e2r_face<N, 8, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
      default: e2r_face<N, 9, OVL>(R, form, k, h, To, Do, xs, nrhs, ftab, tab, TL, L, lane, G1, G2); break;
    }
  }
}

// side s's sums into the element's y: G2 (divided by h) along the normal
// through l_i'(sd), G1 at the side's nodes
template <int N>
__device__ __forceinline__ void e2r_spread(int s, const double* __restrict__ D, const double (&G1)[N],
                                           const double (&G2)[N], double (&Y)[N * N]) {
  constexpr int P = N - 1;
  const int m = s >> 1, sd = s & 1;
  const double* __restrict__ Ds = D + sd * 9;   // l_i'(sd)
  if (m == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int c = 0; c < N; ++c) Y[j * N + c] += Ds[c] * G2[j];
    if (sd == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) Y[j * N] += G1[j];
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) Y[j * N + P] += G1[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int c = 0; c < N; ++c) Y[c * N + j] += Ds[c] * G2[j];
    if (sd == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) Y[j] += G1[j];
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) Y[P * N + j] += G1[j];
    }
  }
}

// volume, y = k (M X K + K X M) over the node rows of X, (row, column) =
// (i1, i0): the row's products with K and M, then its outer products. The 1D
// M and K (in L) are symmetric (up to the rounding of their quadrature sums),
// so their rows serve as columns and are read as contiguous runs.
template <int N, bool PF>
__device__ __forceinline__ void e2r_volume(double k, const double* __restrict__ xe, int nrhs, const E2RLds& L,
                                           double (&Y)[N * N]) {
  constexpr int NN = N * N;
#pragma unroll
  for (int i = 0; i < NN; ++i) Y[i] = 0.0;
  // PF: each row of X loaded one row ahead (more values per lane in flight)
  double xr[N], xq[N];
  if constexpr (PF) {
#pragma unroll
    for (int a = 0; a < N; ++a) xq[a] = xe[(int64_t)a * nrhs];
  }
#pragma unroll
  for (int b = 0; b < N; ++b) {
    double ta[N], tb[N];
    if constexpr (PF) {
#pragma unroll
      for (int a = 0; a < N; ++a) xr[a] = xq[a];
      if (b + 1 < N) {
#pragma unroll
        for (int a = 0; a < N; ++a) xq[a] = xe[(int64_t)((b + 1) * N + a) * nrhs];
      }
    } else {
#pragma unroll
      for (int a = 0; a < N; ++a) xr[a] = xe[(int64_t)(b * N + a) * nrhs];
    }
    // one opaque base per row: the table reads are not kept across rows
    const double* __restrict__ Kr = e2r_opaque(L.K);
    const double* __restrict__ Mr = e2r_opaque(L.M);
#pragma unroll
    for (int i0 = 0; i0 < N; ++i0) {
      const double* __restrict__ Kc = Kr + i0 * N;
      const double* __restrict__ Mc = Mr + i0 * N;
      double sa = 0.0, sb = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        sa += xr[a] * Kc[a];
        sb += xr[a] * Mc[a];
      }
      ta[i0] = sa;
      tb[i0] = sb;
    }
    const double* __restrict__ Mb = Mr + b * N;
    const double* __restrict__ Kb = Kr + b * N;
#pragma unroll
    for (int i1 = 0; i1 < N; ++i1) {
      const double mb = Mb[i1], kb = Kb[i1];
#pragma unroll
      for (int i0 = 0; i0 < N; ++i0) Y[i1 * N + i0] += mb * ta[i0] + kb * tb[i0];
    }
  }
#pragma unroll
  for (int i = 0; i < NN; ++i) Y[i] *= k;
}

template <int N, bool OVL>
__device__ __forceinline__ void e2r_element(int e, int nrhs, int form, const int64_t* __restrict__ off,
                                            const double* __restrict__ hh, const double* __restrict__ kk,
                                            const int32_t* __restrict__ sptr, const FaceRec* __restrict__ recs,
                                            const double* __restrict__ ftab, const double* __restrict__ tab,
                                            const TableLayout& TL, const double* __restrict__ xs,
                                            double* __restrict__ ys, bool act, E2RLds& L, int lane) {
  constexpr int P = N - 1, NN = N * N;
  const double h = hh[e], k = kk[e];
  const int64_t base = off[e];
  e2r_stage<NN>(L.M, tab + TL.mk + P * 162, lane);
  e2r_stage<NN>(L.K, tab + TL.mk + P * 162 + 81, lane);
  if (form == 1) e2r_stage<NN>(L.Mi, tab + TL.minv + P * 81, lane);
  e2r_stage<18>(L.D, tab + TL.dside + P * 18, lane);
  wave_sync();
  const double* __restrict__ xe = xs + base * nrhs;
  double Y[NN];
  e2r_volume<N, OVL>(k, xe, nrhs, L, Y);
  // faces, side by side (m = normal dimension, sd = lower / upper), each
  // side's sums added into y in turn
#pragma unroll 1
  for (int s = 0; s < 4; ++s) {
    double G1[N], G2[N];
    e2r_side<N, OVL>(e, s, nrhs, form, h, k, sptr, recs, ftab, tab, TL, xs, xe, L, lane, G1, G2);
#pragma unroll
    for (int j = 0; j < N; ++j) G2[j] /= h;
    e2r_spread<N>(s, L.D, G1, G2, Y);
  }
  if (act) {
    double* __restrict__ ye = ys + base * nrhs;
#pragma unroll
    for (int i = 0; i < NN; ++i) ye[(int64_t)i * nrhs] = Y[i];
  }
}

// grid: a multiple of 8 workgroups of one wavefront, items (element of
// elist, group of 64 right-hand sides) in XCD-aware order as in k_elem2d.
// NMAX: the largest n compiled in (the registers follow it); elist holds
// elements of n <= NMAX only. OVL: see e2r_face.
template <int NMAX, bool OVL>
__global__ __launch_bounds__(64) void k_elem2d_rhs(int ne, const int32_t* __restrict__ elist, int nrhs, int form,
                                                   const int64_t* __restrict__ off,
                                                   const int8_t* __restrict__ pdeg, const double* __restrict__ hh,
                                                   const double* __restrict__ kk, const int32_t* __restrict__ sptr,
                                                   const FaceRec* __restrict__ recs, const double* __restrict__ ftab,
                                                   const double* __restrict__ tab, TableLayout TL,
                                                   const double* __restrict__ x, double* __restrict__ y) {
  const int ngrp = (nrhs + 63) >> 6;
  const int per = (int)(gridDim.x >> 3);
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= ne * ngrp) return;
  const int il = item / ngrp, g = item - il * ngrp;
  const int e = elist[il];
  const int r = g * 64 + (int)threadIdx.x;
  const bool act = r < nrhs;
  const int rc = act ? r : nrhs - 1;
  const double* xs = x + rc;
  double* ys = y + rc;
  __shared__ E2RLds L;
  const int lane = (int)threadIdx.x;
  switch (pdeg[e]) {
    case 1: e2r_element<2, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
    case 2: e2r_element<3, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
    case 3: e2r_element<4, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
    case 4: e2r_element<5, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
    case 5: e2r_element<6, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
    default:
      if constexpr (NMAX > 6) {
        switch (pdeg[e]) {
          case 6: e2r_element<7, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
          case 7: e2r_element<8, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
          default: e2r_element<9, OVL>(e, nrhs, form, off, hh, kk, sptr, recs, ftab, tab, TL, xs, ys, act, L, lane); break;
        }
      }
      break;
  }
}

// ---------------------------------------------------------- vector kernels
template <typename TI, typename TO>
__global__ void k_cast(int64_t n, const TI* __restrict__ a, TO* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (TO)a[i];
}

// z[i] = d[i / nrhs] * r[i]
template <typename T>
__global__ void k_diag_scale(int64_t n, int nrhs, const T* __restrict__ d, const T* __restrict__ r,
                             T* __restrict__ z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = d[i / nrhs] * r[i];
}

// rt[i] = (T) r[i], z[i] = d[i / nrhs] * rt[i]
template <typename T>
__global__ __launch_bounds__(256) void k_cast_diag_scale(int64_t n, int nrhs, const T* __restrict__ d,
                                                         const double* __restrict__ r, T* __restrict__ rt,
                                                         T* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const T v = (T)r[i];
    rt[i] = v;
    z[i] = d[i / nrhs] * v;
  }
}

// partial dot products per block and per RHS (rhs = index % nrhs); nrhs
// divides 256. part[block * nrhs + r]
__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, int nrhs, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sm[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) acc += a[i] * b[i];
  sm[tid] = acc;
  __syncthreads();
  for (int w = 128; w >= nrhs; w >>= 1) {
    if (tid < w) sm[tid] += sm[tid + w];
    __syncthreads();
  }
  if (tid < nrhs) part[blockIdx.x * nrhs + tid] = sm[tid];
}


// CG scalars on the device, one slot per RHS (SoA, stride 256):
struct CGScal {
  double *rz, *pAp, *rr, *bb, *alpha, *beta, *tol2;
  double* rzn;             // one RHS: the latest r'z (rz holds the one before)
  int *act, *iters, *err;
  double *ahist, *bhist;   // [maxit * hs]: alpha_k, beta_k of RHS c at k * hs + c
  int maxit;               // capacity of the histories in iterations
  int hs;                  // history stride (>= nrhs)
};

// epilogue of a dot product for RHS c with value v
enum { EP_BB = 0, EP_RR0 = 1, EP_RZ0 = 2, EP_PAP = 3, EP_RR = 4, EP_RZ = 5, EP_TRUE = 6 };
__device__ inline void cg_epilogue(int mode, int c, double v, CGScal S) {
  switch (mode) {
    case EP_BB: S.bb[c] = v; break;
    case EP_RR0:
      S.rr[c] = v;
      S.iters[c] = 0;
      S.err[c] = 0;
      S.act[c] = (v > S.tol2[c] * S.bb[c]) ? 1 : 0;
      break;
    case EP_RZ0:
      S.rz[c] = v;
      S.rzn[c] = v;
      if (S.act[c] && !(v > 0.0)) { S.err[c] = 1; S.act[c] = 0; }
      break;
    case EP_PAP:
      S.pAp[c] = v;
      if (S.act[c] && !(v > 0.0)) { S.err[c] = 1; S.act[c] = 0; }
      S.alpha[c] = S.act[c] ? S.rz[c] / v : 0.0;
      break;
    case EP_RR:
      S.rr[c] = v;
      if (S.act[c]) {
        int it = S.iters[c];
        if (it < S.maxit) S.ahist[(int64_t)it * S.hs + c] = S.alpha[c];
        S.iters[c] = it + 1;
        if (!(v > S.tol2[c] * S.bb[c])) S.act[c] = 0;
      }
      break;
    case EP_RZ:
      if (S.act[c]) {
        if (!(v > 0.0)) { S.err[c] = 1; S.act[c] = 0; S.beta[c] = 0.0; break; }
        double b = v / S.rz[c];
        S.beta[c] = b;
        S.rz[c] = v;
        int it = S.iters[c];
        if (it - 1 < S.maxit) S.bhist[(int64_t)(it - 1) * S.hs + c] = b;
      } else {
        S.beta[c] = 0.0;
      }
      break;
    default: S.rr[c] = v; break;   // EP_TRUE: true residual norm^2
  }
}


// sum of p[b * m + c] for b = b0, b0 + bs, ... < n, added in that order; the
// loads are issued eight, then four at a time (same result as the plain loop)
__device__ inline double ordered_sum(const double* __restrict__ p, int b0, int bs, int n, int m, int c) {
  double s = 0.0;
  int b = b0;
  for (; b + 7 * bs < n; b += 8 * bs) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(b + u * bs) * m + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b + 3 * bs < n; b += 4 * bs) {
    const double v0 = p[(int64_t)b * m + c];
    const double v1 = p[(int64_t)(b + bs) * m + c];
    const double v2 = p[(int64_t)(b + 2 * bs) * m + c];
    const double v3 = p[(int64_t)(b + 3 * bs) * m + c];
    s += v0;
    s += v1;
    s += v2;
    s += v3;
  }
  for (; b < n; b += bs) s += p[(int64_t)b * m + c];
  return s;
}

// final stage of a dot product (partials from k_dot_partial) with the scalar
// epilogue; one block of 256 threads, fixed summation order
__global__ __launch_bounds__(256) void k_dot_final_ep(int nblocks, int nrhs, const double* __restrict__ part,
                                                      int mode, CGScal S) {
  __shared__ double sm[256];
  const int t = threadIdx.x;
  const int c = t % nrhs, g = t / nrhs, ng = 256 / nrhs;
  double s = ordered_sum(part, g, ng, nblocks, nrhs, c);
  sm[t] = s;
  __syncthreads();
  for (int w = 128; w >= nrhs; w >>= 1) {
    if (t < w) sm[t] += sm[t + w];
    __syncthreads();
  }
  if (t < nrhs) cg_epilogue(mode, t, sm[t], S);
}

// The two final stages of every CG iteration (one RHS) with their epilogues
// specialised: the scalars an epilogue reads are loaded at the start, beside
// the share loads, instead of after the reduction (the generic epilogue
// reloads them after its own stores, as the scalar arrays may alias). The
// sums and the updates are those of k_dot_final_ep with cg_epilogue.
//
// p'Ap -> pAp, the breakdown flags, alpha = rz / p'Ap while active
__global__ __launch_bounds__(256) void k_dot_final_pap(int nblocks, const double* __restrict__ part, CGScal S) {
  __shared__ double sm[256];
  const int t = threadIdx.x;
  const int act0 = S.act[0];
  const double rz = S.rz[0];
  sm[t] = ordered_sum(part, t, 256, nblocks, 1, 0);
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) sm[t] += sm[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double v = sm[0];
    int act = act0;
    S.pAp[0] = v;
    if (act && !(v > 0.0)) {
      S.err[0] = 1;
      S.act[0] = 0;
      act = 0;
    }
    S.alpha[0] = act ? rz / v : 0.0;
  }
}

// r'r (shares pa) then r'z (shares pb): the residual norm, the iteration
// count and alpha's history, the convergence test, then beta, rz and beta's
// history while active
__global__ __launch_bounds__(256) void k_dot_final_rr_rz(int na, const double* __restrict__ pa, int nb,
                                                         const double* __restrict__ pb, CGScal S) {
  __shared__ double sm[256];
  const int t = threadIdx.x;
  const int act0 = S.act[0], it0 = S.iters[0];
  const double tol2 = S.tol2[0], bb = S.bb[0], rz = S.rz[0], alpha = S.alpha[0];
  double v[2];
  for (int pass = 0; pass < 2; ++pass) {
    sm[t] = ordered_sum(pass ? pb : pa, t, 256, pass ? nb : na, 1, 0);
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (t < w) sm[t] += sm[t + w];
      __syncthreads();
    }
    v[pass] = sm[0];
    __syncthreads();
  }
  if (t == 0) {
    int act = act0, it = it0;
    S.rr[0] = v[0];
    if (act) {
      if (it < S.maxit) S.ahist[(int64_t)it * S.hs] = alpha;
      it = it + 1;
      S.iters[0] = it;
      if (!(v[0] > tol2 * bb)) {
        S.act[0] = 0;
        act = 0;
      }
    }
    if (act) {
      if (!(v[1] > 0.0)) {
        S.err[0] = 1;
        S.act[0] = 0;
        S.beta[0] = 0.0;
      } else {
        const double b = v[1] / rz;
        S.beta[0] = b;
        S.rz[0] = v[1];
        if (it - 1 < S.maxit) S.bhist[(int64_t)(it - 1) * S.hs] = b;
      }
    } else {
      S.beta[0] = 0.0;
    }
  }
}

// x += alpha p ; r -= alpha Ap (alpha = 0 for converged RHS), interleaved
// RHS, with the per-RHS shares of r'r: the grid-stride loop and the
// reduction are those of k_dot_partial (same grid), so the shares are bitwise
// the ones a separate pass over r would give
__global__ __launch_bounds__(256) void k_cg_update2(int64_t n, int nrhs, const double* __restrict__ alpha,
                                                   const double* __restrict__ p, const double* __restrict__ Ap,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ part) {
  __shared__ double sm[256];
  const int tid = threadIdx.x;
  const double al = alpha[tid % nrhs];   // the grid stride is a multiple of nrhs
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] += al * p[i];
    const double ri = r[i] - al * Ap[i];
    r[i] = ri;
    acc += ri * ri;
  }
  sm[tid] = acc;
  __syncthreads();
  for (int w = 128; w >= nrhs; w >>= 1) {
    if (tid < w) sm[tid] += sm[tid + w];
    __syncthreads();
  }
  if (tid < nrhs) part[blockIdx.x * nrhs + tid] = sm[tid];
}

// ------------------------------------------------------------- 3D element
// 3D element kernel: volume and face terms of one element per block of 256
// threads, all degrees in one launch, y written once.
//  volume: y_K = k h (K x M x M + M x K x M + M x M x K) x_K, three 1D
//          contraction phases through LDS.
//  faces:  a face of side (m, s) has tangential slots 0, 1 (the two other
//          dimensions in increasing order); its face-mass matrices are the
//          Kronecker products of the unit-length 1D matrices of the slots,
//          times the area L^2. With own traces To, Do and neighbour traces
//          Tn, Dn (Dn scaled by k_n / h_n) on the face nodes:
//            v    = (A0oo x A1oo) To - (A0on x A1on) Tn          (jump)
//            dsum = k (A0oo x A1oo) Do + (A0on x A1on) Dn        (2 x average)
//          G1 += L^2 (sigma v - c sgn dsum), G2 += -c k sgn L^2 v (c = 1/2
//          inside, 1 on the boundary) for SIPG (Sec. 2); BR2 (Sec. 4.4)
//          replaces sigma v by the liftings
//            c^2 eta k_e L^4 [s_o (A0oo x A1oo)(Mi x Mi) v
//                             + s_n (A0on x A1on)(Mi_n x Mi_n) vn],
//            vn = (A0on x A1on)^T To - (A0nn x A1nn) Tn, s = m00 / h^3.
//          Each Kronecker product is two 1D contractions; the products
//          A Minv of each slot come precomputed from the face table, so a
//          BR2 face takes four barrier-separated stages and an SIPG face two.
//  Memory: records and neighbour traces of up to NM faces are fetched in
//  two parallel rounds into LDS; faces are then applied one after another
//  (a fixed order, so the sums per side node are deterministic).
__device__ inline void tdims3(int m, int& t0, int& t1) {
  t0 = m == 0 ? 1 : 0;
  t1 = m == 2 ? 1 : 2;
}

template <int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NM == 7 ? 7 : 4))) void k_elem3d(int ne, int nrhs, int form, const int64_t* __restrict__ off,
                                                const int8_t* __restrict__ pdeg, const double* __restrict__ hh,
                                                const double* __restrict__ kk, const int32_t* __restrict__ sptr,
                                                const FaceRec* __restrict__ recs, const double* __restrict__ ftab,
                                                const double* __restrict__ tab, TableLayout TL,
                                                const double* __restrict__ x, double* __restrict__ y,
                                                double* __restrict__ pdot, const int32_t* __restrict__ perm) {
  // LDS sized for degree <= NM - 1: volume buffers of NM^3 (reused by the
  // face stage once the volume is done), face slots of F2 = NM^2, KF = NM
  // face records per pass (KF slots of F2 fill a volume buffer)
  constexpr int F2 = NM * NM, V3 = NM * NM * NM, KF = NM;
  static_assert(6 * F2 <= V3, "six face slots must fit a volume buffer");
  __shared__ double sV0[V3], sV1[V3], sV2[V3], sV3[V3];
  __shared__ double sTo[6][F2], sDo[6][F2], sG1[6][F2], sG2[6][F2];
  __shared__ FaceRec sR[KF];
  __shared__ double sRed[4];
  const int per = (int)(gridDim.x >> 3);
  // (element, RHS) items in XCD-aware order; with perm the i-th element
  // position holds element perm[i]
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= ne * nrhs) return;
  const int ei = item / nrhs, rhs = item - ei * nrhs;
  const int e = perm ? perm[ei] : ei;
  const int tid = threadIdx.x;
  const int p = pdeg[e], n = p + 1, n2 = n * n, n3 = n2 * n;
  const double h = hh[e], k = kk[e];
  const int64_t base = off[e];
  int sp[7];
#pragma unroll
  for (int t = 0; t < 7; ++t) sp[t] = sptr[e * 6 + t];
  // the 1D mass and stiffness of the element's degree, staged in the side-sum
  // arrays, which the volume stage does not use (they are cleared after it)
  {
    const double* gMt = tab + TL.mk + (p * 2 + 0) * 81;
    const double* gKt = tab + TL.mk + (p * 2 + 1) * 81;
    for (int i = tid; i < n2; i += 256) {
      (&sG1[0][0])[i] = gMt[i];
      (&sG2[0][0])[i] = gKt[i];
    }
  }
  const double* Mt = &sG1[0][0];
  const double* Kt = &sG2[0][0];
  double* sX = sV0;
  for (int i = tid; i < n3; i += 256) sX[i] = x[(base + i) * nrhs + rhs];
  __syncthreads();
  // phase 1 (dimension 0) and the own traces
  double* sA = sV1;
  double* sB = sV2;
  for (int r = tid; r < n3; r += 256) {
    const int i0 = r % n, i12 = r - i0;
    double a0 = 0.0, b0 = 0.0;
    #pragma unroll 4
    for (int a = 0; a < n; ++a) {
      const double xa = sX[i12 + a];
      a0 += xa * Mt[a * n + i0];
      b0 += xa * Kt[a * n + i0];
    }
    sA[r] = a0;
    sB[r] = b0;
  }
  for (int t = tid; t < 6 * n2; t += 256) {
    const int side = t / n2, q = t - side * n2;
    const int m = side >> 1, s = side & 1;
    int t0, t1;
    tdims3(m, t0, t1);
    const int st[3] = {1, n, n2};
    const int j0 = q % n, j1 = q / n;
    const int o = j0 * st[t0] + j1 * st[t1];
    const double* Ds = tab + TL.dside + (p * 2 + s) * 9;
    double dv = 0.0;
    #pragma unroll 4
    for (int a = 0; a < n; ++a) dv += Ds[a] * sX[o + a * st[m]];
    sTo[side][q] = sX[o + (s ? p : 0) * st[m]];
    sDo[side][q] = dv / h;
  }
  __syncthreads();
  // phase 2 (dimension 1): C into sV0 (x is no longer needed), D into sV3
  double* sC = sV0;
  double* sD = sV3;
  for (int r = tid; r < n3; r += 256) {
    const int i0 = r % n, i1 = (r / n) % n, i2 = r / n2;
    double aa = 0.0, ab = 0.0, ba = 0.0;
    #pragma unroll 4
    for (int b = 0; b < n; ++b) {
      const double av = sA[i0 + n * b + n2 * i2], bv = sB[i0 + n * b + n2 * i2];
      const double mb = Mt[b * n + i1], kb = Kt[b * n + i1];
      aa += av * mb;
      ab += av * kb;
      ba += bv * mb;
    }
    sC[r] = aa;
    sD[r] = ab + ba;
  }
  __syncthreads();
  // phase 3 (dimension 2)
  double yv[3] = {0.0, 0.0, 0.0};
  {
    int c = 0;
    for (int r = tid; r < n3; r += 256, ++c) {
      const int i01 = r % n2, i2 = r / n2;
      double acc = 0.0;
      #pragma unroll 4
      for (int cc = 0; cc < n; ++cc) acc += Kt[cc * n + i2] * sC[i01 + n2 * cc] + Mt[cc * n + i2] * sD[i01 + n2 * cc];
      yv[c] = k * h * acc;
    }
  }
  __syncthreads();
  // the side sums start at zero (the face stage's first barrier orders this
  // before their first use)
  for (int i = tid; i < 6 * F2; i += 256) {
    (&sG1[0][0])[i] = 0.0;
    (&sG2[0][0])[i] = 0.0;
  }
  // face stage: work arrays in the volume buffers
  double* sTn = sV0;                 // [KF][F2]
  double* sDn = sV3;                 // [KF][F2]
  double* U0 = sV1;                  // contraction temporaries
  double* U1 = sV1 + F2;
  double* U2 = sV1 + 2 * F2;
  double* U3 = sV1 + 3 * F2;
  double* Y0 = sV1 + 4 * F2;
  double* Y1 = sV1 + 5 * F2;
  double* Vv = sV2;                  // jump on own face nodes
  double* Vn = sV2 + F2;             // jump on the neighbour's face nodes (BR2)
  double* P0 = sV2 + 2 * F2;
  double* Q0 = sV2 + 3 * F2;
  for (int c0 = sp[0]; c0 < sp[6]; c0 += KF) {
    const int nF = min(KF, sp[6] - c0);
    {
      constexpr int W = (int)(sizeof(FaceRec) / 8);
      const unsigned long long* src = reinterpret_cast<const unsigned long long*>(recs + c0);
      unsigned long long* dst = reinterpret_cast<unsigned long long*>(sR);
      for (int t = tid; t < nF * W; t += 256) dst[t] = src[t];
    }
    __syncthreads();
    // neighbour traces
    for (int t = tid; t < nF * F2; t += 256) {
      const int f = t / F2, q = t - F2 * f;
      const int nb = sR[f].nbr, po = sR[f].pn, no = po + 1;
      if (nb < 0 || q >= no * no) continue;
      const int mm = sR[f].m, so = 1 - sR[f].side;
      int t0, t1;
      tdims3(mm, t0, t1);
      const int st[3] = {1, no, no * no};
      const int a0 = q % no, a1 = q / no;
      const int o = a0 * st[t0] + a1 * st[t1];
      const double* Dso = tab + TL.dside + (po * 2 + so) * 9;
      const double* xn = x + (int64_t)sR[f].nbase * nrhs + rhs;
      double dv = 0.0;
      #pragma unroll 4
      for (int a = 0; a < no; ++a) dv += Dso[a] * xn[(int64_t)(o + a * st[mm]) * nrhs];
      sTn[f * F2 + q] = xn[(int64_t)(o + (so ? po : 0) * st[mm]) * nrhs];
      sDn[f * F2 + q] = sR[f].kho * dv;
    }
    __syncthreads();
    for (int f = 0; f < nF; ++f) {
      const FaceRec& R = sR[f];
      const int m = R.m, s = R.side, side = 2 * m + s;
      const bool inner = R.nbr >= 0;
      const int po = inner ? (int)R.pn : 0, no = po + 1;
      const double area = R.flen * R.flen;
      const double sgn = s ? 1.0 : -1.0;
      const double csym = inner ? 0.5 : 1.0;
      const double* A0oo = ftab + R.foo[0];
      const double* A1oo = ftab + R.foo[1];
      const double* A0on = ftab + R.fon[0];
      const double* A1on = ftab + R.fon[1];
      const double* Tn = sTn + f * F2;
      const double* Dn = sDn + f * F2;
      const bool br2i = form == 1 && inner;
      const double* A0nn = ftab + R.fnn[0];
      const double* A1nn = ftab + R.fnn[1];
      // stage 1: slot-0 contractions of To, Do (own) and Tn, Dn (neighbour);
      // for BR2 also the slot-0 halves of the neighbour's jump
      //   Y0 = A0on^T To (no x n), Y1 = A0nn Tn (no x no)
      for (int t = tid; t < 6 * F2; t += 256) {
        const int which = t / F2, q = t - F2 * which;
        if (which < 2) {
          if (q >= n2) continue;
          const int j0 = q % n, a1 = q / n;
          const double* in = which == 0 ? sTo[side] : sDo[side];
          double sacc = 0.0;
          #pragma unroll 4
          for (int a0 = 0; a0 < n; ++a0) sacc += A0oo[j0 * n + a0] * in[a0 + n * a1];
          (which == 0 ? U0 : U1)[q] = sacc;
        } else if (which < 4) {
          if (!inner || q >= n * no) continue;
          const int j0 = q % n, a1 = q / n;
          const double* in = which == 2 ? Tn : Dn;
          double sacc = 0.0;
          #pragma unroll 4
          for (int a0 = 0; a0 < no; ++a0) sacc += A0on[j0 * no + a0] * in[a0 + no * a1];
          (which == 2 ? U2 : U3)[q] = sacc;
        } else if (which == 4) {
          if (!br2i || q >= no * n) continue;
          const int a0 = q % no, a1 = q / no;      // a1 over own slot-1 nodes
          double sacc = 0.0;
          #pragma unroll 4
          for (int j0 = 0; j0 < n; ++j0) sacc += A0on[j0 * no + a0] * sTo[side][j0 + n * a1];
          Y0[q] = sacc;
        } else {
          if (!br2i || q >= no * no) continue;
          const int a0 = q % no, a1 = q / no;
          double sacc = 0.0;
          #pragma unroll 4
          for (int b0 = 0; b0 < no; ++b0) sacc += A0nn[a0 * no + b0] * Tn[b0 + no * a1];
          Y1[q] = sacc;
        }
      }
      __syncthreads();
      // stage 2: slot-1 contractions; jump, average and the penalty; for BR2
      // the neighbour's jump vn = (A0on x A1on)^T To - (A0nn x A1nn) Tn
      for (int t = tid; t < 2 * F2; t += 256) {
        if (t < F2) {
          const int q = t;
          if (q >= n2) continue;
          const int j0 = q % n, j1 = q / n;
          double v = 0.0, ds = 0.0;
          #pragma unroll 4
          for (int a1 = 0; a1 < n; ++a1) {
            const double w = A1oo[j1 * n + a1];
            v += w * U0[j0 + n * a1];
            ds += k * w * U1[j0 + n * a1];
          }
          if (inner)
            #pragma unroll 4
            for (int a1 = 0; a1 < no; ++a1) {
              const double w = A1on[j1 * no + a1];
              v -= w * U2[j0 + n * a1];
              ds += w * U3[j0 + n * a1];
            }
          double g1 = -area * csym * sgn * ds;
          if (form == 0) g1 += area * R.sig * v;
          sG1[side][q] += g1;
          sG2[side][q] -= csym * k * sgn * area * v;
          Vv[q] = v;
        } else {
          const int q = t - F2;
          if (!br2i || q >= no * no) continue;
          const int a0 = q % no, b1 = q / no;
          double vn = 0.0;
          #pragma unroll 4
          for (int a1 = 0; a1 < n; ++a1) vn += A1on[a1 * no + b1] * Y0[a0 + no * a1];
          #pragma unroll 4
          for (int c1 = 0; c1 < no; ++c1) vn -= A1nn[b1 * no + c1] * Y1[a0 + no * c1];
          Vn[q] = vn;
        }
      }
      __syncthreads();
      if (form == 1) {
        // liftings with the products L = A Minv of each slot:
        //   G1 += L2 [s_o (Loo0 x Loo1) v + s_n (Lon0 x Lon1) vn]
        const double c2 = inner ? 0.25 : 1.0;
        const double L2 = c2 * R.sig * area * area;
        const double* Mi = tab + TL.minv + p * 81;
        const int sk = s ? p : 0;
        const double so = Mi[sk * n + sk] / (h * h * h);
        double sn = 0.0;
        if (inner) {
          const double* Min = tab + TL.minv + po * 81;
          const int skn = (1 - s) ? po : 0;
          sn = Min[skn * no + skn] / (R.hn * R.hn * R.hn);
        }
        const double* L0o = ftab + R.loo[0];
        const double* L1o = ftab + R.loo[1];
        const double* L0n = ftab + R.lon[0];
        const double* L1n = ftab + R.lon[1];
        // stage 3: slot 0
        for (int t = tid; t < 2 * F2; t += 256) {
          const int which = t / F2, q = t - F2 * which;
          if (which == 0) {
            if (q >= n2) continue;
            const int j0 = q % n, a1 = q / n;
            double sacc = 0.0;
            #pragma unroll 4
            for (int a0 = 0; a0 < n; ++a0) sacc += L0o[j0 * n + a0] * Vv[a0 + n * a1];
            P0[q] = sacc;
          } else {
            if (!inner || q >= n * no) continue;
            const int j0 = q % n, a1 = q / n;
            double sacc = 0.0;
            #pragma unroll 4
            for (int a0 = 0; a0 < no; ++a0) sacc += L0n[j0 * no + a0] * Vn[a0 + no * a1];
            Q0[q] = sacc;
          }
        }
        __syncthreads();
        // stage 4: slot 1 and the sum
        for (int q = tid; q < n2; q += 256) {
          const int j0 = q % n, j1 = q / n;
          double so_acc = 0.0, sn_acc = 0.0;
          #pragma unroll 4
          for (int a1 = 0; a1 < n; ++a1) so_acc += L1o[j1 * n + a1] * P0[j0 + n * a1];
          if (inner)
            #pragma unroll 4
            for (int a1 = 0; a1 < no; ++a1) sn_acc += L1n[j1 * no + a1] * Q0[j0 + n * a1];
          sG1[side][q] += L2 * (so * so_acc + sn * sn_acc);
        }
        __syncthreads();
      }
    }
  }
  // lift the side sums into the element: y += D_side(i_m) G2 / h + [i_m on the face] G1
  const double* D0 = tab + TL.dside + (p * 2 + 0) * 9;
  const double* D1 = tab + TL.dside + (p * 2 + 1) * 9;
  double xy = 0.0;
  {
    int c = 0;
    for (int r = tid; r < n3; r += 256, ++c) {
      const int i[3] = {r % n, (r / n) % n, r / n2};
      double v = yv[c];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        int t0, t1;
        tdims3(m, t0, t1);
        const int q = i[t0] + n * i[t1];
        v += (D0[i[m]] * sG2[2 * m][q] + D1[i[m]] * sG2[2 * m + 1][q]) / h;
        if (i[m] == 0) v += sG1[2 * m][q];
        if (i[m] == p) v += sG1[2 * m + 1][q];
      }
      y[(base + r) * nrhs + rhs] = v;
      xy += x[(base + r) * nrhs + rhs] * v;
    }
  }
  if (pdot) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) xy += __shfl_xor(xy, o, 64);
    if ((tid & 63) == 0) sRed[tid >> 6] = xy;
    __syncthreads();
    if (tid == 0) pdot[e] = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
  }
}

// ---------------------------------------------- 3D operator in three passes
// The same operator as k_elem3d (same face arithmetic, same record order of
// the side sums), split so that each pass keeps many items in flight (one
// RHS):
//   k_e3_vol   one workgroup per element: the volume term into y and the
//              element's traces and normal derivatives on its six sides
//              (To, Do = d/dn / h) into the side buffer sb (12 n^2 values per
//              element at sboff[e]; side s holds To then Do);
//   k_e3_face  one wavefront per face record (four per workgroup, only
//              wave-level synchronisation): the record's contributions to the
//              tests of its element's side nodes, g1 (against the trace) and
//              g2 (against the normal derivative), into gbuf at goff[rec];
//   k_e3_lift  one workgroup per element: the side sums of g1, g2 over its
//              records in record order, lifted into the element
//              (y += D_side(i_m) G2 / h + [i_m on the side] G1), with the
//              element's share of x'y.
// Per record the host adds FaceAux: the own element's degree, h and k, and
// the side-buffer offsets of the own side and of the neighbour's side.
struct FaceAux {
  double h, k;        // own element
  int64_t sb_own;     // offset (doubles) of the own side's To in sb
  int64_t sb_nbr;     // the neighbour's side facing this one (-1 on the boundary)
  int64_t goff;       // offset of this record's g1 (g2 follows after n^2) in gbuf
  int32_t p, pad;
};
static_assert(sizeof(FaceAux) == 48, "FaceAux layout");

template <int N, int NM>
__device__ inline void e3v_body(double (*V)[NM * NM * NM], double* tb, int e, const int64_t* __restrict__ off,
                                const double* __restrict__ hh, const double* __restrict__ kk,
                                const int64_t* __restrict__ sboff, const double* __restrict__ tab, TableLayout TL,
                                const double* __restrict__ x, double* __restrict__ y, double* __restrict__ sb) {
  constexpr int N2 = N * N, N3 = N2 * N, p = N - 1;
  const int tid = threadIdx.x;
  const double h = hh[e], k = kk[e];
  const int64_t base = off[e];
  double* sX = V[0];
  for (int i = tid; i < N3; i += 256) sX[i] = x[base + i];
  {
    const double* gM = tab + TL.mk + (p * 2 + 0) * 81;
    const double* gK = tab + TL.mk + (p * 2 + 1) * 81;
    for (int i = tid; i < N2; i += 256) {
      tb[i] = gM[i];
      tb[81 + i] = gK[i];
    }
    if (tid < N) {
      tb[162 + tid] = tab[TL.dside + (p * 2 + 0) * 9 + tid];
      tb[171 + tid] = tab[TL.dside + (p * 2 + 1) * 9 + tid];
    }
  }
  __syncthreads();
  const double* Mt = tb;
  const double* Kt = tb + 81;
  // phase 1 (dimension 0) and the six sides' traces into the side buffer
  {
    double* sA = V[1];
    double* sB = V[2];
    for (int r = tid; r < N3; r += 256) {
      const int i0 = r % N, i12 = r - i0;
      double a0 = 0.0, b0 = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const double xa = sX[i12 + a];
        a0 += xa * Mt[a * N + i0];
        b0 += xa * Kt[a * N + i0];
      }
      sA[r] = a0;
      sB[r] = b0;
    }
    double* out = sb + sboff[e];
    for (int t = tid; t < 6 * N2; t += 256) {
      const int side = t / N2, q = t - side * N2;
      const int m = side >> 1, s = side & 1;
      int t0, t1;
      tdims3(m, t0, t1);
      const int st[3] = {1, N, N2};
      const int j0 = q % N, j1 = q / N;
      const int o = j0 * st[t0] + j1 * st[t1];
      const double* Ds = tb + (s ? 171 : 162);
      double dv = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) dv += Ds[a] * sX[o + a * st[m]];
      out[side * 2 * N2 + q] = sX[o + (s ? p : 0) * st[m]];
      out[side * 2 * N2 + N2 + q] = dv / h;
    }
  }
  __syncthreads();
  // phase 2 (dimension 1): C into V0 (x is no longer needed), D into V3
  {
    const double* sA = V[1];
    const double* sB = V[2];
    double* sC = V[0];
    double* sD = V[3];
    for (int r = tid; r < N3; r += 256) {
      const int i0 = r % N, i1 = (r / N) % N, i2 = r / N2;
      double aa = 0.0, ab = 0.0, ba = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const double av = sA[i0 + N * b + N2 * i2], bv = sB[i0 + N * b + N2 * i2];
        const double mb = Mt[b * N + i1], kb = Kt[b * N + i1];
        aa += av * mb;
        ab += av * kb;
        ba += bv * mb;
      }
      sC[r] = aa;
      sD[r] = ab + ba;
    }
  }
  __syncthreads();
  // phase 3 (dimension 2): the volume term into y
  {
    const double* sC = V[0];
    const double* sD = V[3];
    for (int r = tid; r < N3; r += 256) {
      const int i01 = r % N2, i2 = r / N2;
      double acc = 0.0;
#pragma unroll
      for (int cc = 0; cc < N; ++cc) acc += Kt[cc * N + i2] * sC[i01 + N2 * cc] + Mt[cc * N + i2] * sD[i01 + N2 * cc];
      y[base + r] = k * h * acc;
    }
  }
}

template <int NM>
__global__ __launch_bounds__(256) void k_e3_vol(int ne, const int64_t* __restrict__ off,
                                                const int8_t* __restrict__ pdeg, const double* __restrict__ hh,
                                                const double* __restrict__ kk, const int64_t* __restrict__ sboff,
                                                const double* __restrict__ tab, TableLayout TL,
                                                const double* __restrict__ x, double* __restrict__ y,
                                                double* __restrict__ sb, const int32_t* __restrict__ perm) {
  __shared__ double V[4][NM * NM * NM];
  __shared__ double tb[180];
  const int per = (int)(gridDim.x >> 3);
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);   // XCD-aware order
  if (item >= ne) return;
  const int e = perm ? perm[item] : item;
  switch (pdeg[e]) {
    case 1: e3v_body<2, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb); break;
    case 2: e3v_body<3, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb); break;
    case 3: e3v_body<4, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb); break;
    case 4: e3v_body<5, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb); break;
    case 5: e3v_body<6, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb); break;
    case 6: e3v_body<7, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb); break;
    default:
      if constexpr (NM >= 9) {
        if (pdeg[e] == 7) e3v_body<8, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb);
        else e3v_body<9, NM>(V, tb, e, off, hh, kk, sboff, tab, TL, x, y, sb);
      }
      break;
  }
}

// floor(q / d) for 0 <= q < 128 and 1 <= d <= 9 by a multiply and a shift
// (mul = 65536 / d + 1; exact in that range)
__device__ inline int qdiv(int q, int mul) { return (q * mul) >> 16; }

// one face record per wavefront, the own degree N = n a constant
template <int N, int NM, bool STAGE>
__device__ inline void e3f_body(const FaceRec& r, const FaceAux& ax, int form, double* To, double* Do, double* W,
                                double* Mx, const double* __restrict__ ftab, const double* __restrict__ tab,
                                TableLayout TL, const double* __restrict__ sb, double* __restrict__ gbuf, int lane) {
  constexpr int F2 = NM * NM, n = N, n2 = N * N, p = N - 1;
  const bool inner = r.nbr >= 0;
  const int po = inner ? (int)r.pn : 0, no = po + 1, no2 = no * no;
  const int mno = 65536 / no + 1;
  // the ten 1D face matrices: with STAGE the six of stages 1-2 staged in
  // LDS and the four BR2 lifting matrices (stages 3-4, read once per node)
  // through the caches; without, all ten through the caches
  const double* MP[10];
  if (STAGE) {
#pragma unroll
    for (int k = 0; k < 6; ++k) MP[k] = Mx + k * F2;
    MP[6] = ftab + r.loo[0];
    MP[7] = ftab + r.loo[1];
    MP[8] = ftab + r.lon[0];
    MP[9] = ftab + r.lon[1];
  } else {
    MP[0] = ftab + r.foo[0];
    MP[1] = ftab + r.foo[1];
    MP[2] = ftab + r.fon[0];
    MP[3] = ftab + r.fon[1];
    MP[4] = ftab + r.fnn[0];
    MP[5] = ftab + r.fnn[1];
    MP[6] = ftab + r.loo[0];
    MP[7] = ftab + r.loo[1];
    MP[8] = ftab + r.lon[0];
    MP[9] = ftab + r.lon[1];
  }
  // staging: own side (To, Do), neighbour side (Tn, Dn = k_n Do_n), matrices
  {
    const double* so = sb + ax.sb_own;
    for (int q = lane; q < n2; q += 64) {
      To[q] = so[q];
      Do[q] = so[n2 + q];
    }
    if (inner) {
      const double* sn = sb + ax.sb_nbr;
      const double kn = r.kho * r.hn;
      for (int q = lane; q < no2; q += 64) {
        W[q] = sn[q];
        W[F2 + q] = kn * sn[no2 + q];
      }
    }
    // A0oo A1oo (n x n), A0on A1on (n x no), then for BR2 A0nn A1nn (no x no)
    const int nm = !STAGE ? 0 : form == 1 ? 6 : (inner ? 4 : 2);
    for (int t = lane; t < nm * F2; t += 64) {
      const int kx = t / F2, i = t - kx * F2;
      int sz = n2, o = -1;
      switch (kx) {
        case 0: o = r.foo[0]; break;
        case 1: o = r.foo[1]; break;
        case 2: if (inner) { o = r.fon[0]; sz = n * no; } break;
        case 3: if (inner) { o = r.fon[1]; sz = n * no; } break;
        case 4: if (inner) { o = r.fnn[0]; sz = no2; } break;
        case 5: if (inner) { o = r.fnn[1]; sz = no2; } break;
        case 6: o = r.loo[0]; break;
        case 7: o = r.loo[1]; break;
        case 8: if (inner) { o = r.lon[0]; sz = n * no; } break;
        default: if (inner) { o = r.lon[1]; sz = n * no; } break;
      }
      if (o >= 0 && i < sz) Mx[t] = ftab[o + i];
    }
  }
  wave_sync();
  // stage 1: U0 = A0oo To, U1 = A0oo Do (n x n), U2 = A0on Tn, U3 = A0on Dn
  // (n x no); BR2: Y0 = A0on^T To stored transposed, Y0[a1 + n a0] (a0 < no,
  // a1 < n), Y1 = A0nn Tn (no x no). In two halves: first the products of
  // the own traces (slots 2, 3, 4), then those of the neighbour's into the
  // own traces' slots 6, 7 and slot 5 (a lane forms both products of its
  // node, reading each matrix entry once)
  constexpr int QF = (F2 + 63) / 64;
#pragma unroll
  for (int t = 0; t < QF; ++t) {
    const int q = lane + 64 * t;
    if (q >= n2) break;
    const int j0 = q % n, a1 = q / n;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int a0 = 0; a0 < n; ++a0) {
      const double mv = MP[0][j0 * n + a0];
      s0 += mv * To[a0 + n * a1];
      s1 += mv * Do[a0 + n * a1];
    }
    W[2 * F2 + q] = s0;
    W[3 * F2 + q] = s1;
  }
  if (inner && form == 1) {
    const double* A = MP[2];
    for (int q = lane; q < n * no; q += 64) {
      const int a1 = q % n, a0 = q / n;
      double s = 0.0;
#pragma unroll
      for (int j0 = 0; j0 < n; ++j0) s += A[j0 * no + a0] * To[j0 + n * a1];
      W[4 * F2 + q] = s;
    }
  }
  wave_sync();
  if (inner) {
    const double* A = MP[2];
#pragma unroll
    for (int t = 0; t < QF; ++t) {
      const int q = lane + 64 * t;
      if (q >= n * no) break;
      const int j0 = q % n, a1 = q / n;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int a0 = 0; a0 < NM; ++a0)
        if (a0 < no) {
          const double av = A[j0 * no + a0];
          s0 += av * W[a0 + no * a1];
          s1 += av * W[F2 + a0 + no * a1];
        }
      W[6 * F2 + q] = s0;
      W[7 * F2 + q] = s1;
    }
    if (form == 1) {
      const double* Ann = MP[4];
      for (int q = lane; q < no2; q += 64) {
        const int a1 = qdiv(q, mno), a0 = q - a1 * no;
        double s = 0.0;
#pragma unroll
        for (int b0 = 0; b0 < NM; ++b0)
          if (b0 < no) s += Ann[a0 * no + b0] * W[b0 + no * a1];
        W[5 * F2 + q] = s;
      }
    }
  }
  wave_sync();
  const double area = r.flen * r.flen;
  const double sgn = r.side ? 1.0 : -1.0;
  const double csym = inner ? 0.5 : 1.0;
  const double k = ax.k;
  // stage 2: v, the average and the penalty on the own side nodes; BR2: the
  // neighbour's jump vn = (A0on x A1on)^T To - (A0nn x A1nn) Tn. The
  // record's results g1, g2 stay in registers (node q = lane + 64 t in slot t)
  constexpr int QN = (n2 + 63) / 64;
  double G1[QN], G2[QN];
#pragma unroll
  for (int t = 0; t < QN; ++t) G1[t] = G2[t] = 0.0;
#pragma unroll
  for (int t = 0; t < QN; ++t) {
    const int q = lane + 64 * t;
    if (q >= n2) break;
    const int j0 = q % n, j1 = q / n;
    const double* A1oo = MP[1];
    double v = 0.0, ds = 0.0;
#pragma unroll
    for (int a1 = 0; a1 < n; ++a1) {
      const double wv = A1oo[j1 * n + a1];
      v += wv * W[2 * F2 + j0 + n * a1];
      ds += k * wv * W[3 * F2 + j0 + n * a1];
    }
    if (inner) {
      const double* A1on = MP[3];
#pragma unroll
      for (int a1 = 0; a1 < NM; ++a1)
        if (a1 < no) {
          const double wv = A1on[j1 * no + a1];
          v -= wv * W[6 * F2 + j0 + n * a1];
          ds += wv * W[7 * F2 + j0 + n * a1];
        }
    }
    double g1 = -area * csym * sgn * ds;
    if (form == 0) g1 += area * r.sig * v;
    G1[t] = g1;
    G2[t] = -csym * k * sgn * area * v;
    W[q] = v;
  }
  if (inner && form == 1) {
    const double* A1on = MP[3];
    const double* A1nn = MP[5];
    for (int q = lane; q < no2; q += 64) {
      const int b1 = qdiv(q, mno), a0 = q - b1 * no;
      double vn = 0.0;
#pragma unroll
      for (int a1 = 0; a1 < n; ++a1) vn += A1on[a1 * no + b1] * W[4 * F2 + a1 + n * a0];
#pragma unroll
      for (int c1 = 0; c1 < NM; ++c1)
        if (c1 < no) vn -= A1nn[b1 * no + c1] * W[5 * F2 + a0 + no * c1];
      W[F2 + q] = vn;
    }
  }
  wave_sync();
  if (form == 1) {
    // stage 3: P0 = L0o v (n x n), Q0 = L0n vn (n x no), one lane per node
    {
      const double* L0o = MP[6];
      const double* L0n = MP[8];
#pragma unroll
      for (int t = 0; t < QF; ++t) {
        const int q = lane + 64 * t;
        const int j0 = q % n, a1 = q / n;
        if (q < n2) {
          double s = 0.0;
#pragma unroll
          for (int a0 = 0; a0 < n; ++a0) s += L0o[j0 * n + a0] * W[a0 + n * a1];
          W[2 * F2 + q] = s;
        }
        if (inner && q < n * no) {
          double s = 0.0;
#pragma unroll
          for (int a0 = 0; a0 < NM; ++a0)
            if (a0 < no) s += L0n[j0 * no + a0] * W[F2 + a0 + no * a1];
          W[3 * F2 + q] = s;
        }
      }
    }
    wave_sync();
    // stage 4: slot 1 and the sum into g1
    double so = 0.0, sn = 0.0;
    {
      const double* Mi = tab + TL.minv + p * 81;
      constexpr int dummy = 0;
      (void)dummy;
      const int sk = r.side ? p : 0;
      so = Mi[sk * n + sk] / (ax.h * ax.h * ax.h);
      if (inner) {
        const double* Min = tab + TL.minv + po * 81;
        const int skn = (1 - r.side) ? po : 0;
        sn = Min[skn * no + skn] / (r.hn * r.hn * r.hn);
      }
    }
    const double L2 = (inner ? 0.25 : 1.0) * r.sig * area * area;
    const double* L1o = MP[7];
    const double* L1n = MP[9];
#pragma unroll
    for (int t = 0; t < QN; ++t) {
      const int q = lane + 64 * t;
      if (q >= n2) break;
      const int j0 = q % n, j1 = q / n;
      double so_acc = 0.0, sn_acc = 0.0;
#pragma unroll
      for (int a1 = 0; a1 < n; ++a1) so_acc += L1o[j1 * n + a1] * W[2 * F2 + j0 + n * a1];
      if (inner) {
#pragma unroll
        for (int a1 = 0; a1 < NM; ++a1)
          if (a1 < no) sn_acc += L1n[j1 * no + a1] * W[3 * F2 + j0 + n * a1];
      }
      G1[t] += L2 * (so * so_acc + sn * sn_acc);
    }
  }
  double* g = gbuf + ax.goff;
#pragma unroll
  for (int t = 0; t < QN; ++t) {
    const int q = lane + 64 * t;
    if (q >= n2) break;
    g[q] = G1[t];
    g[n2 + q] = G2[t];
  }
}

// one face record per wavefront (four per workgroup, wave-level
// synchronisation only); NM: largest n of the mesh
template <int NM, bool STAGE>
__global__ __launch_bounds__(256) void k_e3_face(int nrec, int xcd, int form, const FaceRec* __restrict__ recs,
                                                 const FaceAux* __restrict__ aux, const double* __restrict__ ftab,
                                                 const double* __restrict__ tab, TableLayout TL,
                                                 const double* __restrict__ sb, double* __restrict__ gbuf) {
  constexpr int F2 = NM * NM;
  __shared__ FaceRec sR[4];
  __shared__ FaceAux sAx[4];
  __shared__ double sW[4][8][F2];     // 0 Tn -> v, 1 Dn -> vn, 2 U0 -> P0, 3 U1 -> Q0, 4 Y0, 5 Y1, 6 To -> U2, 7 Do -> U3
  __shared__ double sM[STAGE ? 4 : 1][STAGE ? 6 : 1][STAGE ? F2 : 1];    // A0oo A1oo A0on A1on A0nn A1nn
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  // xcd: XCD-aware order (grid a multiple of 8): workgroups go round-robin to
  // the 8 XCDs, so block b takes record group (b % 8) per + b / 8 and each
  // XCD a contiguous range of records (a piece of the mesh, as in k_e3_vol)
  const int grp = xcd ? (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  const int rec = grp * 4 + w;
  if (rec >= nrec) return;            // whole wavefronts only: no block-wide barrier below
  {
    constexpr int WR = (int)(sizeof(FaceRec) / 8), WA = (int)(sizeof(FaceAux) / 8);
    const unsigned long long* s0 = reinterpret_cast<const unsigned long long*>(recs + rec);
    const unsigned long long* s1 = reinterpret_cast<const unsigned long long*>(aux + rec);
    if (lane < WR) reinterpret_cast<unsigned long long*>(&sR[w])[lane] = s0[lane];
    else if (lane < WR + WA) reinterpret_cast<unsigned long long*>(&sAx[w])[lane - WR] = s1[lane - WR];
  }
  wave_sync();
  double* W = &sW[w][0][0];
  double* Mx = STAGE ? &sM[w][0][0] : nullptr;
  double* To = W + 6 * F2;             // last read in the first half of stage 1
  double* Do = W + 7 * F2;
  switch (sAx[w].p) {
    case 1: e3f_body<2, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane); break;
    case 2: e3f_body<3, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane); break;
    case 3: e3f_body<4, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane); break;
    case 4: e3f_body<5, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane); break;
    case 5: e3f_body<6, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane); break;
    case 6: e3f_body<7, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane); break;
    default:
      if constexpr (NM >= 9) {
        if (sAx[w].p == 7) e3f_body<8, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane);
        else e3f_body<9, NM, STAGE>(sR[w], sAx[w], form, To, Do, W, Mx, ftab, tab, TL, sb, gbuf, lane);
      }
      break;
  }
}

template <int N>
__device__ inline void e3l_body(double (*S)[81], int* rside, int64_t* rgoff, int e, const int64_t* __restrict__ off,
                                const double* __restrict__ hh, const int32_t* __restrict__ sptr,
                                const FaceRec* __restrict__ recs, const FaceAux* __restrict__ aux,
                                const double* __restrict__ tab, TableLayout TL, const double* __restrict__ gbuf,
                                const double* __restrict__ x, double* __restrict__ y, double* __restrict__ pdot,
                                double* red) {
  constexpr int N2 = N * N, N3 = N2 * N, p = N - 1;
  const int tid = threadIdx.x;
  const int f0 = sptr[e * 6], f1 = sptr[e * 6 + 6];
  // the element's records (side, offset of g1) in LDS, in record order;
  // elements with more than 64 records take them from memory
  const int nf = f1 - f0;
  if (nf <= 64 && tid < nf) {
    rside[tid] = 2 * recs[f0 + tid].m + recs[f0 + tid].side;
    rgoff[tid] = aux[f0 + tid].goff;
  }
  __syncthreads();
  // side sums, records in order
  for (int t = tid; t < 6 * N2; t += 256) {
    const int side = t / N2, q = t - side * N2;
    double s1 = 0.0, s2 = 0.0;
    for (int f = 0; f < nf; ++f) {
      const int sf = nf <= 64 ? rside[f] : 2 * recs[f0 + f].m + recs[f0 + f].side;
      if (sf != side) continue;
      const double* g = gbuf + (nf <= 64 ? rgoff[f] : aux[f0 + f].goff);
      s1 += g[q];
      s2 += g[N2 + q];
    }
    S[side][q] = s1;
    S[6 + side][q] = s2;
  }
  __syncthreads();
  const double h = hh[e];
  const int64_t base = off[e];
  const double* D0 = tab + TL.dside + (p * 2 + 0) * 9;
  const double* D1 = tab + TL.dside + (p * 2 + 1) * 9;
  double xy = 0.0;
  for (int r = tid; r < N3; r += 256) {
    const int i[3] = {r % N, (r / N) % N, r / N2};
    double v = y[base + r];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int t0, t1;
      tdims3(m, t0, t1);
      const int q = i[t0] + N * i[t1];
      v += (D0[i[m]] * S[6 + 2 * m][q] + D1[i[m]] * S[6 + 2 * m + 1][q]) / h;
      if (i[m] == 0) v += S[2 * m][q];
      if (i[m] == p) v += S[2 * m + 1][q];
    }
    y[base + r] = v;
    xy += x[base + r] * v;
  }
  if (pdot) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) xy += __shfl_xor(xy, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = xy;
    __syncthreads();
    if (tid == 0) pdot[e] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

__global__ __launch_bounds__(256) void k_e3_lift(int ne, int xcd, const int64_t* __restrict__ off,
                                                 const int8_t* __restrict__ pdeg, const double* __restrict__ hh,
                                                 const int32_t* __restrict__ sptr, const FaceRec* __restrict__ recs,
                                                 const FaceAux* __restrict__ aux, const double* __restrict__ tab,
                                                 TableLayout TL, const double* __restrict__ gbuf,
                                                 const double* __restrict__ x, double* __restrict__ y,
                                                 double* __restrict__ pdot) {
  __shared__ double S[12][81];   // G1 of the six sides, then G2
  __shared__ double red[4];
  __shared__ int rside[64];
  __shared__ int64_t rgoff[64];
  // xcd: XCD-aware order (grid a multiple of 8), each XCD a contiguous range
  // of elements as in k_e3_vol and the face pass
  const int e = xcd ? (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  if (e >= ne) return;
  switch (pdeg[e]) {
    case 1: e3l_body<2>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    case 2: e3l_body<3>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    case 3: e3l_body<4>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    case 4: e3l_body<5>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    case 5: e3l_body<6>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    case 6: e3l_body<7>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    case 7: e3l_body<8>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
    default: e3l_body<9>(S, rside, rgoff, e, off, hh, sptr, recs, aux, tab, TL, gbuf, x, y, pdot, red); break;
  }
}

// sum over a block of 256 threads in a fixed order; valid in thread 0
__device__ inline double block_sum256(double v) {
  __shared__ double sw[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((sw[0] + sw[1]) + (sw[2] + sw[3]));
}

// nrhs == 1: x += alpha p ; r -= alpha Ap, and the block's share of r'r;
// with rt also the single-precision copy of r that an FP32 B reads
__global__ __launch_bounds__(256) void k_cg_update_rr(int64_t n, const double* __restrict__ alpha,
                                                     const double* __restrict__ p, const double* __restrict__ Ap,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ part, float* __restrict__ rt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rr = 0.0;
  if (i < n) {
    const double al = alpha[0];
    x[i] += al * p[i];
    const double ri = r[i] - al * Ap[i];
    r[i] = ri;
    if (rt) rt[i] = (float)ri;
    rr = ri * ri;
  }
  const double s = block_sum256(rr);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of n shares in the order of the one-block final stages k_dot_final_pap
// and k_dot_final_rr_rz (each thread's ordered_sum with stride 256, then the
// halving tree): every block that calls it gets the same value, bitwise that
// of those stages.
__device__ inline double shares_sum(const double* __restrict__ part, int n, double* sm) {
  const int t = threadIdx.x;
  sm[t] = ordered_sum(part, t, 256, n, 1, 0);
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) sm[t] += sm[t + w];
    __syncthreads();
  }
  const double v = sm[0];
  __syncthreads();
  return v;
}

// One RHS, the final stages folded into the vector kernels that follow them
// (one launch fewer each): every block repeats the final reduction of the
// shares and takes the same scalar decisions; block 0 stores the scalars.
// No block reads a scalar that another block of the same launch writes,
// except the activity and breakdown flags, which only go from set to
// cleared (activity) or from clear to set (breakdown): a block that already
// sees block 0's store takes the branch block 0 took.
//
// p'Ap from its nsh shares, alpha = r'z / p'Ap while active (r'z from rzn,
// copied to rz), then x += alpha p, r -= alpha Ap and the block's share of
// r'r (and the FP32 copy of r) as k_cg_update_rr. A breakdown sets err here;
// the activity flag is
// cleared by k_cg_dir_rr_rz.
__global__ __launch_bounds__(256) void k_cg_update_pap(int64_t n, int nsh, const double* __restrict__ sh, CGScal S,
                                                       const double* __restrict__ p, const double* __restrict__ Ap,
                                                       double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ part, float* __restrict__ rt) {
  __shared__ double sm[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int act0 = S.act[0];
  const double rz = S.rzn[0];
  double pi = 0.0, api = 0.0, xi = 0.0, ri = 0.0;
  if (i < n) {
    pi = p[i];
    api = Ap[i];
    xi = x[i];
    ri = r[i];
  }
  const double v = shares_sum(sh, nsh, sm);
  const bool ok = act0 && v > 0.0;
  const double al = ok ? rz / v : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.pAp[0] = v;
    S.alpha[0] = al;
    S.rz[0] = rz;
    if (act0 && !(v > 0.0)) S.err[0] = 1;
  }
  double rr = 0.0;
  if (i < n) {
    x[i] = xi + al * pi;
    const double rn = ri - al * api;
    r[i] = rn;
    if (rt) rt[i] = (float)rn;
    rr = rn * rn;
  }
  const double s = block_sum256(rr);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// r'r (na shares pa) and r'z (nb shares pb) as in k_dot_final_rr_rz, then
// p = z + beta p while active. Block 0 stores r'r, alpha's and beta's
// histories, the iteration count, the new r'z (in rzn), beta and the flags
// (including the activity flag after a breakdown in k_cg_update_pap).
__global__ __launch_bounds__(256) void k_cg_dir_rr_rz(int64_t n, int na, const double* __restrict__ pa, int nb,
                                                      const double* __restrict__ pb, CGScal S,
                                                      const double* __restrict__ z, double* __restrict__ p) {
  __shared__ double sm[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int act0 = S.act[0], err0 = S.err[0], it0 = S.iters[0];
  const double tol2 = S.tol2[0], bb = S.bb[0], rz = S.rz[0];
  double zi = 0.0, pi = 0.0;
  if (i < n) {
    zi = z[i];
    pi = p[i];
  }
  const double v0 = shares_sum(pa, na, sm);
  const double v1 = shares_sum(pb, nb, sm);
  const bool run = act0 && !err0;   // active through this iteration's update
  bool act = run && v0 > tol2 * bb;
  const bool brk = act && !(v1 > 0.0);
  act = act && !brk;
  const double beta = act ? v1 / rz : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.rr[0] = v0;
    if (run) {
      if (it0 < S.maxit) S.ahist[(int64_t)it0 * S.hs] = S.alpha[0];
      S.iters[0] = it0 + 1;
    }
    if (act0 && !act) S.act[0] = 0;
    if (brk) S.err[0] = 1;
    S.beta[0] = beta;
    if (act) {
      S.rzn[0] = v1;
      if (it0 < S.maxit) S.bhist[(int64_t)it0 * S.hs] = beta;
    }
  }
  if (i < n && act) p[i] = zi + beta * pi;
}

// p = z + beta p while active
__global__ void k_cg_dir2(int64_t n, int nrhs, const double* __restrict__ beta, const int* __restrict__ act,
                          const double* __restrict__ z, double* __restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % nrhs);
  // all loads issued together; the store depends on the flag only
  const double zi = z[i], pi = p[i], bc = beta[c];
  if (act[c]) p[i] = zi + bc * pi;
}



// x = d . b (pre-smoothing from zero)
template <typename T>
__global__ __launch_bounds__(256) void k_dscale(int n, const T* __restrict__ d, const T* __restrict__ b,
                                                T* __restrict__ x) {
  const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (i < n) x[i] = d[i] * b[i];
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = a[i] - b[i];
}

// ------------------------------------------------------------------- CSR
// modes: 0 y = A x; 1 y = b - A x; 2 y = b + A x;
//        3 (pre-smoother from zero) xo = d.b, y = b - A (d.b);
//        4 (post-smoother) y = x + d.(b - A x);
//        5 y = A [x; b] (columns below nsplit read x, the others b)
// Rows are binned at setup: the first nlong_blk blocks take the long rows
// (one wavefront per row, 4 per block), the others the short rows (LPR
// lanes per row). rows[] lists long rows first, then short rows.
template <typename T, int MODE>
__device__ inline void spmv_row_out(int row, T acc, const T* __restrict__ x, const T* __restrict__ b,
                                    const T* __restrict__ d, T* __restrict__ xo, T* __restrict__ y) {
  if (MODE == 0) y[row] = acc;
  else if (MODE == 1) y[row] = b[row] - acc;
  else if (MODE == 2) y[row] = b[row] + acc;
  else if (MODE == 3) {
    xo[row] = d[row] * x[row];
    y[row] = x[row] - acc;
  } else if (MODE == 4) {
    y[row] = x[row] + d[row] * (b[row] - acc);
  } else {
    y[row] = acc;
  }
}

// operand of one nonzero: MODE 3 scales by d; MODE 5 reads from two vectors,
// columns below nsplit from x and the others from b (shifted by nsplit)
template <typename T, int MODE>
__device__ inline T spmv_src(int j, int nsplit, const T* __restrict__ x, const T* __restrict__ b,
                             const T* __restrict__ d) {
  if (MODE == 3) return d[j] * x[j];
  if (MODE == 5) {
    const T* src = j < nsplit ? x + j : b + (j - nsplit);
    return *src;
  }
  return x[j];
}

// one 4-entry chunk of a padded row, added in entry order
template <typename T, int MODE>
__device__ inline T spmv_chunk(T acc, int c, int nsplit, const int4* __restrict__ idx4, const T* __restrict__ val,
                               const T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ d) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const int4 j = idx4[c];
  const v4 v = reinterpret_cast<const v4*>(val)[c];
  acc += v.x * spmv_src<T, MODE>(j.x, nsplit, x, b, d);
  acc += v.y * spmv_src<T, MODE>(j.y, nsplit, x, b, d);
  acc += v.z * spmv_src<T, MODE>(j.z, nsplit, x, b, d);
  acc += v.w * spmv_src<T, MODE>(j.w, nsplit, x, b, d);
  return acc;
}

// rows padded to multiples of 4 entries: lanes take 4-entry chunks
template <typename T, int MODE, int LPR>
__global__ __launch_bounds__(256) void k_spmv(int nlong, int nlong_blk, int nshort, int nsplit,
                                              const int32_t* __restrict__ rows,
                                              const int32_t* __restrict__ ptr,
                                              const int32_t* __restrict__ idx, const T* __restrict__ val,
                                              const T* __restrict__ x, const T* __restrict__ b,
                                              const T* __restrict__ d, T* __restrict__ xo, T* __restrict__ y) {
  const int4* idx4 = reinterpret_cast<const int4*>(idx);
  if ((int)blockIdx.x < nlong_blk) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= nlong) return;
    const int row = rows[w];
    T acc = 0;
    const int c1 = ptr[row + 1] >> 2;
#pragma unroll 2
    for (int c = (ptr[row] >> 2) + lane; c < c1; c += 64) acc = spmv_chunk<T, MODE>(acc, c, nsplit, idx4, val, x, b, d);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) spmv_row_out<T, MODE>(row, acc, x, b, d, xo, y);
    return;
  }
  const int gt = (blockIdx.x - nlong_blk) * 256 + threadIdx.x;
  const int r = gt / LPR;
  const int sub = gt % LPR;
  if (r >= nshort) return;
  const int row = rows[nlong + r];
  T acc = 0;
  const int c1 = ptr[row + 1] >> 2;
#pragma unroll 2
  for (int c = (ptr[row] >> 2) + sub; c < c1; c += LPR) acc = spmv_chunk<T, MODE>(acc, c, nsplit, idx4, val, x, b, d);
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LPR);
  if (sub == 0) spmv_row_out<T, MODE>(row, acc, x, b, d, xo, y);
}

// same with nrhs interleaved columns: one thread per (row, rhs)
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_spmm(int nrows, int nrhs, int nsplit, const int32_t* __restrict__ ptr,
                                              const int32_t* __restrict__ idx, const T* __restrict__ val,
                                              const T* __restrict__ x, const T* __restrict__ b,
                                              const T* __restrict__ d, T* __restrict__ xo, T* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = t / nrhs;
  const int c = (int)(t - row * nrhs);
  if (row >= nrows) return;
  T acc = 0;
#pragma unroll 4
  for (int q = ptr[row]; q < ptr[row + 1]; ++q) {
    const int64_t j = idx[q];
    T xv;
    if (MODE == 3) xv = d[j] * x[j * nrhs + c];
    else if (MODE == 5) xv = *(j < nsplit ? x + j * nrhs + c : b + (j - nsplit) * nrhs + c);
    else xv = x[j * nrhs + c];
    acc += val[q] * xv;
  }
  const int64_t o = row * nrhs + c;
  if (MODE == 0 || MODE == 5) y[o] = acc;
  else if (MODE == 1) y[o] = b[o] - acc;
  else if (MODE == 2) y[o] = b[o] + acc;
  else if (MODE == 3) {
    xo[o] = d[row] * x[o];
    y[o] = x[o] - acc;
  } else {
    y[o] = x[o] + d[row] * (b[o] - acc);
  }
}

// lane l's value of v, for a wave-uniform l (a scalar)
__device__ __forceinline__ int e_readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float e_readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double e_readlane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// k_spmm for nrhs a multiple of 64: one wavefront per (row, 64 RHS). The
// row's column indices and values are loaded by the lanes, up to 64 at a
// time, and read back as scalars, so the x loads of the row go out together
// instead of each waiting for its index, G at a time; the same terms in the
// same order (bitwise the same results).
template <typename T, int MODE, int G>
__global__ __launch_bounds__(256) void k_spmm64(int nrows, int nrhs, int nsplit, const int32_t* __restrict__ ptr,
                                                const int32_t* __restrict__ idx, const T* __restrict__ val,
                                                const T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ d, T* __restrict__ xo, T* __restrict__ y) {
  const int lane = (int)(threadIdx.x & 63);
  const int ng = nrhs >> 6;
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6));
  const int64_t row = w / ng;
  if (row >= nrows) return;   // the whole wavefront
  const int c = (int)(w - row * ng) * 64 + lane;
  auto xload = [&](int64_t j) -> T {
    if (MODE == 3) return d[j] * x[j * nrhs + c];
    if (MODE == 5) return *(j < nsplit ? x + j * nrhs + c : b + (j - nsplit) * nrhs + c);
    return x[j * nrhs + c];
  };
  const int q0 = ptr[row], q1 = ptr[row + 1];
  T acc = 0;
  for (int qb = q0; qb < q1; qb += 64) {
    const int nq = min(64, q1 - qb);
    const int ql = qb + min(lane, nq - 1);
    const int jl = idx[ql];
    const T vl = val[ql];
    int u = 0;
    for (; u + G <= nq; u += G) {
      T xv[G], vv[G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        vv[k] = e_readlane(vl, u + k);
        xv[k] = xload(e_readlane(jl, u + k));
      }
#pragma unroll
      for (int k = 0; k < G; ++k) acc += vv[k] * xv[k];
    }
    for (; u < nq; ++u) acc += e_readlane(vl, u) * xload(e_readlane(jl, u));
  }
  const int64_t o = row * nrhs + c;
  if (MODE == 0 || MODE == 5) y[o] = acc;
  else if (MODE == 1) y[o] = b[o] - acc;
  else if (MODE == 2) y[o] = b[o] + acc;
  else if (MODE == 3) {
    xo[o] = d[row] * x[o];
    y[o] = x[o] - acc;
  } else {
    y[o] = x[o] + d[row] * (b[o] - acc);
  }
}

// z_out (double) = zb + P e   (prolongation of the conforming correction)
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_out(int nrows, int nrhs, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ idx, const T* __restrict__ val,
                                                     const T* __restrict__ e, const T* __restrict__ zb,
                                                     double* __restrict__ z, const double* __restrict__ rdot,
                                                     double* __restrict__ pdot) {
  // z = z_B + P e; with pdot (nrhs == 1) also the block's share of r'z
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = t / nrhs;
  const int c = (int)(t - row * nrhs);
  double rz = 0.0;
  if (row < nrows) {
    T acc = 0;
#pragma unroll 4
    for (int q = ptr[row]; q < ptr[row + 1]; ++q) acc += val[q] * e[(int64_t)idx[q] * nrhs + c];
    const double zv = (double)(zb[row * nrhs + c] + acc);
    z[row * nrhs + c] = zv;
    if (pdot) rz = rdot[row] * zv;
  }
  if (pdot) {
    const double s = block_sum256(rz);
    if (threadIdx.x == 0) pdot[blockIdx.x] = s;
  }
}


// front of B (nrhs == 1): three independent pieces in one launch, split by
// block index: [0, nb_diag) point Jacobi z = dinv . r on all DOFs,
// [nb_diag, nb_diag + nb_blk) V_e block solves (LPR lanes per block row),
// the rest r_c = P^T r (binned rows as in k_spmv).
template <typename T, int LPRB, int LPRP>
__global__ __launch_bounds__(256) void k_front(int64_t ndof, int nb_diag, const T* __restrict__ dinv,
                                               int64_t brows, int nb_blk, const int32_t* __restrict__ row_blk,
                                               const int32_t* __restrict__ row_loc,
                                               const int64_t* __restrict__ bptr, const int64_t* __restrict__ boff,
                                               const int32_t* __restrict__ bdof, const int32_t* __restrict__ bout,
                                               const T* __restrict__ binv, int nlong, int nlong_blk, int nshort,
                                               const int32_t* __restrict__ rows, const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ idx, const T* __restrict__ val,
                                               const T* __restrict__ r, T* __restrict__ z, T* __restrict__ rc) {
  int b = blockIdx.x;
  if (b < nb_diag) {
    // V_e DOFs carry dinv = -0.0 and are written by the block part only
    int64_t i = (int64_t)b * 256 + threadIdx.x;
    if (i < ndof) {
      T d = dinv[i];
      if (!signbit(d)) z[i] = d * r[i];
    }
    return;
  }
  b -= nb_diag;
  if (b < nb_blk) {
    const int64_t gt = (int64_t)b * 256 + threadIdx.x;
    const int64_t rw = gt / LPRB;
    const int sub = (int)(gt % LPRB);
    if (rw >= brows) return;
    const int bk = row_blk[rw];
    const int i = row_loc[rw];
    const int64_t s0 = bptr[bk];
    const int m = (int)(bptr[bk + 1] - s0);
    const T* row = binv + boff[bk] + (int64_t)i * blk_ld(m);
    T acc = 0;
#pragma unroll 4
    for (int j = sub; j < m; j += LPRB) acc += row[j] * r[bdof[s0 + j]];
#pragma unroll
    for (int o = LPRB / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LPRB);
    // V_e DOFs have dinv = 0, so the block result is the whole value there
    if (sub == 0) z[bout[s0 + i]] = acc;
    return;
  }
  b -= nb_blk;
  const int4* idx4 = reinterpret_cast<const int4*>(idx);
  if (b < nlong_blk) {
    const int w = b * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= nlong) return;
    const int row = rows[w];
    T acc = 0;
    const int c1 = ptr[row + 1] >> 2;
#pragma unroll 2
    for (int c = (ptr[row] >> 2) + lane; c < c1; c += 64)
      acc = spmv_chunk<T, 0>(acc, c, 0, idx4, val, r, nullptr, nullptr);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) rc[row] = acc;
    return;
  }
  b -= nlong_blk;
  const int gt = b * 256 + threadIdx.x;
  const int rr = gt / LPRP;
  const int sub = gt % LPRP;
  if (rr >= nshort) return;
  const int row = rows[nlong + rr];
  T acc = 0;
  const int c1 = ptr[row + 1] >> 2;
#pragma unroll 2
  for (int c = (ptr[row] >> 2) + sub; c < c1; c += LPRP) acc = spmv_chunk<T, 0>(acc, c, 0, idx4, val, r, nullptr, nullptr);
#pragma unroll
  for (int o = LPRP / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LPRP);
  if (sub == 0) rc[row] = acc;
}

// exact V_e solves, interleaved RHS: one thread per (block row, rhs)
template <typename T>
__global__ __launch_bounds__(256) void k_block_gemv(int64_t nrows, int nrhs, const int32_t* __restrict__ row_blk,
                                                    const int32_t* __restrict__ row_loc,
                                                    const int64_t* __restrict__ bptr,
                                                    const int64_t* __restrict__ boff,
                                                    const int32_t* __restrict__ bdof, const int32_t* __restrict__ bout,
                                                    const T* __restrict__ binv, const T* __restrict__ r,
                                                    T* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t rw = t / nrhs;
  const int c = (int)(t - rw * nrhs);
  if (rw >= nrows) return;
  const int b = row_blk[rw];
  const int i = row_loc[rw];
  const int64_t s0 = bptr[b];
  const int m = (int)(bptr[b + 1] - s0);
  const T* row = binv + boff[b] + (int64_t)i * blk_ld(m);
  T acc = 0;
#pragma unroll 4
  for (int j = 0; j < m; ++j) acc += row[j] * r[(int64_t)bdof[s0 + j] * nrhs + c];
  z[(int64_t)bout[s0 + i] * nrhs + c] = acc;
}

// exact V_e solves, interleaved RHS: one workgroup per block; the block's
// r values (m x nrhs) are staged in LDS once and every (row, rhs) pair of the
// block reads them from there (dynamic LDS: m_max * nrhs values)
template <typename T>
__global__ __launch_bounds__(256) void k_block_gemm(int nblocks, int nrhs, const int64_t* __restrict__ bptr,
                                                    const int64_t* __restrict__ boff,
                                                    const int32_t* __restrict__ bdof, const int32_t* __restrict__ bout,
                                                    const T* __restrict__ binv, const T* __restrict__ r,
                                                    T* __restrict__ z) {
  extern __shared__ unsigned char blk_lds[];
  T* rl = reinterpret_cast<T*>(blk_lds);
  const int b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t s0 = bptr[b];
  const int m = (int)(bptr[b + 1] - s0);
  for (int t = threadIdx.x; t < m * nrhs; t += 256) {
    const int j = t / nrhs, c = t - j * nrhs;
    rl[t] = r[(int64_t)bdof[s0 + j] * nrhs + c];
  }
  __syncthreads();
  const T* B = binv + boff[b];
  const int ld = blk_ld(m);
  for (int t = threadIdx.x; t < m * nrhs; t += 256) {
    const int i = t / nrhs, c = t - i * nrhs;
    T acc = 0;
    for (int j = 0; j < m; ++j) acc += B[(int64_t)i * ld + j] * rl[j * nrhs + c];
    z[(int64_t)bout[s0 + i] * nrhs + c] = acc;
  }
}

// exact V_e solves for many RHS (nrhs a multiple of 16) on the matrix cores:
// Z_b = B_b R_b per block in 16 x 16 output tiles (block rows x right-hand
// sides), each a chain of 16x16x4 MFMA steps over the block's columns. The
// stored inverse B_b is exactly symmetric, so the A operand B_b[i][k] is read
// as B_b[k][i]: 16 consecutive entries of a row per lane group. Operand
// layout of the 16x16x4 steps on gfx950 (one 64-lane wavefront, checked by a
// lane probe): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its
// accumulator entry v holds D[row][l % 16] with row = 4 (l / 16) + v for FP32
// and row = l / 16 + 4 v for FP64. One workgroup (4 wavefronts) per block;
// the block's DOF list is staged in LDS (dynamic, m int32).
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};
template <>
struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return lk + 4 * v; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_block_mfma(int nblocks, int nrhs, const int64_t* __restrict__ bptr,
                                                    const int64_t* __restrict__ boff,
                                                    const int32_t* __restrict__ bdof, const int32_t* __restrict__ bout,
                                                    const T* __restrict__ binv, const T* __restrict__ r,
                                                    T* __restrict__ z) {
  extern __shared__ unsigned char blk_lds[];
  int32_t* sdof = reinterpret_cast<int32_t*>(blk_lds);
  const int b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t s0 = bptr[b];
  const int m = (int)(bptr[b + 1] - s0);
  for (int t = threadIdx.x; t < m; t += 256) sdof[t] = bdof[s0 + t];
  __syncthreads();
  const T* B = binv + boff[b];
  const int ld = blk_ld(m);
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int nti = (m + 15) >> 4, ntj = nrhs >> 4;
  for (int tile = wv; tile < nti * ntj; tile += 4) {
    const int i0 = (tile % nti) * 16, j0 = (tile / nti) * 16;
    const int i = i0 + li;
    typename Mfma16<T>::v4 acc = {0, 0, 0, 0};
    // four k-steps per pass: their eight operand loads in flight together
    for (int k0 = 0; k0 < m; k0 += 16) {
      T a[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + lk;
        a[u] = 0;
        bv[u] = 0;
        if (k < m) {
          if (i < m) a[u] = B[(int64_t)k * ld + i];
          bv[u] = r[(int64_t)sdof[k] * nrhs + j0 + li];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = Mfma16<T>::step(a[u], bv[u], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + Mfma16<T>::row(lk, v);
      if (row < m) z[(int64_t)bout[s0 + row] * nrhs + j0 + li] = acc[v];
    }
  }
}

// exact V_e solves for one RHS, one workgroup per block (blocks listed by
// order[], largest first): the block's r values are gathered into LDS once
// (zeros up to the padded row length), then LPR lanes per row stream the row
// of the stored inverse against them in 4-entry vector loads and add their
// parts in a fixed order. Each lane group takes four rows per pass, so that
// four rows' loads are in flight together. Dynamic LDS: blk_ld(m_max)
// values.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_block_rows(int nblocks, const int32_t* __restrict__ order,
                                                    const int64_t* __restrict__ bptr,
                                                    const int64_t* __restrict__ boff,
                                                    const int32_t* __restrict__ bdof, const int32_t* __restrict__ bout,
                                                    const T* __restrict__ binv, const T* __restrict__ r,
                                                    T* __restrict__ z) {
  extern __shared__ unsigned char blk_lds[];
  T* rl = reinterpret_cast<T*>(blk_lds);
  if ((int)blockIdx.x >= nblocks) return;
  const int b = order[blockIdx.x];
  const int64_t s0 = bptr[b];
  const int m = (int)(bptr[b + 1] - s0);
  const int q = blk_ld(m) >> 2;
  for (int t = threadIdx.x; t < 4 * q; t += 256) rl[t] = t < m ? r[bdof[s0 + t]] : T(0);
  __syncthreads();
  typedef T v4 __attribute__((ext_vector_type(4)));
  const v4* B = reinterpret_cast<const v4*>(binv + boff[b]);
  const v4* r4 = reinterpret_cast<const v4*>(rl);
  const int sub = (int)(threadIdx.x % LPR);
  constexpr int G = 256 / LPR, R = 4;
  for (int i0 = (int)(threadIdx.x / LPR); i0 < m; i0 += R * G) {
    T acc[R];
#pragma unroll
    for (int u = 0; u < R; ++u) acc[u] = 0;
    for (int j = sub; j < q; j += LPR) {
      const v4 x = r4[j];
      v4 a[R];
#pragma unroll
      for (int u = 0; u < R; ++u)
        if (i0 + u * G < m) a[u] = B[(int64_t)(i0 + u * G) * q + j];
#pragma unroll
      for (int u = 0; u < R; ++u)
        if (i0 + u * G < m) {
          acc[u] += a[u].x * x.x;
          acc[u] += a[u].y * x.y;
          acc[u] += a[u].z * x.z;
          acc[u] += a[u].w * x.w;
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
#pragma unroll
      for (int o = LPR / 2; o > 0; o >>= 1) acc[u] += __shfl_xor(acc[u], o, LPR);
      if (sub == 0 && i0 + u * G < m) z[bout[s0 + i0 + u * G]] = acc[u];
    }
  }
}

// overlapping V_e (3D): the block solves write one slot per block row past
// the DG vector; every N-DOF then sums the slots of the blocks that hold it,
// in block order (fixed, so results do not depend on scheduling):
// z[dof] = sum_q z[slot_q] (interleaved RHS)
template <typename T>
__global__ __launch_bounds__(256) void k_block_gather(int ndofs, int nrhs, const int32_t* __restrict__ gdof,
                                                      const int32_t* __restrict__ gptr,
                                                      const int32_t* __restrict__ gslot, T* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = t / nrhs;
  const int c = (int)(t - row * nrhs);
  if (row >= ndofs) return;
  T acc = 0;
  for (int q = gptr[row]; q < gptr[row + 1]; ++q) acc += z[(int64_t)gslot[q] * nrhs + c];
  z[(int64_t)gdof[row] * nrhs + c] = acc;
}

// dense x = C b for many RHS (nrhs a multiple of 16) on the matrix cores: one
// workgroup per 16 x 16 output tile (rows x right-hand sides); its four
// wavefronts take a quarter of the columns of C each (16x16x4 MFMA steps, four
// per pass) and their partial tiles are added in wavefront order through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_mfma(int n, int nrhs, const T* __restrict__ C,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  __shared__ T red[4][64][4];
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int i = i0 + li;
  const int kq = (((n + 3) / 4 + 15) / 16) * 16;   // columns per wavefront, a multiple of 16
  const int ka = wv * kq, kb = min(n, ka + kq);
  typename Mfma16<T>::v4 acc = {0, 0, 0, 0};
  for (int k0 = ka; k0 < kb; k0 += 16) {
    T a[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + lk;
      a[u] = 0;
      bv[u] = 0;
      if (k < kb) {
        if (i < n) a[u] = C[(int64_t)i * n + k];
        bv[u] = b[(int64_t)k * nrhs + j0 + li];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = Mfma16<T>::step(a[u], bv[u], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][lane][v] = acc[v];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T sum = ((red[0][lane][v] + red[1][lane][v]) + red[2][lane][v]) + red[3][lane][v];
      const int row = i0 + Mfma16<T>::row(lk, v);
      if (row < n) x[(int64_t)row * nrhs + j0 + li] = sum;
    }
  }
}

// coarsest level, interleaved RHS: a workgroup per row, its 256 / nrhs lane
// groups split the row and add their parts in a fixed order
template <typename T>
__global__ __launch_bounds__(256) void k_dense_gemm(int n, int nrhs, const T* __restrict__ C,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  __shared__ T part[256];
  const int row = blockIdx.x;
  const int c = threadIdx.x % nrhs, g = threadIdx.x / nrhs, ng = 256 / nrhs;
  T acc = 0;
#pragma unroll 4
  for (int j = g; j < n; j += ng) acc += C[(int64_t)row * n + j] * b[(int64_t)j * nrhs + c];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (g == 0) {
    T s = part[c];
    for (int q = 1; q < ng; ++q) s += part[q * nrhs + c];
    x[(int64_t)row * nrhs + c] = s;
  }
}

// final stage of a dot product for many RHS: one workgroup per RHS, fixed
// summation order, then the scalar epilogue
__global__ __launch_bounds__(256) void k_dot_final_rhs(int nblocks, int nrhs, const double* __restrict__ part,
                                                       int mode, CGScal S) {
  __shared__ double sm[256];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  double s = ordered_sum(part, t, 256, nblocks, nrhs, c);
  sm[t] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) sm[t] += sm[t + w];
    __syncthreads();
  }
  if (t == 0) cg_epilogue(mode, c, sm[0], S);
}

// coarsest level: x = C b (dense inverse). nrhs == 1: one wavefront per row
// (coalesced row reads); otherwise one thread per (row, rhs)
template <typename T>
__global__ __launch_bounds__(256) void k_dense_gemv1(int n, const T* __restrict__ C, const T* __restrict__ b,
                                                     T* __restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  T acc = 0;
#pragma unroll 4
  for (int j = lane; j < n; j += 64) acc += C[(int64_t)row * n + j] * b[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) x[row] = acc;
}


}  // namespace hpdg
