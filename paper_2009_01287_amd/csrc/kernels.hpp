// Device-side data layout shared by the HIP kernels and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpdg {

// One face as seen from one of its two elements (or the only one on the
// boundary). 88 bytes; the neighbour's degree, first DOF and coefficient are
// copied in so that the element kernel needs no second lookup.
struct FaceRec {
  int32_t nbr;      // neighbour element, -1 on the boundary
  int8_t side;      // side of the own element: 0 lower (normal -e_m), 1 upper
  int8_t m;         // normal dimension
  int8_t q;         // Gauss points per tangential dimension (max p + 1)
  int8_t pn;        // neighbour degree (0 on the boundary)
  uint8_t oc[2];    // sub-interval code of the face inside the own side, per tangential slot
  uint8_t nc[2];    // same inside the neighbour's side
  int32_t nbase;    // first DOF of the neighbour
  int32_t foo[2];   // per tangential slot: offsets (doubles) in the face-matrix table of
  int32_t fon[2];   //   the unit-length 1D face-mass matrices A_oo (own x own),
  int32_t fnn[2];   //   A_on (own x neighbour), A_nn (neighbour x neighbour)
  int32_t loo[2];   // per slot: A_oo Minv_own and A_on Minv_nbr (BR2 liftings)
  int32_t lon[2];
  double flen;      // physical face side length
  double sig;       // SIPG penalty sigma, or eta*k_e for BR2
  double kho;       // neighbour k / h (0 on the boundary)
  double hn;        // neighbour h (1 on the boundary)
};
static_assert(sizeof(FaceRec) == 88, "FaceRec layout");

// Stored V_e block inverses: block b (m x m, row-major) starts at boff[b]
// with its rows padded to blk_ld(m) entries (zeros past column m), so that
// every row starts on a 4-entry boundary for vector loads.
__host__ __device__ inline int blk_ld(int m) { return (m + 3) & ~3; }

// Tables of the 1D basis, all degrees, in one device buffer (doubles).
struct TableLayout {
  int64_t dside;      // l_i'(0), l_i'(1): dside[(p*2+s)*9+i]
  int64_t minv;       // inverse 1D mass: minv[p*81+i*(p+1)+j]
  int64_t mk;         // M, K: mk[(p*2+0)*81 + i*(p+1)+j] is M, +1 is K
  int64_t total;
};


}  // namespace hpdg
