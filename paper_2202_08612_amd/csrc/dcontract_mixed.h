// Mixed-precision (FP32 MFMA) d-contraction of the triples intermediate.
#pragma once
#include "mlcc3_internal.h"

namespace mlcc3 {

// one product term: A[m][k] (FP32, row pitch lda) times B[z][k][n] (FP32, row pitch ldb,
// batch pitch bbatch); k < Kp, where rows K <= k < Kp of B and columns of A are zero padding;
// B columns N <= n < Np are padding.  Kp, Np, lda, ldb, bbatch multiples of 4, bases 16-byte aligned.
// (vector v: A + v*avec, B + v*bvec)
struct MixSeg {
  const float *A = nullptr;
  long long lda = 0, avec = 0;
  const float *B = nullptr;
  long long ldb = 0, bbatch = 0, bvec = 0;
  int Kp = 0, Np = 0;
};

// C[z*cbatch + cmap(m) + n] = sum_seg sum_k A_seg[m][k] B_seg[z][k][n]  (FP32 MFMA; FP32 sums over
// 32-deep K slabs, added in FP64)
// for every vector v < nvec: C + v*cvec; persist > 0 caps the grid (workgroups loop over tiles)
struct MixGemm {
  int M = 0, N = 0, nbatch = 1, nseg = 0, nvec = 1;
  MixSeg seg[2];
  double *C = nullptr;
  Idx2 cmap;
  long long cbatch = 0, cvec = 0;
  int persist = 0;
  // core-valence separation: skip tiles whose (p,q,r) are all valence (see TileGemm)
  int cvs = 0, cvs_no = 0, cvs_nv = 0;
  unsigned long long cvs_bits = 0;
};

hipError_t dcontract_f32(const MixGemm &g, hipStream_t s);
// dst[b][r][c] (b < nb, r < Rp, c < Cp) = FP32 of src[b][r][c] inside R x C, zero outside
hipError_t pad_to_f32(const double *src, int nb, int R, int C, float *dst, int Rp, int Cp, hipStream_t s);

}  // namespace mlcc3
