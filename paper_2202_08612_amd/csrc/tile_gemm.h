// Large-tile FP64 MFMA GEMM for the O(n_o^3 n_v^3 N) contractions of the triples path.
#pragma once
#include "mlcc3_internal.h"

namespace mlcc3 {

// one product term of a TileGemm.  B(k,n) = B[z*bbatch + k*ldb + n];
// A(m,k) = A[z*abatch + amap(m) + k] when TileGemm::ak, else A[z*abatch + amap(k) + m]
struct TgSeg {
  const double *A = nullptr;
  Idx2 amap;
  long long abatch = 0;
  const double *B = nullptr;
  long long ldb = 0, bbatch = 0;
  int K = 0;
};

// C[z*cbatch + cmap(m) + n] = alpha * sum_seg sum_k A_seg(m,k) B_seg(k,n) + beta * C[...]
// for m < M, n < N, z < nbatch
struct TileGemm {
  int M = 0, N = 0, nbatch = 1, nseg = 0;
  TgSeg seg[2];
  int ak = 1;
  double *C = nullptr;
  Idx2 cmap;
  long long cbatch = 0;
  double alpha = 1.0, beta = 0.0;
  int dcontract = 0;   // the d-contraction of the triples: launched under its own kernel symbol
  // split-K: batch index zz of the launch = z * ksplit + part; part takes the part-th slice of
  // every segment's K (multiples of 16).  The host points C at a partial buffer for it.
  int ksplit = 1;
};

hipError_t tile_gemm_f64(const TileGemm &g, hipStream_t s);
long long tile_gemm_blocks(const TileGemm &g);

}  // namespace mlcc3
