// The d-contraction of the triples intermediate as a dedicated FP64 MFMA kernel.
#pragma once
#include "mlcc3_internal.h"

namespace mlcc3 {

// one product term: A[m][k] (row pitch lda, the same for every batch) times
// B[z][k][n] (row pitch ldb, batch pitch bbatch), k < K
struct DcSeg {
  const double *A = nullptr;
  long long lda = 0;
  const double *B = nullptr;
  long long ldb = 0, bbatch = 0;
  int K = 0;
};

// C[z][crow(m) + n] = sum_seg sum_k A_seg[m][k] B_seg[z][k][n], m < M, n < N, z < nbatch,
// crow(m) = (m / crow_d) * crow_s1 + (m % crow_d) * crow_s0 (C is overwritten)
struct Dcontract {
  int M = 0, N = 0, nbatch = 1, nseg = 0;
  DcSeg seg[2];
  double *C = nullptr;
  int crow_d = 1;
  long long crow_s1 = 0, crow_s0 = 0, cbatch = 0;
  int remap = 1;   // XCD-aware workgroup order
};

hipError_t dcontract_f64(const Dcontract &g, hipStream_t s);
long long dcontract_blocks(const Dcontract &g);

}  // namespace mlcc3
