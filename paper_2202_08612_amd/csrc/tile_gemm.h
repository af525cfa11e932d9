// Large-tile FP64 MFMA GEMM for the O(n_o^3 n_v^3 N) contractions of the triples path.
#pragma once
#include "mlcc3_internal.h"

namespace mlcc3 {

// one product term of a TileGemm, for vector v < nvec and batch z < nbatch:
// B(k,n) = B[v*bvec + z*bbatch + k*ldb + n];
// A(m,k) = A[v*avec + z*abatch + amap(m) + k] when TileGemm::ak, else A[... + amap(k) + m]
struct TgSeg {
  const double *A = nullptr;
  const float *Af = nullptr;  // A of float elements at the same offsets instead of A (then A unused)
  Idx2 amap;
  long long abatch = 0, avec = 0;
  const double *B = nullptr;
  long long ldb = 0, bbatch = 0, bvec = 0;
  int K = 0;
};

// C[v*cvec + z*cbatch + cmap(m) + n] = alpha * sum_seg sum_k A_seg(m,k) B_seg(k,n) + beta * C[...]
// for m < M, n < N, z < nbatch, v < nvec (several trial vectors in one launch)
struct TileGemm {
  int M = 0, N = 0, nbatch = 1, nseg = 0, nvec = 1;
  TgSeg seg[2];
  int ak = 1;
  double *C = nullptr;
  Idx2 cmap;
  long long cbatch = 0, cvec = 0;
  double alpha = 1.0, beta = 0.0;
  int dcontract = 0;   // the d-contraction of the triples: launched under its own kernel symbol
  // split-K: part < ksplit takes the part-th slice of every segment's K (multiples of 16) and
  // writes at C + part*cpart; the host points C at a partial buffer for it.
  int ksplit = 1;
  long long cpart = 0;
  // persistent launch: at most this many workgroups, each looping over tiles (0: one per tile)
  int persist = 0;
  // rows (p,q,a), batch r: tiles of ordered triples the call does not need (outside its triple
  // range, or all valence under core-valence separation) are skipped, or written as zeros
  // (tf.zero; only without beta)
  TripleFilter tf;
};

hipError_t tile_gemm_f64(const TileGemm &g, hipStream_t s);
long long tile_gemm_blocks(const TileGemm &g);

}  // namespace mlcc3
