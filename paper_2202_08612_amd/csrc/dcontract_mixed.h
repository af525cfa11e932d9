// Mixed-precision d-contractions of the triples intermediate: FP32 MFMA, and split-bf16
// products (three or six bf16 MFMA products per FP64 product).
#pragma once
#include <stdint.h>
#include "mlcc3_internal.h"

namespace mlcc3 {

// offset of row x under a two-level map: (x / d) s1 + (x % d) s0
__device__ __forceinline__ long long mix_moff(const Idx2 &f, int x) {
  const int q = x / f.d;
  return (long long)q * f.s1 + (long long)(x - q * f.d) * f.s0;
}

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
  // A read in place instead (K > 0): element (m, k) of batch z at A + v*avec + z*abatch +
  // amap(m) + k for k < K (zero for K <= k < Kp); lda unused, no padding needed
  Idx2 amap;
  long long abatch = 0;
  int K = 0;
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
  // ordered triples the call does not need are skipped (see TileGemm); tf.zero writes the
  // skipped tiles as zeros
  TripleFilter tf;
};

hipError_t dcontract_f32(const MixGemm &g, hipStream_t s);
// dst[b][r][c] (b < nb, r < Rp, c < Cp) = FP32 of src[b][r][c] inside R x C, zero outside
hipError_t pad_to_f32(const double *src, int nb, int R, int C, float *dst, int Rp, int Cp, hipStream_t s);

// ---- split-bf16 form (Henry, Tang and Heinecke, ARITH 2019) ----
// Every FP64 operand element is split into ns bf16 planes, x ~ x_0 + ... + x_{ns-1}, with
// x_0 = bf16(x) and x_s = bf16 of the (exact, FP64) remainder after x_0..x_{s-1}.  The product
// keeps the plane pairs (s, t) with s + t < ns: ns = 2 gives three products (about 2^-16
// relative per product), ns = 3 six (about 2^-24).
constexpr int BF_BM = 128, BF_BN = 64, BF_BK = 32;

// one product term: A plane s at A + s*aplane, rows [m][k] with pitch Kp (Mp >= M rows, a
// multiple of BF_BM, zero beyond M and K); B plane s at B + s*bplane, batch z at + z*bbatch,
// stored TRANSPOSED as [n][k] with pitch Kp (Np >= N rows, a multiple of BF_BN, zero padded).
// Kp a multiple of BF_BK; bases 16-byte aligned.  Vector v: A + v*avec, B + v*bvec.
struct BfSeg {
  const uint16_t *A = nullptr;
  long long aplane = 0, avec = 0;
  const uint16_t *B = nullptr;
  long long bplane = 0, bbatch = 0, bvec = 0;
  int Kp = 0;
  long long abatch = 0;  // batch z of the A planes at + z*abatch (0: shared by all batches)
  // B given in FP64 instead (B64 != NULL): row n, k < K at B64 + v*bvec + z*bbatch + bmap(n) + k
  // (zero for k >= K or n >= N), split into planes while it is staged; B and bplane unused
  const double *B64 = nullptr;
  const float *B32 = nullptr;  // instead of B64: float elements at the same offsets
  Idx2 bmap;
  int K = 0;
  // with B64 or B32 only: kd > 0 maps k to (k / kd) ks + k % kd (element k of row n at
  // bmap(n) + (k / kd) ks + k % kd instead of bmap(n) + k)
  int kd = 0;
  long long ks = 0;
};

// C[z*cbatch + cmap(m) + n] = sum_seg sum_(s,t) sum_k A_seg,s[m][k] B_seg,t[z][n][k] (bf16 MFMA,
// FP32 sums over 64-deep K steps, added in FP64), for every vector v < nvec (C + v*cvec)
struct BfGemm {
  int M = 0, N = 0, nbatch = 1, nseg = 0, nvec = 1, ns = 2;
  BfSeg seg[2];
  double *C = nullptr;
  Idx2 cmap;
  long long cbatch = 0, cvec = 0;
  int persist = 0;
  // ordered triples the call does not need: the filter applies to the rows (p,q,a) with batch r,
  // or, with B in FP64, to the columns; tf.zero writes the skipped tiles as zeros
  TripleFilter tf;
};

hipError_t dcontract_bf16(const BfGemm &g, hipStream_t s);
// planes of src[b][r][c] (b < nb, inside R x C; zero outside) into dst + s*plane, layout
// [b][Rp][Cp]; transpose = 1 writes [b][Cp][Rp] instead (src columns become rows)
hipError_t split_bf16(const double *src, int nb, int R, int C, uint16_t *dst, int Rp, int Cp, long long plane,
                      int ns, int transpose, hipStream_t s);

}  // namespace mlcc3
