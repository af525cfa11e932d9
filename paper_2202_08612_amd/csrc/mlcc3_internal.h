// Internal declarations of libmlcc3 (not part of the public C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlcc3 {

// Two-level index map used for every GEMM operand: off(x) = (x / d) * s1 + (x % d) * s0,
// or x * s0 when d <= 0.  It lets one kernel read and write the blocked tensor layouts of
// the triples path (ordered triple blocks, integral blocks) without repacking.
struct Idx2 {
  long long s0 = 0, s1 = 0;
  int d = 0;
};

inline Idx2 plain(long long s0) { Idx2 f; f.s0 = s0; f.d = 0; return f; }
__host__ __device__ __forceinline__ long long ioff(const Idx2 &f, int x) {
  if (f.d <= 0) return (long long)x * f.s0;
  const int q = x / f.d;
  return (long long)q * f.s1 + (long long)(x - q * f.d) * f.s0;
}
inline Idx2 split(int d, long long s1, long long s0) { Idx2 f; f.d = d; f.s1 = s1; f.s0 = s0; return f; }

// A(m,k) = p[row(m) + col(k) + z*batch]; B(k,n) = p[row(k) + col(n) + z*batch]
struct Operand {
  const double *p = nullptr;
  Idx2 row, col;
  long long batch = 0;
};

struct Seg {
  Operand A, B;
  int K = 0;
  double scale = 1.0;   // applied to this segment's products
};

struct Gemm {
  int M = 0, N = 0, nbatch = 1, nseg = 0;
  Seg seg[2];
  double *C = nullptr;
  Idx2 crow, ccol;
  long long cbatch = 0;
  double alpha = 1.0, beta = 0.0;   // C = alpha * sum_seg scale*A*B + beta * C
  // split-K: ksplit > 1 gives each (batch, part) workgroup a slice of every segment's K;
  // partial tiles go to P[batch][part][M][N] and a fixed-order reduction applies alpha/beta.
  int ksplit = 1;
  double *P = nullptr;
  // block tile (32 tm) x (32 tn), tm, tn in {1, 2, 4}; 0 = chosen from the sizes
  int tm = 0, tn = 0;
};

// FP64 MFMA GEMM (v_mfma_f64_16x16x4_f64), LDS-staged, 256 threads per block.
hipError_t gemm_f64(const Gemm &g, hipStream_t s);
// C = alpha * sum_{part < ksplit} P[batch][part][M][N] + beta * C through g's output maps
hipError_t gemm_reduce_parts(const Gemm &g, hipStream_t s);
// number of workgroups gemm_f64 launches for g with ksplit = 1
long long gemm_tiles(const Gemm &g);

// Dry-run mode (environment MLCC3_DRYRUN=1): no device calls, no kernel launches; the
// host orchestration and its bounds self-checks still run.  Used to validate every
// launch descriptor on a host without a GPU.
extern bool g_dry;

}  // namespace mlcc3
