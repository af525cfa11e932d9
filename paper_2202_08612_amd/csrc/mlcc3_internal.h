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
  const float *pf = nullptr;  // A operands only: float elements at the same offsets instead of p
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

// Position of the unique occupied triple i >= j >= k (not all equal) in the canonical list
// (i outer, k inner, the all-equal triples left out): the triples before it with first index
// below i number C(i+2,3) - i, those with first index i and second below j number j(j+1)/2.
__host__ __device__ __forceinline__ long long canon_index(int i, int j, int k) {
  return (long long)i * (i + 1) * (i + 2) / 6 - i + (long long)j * (j + 1) / 2 + k;
}

// Which ordered occupied triples a GEMM over rows (p,q,a) (p*no + q pairs, nv values of a per
// pair) and batch r has to produce: the triple (p,q,r) is needed when it is not all-equal, its
// canonical position lies in [tb, te), and (core != 0) one of p, q, r is a core orbital (bit of
// core).  A tile none of whose rows is needed is skipped; with zero set it writes zeros instead
// (for outputs that are summed over the batch afterwards).
struct TripleFilter {
  int on = 0, no = 0, nv = 0, zero = 0;
  unsigned long long core = 0;
  long long tb = 0, te = 0;
  int pq0 = 0;  // the rows start at pair pq0 (an occupied slab: pq0 = p0 n_o)
};

__device__ __forceinline__ bool triple_needed(const TripleFilter &f, int p, int q, int r) {
  if (p == q && q == r) return false;
  if (f.core && !(((f.core >> p) | (f.core >> q) | (f.core >> r)) & 1ULL)) return false;
  const int i = max(p, max(q, r)), k = min(p, min(q, r)), j = p + q + r - i - k;
  const long long c = canon_index(i, j, k);
  return c >= f.tb && c < f.te;
}

// is any row of [m0, m1) of batch r needed?
__device__ __forceinline__ bool tile_needed(const TripleFilter &f, int r, int m0, int m1) {
  for (int pq = m0 / f.nv + f.pq0; pq <= (m1 - 1) / f.nv + f.pq0; pq++)
    if (triple_needed(f, pq / f.no, pq % f.no, r)) return true;
  return false;
}

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
