// FP64 MFMA kernel of the virtual-index contraction that builds the triples intermediate
//   W[p][q][r][a][b][c] = sum_seg sum_D x_seg[(p,q,a)][D] G_seg[r][D][(b,c)]
// (Implementation section: the O(N_V n_v^3 n_o^3) d-contraction, here over all ordered
// active occupied triples at once; one GEMM per r with M = n_o^2 n_v, N = n_v^2, K = N_V).
//
// gfx950 mapping: 256 threads = 4 waves in a 2x2 arrangement, 128x128 block tile, each wave
// a 64x64 sub-tile of 4x4 v_mfma_f64_16x16x4_f64 tiles (accumulators in AGPRs), K in slabs
// of 16 staged through LDS with a register prefetch of the next slab and one barrier per
// slab.  Launch bounds ask for two workgroups per CU so that one workgroup's global loads
// and barrier overlap the other's MFMAs; 72 KB of LDS per workgroup keeps two resident.
//  - A slab in LDS as [m][k] (row pitch 17 doubles): the fragment reads of 16 rows x 2 k
//    hit 32 distinct bank pairs.
//  - B slab in LDS as [k][n] (row pitch 144 doubles = 32 banks mod 64): rows k and k+1
//    fall in opposite bank halves.
//  - Global loads are 16-byte vectors along the unit-stride index (K for A, N for B).
//  - Tiles are ordered batch-major, then in groups of 8 M-tiles with N inside, and the
//    workgroup index is remapped so that each XCD (workgroups are dealt round-robin over
//    the 8 XCDs) walks a contiguous range of that order: the tiles in flight on one XCD
//    share A rows and B columns in its L2.
#include "dcontract.h"

namespace mlcc3 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PA = BK + 1;   // A slab row pitch (doubles)
constexpr int PB = BN + 16;  // B slab row pitch (doubles)
constexpr int GM = 8;        // M-tiles per group in the tile order
constexpr int NXCD = 8;

// logical tile of workgroup `bid` out of T: XCD x = bid % 8 gets the contiguous range
// [start(x), start(x+1)) of the logical order, start(x) = x*floor(T/8) + min(x, T%8)
__device__ __forceinline__ long long xcd_remap(long long bid, long long T) {
  const long long x = bid % NXCD, slot = bid / NXCD;
  const long long q = T / NXCD, rem = T % NXCD;
  return x * q + (x < rem ? x : rem) + slot;
}

template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_dcontract_f64(const Dcontract g) {
  __shared__ double As[2][BM * PA];
  __shared__ double Bs[2][BK * PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mt = (g.M + BM - 1) / BM, nt = (g.N + BN - 1) / BN;
  const long long T = (long long)mt * nt * g.nbatch;
  long long L = g.remap ? xcd_remap(blockIdx.x, T) : (long long)blockIdx.x;
  const int z = (int)(L / ((long long)mt * nt));
  int t = (int)(L - (long long)z * mt * nt);
  // groups of GM M-tiles, N-tiles inside a group
  const int grp = t / (GM * nt), gbase = grp * GM;
  const int gsz = min(GM, mt - gbase);
  t -= grp * GM * nt;
  const int m0 = (gbase + t % gsz) * BM, n0 = (t / gsz) * BN;
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // staging assignment: A rows ar + 32u, k pair 2*akp; B rows bk + 4u, n pair 2*bnp
  const int akp = tid & 7, ar = tid >> 3;
  const int bnp = tid & 63, bk = tid >> 6;
  d2 ra[4], rb[4];

  for (int s = 0; s < g.nseg; s++) {
    const DcSeg &sg = g.seg[s];
    const int K = sg.K;
    const double *Ap = sg.A;
    const double *Bp = sg.B + (long long)z * sg.bbatch;
    const int nkt = (K + BK - 1) / BK;

    auto load = [&](int kt) {
      const int k = kt * BK + 2 * akp;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int m = m0 + ar + 32 * u;
        d2 v = d2{0.0, 0.0};
        if (m < g.M) {
          const double *p = Ap + (long long)m * sg.lda + k;
          if (VEC && k + 1 < K) {
            v = *(const d2 *)p;
          } else {
            if (k < K) v.x = p[0];
            if (k + 1 < K) v.y = p[1];
          }
        }
        ra[u] = v;
      }
      const int n = n0 + 2 * bnp;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int k2 = kt * BK + bk + 4 * u;
        d2 v = d2{0.0, 0.0};
        if (k2 < K) {
          const double *p = Bp + (long long)k2 * sg.ldb + n;
          if (VEC && n + 1 < g.N) {
            v = *(const d2 *)p;
          } else {
            if (n < g.N) v.x = p[0];
            if (n + 1 < g.N) v.y = p[1];
          }
        }
        rb[u] = v;
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int u = 0; u < 4; u++) {
        double *pa = &As[buf][(ar + 32 * u) * PA + 2 * akp];
        pa[0] = ra[u].x;
        pa[1] = ra[u].y;
      }
#pragma unroll
      for (int u = 0; u < 4; u++) *(d2 *)&Bs[buf][(bk + 4 * u) * PB + 2 * bnp] = rb[u];
    };

    __syncthreads();  // the previous segment's readers are done with both buffers
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; kt++) {
      const int cur = kt & 1;
      if (kt + 1 < nkt) load(kt + 1);
      const double *as = &As[cur][(wm0 + (lane & 15)) * PA + (lane >> 4)];
      const double *bs = &Bs[cur][(lane >> 4) * PB + wn0 + (lane & 15)];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; i++) a[i] = as[16 * i * PA + kk];
#pragma unroll
        for (int j = 0; j < 4; j++) b[j] = bs[kk * PB + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (kt + 1 < nkt) store(cur ^ 1);
      __syncthreads();
    }
  }

  // lane l, register v of a 16x16 f64 MFMA tile: row l/16 + 4v, column l%16
  double *Cp = g.C + (long long)z * g.cbatch;
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int m = m0 + wm0 + 16 * i + (lane >> 4) + 4 * v;
      if (m >= g.M) continue;
      const int mq = m / g.crow_d;
      double *crow = Cp + (long long)mq * g.crow_s1 + (long long)(m - mq * g.crow_d) * g.crow_s0;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int n = n0 + wn0 + 16 * j + (lane & 15);
        if (n < g.N) crow[n] = acc[i][j][v];
      }
    }
}

}  // namespace

long long dcontract_blocks(const Dcontract &g) {
  return (long long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.nbatch;
}

hipError_t dcontract_f64(const Dcontract &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0 || g_dry) return hipSuccess;
  if (g.nseg < 1 || g.nseg > 2 || g.crow_d < 1) return hipErrorInvalidValue;
  const long long T = dcontract_blocks(g);
  if (T > 0x7fffffffLL) return hipErrorInvalidValue;
  bool vec = g.N % 2 == 0;
  for (int i = 0; i < g.nseg; i++) {
    const DcSeg &sg = g.seg[i];
    vec = vec && sg.lda % 2 == 0 && sg.ldb % 2 == 0 && sg.bbatch % 2 == 0 && (uintptr_t)sg.A % 16 == 0 &&
          (uintptr_t)sg.B % 16 == 0;
  }
  if (vec) hipLaunchKernelGGL(k_dcontract_f64<true>, dim3((unsigned)T), dim3(256), 0, s, g);
  else hipLaunchKernelGGL(k_dcontract_f64<false>, dim3((unsigned)T), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace mlcc3
