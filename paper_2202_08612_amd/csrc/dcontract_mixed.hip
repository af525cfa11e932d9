// Mixed-precision d-contraction of the triples intermediate (FP32 MFMA; FP32 partial sums over
// 32-deep K slabs, FP64 across slabs):
//   W[p][q][r][a][b][c] = sum_seg sum_D x_seg[(p,q,a)][D] G_seg[r][D][(b,c)]
// The operands are FP32 copies of the FP64 blocks (rounded to nearest), padded to multiples
// of 4 in K and N so that every staged load is a 16-byte vector; W is written in FP64.  The
// same kernel runs the N_V-wide back-contraction of the FP32 contravariant blocks in the FP32
// form, with A read in place through its row map (MixSeg::K > 0: loads masked at K, 16-byte
// vectors where the offset allows).
//
// gfx950 mapping: v_mfma_f32_16x16x4_f32 (operand lane l: A row l%16, k l/16; B k l/16,
// column l%16; result register v of lane l: row 4(l/16) + v, column l%16).  256 threads in a
// 2x2 wave arrangement, 128x64 block tile, each wave 4x2 MFMA tiles; K in slabs of 32.  The
// MFMAs accumulate one slab in FP32; after every slab the FP32 tile is added into an FP64
// accumulator, so FP32 rounding accumulates over 32 products only (the error of the result is
// then dominated by the rounding of the operands, about 1e-7 relative).
//  - A slab in LDS as [m][k], row pitch 36 floats: the 16 rows x 4 k of a fragment read fall
//    in 64 distinct banks.
//  - B slab as [k][n], row pitch 80 floats (16 banks mod 64): the 4 k rows of a fragment read
//    fall in distinct bank quarters.
#include "dcontract_mixed.h"

namespace mlcc3 {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 128, BN = 64, BK = 32;
constexpr int PA = BK + 4;
constexpr int PB = BN + 16;
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int GM = 8;

__global__ __launch_bounds__(256, 2) void k_dcontract_f32(const MixGemm g) {
  __shared__ float As[2][BM * PA];
  __shared__ float Bs[2][BK * PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mt = (g.M + BM - 1) / BM, nt = (g.N + BN - 1) / BN;
  const long long ntiles = (long long)mt * nt * g.nbatch * g.nvec;
  for (long long L = blockIdx.x; L < ntiles; L += gridDim.x) {
    const long long zf = L / (mt * nt);
    const int vv = (int)(zf / g.nbatch), z = (int)(zf - (long long)vv * g.nbatch);
    int t = (int)(L - zf * (mt * nt));
    const int grp = t / (GM * nt), gbase = grp * GM;
    const int gsz = min(GM, mt - gbase);
    t -= grp * GM * nt;
    const int m0 = (gbase + t % gsz) * BM, n0 = (t / gsz) * BN;
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 32;
    const bool skip = g.tf.on && !tile_needed(g.tf, z, m0, min(g.M, m0 + BM));  // uniform per workgroup
    if (skip && !g.tf.zero) continue;

    f4 acc[4][2];
    d4 acc64[4][2];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 2; j++) {
        acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      }

    // staging: A rows ar + 32u with k quad 4*aq; B rows (k) br + 16u with n quad 4*bq
    const int aq = tid & 7, ar = tid >> 3;
    const int bq = tid & 15, br = tid >> 4;
    f4 ra[4], rb[2];

    for (int s = 0; s < (skip ? 0 : g.nseg); s++) {
      const MixSeg &sg = g.seg[s];
      const int Kp = sg.Kp;
      const bool inplace = sg.K > 0;  // uniform
      const float *Ap = sg.A + vv * sg.avec + (inplace ? (long long)z * sg.abatch : 0);
      const float *Bp = sg.B + vv * sg.bvec + (long long)z * sg.bbatch;
      const int nkt = (Kp + BK - 1) / BK;
      long long arow[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int m = m0 + ar + 32 * u;
        arow[u] = m >= g.M ? -1 : (inplace ? mix_moff(sg.amap, m) : (long long)m * sg.lda);
      }
      auto load = [&](int kt) {
        const int k = kt * BK + 4 * aq;
#pragma unroll
        for (int u = 0; u < 4; u++) {
          if (!inplace) {
            ra[u] = (arow[u] >= 0 && k < Kp) ? *(const f4 *)(Ap + arow[u] + k) : f4{0.f, 0.f, 0.f, 0.f};
          } else if (arow[u] >= 0 && k + 4 <= sg.K && ((arow[u] + k) & 3) == 0) {
            ra[u] = *(const f4 *)(Ap + arow[u] + k);
          } else {
            f4 v = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; e++) v[e] = (arow[u] >= 0 && k + e < sg.K) ? Ap[arow[u] + k + e] : 0.f;
            ra[u] = v;
          }
        }
        const int n = n0 + 4 * bq;
#pragma unroll
        for (int u = 0; u < 2; u++) {
          const int k2 = kt * BK + br + 16 * u;
          rb[u] = (k2 < Kp && n < sg.Np) ? *(const f4 *)(Bp + (long long)k2 * sg.ldb + n) : f4{0.f, 0.f, 0.f, 0.f};
        }
      };
      auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; u++) *(f4 *)&As[buf][(ar + 32 * u) * PA + 4 * aq] = ra[u];
#pragma unroll
        for (int u = 0; u < 2; u++) *(f4 *)&Bs[buf][(br + 16 * u) * PB + 4 * bq] = rb[u];
      };

      __syncthreads();  // the previous segment's readers are done with both buffers
      load(0);
      store(0);
      __syncthreads();
      for (int kt = 0; kt < nkt; kt++) {
        const int cur = kt & 1;
        if (kt + 1 < nkt) load(kt + 1);
        const float *as = &As[cur][(wm0 + (lane & 15)) * PA + (lane >> 4)];
        const float *bs = &Bs[cur][(lane >> 4) * PB + wn0 + (lane & 15)];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          float a[4], b[2];
#pragma unroll
          for (int i = 0; i < 4; i++) a[i] = as[16 * i * PA + kk];
#pragma unroll
          for (int j = 0; j < 2; j++) b[j] = bs[kk * PB + 16 * j];
#pragma unroll
          for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nkt) store(cur ^ 1);
        // slab done: move the FP32 partial sums into the FP64 accumulator
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 2; j++) {
#pragma unroll
            for (int v = 0; v < 4; v++) acc64[i][j][v] += (double)acc[i][j][v];
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          }
        __syncthreads();
      }
    }

    double *Cp = g.C + vv * g.cvec + (long long)z * g.cbatch;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int m = m0 + wm0 + 16 * i + 4 * (lane >> 4) + v;
        if (m >= g.M) continue;
        double *crow = Cp + mix_moff(g.cmap, m);
#pragma unroll
        for (int j = 0; j < 2; j++) {
          const int n = n0 + wn0 + 16 * j + (lane & 15);
          if (n < g.N) crow[n] = acc64[i][j][v];
        }
      }
  }  // tiles of a persistent workgroup
}

// dst[b][r][c] = src[b][r][c] rounded to FP32 for r < R, c < C; zero for R <= r < Rp, C <= c < Cp
__global__ void k_pad_f32(const double *__restrict__ src, int R, int C, float *__restrict__ dst, int Rp, int Cp,
                          long long n) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int c = (int)(id % Cp);
  const long long t = id / Cp;
  const int r = (int)(t % Rp);
  const long long b = t / Rp;
  dst[id] = (r < R && c < C) ? (float)src[(b * R + r) * (long long)C + c] : 0.0f;
}

}  // namespace

hipError_t pad_to_f32(const double *src, int nb, int R, int C, float *dst, int Rp, int Cp, hipStream_t s) {
  const long long n = (long long)nb * Rp * Cp;
  if (n <= 0 || g_dry) return hipSuccess;
  hipLaunchKernelGGL(k_pad_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, R, C, dst, Rp, Cp, n);
  return hipGetLastError();
}

hipError_t dcontract_f32(const MixGemm &g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.nbatch <= 0 || g0.nvec <= 0) return hipSuccess;
  if (g0.tf.on && (g0.tf.no < 1 || g0.tf.nv < 1)) return hipErrorInvalidValue;
  if (g0.nseg < 1 || g0.nseg > 2) return hipErrorInvalidValue;
  MixGemm g = g0;
  for (int i = 0; i < g.nseg; i++) {
    const MixSeg &sg = g.seg[i];
    if (sg.Kp % 4 || sg.Np % 4 || sg.lda % 4 || sg.ldb % 4 || sg.bbatch % 4 || sg.avec % 4 || sg.bvec % 4 ||
        sg.Np < g.N || (uintptr_t)sg.A % 16 || (uintptr_t)sg.B % 16)
      return hipErrorInvalidValue;
    if (sg.K < 0 || sg.K > sg.Kp || sg.abatch < 0) return hipErrorInvalidValue;
  }
  for (int i = 0; i < g.nseg; i++)
    if (g.seg[i].K > 0 && g.seg[i].amap.d <= 0) {  // one-level map: no division in the kernel
      g.seg[i].amap.d = 0x7fffffff;
      g.seg[i].amap.s1 = 0;
    }
  if (g.cmap.d <= 0) {
    g.cmap.d = 0x7fffffff;
    g.cmap.s1 = 0;
  }
  const long long T = (long long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.nbatch * g.nvec;
  if (T > 0x7fffffffLL) return hipErrorInvalidValue;
  if (g_dry) return hipSuccess;  // host sizing run: arguments checked, nothing launched
  hipLaunchKernelGGL(k_dcontract_f32, dim3((unsigned)(g.persist > 0 && g.persist < T ? g.persist : T)), dim3(256), 0,
                     s, g);
  return hipGetLastError();
}

}  // namespace mlcc3
