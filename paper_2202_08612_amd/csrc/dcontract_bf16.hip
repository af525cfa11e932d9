// Split-bf16 d-contraction of the triples intermediate:
//   W[p][q][r][a][b][c] = sum_seg sum_D x_seg[(p,q,a)][D] G_seg[r][D][(b,c)]
// with every FP64 operand written as a sum of ns bf16 planes (the split-bf16 products of Henry,
// Tang and Heinecke, ARITH 2019) and the plane pairs (s, t) with s + t < ns multiplied in bf16
// MFMA: ns = 2 is the three-product form (hi*hi + hi*lo + lo*hi), ns = 3 the six-product form.
// Products of bf16 planes are exact in FP32; the MFMA sums them in FP32 over two 32-deep K
// slabs, after which the FP32 tile is added into an FP64 accumulator.  W is written in FP64.
// The same kernel runs the N_V-wide back-contractions with the triples operand split while it
// is staged (BMODE 1, 2).
//
// gfx950 mapping: v_mfma_f32_16x16x32_bf16 (operand lane l: A row l%16 and B column l%16, the
// 8 consecutive k of chunk l/16; result register v of lane l: row 4(l/16) + v, column l%16).
// 256 threads in a 2x2 wave arrangement, 128x64 block tile, each wave 4x2 MFMA tiles.  Both
// operands are staged K-contiguous (B planes are stored transposed, [n][k]), so every fragment
// is one 16-byte LDS read.  LDS rows are 64 bytes (32 k) with the four 16-byte chunks of row R
// permuted by XOR with (R / 4) % 4, which puts the 16 rows of a fragment read in 16 distinct
// groups of 4 banks without padding.  LDS holds two slab buffers (double buffering, one barrier
// per slab): 48 KB for two planes, 72 KB for three, so two workgroups fit on a CU either way.
#include "dcontract_mixed.h"

namespace mlcc3 {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int BM = BF_BM, BN = BF_BN, BK = BF_BK;
constexpr int PW = BK / 2;      // LDS row pitch in 4-byte words (64 bytes)
constexpr int GM = 8;           // M-tiles per group of the tile order
constexpr int FLUSH = 2;        // K slabs summed in FP32 before the FP64 add

__device__ __forceinline__ bf8 as_bf8(const u4 &x) { return __builtin_bit_cast(bf8, x); }

// word offset of 16-byte chunk c (0..3) of LDS row r
__device__ __forceinline__ int swz(int r, int c) { return r * PW + 4 * (c ^ ((r >> 2) & 3)); }

// LDS word offsets of the A and B plane s of slab buffer b
template <int NS>
__device__ __forceinline__ int a_off(int b, int s) {
  return (b * NS + s) * BM * PW;
}
template <int NS>
__device__ __forceinline__ int b_off(int b, int s) {
  return 2 * NS * BM * PW + (b * NS + s) * BN * PW;
}

// round-to-nearest-even FP32 -> bf16 (finite inputs)
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf16_value(uint16_t h) { return (double)__uint_as_float((unsigned)h << 16); }

// x = x_0 + ... + x_{ns-1} + remainder; each remainder is exact in FP64
template <int NS>
__device__ __forceinline__ void split_planes(double x, uint16_t *o) {
#pragma unroll
  for (int s = 0; s < NS; s++) {
    o[s] = bf16_rne((float)x);
    x -= bf16_value(o[s]);
  }
}

// eight FP64 values as the 16-byte chunks (eight bf16) of the NS planes
template <int NS>
__device__ __forceinline__ void split8(const double (&x)[8], u4 (&o)[NS]) {
#pragma unroll
  for (int w = 0; w < 4; w++) {
    uint16_t lo[NS], hi[NS];
    split_planes<NS>(x[2 * w], lo);
    split_planes<NS>(x[2 * w + 1], hi);
#pragma unroll
    for (int s = 0; s < NS; s++) o[s][w] = (unsigned)lo[s] | ((unsigned)hi[s] << 16);
  }
}

// BMODE 0: B given as bf16 planes; 1: the B operand of every segment is read in FP64
// (BfSeg::B64), 2: in FP32 (BfSeg::B32), and split into planes while staged
template <int NS, int BMODE>
__global__ __launch_bounds__(256, 2) void k_dcontract_bf16(const BfGemm g) {
  constexpr bool BF64 = BMODE != 0;
  __shared__ u4 lds[2 * NS * (BM + BN) * PW / 4];
  unsigned *ldw = (unsigned *)lds;

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
    const bool skip = g.tf.on && (BF64 ? !tile_needed(g.tf, z, n0, min(g.N, n0 + BN))
                                       : !tile_needed(g.tf, z, m0, min(g.M, m0 + BM)));  // uniform per workgroup
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

    // staging: 16-byte chunk kc (8 k values) of rows sr and sr + 64 (A) and of row sr (B)
    const int kc = tid & 3, sr = tid >> 2;
    u4 ra[NS][2], rb[NS];
    double xb[8];
    float xf[8];  // B32 elements as loaded

    for (int sg_i = 0; sg_i < (skip ? 0 : g.nseg); sg_i++) {
      const BfSeg &sg = g.seg[sg_i];
      const int Kp = sg.Kp, nkt = Kp / BK;
      const uint16_t *Ap = sg.A + vv * sg.avec + (long long)z * sg.abatch + (long long)m0 * Kp;
      const uint16_t *Bp = BF64 ? nullptr : sg.B + vv * sg.bvec + (long long)z * sg.bbatch + (long long)n0 * Kp;
      const double *B64 = BMODE == 1 ? sg.B64 + vv * sg.bvec + (long long)z * sg.bbatch : nullptr;
      const float *B32 = BMODE == 2 ? sg.B32 + vv * sg.bvec + (long long)z * sg.bbatch : nullptr;
      long long brow = -1;
      if (BF64) {
        const int n = n0 + sr;
        brow = n < g.N ? mix_moff(sg.bmap, n) : -1;
      }
      // offset of element k of a B row (the K map, if any)
      auto koff = [&](int k) -> long long {
        return sg.kd > 0 ? (long long)(k / sg.kd) * sg.ks + k % sg.kd : (long long)k;
      };
      auto load = [&](int kt) {
        const int k = kt * BK + 8 * kc;
        // the two halves of the 8 k values: each lies in one run of the K map when kd % 4 == 0
        const bool full = brow >= 0 && k + 8 <= sg.K && sg.kd % 4 == 0;
        const long long o0 = full ? brow + koff(k) : 0, o1 = full ? brow + koff(k + 4) : 0;
        if (BMODE == 1) {
          if (full && ((o0 | o1) & 1) == 0) {  // four 16-byte loads
#pragma unroll
            for (int h = 0; h < 2; h++) {
              const double2 *q = (const double2 *)(B64 + (h ? o1 : o0));
#pragma unroll
              for (int e = 0; e < 2; e++) {
                const double2 v = q[e];
                xb[4 * h + 2 * e] = v.x;
                xb[4 * h + 2 * e + 1] = v.y;
              }
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; e++) xb[e] = (brow >= 0 && k + e < sg.K) ? B64[brow + koff(k + e)] : 0.0;
          }
        } else if (BMODE == 2) {
          // kept as float until the store: a conversion here would wait for the loads
          if (full && ((o0 | o1) & 3) == 0) {  // two 16-byte loads
#pragma unroll
            for (int h = 0; h < 2; h++) {
              const float4 v = *(const float4 *)(B32 + (h ? o1 : o0));
              xf[4 * h] = v.x;
              xf[4 * h + 1] = v.y;
              xf[4 * h + 2] = v.z;
              xf[4 * h + 3] = v.w;
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; e++) xf[e] = (brow >= 0 && k + e < sg.K) ? B32[brow + koff(k + e)] : 0.0f;
          }
        }
#pragma unroll
        for (int s = 0; s < NS; s++) {
#pragma unroll
          for (int u = 0; u < 2; u++) ra[s][u] = *(const u4 *)(Ap + s * sg.aplane + (long long)(sr + 64 * u) * Kp + k);
          if (!BF64) rb[s] = *(const u4 *)(Bp + s * sg.bplane + (long long)sr * Kp + k);
        }
      };
      auto store = [&](int buf) {
        if (BMODE == 2)
#pragma unroll
          for (int e = 0; e < 8; e++) xb[e] = (double)xf[e];
        if (BF64) split8<NS>(xb, rb);
#pragma unroll
        for (int s = 0; s < NS; s++) {
#pragma unroll
          for (int u = 0; u < 2; u++) *(u4 *)&ldw[a_off<NS>(buf, s) + swz(sr + 64 * u, kc)] = ra[s][u];
          *(u4 *)&ldw[b_off<NS>(buf, s) + swz(sr, kc)] = rb[s];
        }
      };

      __syncthreads();  // the previous segment's readers are done with both buffers
      load(0);
      store(0);
      __syncthreads();
      for (int kt = 0; kt < nkt; kt++) {
        const int cur = kt & 1;
        if (kt + 1 < nkt) load(kt + 1);
        u4 af[NS][4], bq[NS][2];
#pragma unroll
        for (int s = 0; s < NS; s++) {
#pragma unroll
          for (int i = 0; i < 4; i++)
            af[s][i] = *(const u4 *)&ldw[a_off<NS>(cur, s) + swz(wm0 + 16 * i + (lane & 15), lane >> 4)];
#pragma unroll
          for (int j = 0; j < 2; j++)
            bq[s][j] = *(const u4 *)&ldw[b_off<NS>(cur, s) + swz(wn0 + 16 * j + (lane & 15), lane >> 4)];
        }
        // plane pairs (sa, sb) with sa + sb = dg, smallest products first
#pragma unroll
        for (int dg = NS - 1; dg >= 0; dg--)
#pragma unroll
          for (int sa = 0; sa <= dg; sa++)
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
              for (int j = 0; j < 2; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(af[sa][i]), as_bf8(bq[dg - sa][j]),
                                                                     acc[i][j], 0, 0, 0);
        if (kt + 1 < nkt) store(cur ^ 1);
        if ((kt + 1) % FLUSH == 0 || kt + 1 == nkt) {
#pragma unroll
          for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) {
#pragma unroll
              for (int v = 0; v < 4; v++) acc64[i][j][v] += (double)acc[i][j][v];
              acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            }
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

// planes of src[b][r][c] into dst[s*plane + (b*Rp + r)*Cp + c], zero outside R x C
template <int NS>
__global__ void k_split_rows(const double *__restrict__ src, int R, int C, uint16_t *__restrict__ dst, int Rp, int Cp,
                             long long plane, long long n) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int c = (int)(id % Cp);
  const long long t = id / Cp;
  const int r = (int)(t % Rp);
  const long long b = t / Rp;
  uint16_t o[NS];
  split_planes<NS>((r < R && c < C) ? src[(b * R + r) * (long long)C + c] : 0.0, o);
#pragma unroll
  for (int s = 0; s < NS; s++) dst[s * plane + id] = o[s];
}

// planes of src[b][r][c], transposed: dst[s*plane + (b*Cp + c)*Rp + r]; 32x32 tiles through LDS
template <int NS>
__global__ void k_split_T(const double *__restrict__ src, int R, int C, uint16_t *__restrict__ dst, int Rp, int Cp,
                          long long plane) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const long long b = blockIdx.z;
#pragma unroll
  for (int y = 0; y < 32; y += 8) {
    const int r = r0 + ty + y, c = c0 + tx;
    tile[ty + y][tx] = (r < R && c < C) ? src[(b * R + r) * (long long)C + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int y = 0; y < 32; y += 8) {
    const int c = c0 + ty + y, r = r0 + tx;
    if (c < Cp && r < Rp) {
      uint16_t o[NS];
      split_planes<NS>(tile[tx][ty + y], o);
#pragma unroll
      for (int s = 0; s < NS; s++) dst[s * plane + (b * Cp + c) * (long long)Rp + r] = o[s];
    }
  }
}

}  // namespace

hipError_t split_bf16(const double *src, int nb, int R, int C, uint16_t *dst, int Rp, int Cp, long long plane,
                      int ns, int transpose, hipStream_t s) {
  if (nb <= 0 || Rp <= 0 || Cp <= 0 || g_dry) return hipSuccess;
  if (ns != 2 && ns != 3) return hipErrorInvalidValue;
  if (transpose) {
    if (nb > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((Cp + 31) / 32), (unsigned)((Rp + 31) / 32), (unsigned)nb);
    if (ns == 2)
      hipLaunchKernelGGL(k_split_T<2>, grid, dim3(256), 0, s, src, R, C, dst, Rp, Cp, plane);
    else
      hipLaunchKernelGGL(k_split_T<3>, grid, dim3(256), 0, s, src, R, C, dst, Rp, Cp, plane);
  } else {
    const long long n = (long long)nb * Rp * Cp;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (ns == 2)
      hipLaunchKernelGGL(k_split_rows<2>, grid, dim3(256), 0, s, src, R, C, dst, Rp, Cp, plane, n);
    else
      hipLaunchKernelGGL(k_split_rows<3>, grid, dim3(256), 0, s, src, R, C, dst, Rp, Cp, plane, n);
  }
  return hipGetLastError();
}

hipError_t dcontract_bf16(const BfGemm &g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.nbatch <= 0 || g0.nvec <= 0) return hipSuccess;
  if (g0.tf.on && (g0.tf.no < 1 || g0.tf.nv < 1)) return hipErrorInvalidValue;
  if (g0.nseg < 1 || g0.nseg > 2 || (g0.ns != 2 && g0.ns != 3)) return hipErrorInvalidValue;
  BfGemm g = g0;
  for (int i = 0; i < g.nseg; i++) {
    const BfSeg &sg = g.seg[i];
    if (sg.Kp <= 0 || sg.Kp % BK || sg.aplane % 8 || sg.avec % 8 || sg.abatch % 8 || (uintptr_t)sg.A % 16)
      return hipErrorInvalidValue;
    if (!sg.B64 && !sg.B32 && (sg.bplane % 8 || sg.bbatch % 8 || sg.bvec % 8 || (uintptr_t)sg.B % 16))
      return hipErrorInvalidValue;
    // the 16-byte loads test the alignment of the element offset only
    if ((sg.B64 && (uintptr_t)sg.B64 % 16) || (sg.B32 && (uintptr_t)sg.B32 % 16)) return hipErrorInvalidValue;
    if (sg.kd < 0 || sg.ks < 0 || (sg.kd > 0 && !sg.B64 && !sg.B32)) return hipErrorInvalidValue;
  }
  if (g.cmap.d <= 0) {
    g.cmap.d = 0x7fffffff;
    g.cmap.s1 = 0;
  }
  const long long T = (long long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.nbatch * g.nvec;
  if (T > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(g.persist > 0 && g.persist < T ? g.persist : T));
  const int bmode = g.seg[0].B64 ? 1 : (g.seg[0].B32 ? 2 : 0);
  for (int i = 0; i < g.nseg; i++) {
    const BfSeg &sg = g.seg[i];
    if ((sg.B64 ? 1 : (sg.B32 ? 2 : 0)) != bmode || (sg.B64 && sg.B32) ||
        (bmode && (sg.K <= 0 || sg.K > sg.Kp)))
      return hipErrorInvalidValue;
  }
  if (g_dry) return hipSuccess;  // host sizing run: arguments checked, nothing launched
  if (bmode) {
    for (int i = 0; i < g.nseg; i++)
      if (g.seg[i].bmap.d <= 0) {
        g.seg[i].bmap.d = 0x7fffffff;
        g.seg[i].bmap.s1 = 0;
      }
  }
#define MLCC3_BF(NS_, M_) \
  if (g.ns == NS_ && bmode == M_) hipLaunchKernelGGL((k_dcontract_bf16<NS_, M_>), grid, dim3(256), 0, s, g);
  MLCC3_BF(2, 0) MLCC3_BF(3, 0) MLCC3_BF(2, 1) MLCC3_BF(3, 1) MLCC3_BF(2, 2) MLCC3_BF(3, 2)
#undef MLCC3_BF
  return hipGetLastError();
}

}  // namespace mlcc3
