// Large-tile FP64 MFMA GEMM of the triples path.  Its main user is the virtual-index
// contraction that builds the triples intermediate
//   W[p][q][r][a][b][c] = sum_seg sum_D x_seg[(p,q,a)][D] G_seg[r][D][(b,c)]
// (Implementation section: the O(N_V n_v^3 n_o^3) d-contraction, here over all ordered
// active occupied triples at once; one GEMM per r with M = n_o^2 n_v, N = n_v^2, K = N_V);
// the back-contractions of the contravariant triples with integrals and amplitudes of the
// same size (K = n_v^2 or n_o^2 n_v) use it too.
//
// gfx950 mapping: 256 threads = 4 waves in a 2x2 arrangement, 128x128 block tile, each wave
// a 64x64 sub-tile of 4x4 v_mfma_f64_16x16x4_f64 tiles, K in slabs of 16 staged through
// LDS with a register prefetch of the next slab and one barrier per slab.  Launch bounds
// ask for two workgroups per CU (at most 256 VGPRs per lane, 70-72 KB of LDS per workgroup) so
// that one workgroup's global loads and barrier overlap the other's MFMAs.
//  - A K-contiguous: slab in LDS as [m][k], row pitch 17 doubles, so the fragment reads of
//    16 rows x 2 k hit 32 distinct bank pairs.
//  - A M-contiguous and B: slab as [k][m|n], row pitch 144 doubles (32 banks mod 64), so
//    rows k and k+1 of one fragment read fall in opposite bank halves.
//  - Global loads are 16-byte vectors along the unit-stride index when the layout allows.
//  - Tiles are ordered batch-major, then in groups of 8 M-tiles with the N-tiles inside a
//    group, so that the workgroups in flight share A rows and B columns in L2.  (An
//    XCD-aware remap of the workgroup index was measured on the d-contraction shapes and
//    gave no gain: all operands of one batch fit in the last-level cache.)
#include "tile_gemm.h"

namespace mlcc3 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PA = BK + 1;   // [m][k] slab row pitch (doubles)
constexpr int PB = BN + 16;  // [k][m|n] slab row pitch (doubles)
constexpr int GM = 8;        // M-tiles per group in the tile order

// two-level map without a branch: the host turns a one-level map into d = INT_MAX, s1 = 0
__device__ __forceinline__ long long moff(const Idx2 &f, int x) {
  const int q = x / f.d;
  return (long long)q * f.s1 + (long long)(x - q * f.d) * f.s0;
}

// AF: the A operand of every segment holds float elements (TgSeg::Af), widened when staged
template <bool AK, bool VEC, bool BETA, bool AF = false>
__device__ __forceinline__ void tile_body(const TileGemm &g) {
  __shared__ double As[2][AK ? BM * PA : BK * PB];
  __shared__ double Bs[2][BK * PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mt = (g.M + BM - 1) / BM, nt = (g.N + BN - 1) / BN;
  const long long ntiles = (long long)mt * nt * g.nbatch * g.nvec * g.ksplit;
  for (long long L = blockIdx.x; L < ntiles; L += gridDim.x) {
    const long long zz = L / (mt * nt);
    const long long zf = zz / g.ksplit;
    const int part = (int)(zz - zf * g.ksplit);
    const int vv = (int)(zf / g.nbatch), z = (int)(zf - (long long)vv * g.nbatch);
    int t = (int)(L - zz * (mt * nt));
    const int grp = t / (GM * nt), gbase = grp * GM;
    const int gsz = min(GM, mt - gbase);
    t -= grp * GM * nt;
    const int m0 = (gbase + t % gsz) * BM, n0 = (t / gsz) * BN;
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
    const bool skip = g.tf.on && !tile_needed(g.tf, z, m0, min(g.M, m0 + BM));  // uniform per workgroup
    if (skip && !g.tf.zero) continue;

    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // staging: A K-contiguous: rows ar + 32u, k pair 2*akp; A M-contiguous and B: rows (k)
    // kr + 4u, pair 2*np along m or n
    const int akp = tid & 7, ar = tid >> 3;
    const int np = tid & 63, kr = tid >> 6;
    d2 ra[4], rb[4];
    // float A is kept as loaded until the LDS store: a conversion at the load would wait for
    // the load there and take the next K-step's prefetch out of the shadow of the MFMAs
    float2 raf[4];

    for (int s = 0; s < (skip ? 0 : g.nseg); s++) {
      const TgSeg &sg = g.seg[s];
      // K slice [kb, K) of this part
      const int chunk = ((sg.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
      const int kb = part * chunk;
      const int K = min(sg.K, kb + chunk);
      if (kb >= K) continue;  // uniform over the workgroup
      const double *Ap = AF ? nullptr : sg.A + vv * sg.avec + (long long)z * sg.abatch;
      const float *Afp = AF ? sg.Af + vv * sg.avec + (long long)z * sg.abatch : nullptr;
      const double *Bp = sg.B + vv * sg.bvec + (long long)z * sg.bbatch;
      const int nkt = (K - kb + BK - 1) / BK;
      long long aoff[4];
      if (AK) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int m = m0 + ar + 32 * u;
          aoff[u] = m < g.M ? moff(sg.amap, m) : -1;
        }
      }

      auto load = [&](int kt) {
        if (AK) {
          const int k = kb + kt * BK + 2 * akp;
#pragma unroll
          for (int u = 0; u < 4; u++) {
            d2 v = d2{0.0, 0.0};
            float2 f = make_float2(0.0f, 0.0f);
            if (aoff[u] >= 0) {
              if (AF) {
                const float *p = Afp + aoff[u] + k;
                if (VEC && k + 1 < K) {
                  f = *(const float2 *)p;
                } else {
                  if (k < K) f.x = p[0];
                  if (k + 1 < K) f.y = p[1];
                }
              } else {
                const double *p = Ap + aoff[u] + k;
                if (VEC && k + 1 < K) {
                  v = *(const d2 *)p;
                } else {
                  if (k < K) v.x = p[0];
                  if (k + 1 < K) v.y = p[1];
                }
              }
            }
            if (AF) raf[u] = f;
            else ra[u] = v;
          }
        } else {
          const int m = m0 + 2 * np;
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int k = kb + kt * BK + kr + 4 * u;
            d2 v = d2{0.0, 0.0};
            float2 f = make_float2(0.0f, 0.0f);
            if (k < K) {
              if (AF) {
                const float *p = Afp + moff(sg.amap, k) + m;
                if (VEC && m + 1 < g.M) {
                  f = *(const float2 *)p;
                } else {
                  if (m < g.M) f.x = p[0];
                  if (m + 1 < g.M) f.y = p[1];
                }
              } else {
                const double *p = Ap + moff(sg.amap, k) + m;
                if (VEC && m + 1 < g.M) {
                  v = *(const d2 *)p;
                } else {
                  if (m < g.M) v.x = p[0];
                  if (m + 1 < g.M) v.y = p[1];
                }
              }
            }
            if (AF) raf[u] = f;
            else ra[u] = v;
          }
        }
        const int n = n0 + 2 * np;
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int k = kb + kt * BK + kr + 4 * u;
          d2 v = d2{0.0, 0.0};
          if (k < K) {
            const double *p = Bp + (long long)k * sg.ldb + n;
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
          const d2 av = AF ? d2{(double)raf[u].x, (double)raf[u].y} : ra[u];
          if (AK) {
            double *pa = &As[buf][(ar + 32 * u) * PA + 2 * akp];
            pa[0] = av.x;
            pa[1] = av.y;
          } else {
            *(d2 *)&As[buf][(kr + 4 * u) * PB + 2 * np] = av;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) *(d2 *)&Bs[buf][(kr + 4 * u) * PB + 2 * np] = rb[u];
      };

      __syncthreads();  // the previous segment's readers are done with both buffers
      load(0);
      store(0);
      __syncthreads();
      for (int kt = 0; kt < nkt; kt++) {
        const int cur = kt & 1;
        if (kt + 1 < nkt) load(kt + 1);
        const double *as = AK ? &As[cur][(wm0 + (lane & 15)) * PA + (lane >> 4)]
                              : &As[cur][(lane >> 4) * PB + wm0 + (lane & 15)];
        const double *bs = &Bs[cur][(lane >> 4) * PB + wn0 + (lane & 15)];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          double a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; i++) a[i] = AK ? as[16 * i * PA + kk] : as[kk * PB + 16 * i];
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
    double *Cp = g.C + vv * g.cvec + (long long)z * g.cbatch + part * g.cpart;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int m = m0 + wm0 + 16 * i + (lane >> 4) + 4 * v;
        if (m >= g.M) continue;
        double *crow = Cp + moff(g.cmap, m);
        double old[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int n = n0 + wn0 + 16 * j + (lane & 15);
          old[j] = (BETA && n < g.N) ? crow[n] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int n = n0 + wn0 + 16 * j + (lane & 15);
          if (n < g.N) crow[n] = BETA ? g.alpha * acc[i][j][v] + g.beta * old[j] : g.alpha * acc[i][j][v];
        }
      }
  }  // tiles of a persistent workgroup
}

template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_dcontract_f64(const TileGemm g) {
  tile_body<true, VEC, false>(g);
}

template <bool AK, bool VEC, bool BETA, bool AF = false>
__global__ __launch_bounds__(256, 2) void k_tile_gemm_f64(const TileGemm g) {
  tile_body<AK, VEC, BETA, AF>(g);
}

bool even_map(const Idx2 &f) { return f.s0 % 2 == 0 && (f.d <= 0 || f.s1 % 2 == 0); }

Idx2 branchless(Idx2 f) {
  if (f.d <= 0) {
    f.d = 0x7fffffff;
    f.s1 = 0;
  }
  return f;
}

}  // namespace

long long tile_gemm_blocks(const TileGemm &g) {
  return (long long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.nbatch * g.nvec * g.ksplit;
}

hipError_t tile_gemm_f64(const TileGemm &g0, hipStream_t s) {
  TileGemm g = g0;
  if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0 || g.nvec <= 0) return hipSuccess;
  if (g.nseg < 1 || g.nseg > 2) return hipErrorInvalidValue;
  if (g.dcontract && !g.ak) return hipErrorInvalidValue;
  if (g.ksplit < 1 || (g.ksplit > 1 && g.beta != 0.0)) return hipErrorInvalidValue;
  if (g.tf.on && (g.tf.no < 1 || g.tf.nv < 1 || (g.tf.zero && g.beta != 0.0))) return hipErrorInvalidValue;
  const long long T = tile_gemm_blocks(g);
  if (T > 0x7fffffffLL) return hipErrorInvalidValue;
  // 16-byte loads need even offsets of every loaded pair and 16-byte aligned bases (8-byte ones
  // for a float A)
  const bool af = g.seg[0].Af != nullptr;
  bool vec = g.N % 2 == 0;
  for (int i = 0; i < g.nseg; i++) {
    const TgSeg &sg = g.seg[i];
    if ((sg.Af != nullptr) != af) return hipErrorInvalidValue;
    const bool abase = af ? (uintptr_t)sg.Af % 8 == 0 : (uintptr_t)sg.A % 16 == 0;
    vec = vec && even_map(sg.amap) && sg.ldb % 2 == 0 && sg.abatch % 2 == 0 && sg.bbatch % 2 == 0 &&
          sg.avec % 2 == 0 && sg.bvec % 2 == 0 && abase && (uintptr_t)sg.B % 16 == 0;
  }
  if (af && g.dcontract) return hipErrorInvalidValue;
  for (int i = 0; i < g.nseg; i++) g.seg[i].amap = branchless(g.seg[i].amap);
  g.cmap = branchless(g.cmap);
  if (g.dcontract && g.beta != 0.0) return hipErrorInvalidValue;
  if (g_dry) return hipSuccess;  // host sizing run: arguments checked, nothing launched
  const dim3 grid((unsigned)(g.persist > 0 && g.persist < T ? g.persist : T)), block(256);
  const bool beta = g.beta != 0.0;
  if (g.dcontract) {
    if (beta) return hipErrorInvalidValue;
    if (vec) hipLaunchKernelGGL(k_dcontract_f64<true>, grid, block, 0, s, g);
    else hipLaunchKernelGGL(k_dcontract_f64<false>, grid, block, 0, s, g);
  }
#define MLCC3_TG(A_, V_, B_, F_) \
  else if ((g.ak != 0) == A_ && vec == V_ && beta == B_ && af == F_) \
    hipLaunchKernelGGL((k_tile_gemm_f64<A_, V_, B_, F_>), grid, block, 0, s, g);
  MLCC3_TG(true, true, false, false) MLCC3_TG(true, true, true, false) MLCC3_TG(true, false, false, false)
  MLCC3_TG(true, false, true, false) MLCC3_TG(false, true, false, false) MLCC3_TG(false, true, true, false)
  MLCC3_TG(false, false, false, false) MLCC3_TG(false, false, true, false)
  MLCC3_TG(true, true, false, true) MLCC3_TG(true, false, false, true) MLCC3_TG(false, true, false, true)
  MLCC3_TG(false, false, false, true) MLCC3_TG(false, true, true, true) MLCC3_TG(false, false, true, true)
  else return hipErrorInvalidValue;  // no instantiation for this combination
#undef MLCC3_TG
  return hipGetLastError();
}

}  // namespace mlcc3
