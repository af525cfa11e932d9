// FP64 MFMA GEMM for gfx950 (CDNA4) with strided two-level operand maps.
//
// C[m,n] = alpha * sum_seg scale_seg * sum_k A_seg(m,k) B_seg(k,n) + beta * C[m,n]
//
// 256 threads = 4 waves (64 lanes) in a 2x2 arrangement; each wave owns a
// (16*TM) x (16*TN) sub-tile built from v_mfma_f64_16x16x4_f64 tiles, so the block tile
// is (32*TM) x (32*TN).  K advances in slabs of 16 staged through LDS with a
// register prefetch of the next slab (two LDS buffers, one barrier per slab).
// Global loads are coalesced along whichever operand index is unit-stride.
#include <type_traits>

#include "mlcc3_internal.h"

namespace mlcc3 {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;

typedef float f4 __attribute__((ext_vector_type(4)));

// AF: the A operand of every segment holds float elements (Operand::pf) (the contravariant
// triples of the reduced-precision forms); the product then runs as v_mfma_f32_16x16x4_f32 on
// FP32 slabs in LDS (B rounded to FP32 when staged), each 16-deep K slab summed in FP32 and
// added into the FP64 accumulators.  Result register v of lane l: row 4(l/16) + v (FP32 MFMA)
// or l/16 + 4v (FP64 MFMA), column l%16.
template <int TM, int TN, bool AKF, bool BNF, bool AF>
__device__ __forceinline__ void gemm_body(const Gemm &g) {
  typedef typename std::conditional<AF, float, double>::type LT;
  constexpr int BM = 32 * TM, BN = 32 * TN;
  // row pitches: 2 doubles, or 16 floats, of padding so that the 4 rows of a fragment read
  // fall in different banks
  constexpr int PA = BM + (AF ? 16 : 2), PB = BN + (AF ? 16 : 2);
  constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
  __shared__ LT As[2][BK][PA];
  __shared__ LT Bs[2][BK][PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int z = blockIdx.z / g.ksplit, part = blockIdx.z % g.ksplit;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm0 = (wave >> 1) * (BM / 2), wn0 = (wave & 1) * (BN / 2);

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[NA], rb[NB];
  // float A stays as loaded until the LDS store (a conversion at the load would wait for it)
  float raf[NA];

  for (int s = 0; s < g.nseg; s++) {
    const Seg &sg = g.seg[s];
    // K slice of this part (multiples of BK); loads beyond K are masked
    const int chunk = ((sg.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    const int kbeg = part * chunk;
    const int K = min(sg.K, kbeg + chunk);
    if (kbeg >= K) continue;
    const double *Ap = AF ? nullptr : sg.A.p + (long long)z * sg.A.batch;
    const float *Af = AF ? sg.A.pf + (long long)z * sg.A.batch : nullptr;
    const double *Bp = sg.B.p + (long long)z * sg.B.batch;
    const double scale = sg.scale;
    // hoisted offsets of the fixed (non-K) index of each staged element
    long long aoff[NA], boff[NB];
    bool aok[NA], bok[NB];
#pragma unroll
    for (int u = 0; u < NA; u++) {
      const int m = AKF ? (m0 + tid / BK + u * (256 / BK)) : (m0 + tid % BM);
      aok[u] = m < g.M;
      aoff[u] = aok[u] ? ioff(sg.A.row, m) : 0;
    }
#pragma unroll
    for (int u = 0; u < NB; u++) {
      const int n = BNF ? (n0 + tid % BN) : (n0 + tid / BK + u * (256 / BK));
      bok[u] = n < g.N;
      bok[u] = bok[u];
      boff[u] = bok[u] ? ioff(sg.B.col, n) : 0;
    }
    auto load = [&](int kt) {
      const int kb = kbeg + kt * BK;
      if (AKF) {
        const int k = kb + tid % BK;
        const bool kin = k < K;
        const long long ko = kin ? ioff(sg.A.col, k) : 0;
#pragma unroll
        for (int u = 0; u < NA; u++) {
          if (AF) raf[u] = (kin && aok[u]) ? Af[aoff[u] + ko] : 0.0f;
          else ra[u] = (kin && aok[u]) ? Ap[aoff[u] + ko] : 0.0;
        }
      } else {
#pragma unroll
        for (int u = 0; u < NA; u++) {
          const int k = kb + tid / BM + u * (256 / BM);
          if (AF) raf[u] = (k < K && aok[u]) ? Af[aoff[u] + ioff(sg.A.col, k)] : 0.0f;
          else ra[u] = (k < K && aok[u]) ? Ap[aoff[u] + ioff(sg.A.col, k)] : 0.0;
        }
      }
      if (BNF) {
#pragma unroll
        for (int u = 0; u < NB; u++) {
          const int k = kb + tid / BN + u * (256 / BN);
          rb[u] = (k < K && bok[u]) ? Bp[ioff(sg.B.row, k) + boff[u]] : 0.0;
        }
      } else {
        const int k = kb + tid % BK;
        const bool kin = k < K;
        const long long ko = kin ? ioff(sg.B.row, k) : 0;
#pragma unroll
        for (int u = 0; u < NB; u++) rb[u] = (kin && bok[u]) ? Bp[ko + boff[u]] : 0.0;
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int u = 0; u < NA; u++) {
        const double av = AF ? (double)raf[u] : ra[u];
        if (AKF) As[buf][tid % BK][tid / BK + u * (256 / BK)] = (LT)(av * scale);
        else As[buf][tid / BM + u * (256 / BM)][tid % BM] = (LT)(av * scale);
      }
#pragma unroll
      for (int u = 0; u < NB; u++) {
        if (BNF) Bs[buf][tid / BN + u * (256 / BN)][tid % BN] = (LT)rb[u];
        else Bs[buf][tid % BK][tid / BK + u * (256 / BK)] = (LT)rb[u];
      }
    };

    const int nkt = (K - kbeg + BK - 1) / BK;
    __syncthreads();  // previous segment's readers are done with both buffers
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; kt++) {
      const int cur = kt & 1;
      if (kt + 1 < nkt) load(kt + 1);
      if constexpr (AF) {
        f4 acc32[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
          for (int j = 0; j < TN; j++) acc32[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          float a[TM], b[TN];
#pragma unroll
          for (int i = 0; i < TM; i++) a[i] = As[cur][kk + (lane >> 4)][wm0 + 16 * i + (lane & 15)];
#pragma unroll
          for (int j = 0; j < TN; j++) b[j] = Bs[cur][kk + (lane >> 4)][wn0 + 16 * j + (lane & 15)];
#pragma unroll
          for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++)
              acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc32[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
          for (int j = 0; j < TN; j++)
#pragma unroll
            for (int v = 0; v < 4; v++) acc[i][j][v] += (double)acc32[i][j][v];
      } else {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          double a[TM], b[TN];
#pragma unroll
          for (int i = 0; i < TM; i++) a[i] = As[cur][kk + (lane >> 4)][wm0 + 16 * i + (lane & 15)];
#pragma unroll
          for (int j = 0; j < TN; j++) b[j] = Bs[cur][kk + (lane >> 4)][wn0 + 16 * j + (lane & 15)];
#pragma unroll
          for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      }
      if (kt + 1 < nkt) store(cur ^ 1);
      __syncthreads();
    }
  }

  // epilogue: lane l, register v of a 16x16 tile holds row l/16 + 4v (FP64 MFMA) or 4(l/16) + v
  // (FP32 MFMA), column l%16.  All old C values are loaded before the first store so the loads
  // are not serialised behind stores to the same array.
  auto row_of = [&](int i, int v) {
    return m0 + wm0 + 16 * i + (AF ? 4 * (lane >> 4) + v : (lane >> 4) + 4 * v);
  };
  if (g.ksplit > 1) {
    double *Pp = g.P + ((long long)z * g.ksplit + part) * (long long)g.M * g.N;
#pragma unroll
    for (int j = 0; j < TN; j++) {
      const int n = n0 + wn0 + 16 * j + (lane & 15);
      if (n >= g.N) continue;
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int m = row_of(i, v);
          if (m < g.M) Pp[(long long)m * g.N + n] = acc[i][j][v];
        }
    }
    return;
  }
  double *Cp = g.C + (long long)z * g.cbatch;
  long long ro[TM][4], co[TN];
  bool rok[TM][4], cok[TN];
#pragma unroll
  for (int j = 0; j < TN; j++) {
    const int n = n0 + wn0 + 16 * j + (lane & 15);
    cok[j] = n < g.N;
    co[j] = cok[j] ? ioff(g.ccol, n) : 0;
  }
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int m = row_of(i, v);
      rok[i][v] = m < g.M;
      ro[i][v] = rok[i][v] ? ioff(g.crow, m) : 0;
    }
  if (g.beta != 0.0) {
    double old[TM][TN][4];
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) old[i][j][v] = (cok[j] && rok[i][v]) ? Cp[ro[i][v] + co[j]] : 0.0;
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int v = 0; v < 4; v++)
          if (cok[j] && rok[i][v]) Cp[ro[i][v] + co[j]] = g.alpha * acc[i][j][v] + g.beta * old[i][j][v];
  } else {
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int v = 0; v < 4; v++)
          if (cok[j] && rok[i][v]) Cp[ro[i][v] + co[j]] = g.alpha * acc[i][j][v];
  }
}

template <int TM, int TN, bool AKF, bool BNF, bool AF = false>
__global__ __launch_bounds__(256) void k_gemm_f64(const Gemm g) {
  gemm_body<TM, TN, AKF, BNF, AF>(g);
}

// C = alpha * sum_part P[batch][part] + beta * C through the output maps (fixed order)
__global__ void k_splitk_reduce(const Gemm g) {
  const long long MN = (long long)g.M * g.N;
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= MN * g.nbatch) return;
  const int z = (int)(id / MN);
  const long long e = id - (long long)z * MN;
  const int m = (int)(e / g.N), n = (int)(e - (long long)m * g.N);
  const double *P = g.P + (long long)z * g.ksplit * MN + e;
  double acc = 0.0;
  for (int p = 0; p < g.ksplit; p++) acc += P[p * MN];
  double *Cp = g.C + (long long)z * g.cbatch + ioff(g.crow, m) + ioff(g.ccol, n);
  double r = g.alpha * acc;
  if (g.beta != 0.0) r += g.beta * *Cp;
  *Cp = r;
}

template <int TM, int TN>
static hipError_t launch_tiles(const Gemm &g, hipStream_t s, bool akf, bool bnf, bool af) {
  dim3 grid((g.N + 32 * TN - 1) / (32 * TN), (g.M + 32 * TM - 1) / (32 * TM), g.nbatch * g.ksplit);
  if (af) {  // float A (contravariant triples of the reduced-precision forms)
    if (akf && bnf) hipLaunchKernelGGL((k_gemm_f64<TM, TN, true, true, true>), grid, dim3(256), 0, s, g);
    else if (akf) hipLaunchKernelGGL((k_gemm_f64<TM, TN, true, false, true>), grid, dim3(256), 0, s, g);
    else if (bnf) hipLaunchKernelGGL((k_gemm_f64<TM, TN, false, true, true>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_gemm_f64<TM, TN, false, false, true>), grid, dim3(256), 0, s, g);
  } else if (akf && bnf) hipLaunchKernelGGL((k_gemm_f64<TM, TN, true, true>), grid, dim3(256), 0, s, g);
  else if (akf) hipLaunchKernelGGL((k_gemm_f64<TM, TN, true, false>), grid, dim3(256), 0, s, g);
  else if (bnf) hipLaunchKernelGGL((k_gemm_f64<TM, TN, false, true>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((k_gemm_f64<TM, TN, false, false>), grid, dim3(256), 0, s, g);
  if (g.ksplit > 1) {
    const long long n = (long long)g.M * g.N * g.nbatch;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// unit stride inside each run of the index (two-level maps with s0 = 1 are contiguous in runs of d)
hipError_t gemm_reduce_parts(const Gemm &g, hipStream_t s) {
  if (g_dry || g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.ksplit < 1 || !g.P) return hipErrorInvalidValue;
  const long long n = (long long)g.M * g.N * g.nbatch;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

static bool unit(const Idx2 &f) { return f.s0 == 1; }

bool g_dry = false;

static int pick(int n) { return n <= 32 ? 1 : (n <= 64 ? 2 : 4); }

long long gemm_tiles(const Gemm &g) {
  int tm = pick(g.M), tn = pick(g.N);
  long long ktot = 0;
  for (int i = 0; i < g.nseg; i++) ktot += g.seg[i].K;
  if (ktot <= 64) { tm = tm > 2 ? 2 : tm; tn = tn > 2 ? 2 : tn; }
  auto blocks = [&](int a, int b) {
    return (long long)((g.M + 32 * a - 1) / (32 * a)) * ((g.N + 32 * b - 1) / (32 * b)) * g.nbatch;
  };
  while (blocks(tm, tn) < 512 && (tm > 2 || tn > 2)) {
    if (tm >= tn) tm /= 2; else tn /= 2;
  }
  if (g.tm > 0 && g.tn > 0) {
    tm = g.tm;
    tn = g.tn;
  }
  return blocks(tm, tn);
}

hipError_t gemm_f64(const Gemm &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0) return hipSuccess;
  if (g.nseg < 1 || g.nseg > 2 || g.ksplit < 1 || (g.ksplit > 1 && !g.P)) return hipErrorInvalidValue;
  const bool akf = unit(g.seg[0].A.col);
  const bool bnf = unit(g.seg[0].B.col);
  const bool af = g.seg[0].A.pf != nullptr;
  for (int i = 0; i < g.nseg; i++)
    if ((g.seg[i].A.pf != nullptr) != af) return hipErrorInvalidValue;
  int tm = pick(g.M), tn = pick(g.N);
  long long ktot = 0;
  for (int i = 0; i < g.nseg; i++) ktot += g.seg[i].K;
  // short K is bound by the C traffic: smaller tiles give more waves per SIMD
  if (ktot <= 64) { tm = tm > 2 ? 2 : tm; tn = tn > 2 ? 2 : tn; }
  auto blocks = [&](int a, int b) {
    return (long long)((g.M + 32 * a - 1) / (32 * a)) * ((g.N + 32 * b - 1) / (32 * b)) * g.nbatch;
  };
  while (blocks(tm, tn) < 512 && (tm > 2 || tn > 2)) {
    if (tm >= tn) tm /= 2; else tn /= 2;
  }
  if (g.tm > 0 && g.tn > 0) {  // caller's choice
    tm = g.tm;
    tn = g.tn;
  }
  if (g_dry) return hipSuccess;  // host sizing run: arguments checked, nothing launched
#define MLCC3_TILE(a, b) \
  if (tm == a && tn == b) return launch_tiles<a, b>(g, s, akf, bnf, af);
  MLCC3_TILE(4, 4) MLCC3_TILE(4, 2) MLCC3_TILE(4, 1) MLCC3_TILE(2, 4) MLCC3_TILE(2, 2) MLCC3_TILE(2, 1)
  MLCC3_TILE(1, 4) MLCC3_TILE(1, 2) MLCC3_TILE(1, 1)
#undef MLCC3_TILE
  return hipErrorInvalidValue;
}

}  // namespace mlcc3
