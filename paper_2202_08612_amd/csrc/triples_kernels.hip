// Element-wise and reduction kernels of the MLCC3 triples path (gfx950).
//
// Layout of the ordered-triple buffers used throughout: X[p][q][r][a][b][c]
// (every ordered active occupied triple (p,q,r), including p=q=r, holds one
// contiguous n_v^3 block).
#include "mlcc3_internal.h"
#include "triples_kernels.h"

namespace mlcc3 {

static inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- T1 transform
// first term of Lhat_vO: LhvO[J][c][K] = L_OV[J][K][c] (the GEMMs add the rest)
__global__ void k_lhat_vO_init(const double *LOV, int nc, int NO, int NV, int nv, double *LhvO) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)nc * nv * NO) return;
  const int K = id % NO, c = (id / NO) % nv;
  const long long J = id / ((long long)nv * NO);
  LhvO[id] = LOV[(J * NO + K) * NV + c];
}

// --------------------------------------------- X_kc = sum_LD (2 g_kcLD - g_kDLc) x^D_L
// with bare (ov|ov) = sum_J L_kc L_LD:  s_J = sum_LD L^J_LD x^D_L,
// y^J_kL = sum_D L^J_kD x^D_L,  X_kc = sum_J (2 L^J_kc s_J - sum_L y^J_kL L^J_Lc)
// s_J as a dot product of the contiguous block L^J [L][D] with xT[L][D] = x^D_L
__global__ void k_fock_s(const double *__restrict__ LOV, const double *__restrict__ xT, int nc, int NO, int NV,
                         double *s) {
  const int J = blockIdx.x;
  __shared__ double red[256];
  double acc = 0.0;
  const long long n = (long long)NO * NV;
  const double *l = LOV + (long long)J * n;
  for (long long e = threadIdx.x; e < n; e += 256) acc += l[e] * xT[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) s[J] = red[0];
}

__global__ void k_fock_z(const double *LOV, const double *s, const double *y, int nc, int NO, int NV, int no,
                         int nv, double *z) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)nc * no * nv) return;
  const int c = id % nv, k = (id / nv) % no;
  const long long J = id / ((long long)no * nv);
  const double *l = LOV + J * NO * NV;
  double e = 2.0 * l[(long long)k * NV + c] * s[J];
  const double *yy = y + (J * no + k) * NO;
  for (int L = 0; L < NO; L++) e -= yy[L] * l[(long long)L * NV + c];
  z[id] = e;
}

// out[k][c] = sum_J z[J][k][c]  (fixed summation order)
__global__ void k_sum_rows(const double *z, long long rows, long long n, double *out) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= n) return;
  double acc = 0.0;
  for (long long J = 0; J < rows; J++) acc += z[J * n + id];
  out[id] = acc;
}

// ------------------------------------------------------------------ repacks
// xA[p][q][a][D] = f * x^{aD}_{pq},  f = 1 + delta_{aD} delta_{pq} when rbar
__global__ void k_pack_vVoo(const double *x, int no, int nv, int NV, int rbar, double *xA) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)no * no * nv * NV) return;
  const int D = id % NV, a = (id / NV) % nv;
  const int q = (id / ((long long)NV * nv)) % no, p = id / ((long long)NV * nv * no);
  double v = x[(((long long)a * NV + D) * no + p) * no + q];
  if (rbar && a == D && p == q) v *= 2.0;
  xA[id] = v;
}

// xB[a][b][p][L] = (1 + delta_{ab} delta_{pL}) x^{ab}_{pL}
__global__ void k_rbar_vvoO(const double *x, int no, int nv, int NO, double *xB) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)nv * nv * no * NO) return;
  const int L = id % NO, p = (id / NO) % no, b = (id / ((long long)NO * no)) % nv,
            a = id / ((long long)NO * no * nv);
  double v = x[id];
  if (a == b && p == L) v *= 2.0;
  xB[id] = v;
}

// xV[p][q][a][b] = x^{ab}_{pq} (all-active block); mode 1: (1 + delta_{ab} delta_{pq}) x,
// mode 2: contravariant doubles 2 x^{ab}_{pq} - x^{ba}_{pq}
__global__ void k_pack_vvoo(const double *x, int no, int nv, int NV, int mode, double *xV) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)no * no * nv * nv) return;
  const int b = id % nv, a = (id / nv) % nv, q = (id / ((long long)nv * nv)) % no,
            p = id / ((long long)nv * nv * no);
  double v = x[(((long long)a * NV + b) * no + p) * no + q];
  if (mode == 1 && a == b && p == q) v *= 2.0;
  if (mode == 2) v = 2.0 * v - x[(((long long)b * NV + a) * no + p) * no + q];
  xV[id] = v;
}

// deterministic dot product: per-block partial sums, then one block adds them in order
__global__ void k_dot_partial(const double *a, const double *b, long long n, double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_dot_final(const double *part, int np, double scale, double *out) {
  if (threadIdx.x != 0) return;
  double acc = 0.0;
  for (int i = 0; i < np; i++) acc += part[i];
  out[0] = scale * acc;
}

// transition moments of state m, component x (one workgroup each, fixed-order reduction):
//   Tm0[m][x] = sum_pq Dm0[m][p][q] A[x][p][q]
//   T0m[m][x] = sum_pq (D0m[m][p][q] - s[m] D00[p][q]) A[x][p][q]
__global__ void k_moments(const double *__restrict__ A, long long NN, int ncomp, const double *__restrict__ Dm0,
                          const double *__restrict__ D0m, const double *__restrict__ D00, const double *sv,
                          double *Tm0, double *T0m) {
  __shared__ double r1[256], r2[256], r3[256];
  const int x = blockIdx.x, m = blockIdx.y;
  const double *a = A + (long long)x * NN, *dl = Dm0 + (long long)m * NN, *dr = D0m + (long long)m * NN;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (long long i = threadIdx.x; i < NN; i += blockDim.x) {
    s1 += dl[i] * a[i];
    s2 += dr[i] * a[i];
    s3 += D00[i] * a[i];
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  r3[threadIdx.x] = s3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
      r3[threadIdx.x] += r3[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Tm0[(long long)m * ncomp + x] = r1[0];
    T0m[(long long)m * ncomp + x] = r2[0] - sv[m] * r3[0];
  }
}

// f[m] = (2/3) omega[m] sum_x T0m[m][x] Tm0[m][x]
__global__ void k_strength(const double *Tm0, const double *T0m, const double *om, int ncomp, int nstate,
                           double *f) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nstate) return;
  double acc = 0.0;
  for (int x = 0; x < ncomp; x++) acc += T0m[(long long)m * ncomp + x] * Tm0[(long long)m * ncomp + x];
  f[m] = (2.0 / 3.0) * om[m] * acc;
}

// D[L][L] += f * s[0] for all L < NO (row stride N)
__global__ void k_add_diag(double *D, int NO, int N, const double *s, double f) {
  int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L < NO) D[(long long)L * N + L] += f * s[0];
}

// D[N_O + c][k] += f * Y[k][c]
__global__ void k_add_vo(double *D, int NO, int N, int no, int nv, const double *Y, double f) {
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= no * nv) return;
  const int c = id % nv, k = id / nv;
  D[(long long)(NO + c) * N + k] += f * Y[id];
}

// ------------------------------------------ permutation / denominator / contravariant
// Two LDS-tiled passes over 16^3 sub-cubes of the virtual index space.
//
// pass 1 (k_sym_denom): for unique triple o and output tile (TA,TB,TC)
//   X_o[v] = -(sum over the six pair permutations s of W_{o.s}[v.s]) / (eps - omega)   (P, eq. tau3)
//   Each source sub-cube W_{o.s}[tile.s] is read coalesced (c fastest) into LDS and
//   gathered through the permuted local index.
// pass 2 (k_contra_scatter): X~_o[v] = 4X - 2X^{bac} - 2X^{cba} - 2X^{acb} + X^{cab} + X^{bca}
//   (virtual permutations t at fixed ijk, same LDS gather), then X~ is written to every
//   distinct ordering o.s at index v.s (X~ is pair-symmetric), staged through LDS so the
//   global stores are coalesced.  All-equal triples and triples outside the requested
//   range produce zero blocks.
__device__ __constant__ int c_perm[6][3] = {{0, 1, 2}, {1, 0, 2}, {2, 1, 0}, {0, 2, 1}, {2, 0, 1}, {1, 2, 0}};
__device__ __constant__ double c_coef[6] = {4.0, -2.0, -2.0, -2.0, 1.0, 1.0};

constexpr int TT = 16;              // sub-cube edge

// Work item of workgroup blockIdx.x in the passes over (vector, unique triple, sub-cube):
// workgroups are dealt round-robin over the 8 XCDs, so XCD x is given the contiguous range
// [x*floor(n/8) + min(x, n%8), ...) of the order (vector, triple, T0, T1, T2) with T2 (the
// unit-stride index c) fastest.  The sub-cubes that share cache lines of a row (rows of n_v
// doubles are not 128-byte aligned in general) then run on the same XCD at about the same
// time, and the partial lines they write are merged in its L2.
__device__ __forceinline__ void pass_item(int nvec, int nu, int nt, int &vec, int &tri, int (&T)[3]) {
  const int nt3 = nt * nt * nt;
  const long long n = (long long)nvec * nu * nt3, bid = blockIdx.x;
  const long long x = bid % 8, slot = bid / 8, q = n / 8, rem = n % 8;
  const long long L = x * q + (x < rem ? x : rem) + slot;
  const long long vt = L / nt3;
  vec = (int)(vt / nu);
  tri = (int)(vt - (long long)vec * nu);
  const int t = (int)(L - vt * nt3);
  T[0] = t / (nt * nt);
  T[1] = (t / nt) % nt;
  T[2] = t % nt;
}
constexpr int LY = TT + 1, LX = (TT + 1) * (TT + 1);  // odd strides (in doubles) against bank conflicts
constexpr int SUB = TT * LX;

// sub-cube of block src (rows of pitch rp >= n_v) starting at (X0,Y0,Z0): thread (y,z) =
// (tid/16, tid%16) loads the 16 x-values of its (y,z) line into registers; cube_store puts them
// at lds[x*LX + y*LY + z]
__device__ __forceinline__ void cube_load(const double *__restrict__ src, int nv, int rp, int X0, int Y0, int Z0,
                                          double (&v)[TT]) {
  const int tid = threadIdx.x;
  const int y = tid >> 4, z = tid & 15;
  const long long nv2 = (long long)nv * rp;
  const bool yz = (Y0 + y) < nv && (Z0 + z) < nv;
  const double *row = src + (long long)(Y0 + y) * rp + (Z0 + z);
#pragma unroll
  for (int x = 0; x < TT; x++) v[x] = (yz && X0 + x < nv) ? row[(X0 + x) * nv2] : 0.0;
}

__device__ __forceinline__ void cube_store(const double (&v)[TT], double *lds) {
  const int tid = threadIdx.x;
  const int y = tid >> 4, z = tid & 15;
#pragma unroll
  for (int x = 0; x < TT; x++) lds[x * LX + y * LY + z] = v[x];
}

typedef double d4v __attribute__((ext_vector_type(4)));

// cube[x][y][z] -= sum_L xT[p][X0+x][L][Y0+y] G[L][q][r][Z0+z] for the sub-cube in LDS (xT rows of
// pitch occ_pitch(n_v)); wave w
// takes the x-slices w, w+4, w+8, w+12, each a 16x16 (y,z) tile of v_mfma_f64_16x16x4_f64
// (operand lane l: A row y = l%16, k = l/16; B k = l/16, column z = l%16; result row
// l/16 + 4v, column l%16).
__device__ __forceinline__ void occ_term_cube(const OccTerm &ot, int vec, int no, int nv, int p, int q, int r, int X0,
                                              int Y0, int Z0, double *cube) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ly = lane & 15, lk = lane >> 4;
  const int NO = ot.NO;
  const int gy = Y0 + ly, gz = Z0 + ly;
  const int nvp = occ_pitch(nv);  // b pitch of xT
  constexpr int KC = 4;  // k-steps per chunk (16 values of L)
  constexpr int XS = TT / 4;  // x-slices per wave: w, w+4, w+8, w+12, taken two at a time
  const long long qr = (long long)no * no * nv;  // L stride of G
#pragma unroll
  for (int h = 0; h < XS; h += 2) {
    d4v acc[2];
    acc[0] = d4v{0.0, 0.0, 0.0, 0.0};
    acc[1] = acc[0];
    for (int sg = 0; sg < ot.nseg; sg++) {
      const double *gb = ot.G[sg] + vec * ot.gv[sg] + (long long)(q * no + r) * nv + gz;
      for (int k0 = 0; k0 < NO; k0 += 4 * KC) {
        double a[2][KC], b[KC];
#pragma unroll
        for (int u = 0; u < KC; u++) {
          const int L = k0 + 4 * u + lk;
          b[u] = (L < NO && gz < nv) ? gb[L * qr] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 2; e++) {
          const int gx = X0 + wave + 4 * (h + e);
          const double *xa = ot.x[sg] + vec * ot.xv[sg] + ((long long)p * nv + gx) * NO * nvp + gy;
#pragma unroll
          for (int u = 0; u < KC; u++) {
            const int L = k0 + 4 * u + lk;
            a[e][u] = (L < NO && gy < nv && gx < nv) ? xa[L * nvp] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < KC; u++)
#pragma unroll
          for (int e = 0; e < 2; e++) acc[e] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e][u], b[u], acc[e], 0, 0, 0);
      }
    }
#pragma unroll
    for (int e = 0; e < 2; e++)
#pragma unroll
      for (int v = 0; v < 4; v++) cube[(wave + 4 * (h + e)) * LX + (lk + 4 * v) * LY + ly] -= acc[e][v];
  }
}

typedef float f4v __attribute__((ext_vector_type(4)));

// occ_term_cube from the FP32 copies of the operands (reduced-precision forms) with
// v_mfma_f32_16x16x4_f32: operand lanes as in the FP64 form, result register v of lane l at row
// 4(l/16) + v, column l%16.  Each segment's sum over its N_O values of L is formed in FP32 and
// added in FP64.
__device__ __forceinline__ void occ_term_cube_f32(const OccTerm &ot, int vec, int no, int nv, int p, int q, int r,
                                                  int X0, int Y0, int Z0, double *cube) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ly = lane & 15, lk = lane >> 4;
  const int NO = ot.NO;
  const int gy = Y0 + ly, gz = Z0 + ly;
  const int nvp = occ_pitch(nv);
  constexpr int KC = 4;
  constexpr int XS = TT / 4;
  const long long qr = (long long)no * no * nv;
#pragma unroll
  for (int h = 0; h < XS; h += 2) {
    d4v sum[2];
    sum[0] = d4v{0.0, 0.0, 0.0, 0.0};
    sum[1] = sum[0];
    for (int sg = 0; sg < ot.nseg; sg++) {
      f4v acc[2];
      acc[0] = f4v{0.f, 0.f, 0.f, 0.f};
      acc[1] = acc[0];
      const float *gb = ot.Gs[sg] + vec * ot.gsv[sg] + (long long)(q * no + r) * nv + gz;
      for (int k0 = 0; k0 < NO; k0 += 4 * KC) {
        float a[2][KC], b[KC];
#pragma unroll
        for (int u = 0; u < KC; u++) {
          const int L = k0 + 4 * u + lk;
          b[u] = (L < NO && gz < nv) ? gb[L * qr] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 2; e++) {
          const int gx = X0 + wave + 4 * (h + e);
          const float *xa = ot.xs[sg] + vec * ot.xsv[sg] + ((long long)p * nv + gx) * NO * nvp + gy;
#pragma unroll
          for (int u = 0; u < KC; u++) {
            const int L = k0 + 4 * u + lk;
            a[e][u] = (L < NO && gy < nv && gx < nv) ? xa[L * nvp] : 0.f;
          }
        }
#pragma unroll
        for (int u = 0; u < KC; u++)
#pragma unroll
          for (int e = 0; e < 2; e++) acc[e] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e][u], b[u], acc[e], 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 2; e++)
#pragma unroll
        for (int v = 0; v < 4; v++) sum[e][v] += (double)acc[e][v];
    }
#pragma unroll
    for (int e = 0; e < 2; e++)
#pragma unroll
      for (int v = 0; v < 4; v++) cube[(wave + 4 * (h + e)) * LX + (4 * lk + v) * LY + ly] -= sum[e][v];
  }
}

__device__ __forceinline__ int sel3(int a0, int a1, int a2, int i) { return i == 0 ? a0 : (i == 1 ? a1 : a2); }

// OF32: the occupied term from the FP32 operand copies (occ_term_cube_f32)
template <bool OF32>
__global__ __launch_bounds__(256, 4) void k_sym_denom(const double *__restrict__ W, double *__restrict__ Xu,
                                                      const UniqueTriple *ut, int no, int nv, const double *eps_o,
                                                      const double *eps_v, VecBatch vb, long long tb, long long te,
                                                      LocalTerms lt, OccTerm ot, int nu) {
  __shared__ double cube[SUB];
  const int nt = (nv + TT - 1) / TT;
  int vec, tri, T[3];
  pass_item(vb.nvec, vb.tl ? vb.ntl : nu, nt, vec, tri, T);
  if (vb.tl) tri = vb.tl[tri];
  W += vec * vb.w;
  Xu += vec * vb.xu;
  const double omega = vb.omega[vec];
  const double *L1 = lt.L1 + vec * lt.L1v, *LV = lt.LV + vec * lt.LVv;
  const int T0 = T[0], T1 = T[1], T2 = T[2];
  const UniqueTriple u = ut[tri];
  const long long nv2 = (long long)nv * nv, nv3 = nv2 * nv;
  const bool keep = !vb.cvs || (((vb.core_bits >> u.i) | (vb.core_bits >> u.j) | (vb.core_bits >> u.k)) & 1ULL);
  const bool active = !(u.i == u.j && u.j == u.k) && u.canon >= tb && u.canon < te && keep;
  // occupied slab: orderings whose first index lies outside it are left to the other slabs; a
  // later slab (p0 > 0) adds into Xu and skips the triples none of whose orderings it holds
  const int sp0 = vb.p0, sp1 = vb.np > 0 ? vb.p0 + vb.np : no;
  if (vb.np > 0 && !((u.i >= sp0 && u.i < sp1) || (u.j >= sp0 && u.j < sp1) || (u.k >= sp0 && u.k < sp1))) return;
  const int tid = threadIdx.x, lb = tid >> 4, lc = tid & 15;
  double acc[TT];
#pragma unroll
  for (int r = 0; r < TT; r++) acc[r] = 0.0;
  if (active) {
    for (int s = 0; s < 6; s++) {
      const int s0 = c_perm[s][0], s1 = c_perm[s][1], s2 = c_perm[s][2];
      const int p = sel3(u.i, u.j, u.k, s0), q = sel3(u.i, u.j, u.k, s1), rr = sel3(u.i, u.j, u.k, s2);
      if (p < sp0 || p >= sp1) continue;  // uniform over the workgroup
      const int X0 = TT * sel3(T0, T1, T2, s0), Y0 = TT * sel3(T0, T1, T2, s1), Z0 = TT * sel3(T0, T1, T2, s2);
      {
        double v[TT];
        cube_load(W + ((long long)((p - sp0) * no + q) * no + rr) * nv3, nv, nv, X0, Y0, Z0, v);
        __syncthreads();
        cube_store(v, cube);
      }
      if (ot.nseg > 0) {
        __syncthreads();
        if (OF32) occ_term_cube_f32(ot, vec, no, nv, p, q, rr, X0, Y0, Z0, cube);
        else occ_term_cube(ot, vec, no, nv, p, q, rr, X0, Y0, Z0, cube);
      }
      __syncthreads();
      // output local index v = (r, lb, lc) reads the source cube at (v_{s0}, v_{s1}, v_{s2})
      const int w0 = s0 == 0 ? LX : (s1 == 0 ? LY : 1);
      const int w1 = s0 == 1 ? LX : (s1 == 1 ? LY : 1);
      const int w2 = s0 == 2 ? LX : (s1 == 2 ? LY : 1);
      const double *cb = cube + lb * w1 + lc * w2;
#pragma unroll
      for (int r = 0; r < TT; r++) acc[r] += cb[r * w0];
      if (lt.L1) {  // local terms of the left triples: L^x_p g_qyrz + L^{xy}_{pq} F_rz
        const int gb = TT * T1 + lb, gc = TT * T2 + lc;
#pragma unroll
        for (int r = 0; r < TT; r++) {
          const int ga = TT * T0 + r;
          if (ga >= nv || gb >= nv || gc >= nv) continue;
          const int x = sel3(ga, gb, gc, s0), y = sel3(ga, gb, gc, s1), z = sel3(ga, gb, gc, s2);
          acc[r] += L1[(long long)x * lt.NO + p] * lt.gov[(((long long)q * no + rr) * nv + y) * nv + z] +
                    LV[(((long long)p * no + q) * nv + x) * nv + y] * lt.F[(long long)rr * nv + z];
        }
      }
    }
  }
  const double eocc = eps_o[u.i] + eps_o[u.j] + eps_o[u.k];
  const int up = occ_pitch(nv);  // row pitch of the unique-triple blocks
  double *dst = Xu + (long long)tri * nv * nv * up;
  const int gb = TT * T1 + lb, gc = TT * T2 + lc;
  if (gb >= nv || gc >= nv) return;
#pragma unroll
  for (int r = 0; r < TT; r++) {
    const int ga = TT * T0 + r;
    if (ga >= nv) break;
    const double den = eps_v[ga] + eps_v[gb] + eps_v[gc] - eocc - omega;
    const double x = active ? -acc[r] / den : 0.0;
    if (vb.np > 0) dst[((long long)ga * nv + gb) * up + gc] += x;
    else dst[((long long)ga * nv + gb) * up + gc] = x;
  }
}

// OT: element type of the ordered blocks written (double, or float for the reduced-precision
// forms of the right and left transforms and the ground residual)
template <typename OT>
__global__ __launch_bounds__(256) void k_contra_scatter(const double *__restrict__ Xu, OT *__restrict__ Xt,
                                                        const UniqueTriple *ut, int no, int nv, int covariant, int nu,
                                                        int nvec, long long xuv, long long xtv, int sp0, int sp1,
                                                        const int *tl) {
  __shared__ double cube[SUB];
  const int nt = (nv + TT - 1) / TT;
  int vec, tri, T[3];
  pass_item(nvec, nu, nt, vec, tri, T);
  if (tl) tri = tl[tri];
  Xu += vec * xuv;
  Xt += vec * xtv;
  const UniqueTriple u = ut[tri];
  // occupied slab [sp0, sp1): only the orderings whose first index lies in it are written
  if (!((u.i >= sp0 && u.i < sp1) || (u.j >= sp0 && u.j < sp1) || (u.k >= sp0 && u.k < sp1))) return;
  const long long nv2 = (long long)nv * nv, nv3 = nv2 * nv;
  const int o[3] = {u.i, u.j, u.k};
  const int tid = threadIdx.x, lb = tid >> 4, lc = tid & 15;
  const int up = occ_pitch(nv);  // row pitch of the unique-triple blocks
  const double *src = Xu + (long long)tri * nv * nv * up;
  double acc[TT];
#pragma unroll
  for (int r = 0; r < TT; r++) acc[r] = 0.0;
  const int nterm = covariant ? 1 : 6;  // covariant mode copies X itself to every ordering
  // the sub-cube of term t+1 is loaded into registers while term t is gathered
  double nxt[TT];
  cube_load(src, nv, up, TT * T[0], TT * T[1], TT * T[2], nxt);
  for (int t = 0; t < nterm; t++) {
    const int t0 = c_perm[t][0], t1 = c_perm[t][1], t2 = c_perm[t][2];
    __syncthreads();
    cube_store(nxt, cube);
    if (t + 1 < nterm) {
      const int u0 = c_perm[t + 1][0], u1 = c_perm[t + 1][1], u2 = c_perm[t + 1][2];
      cube_load(src, nv, up, TT * T[u0], TT * T[u1], TT * T[u2], nxt);
    }
    __syncthreads();
    const double cf = covariant ? 1.0 : c_coef[t];
#pragma unroll
    for (int r = 0; r < TT; r++) {
      const int v[3] = {r, lb, lc};
      acc[r] += cf * cube[v[t0] * LX + v[t1] * LY + v[t2]];
    }
  }
  // stage X~ of this tile (local index v) and write each distinct ordering coalesced
  __syncthreads();
#pragma unroll
  for (int r = 0; r < TT; r++) cube[r * LX + lb * LY + lc] = acc[r];
  __syncthreads();
  for (int s = 0; s < 6; s++) {
    if (!((u.mask >> s) & 1)) continue;
    const int s0 = c_perm[s][0], s1 = c_perm[s][1], s2 = c_perm[s][2];
    if (o[s0] < sp0 || o[s0] >= sp1) continue;
    OT *dst = Xt + ((long long)((o[s0] - sp0) * no + o[s1]) * no + o[s2]) * nv3;
    // output local index w = v.s, i.e. w_n = v_{s_n}; the writer of w reads v with v_{s_n} = w_n
    const int W0 = TT * T[s0], W1 = TT * T[s1], W2 = TT * T[s2];
    for (int r = 0; r < TT; r++) {
      const int w[3] = {r, lb, lc};
      if (W0 + w[0] >= nv || W1 + w[1] >= nv || W2 + w[2] >= nv) continue;
      int v[3];
      v[s0] = w[0]; v[s1] = w[1]; v[s2] = w[2];
      dst[(W0 + w[0]) * nv2 + (long long)(W1 + w[1]) * nv + (W2 + w[2])] = (OT)cube[v[0] * LX + v[1] * LY + v[2]];
    }
  }
}

// CVS projection (one thread per element of the three arrays)
__global__ void k_cvs_project(const double *x1, const double *x2a, const double *x2b, double *y1, double *y2a,
                              double *y2b, const unsigned char *core, int no, int nv, int NO, int NV) {
  const long long n1 = (long long)NV * NO, na = (long long)nv * NV * no * no, nb = (long long)nv * nv * no * NO;
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id < n1) {
    const int I = (int)(id % NO);
    y1[id] = core[I] ? x1[id] : 0.0;
  } else if (id < n1 + na) {
    const long long e = id - n1;
    const int j = (int)(e % no), i = (int)((e / no) % no);
    y2a[e] = (core[i] || core[j]) ? x2a[e] : 0.0;
  } else if (id < n1 + na + nb) {
    const long long e = id - n1 - na;
    const int L = (int)(e % NO), i = (int)((e / NO) % no);
    y2b[e] = (core[i] || core[L]) ? x2b[e] : 0.0;
  }
}

// xT[p][a][L][b] = x[a][b][p][L]
__global__ void k_occ_xT(const double *__restrict__ x, int no, int nv, int NO, double *__restrict__ xT) {
  const int nvp = occ_pitch(nv);
  const long long n = (long long)no * nv * NO * nvp;
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int b = (int)(id % nvp);
  long long t = id / nvp;
  const int L = (int)(t % NO);
  t /= NO;
  const int a = (int)(t % nv), p = (int)(t / nv);
  xT[id] = b < nv ? x[(((long long)a * nv + b) * no + p) * NO + L] : 0.0;
}

// ------------------------------------------------- pairing maps of doubles vectors
// The doubles X^{AB}_{IJ} = X^{BA}_{JI} are stored on two overlapping blocks,
// A2[a][D][i][j] = X^{aD}_{ij} and B2[a][b][i][L] = X^{ab}_{iL}.  An amplitude (A,I,B,J) sits at
// up to four positions: A2(A,B,I,J) if A < n_v, J < n_o; A2(B,A,J,I) if B < n_v, I < n_o;
// B2(A,B,I,J) if A, B < n_v, I < n_o; B2(B,A,J,I) if A, B < n_v, J < n_o (coinciding
// positions count once).
struct PosList {
  int n = 0;
  long long off[4];  // offsets into A2 (>= 0) or B2 (encoded as -1 - offset)
};

__device__ __forceinline__ void amp_positions(int A, int I, int B, int J, int no, int nv, int NO, int NV,
                                              PosList &pl) {
  long long cand[4];
  int nc = 0;
  if (A < nv && I < no && J < no) cand[nc++] = (((long long)A * NV + B) * no + I) * no + J;
  if (B < nv && I < no && J < no) cand[nc++] = (((long long)B * NV + A) * no + J) * no + I;
  if (A < nv && B < nv && I < no) cand[nc++] = -1 - ((((long long)A * nv + B) * no + I) * NO + J);
  if (A < nv && B < nv && J < no) cand[nc++] = -1 - ((((long long)B * nv + A) * no + J) * NO + I);
  pl.n = 0;
  for (int c = 0; c < nc; c++) {
    bool dup = false;
    for (int e = 0; e < pl.n; e++) dup = dup || (pl.off[e] == cand[c]);
    if (!dup) pl.off[pl.n++] = cand[c];
  }
}

__device__ __forceinline__ double pos_val(const double *A2, const double *B2, long long o) {
  return o >= 0 ? A2[o] : B2[-1 - o];
}

// mode 0: average over the positions of each amplitude (a consistent, pair-symmetric vector)
// mode 1: Euclidean gradient g -> left vector L with G(L, y) = <g, y> on consistent y:
//         L = (2 s + s^{BA}_{IJ}) / 3, s = sum of g over the positions of the amplitude
// mode 2: consistent vector S -> representer h with <h, y> = G(S, y) on consistent y:
//         h = (2 S - S^{BA}_{IJ}) / (number of positions)
__global__ void k_vec_map(const double *__restrict__ A2, const double *__restrict__ B2, int no, int nv, int NO, int NV,
                          int mode, double *__restrict__ oA, double *__restrict__ oB) {
  const long long nA = (long long)nv * NV * no * no, nB = (long long)nv * nv * no * NO;
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= nA + nB) return;
  int A, I, B, J;
  if (id < nA) {
    long long t = id;
    J = (int)(t % no); t /= no;
    I = (int)(t % no); t /= no;
    B = (int)(t % NV);
    A = (int)(t / NV);
  } else {
    long long t = id - nA;
    J = (int)(t % NO); t /= NO;
    I = (int)(t % no); t /= no;
    B = (int)(t % nv);
    A = (int)(t / nv);
  }
  PosList pu, ps;
  amp_positions(A, I, B, J, no, nv, NO, NV, pu);
  double r;
  if (mode == 0) {
    double sum = 0.0;
    for (int e = 0; e < pu.n; e++) sum += pos_val(A2, B2, pu.off[e]);
    r = sum / pu.n;
  } else if (mode == 1) {
    amp_positions(B, I, A, J, no, nv, NO, NV, ps);
    double su = 0.0, ss = 0.0;
    for (int e = 0; e < pu.n; e++) su += pos_val(A2, B2, pu.off[e]);
    for (int e = 0; e < ps.n; e++) ss += pos_val(A2, B2, ps.off[e]);
    r = (2.0 * su + ss) / 3.0;
  } else {
    amp_positions(B, I, A, J, no, nv, NO, NV, ps);
    const double self = id < nA ? A2[id] : B2[id - nA];
    r = (2.0 * self - pos_val(A2, B2, ps.off[0])) / pu.n;
  }
  if (id < nA) oA[id] = r;
  else oB[id - nA] = r;
}

// Contravariant pass over one orbit of sub-cube tiles: the distinct permutations of a tile
// triple A >= B >= C.  The six virtual permutations of an output tile read sub-cubes of X_u at
// the permuted tile positions, which are the members of its orbit; so one workgroup per orbit
// reads each input sub-cube of X_u once (instead of once per output tile) and keeps the
// contravariant tiles of the whole orbit in registers, then scatters each of them to every
// distinct ordering of the triple as k_contra_scatter does.
constexpr int kPerm[6][3] = {{0, 1, 2}, {1, 0, 2}, {2, 1, 0}, {0, 2, 1}, {2, 0, 1}, {1, 2, 0}};
constexpr double kCoef[6] = {4.0, -2.0, -2.0, -2.0, 1.0, 1.0};

__device__ __forceinline__ int tile_code(int x, int y, int z, int nt) { return (x * nt + y) * nt + z; }

template <typename OT>
__global__ __launch_bounds__(256, 2) void k_contra_orbit(const double *__restrict__ Xu, OT *__restrict__ Xt,
                                                         const UniqueTriple *ut, int no, int nv, int nu, int nvec,
                                                         long long xuv, long long xtv, int sp0, int sp1,
                                                         const int *tl) {
  __shared__ double cube[SUB];
  const int nt = (nv + TT - 1) / TT;
  const int norb = nt * (nt + 1) * (nt + 2) / 6;
  // work item (vector, triple, orbit), dealt over the XCDs in contiguous ranges
  const long long n = (long long)nvec * nu * norb, bid = blockIdx.x;
  const long long x8 = bid % 8, slot = bid / 8, q8 = n / 8, rem = n % 8;
  const long long L = x8 * q8 + (x8 < rem ? x8 : rem) + slot;
  const long long vt = L / norb;
  const int vec = (int)(vt / nu), tri = tl ? tl[vt - (long long)vec * nu] : (int)(vt - (long long)vec * nu);
  int orb = (int)(L - vt * norb), A = 0, B = 0, C = 0;
  for (int a = 0, idx = 0; a < nt; a++)
    for (int b = 0; b <= a; b++)
      for (int c = 0; c <= b; c++, idx++)
        if (idx == orb) { A = a; B = b; C = c; }
  // orbit members (distinct permutations of (A,B,C)) as tile codes
  const int t3[3] = {A, B, C};
  int mem[6] = {-1, -1, -1, -1, -1, -1}, nm = 0;
#pragma unroll
  for (int s = 0; s < 6; s++) {
    const int code = tile_code(t3[kPerm[s][0]], t3[kPerm[s][1]], t3[kPerm[s][2]], nt);
    bool dup = false;
#pragma unroll
    for (int e = 0; e < 6; e++) dup = dup || (mem[e] == code);
#pragma unroll
    for (int e = 0; e < 6; e++)
      if (!dup && e == nm) mem[e] = code;
    nm += dup ? 0 : 1;
  }
  const UniqueTriple u = ut[tri];
  // occupied slab [sp0, sp1): only the orderings whose first index lies in it are written
  if (!((u.i >= sp0 && u.i < sp1) || (u.j >= sp0 && u.j < sp1) || (u.k >= sp0 && u.k < sp1))) return;
  const long long nv2 = (long long)nv * nv, nv3 = nv2 * nv;
  const int o[3] = {u.i, u.j, u.k};
  const int tid = threadIdx.x, lb = tid >> 4, lc = tid & 15;
  const int up = occ_pitch(nv);  // row pitch of the unique-triple blocks
  const double *src = Xu + vec * xuv + (long long)tri * nv * nv * up;
  Xt += vec * xtv;
  double acc[6][TT];
#pragma unroll
  for (int t = 0; t < 6; t++)
#pragma unroll
    for (int r = 0; r < TT; r++) acc[t][r] = 0.0;
#pragma unroll
  for (int j = 0; j < 6; j++) {
    if (j >= nm) break;
    const int J = mem[j];
    const int J0 = J / (nt * nt), J1 = (J / nt) % nt, J2 = J % nt;
    double v[TT];
    cube_load(src, nv, up, TT * J0, TT * J1, TT * J2, v);
    __syncthreads();
    cube_store(v, cube);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 6; t++) {
      if (t >= nm) break;
      const int T = mem[t];
      const int tt[3] = {T / (nt * nt), (T / nt) % nt, T % nt};
#pragma unroll
      for (int pi = 0; pi < 6; pi++) {
        if (tile_code(tt[kPerm[pi][0]], tt[kPerm[pi][1]], tt[kPerm[pi][2]], nt) != J) continue;
        // output local (r, lb, lc) reads the input cube at (v_{pi0}, v_{pi1}, v_{pi2})
        const int w0 = kPerm[pi][0] == 0 ? LX : (kPerm[pi][1] == 0 ? LY : 1);
        const int w1 = kPerm[pi][0] == 1 ? LX : (kPerm[pi][1] == 1 ? LY : 1);
        const int w2 = kPerm[pi][0] == 2 ? LX : (kPerm[pi][1] == 2 ? LY : 1);
        const double *cb = cube + lb * w1 + lc * w2;
#pragma unroll
        for (int r = 0; r < TT; r++) acc[t][r] += kCoef[pi] * cb[r * w0];
      }
    }
    __syncthreads();
  }
  // stage each output tile and write it to every distinct ordering
#pragma unroll
  for (int t = 0; t < 6; t++) {
    if (t >= nm) break;
    const int T = mem[t];
    const int TT3[3] = {T / (nt * nt), (T / nt) % nt, T % nt};
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TT; r++) cube[r * LX + lb * LY + lc] = acc[t][r];
    __syncthreads();
    for (int s = 0; s < 6; s++) {
      if (!((u.mask >> s) & 1)) continue;
      const int s0 = c_perm[s][0], s1 = c_perm[s][1], s2 = c_perm[s][2];
      if (o[s0] < sp0 || o[s0] >= sp1) continue;
      OT *dst = Xt + ((long long)((o[s0] - sp0) * no + o[s1]) * no + o[s2]) * nv3;
      const int W0 = TT * sel3(TT3[0], TT3[1], TT3[2], s0), W1 = TT * sel3(TT3[0], TT3[1], TT3[2], s1),
                W2 = TT * sel3(TT3[0], TT3[1], TT3[2], s2);
      // output local w = (r, lb, lc) sits at v with v_{s_n} = w_n: LDS weight of w_n is that of axis s_n
      const int ax[3] = {LX, LY, 1};
      const int q0 = sel3(ax[0], ax[1], ax[2], s0), q1 = sel3(ax[0], ax[1], ax[2], s1),
                q2 = sel3(ax[0], ax[1], ax[2], s2);
      if (W1 + lb >= nv || W2 + lc >= nv) continue;
      OT *drow = dst + (long long)(W1 + lb) * nv + (W2 + lc);
      const double *cb = cube + lb * q1 + lc * q2;
      for (int r = 0; r < TT; r++) {
        if (W0 + r >= nv) break;
        drow[(W0 + r) * nv2] = (OT)cb[r * q0];
      }
    }
  }
}

// -------------------------------------------------------------- wave helpers
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ρ-type small contractions over ordered blocks, one workgroup per (p, q, group of AG values of a):
//   part1[p][q][a]   = sum_{r,b,c} X~^{abc}_{pqr} g_qbrc
//   Yvv[p][q][a][b]  = sum_{r,c} (X~^{abc}_{pqr} F_rc + T~^{abc}_{pqr} U_rc)
// Each of the four waves takes every fourth row b; its lanes run over the n_o n_v pairs (r, c)
// of the row, 64 at a time, and each lane applies the g, F and U values it loads to the AG
// values of a of its group (AG independent loads of X~ per position, and g read once per group
// instead of once per a).  A row costs one cross-lane reduction per a.  (Measured at n_v = 60:
// AG = 4 saves 0.8 ms per FP64 step; with FP32 blocks it cost 1.9 ms, so those keep AG = 1.)
template <bool HAS_T, typename XT_, int SR_AG>
__global__ __launch_bounds__(256) void k_small_right(const XT_ *__restrict__ X, const XT_ *__restrict__ T,
                                                     const double *__restrict__ gov, const double *__restrict__ F,
                                                     const double *__restrict__ U, int no, int nv,
                                                     double *__restrict__ part1, double *__restrict__ Yvv, int yacc) {
  const int nag = (nv + SR_AG - 1) / SR_AG;
  const int id = blockIdx.x;
  const int ag = id % nag, q = (id / nag) % no, p = id / (nag * no);
  const int a0 = ag * SR_AG, na = min(SR_AG, nv - a0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nv2 = (long long)nv * nv, nv3 = nv2 * nv;
  const long long off = ((long long)p * no + q) * no * nv3 + (long long)a0 * nv2;  // r = 0, a = a0, b = 0
  const XT_ *x0 = X + off;
  const XT_ *t0 = HAS_T ? T + off : nullptr;
  const double *g0 = gov + (long long)q * no * nv2;
  const int nrc = no * nv;
  const int r0 = lane / nv, c0 = lane - r0 * nv;  // (r, c) of position e = lane
  __shared__ double rpart[4][SR_AG];
  double racc[SR_AG];
#pragma unroll
  for (int t = 0; t < SR_AG; t++) racc[t] = 0.0;
  for (int b = wv; b < nv; b += 4) {
    const long long bo = (long long)b * nv;
    double yb[SR_AG];
#pragma unroll
    for (int t = 0; t < SR_AG; t++) yb[t] = 0.0;
    int r = r0, c = c0;
#pragma unroll 2
    for (int e = lane; e < nrc; e += 64) {
      const long long o = (long long)r * nv3 + bo + c;
      const double gv = g0[(long long)r * nv2 + bo + c], fv = F[r * nv + c];
      const double uv = HAS_T ? U[r * nv + c] : 0.0;
      double xv[SR_AG], tv[SR_AG];
#pragma unroll
      for (int t = 0; t < SR_AG; t++) {
        xv[t] = t < na ? (double)x0[o + t * nv2] : 0.0;
        tv[t] = (HAS_T && t < na) ? (double)t0[o + t * nv2] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < SR_AG; t++) {
        racc[t] += xv[t] * gv;
        yb[t] += xv[t] * fv;
        if (HAS_T) yb[t] += tv[t] * uv;
      }
      // advance the position by 64: c += 64 with the carry into r
      c += 64;
      while (c >= nv) {
        c -= nv;
        r++;
      }
    }
#pragma unroll
    for (int t = 0; t < SR_AG; t++) {
      const double y = wave_sum(yb[t]);
      if (lane == 0 && t < na) {
        double &yo = Yvv[(((long long)p * no + q) * nv + a0 + t) * nv + b];
        yo = yacc ? yo + y : y;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < SR_AG; t++) {
    const double v = wave_sum(racc[t]);
    if (lane == 0) rpart[wv][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < na)
    part1[((long long)p * no + q) * nv + a0 + threadIdx.x] =
        (rpart[0][threadIdx.x] + rpart[1][threadIdx.x]) + (rpart[2][threadIdx.x] + rpart[3][threadIdx.x]);
}

// Occupied Gram block of two ordered-triple buffers (n_o <= 16), one partial per workgroup:
//   P[w][k][l] = sum_{e in chunk} X1[i][j][k][e] X2[i][j][l][e],  w = (i n_o + j) nch + chunk,
// e running over the n_v^3 virtual triples.  Each wave accumulates one 16x16 tile with
// v_mfma_f64_16x16x4_f64: lane l holds row l%16 (k of X1 as the A operand, l of X2 as the B
// operand) at four consecutive e, so the four lanes of a row read 128 contiguous bytes and the
// k index of each MFMA is a set of four e values shared by both operands.  Rows k >= n_o and
// positions past the chunk load zeros.  The four waves' tiles are summed in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_gram_kl(const double *__restrict__ X1, const double *__restrict__ X2, int no,
                                                long long ne, long long chunk, int nch, double *__restrict__ P) {
  __shared__ double red[4][16][17];
  const int w = blockIdx.x;
  const int ij = w / nch, ch = w - ij * nch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, q = lane >> 4;
  const long long e0 = (long long)ch * chunk, e1 = min(ne, e0 + chunk);
  const bool valid = row < no;
  const long long roff = ((long long)ij * no + (valid ? row : 0)) * ne;
  const double *x1 = X1 + roff, *x2 = X2 + roff;
  d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
  // the trip count is uniform over the wave (the MFMA reads every lane's operands whatever the
  // exec mask): positions past the chunk load zeros
  for (long long eb = e0 + 16 * wave; eb < e1; eb += 64) {
    const long long e = eb + 4 * q;
    double a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const bool in = valid && e + c < e1;
      a[c] = in ? x1[e + c] : 0.0;
      b[c] = in ? x2[e + c] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; c++) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b[c], acc, 0, 0, 0);
  }
  // lane l, register v: row l/16 + 4v, column l%16
#pragma unroll
  for (int v = 0; v < 4; v++) red[wave][q + 4 * v][row] = acc[v];
  __syncthreads();
  const int k = threadIdx.x >> 4, l = threadIdx.x & 15;
  if (k < no && l < no)
    P[((long long)w * no + k) * no + l] = (red[0][k][l] + red[1][k][l]) + (red[2][k][l] + red[3][k][l]);
}

// Virtual Gram block of two ordered-triple buffers seen as row sets, for 64 < n <= 160:
//   P[w][c][d] = sum_{k in chunk w} X1[k][c] X2[k][d],  rows k of n contiguous values
// (n = n_v, k running over (i,j,k,a,b)).  The whole n x n output lives in one workgroup: 8 waves
// share its 16x16 v_mfma_f64_16x16x4_f64 tiles (tile t = wave + 8 j), so each slab of 16 rows
// (a contiguous block of 16 n values per operand) is read from HBM once and staged in LDS.
constexpr int GCD_TMAX = 10;                          // 16-wide tiles per dimension (n <= 160)
constexpr int GCD_LDP = 16 * GCD_TMAX + 4;            // LDS row pitch (doubles)
constexpr int GCD_SLOTS = (GCD_TMAX * GCD_TMAX + 7) / 8;  // tiles per wave
__global__ __launch_bounds__(512, 1) void k_gram_cd(const double *__restrict__ X1, const double *__restrict__ X2,
                                                   int n, long long nrows, long long chunk,
                                                   double *__restrict__ P) {
  __shared__ double As[2][16][GCD_LDP];
  __shared__ double Bs[2][16][GCD_LDP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = (n + 15) / 16, ntile = nt * nt;
  const long long k0 = (long long)blockIdx.x * chunk, k1 = min(nrows, k0 + chunk);
  const int nslab = (int)((k1 - k0 + 15) / 16);
  const int sn = 16 * n;  // values per slab and operand
  // zero both buffers once: the columns n .. 16 nt - 1 stay zero
  for (int e = tid; e < 2 * 16 * GCD_LDP; e += 512) {
    (&As[0][0][0])[e] = 0.0;
    (&Bs[0][0][0])[e] = 0.0;
  }
  constexpr int PER = (16 * 16 * GCD_TMAX + 511) / 512;  // staged values per thread and operand
  double ra[PER], rb[PER];
  auto load = [&](int sl) {
    const long long base = (k0 + 16LL * sl) * n;
    const long long lim = (k1 - k0 - 16LL * sl) * n;  // values of this slab inside the chunk
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 512 * u;
      const bool in = e < sn && e < lim;
      ra[u] = in ? X1[base + e] : 0.0;
      rb[u] = in ? X2[base + e] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 512 * u;
      if (e < sn) {
        const int r = e / n, c = e - (e / n) * n;
        As[buf][r][c] = ra[u];
        Bs[buf][r][c] = rb[u];
      }
    }
  };
  d4v acc[GCD_SLOTS];
#pragma unroll
  for (int j = 0; j < GCD_SLOTS; j++) acc[j] = d4v{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  if (nslab > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int sl = 0; sl < nslab; sl++) {
    const int cur = sl & 1;
    if (sl + 1 < nslab) load(sl + 1);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int j = 0; j < GCD_SLOTS; j++) {
        const int t = wave + 8 * j;
        if (t < ntile) {  // uniform over the wave
          const int ti = t / nt, tj = t - (t / nt) * nt;
          const double a = As[cur][kr][16 * ti + (lane & 15)];
          const double b = Bs[cur][kr][16 * tj + (lane & 15)];
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
      }
    }
    if (sl + 1 < nslab) store(cur ^ 1);
    __syncthreads();
  }
  // lane l, register v: row (c) 16 ti + l/16 + 4 v, column (d) 16 tj + l%16
  double *Pw = P + (long long)blockIdx.x * n * n;
#pragma unroll
  for (int j = 0; j < GCD_SLOTS; j++) {
    const int t = wave + 8 * j;
    if (t < ntile) {
      const int ti = t / nt, tj = t - (t / nt) * nt;
      const int d = 16 * tj + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int c = 16 * ti + (lane >> 4) + 4 * v;
        if (c < n && d < n) Pw[(long long)c * n + d] = acc[j][v];
      }
    }
  }
}

// C[k][l] = alpha sum_w P[w][k][l] + beta C[k][l] (row stride ldc): one workgroup per (k,l),
// thread t sums w = t, t+256, ... and a fixed tree adds the 256 partial sums
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ P, int nw, int no, double alpha,
                                                     double beta, double *C, long long ldc) {
  __shared__ double red[256];
  const int id = blockIdx.x, k = id / no, l = id - k * no;
  const long long n2 = (long long)no * no;
  double s = 0.0;
  for (int w = threadIdx.x; w < nw; w += 256) s += P[w * n2 + id];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *c = C + (long long)k * ldc + l;
    *c = alpha * red[0] + (beta != 0.0 ? beta * *c : 0.0);
  }
}

// x1[A][I] = sum_q part1[I][q][A] on the active block, 0 elsewhere
__global__ void k_singles_out(const double *part1, int no, int nv, int NO, int NV, double *x1) {
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= NV * NO) return;
  const int I = id % NO, A = id / NO;
  double s = 0.0;
  if (A < nv && I < no)
    for (int q = 0; q < no; q++) s += part1[((long long)I * no + q) * nv + A];
  x1[id] = s;
}

// raw full-space doubles Y^{AB}_{IJ} from the blocks YvV[i][j][a][D], YvO[i][a][b][L], Yvv[i][j][a][b]
__device__ __forceinline__ double yfull(const DoublesRaw &y, int A, int B, int I, int J) {
  double s = 0.0;
  const int no = y.no, nv = y.nv, NO = y.NO, NV = y.NV;
  if (A < nv && I < no && J < no) {
    s += y.YvV[(((long long)I * no + J) * nv + A) * NV + B];
    if (B < nv && y.Yvv) s += y.Yvv[(((long long)I * no + J) * nv + A) * nv + B];
  }
  if (A < nv && B < nv && I < no && y.YvO) s += y.YvO[(((long long)I * nv + A) * nv + B) * NO + J];
  return s;
}
__device__ __forceinline__ double xcontra(const DoublesRaw &y, int A, int B, int I, int J) {
  double s = yfull(y, A, B, I, J) + yfull(y, B, A, J, I);
  if (y.delta && A == B && I == J) s *= 0.5;
  return s;
}
__device__ __forceinline__ double xcov(const DoublesRaw &y, int A, int B, int I, int J) {
  return (2.0 * xcontra(y, A, B, I, J) + xcontra(y, B, A, I, J)) * (1.0 / 3.0);
}

// covariant output blocks: out_a[a][D][i][j], out_b[a][b][i][L]
__global__ void k_doubles_out(DoublesRaw y, double *out_a, double *out_b) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int no = y.no, nv = y.nv, NO = y.NO, NV = y.NV;
  const long long na = (long long)nv * NV * no * no, nb = (long long)nv * nv * no * NO;
  if (id < na) {
    const int j = id % no, i = (id / no) % no, D = (id / ((long long)no * no)) % NV,
              a = id / ((long long)no * no * NV);
    out_a[id] = xcov(y, a, D, i, j);
  } else if (id < na + nb) {
    const long long e = id - na;
    const int L = e % NO, i = (e / NO) % no, b = (e / ((long long)NO * no)) % nv,
              a = e / ((long long)NO * no * nv);
    out_b[e] = xcov(y, a, b, i, L);
  }
}

// V[r][c] = sum_q Q[q][r][c][q]   (Q stored [q][r][c][L], L over all occupied)
__global__ void k_diag_sum(const double *Q, int no, int nv, int NO, double *V) {
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= no * nv) return;
  const int c = id % nv, r = id / nv;
  double acc = 0.0;
  for (int q = 0; q < no; q++) acc += Q[(((long long)q * no + r) * nv + c) * NO + q];
  V[id] = acc;
}

// Z[J][k][d] = sum_j Am[j][J][k][d] - Hp[k][J][d]
__global__ void k_left_Z(const double *Am, const double *Hp, int nc, int no, int nv, double *Z) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)nc * no * nv) return;
  const int dd = id % nv, k = (id / nv) % no;
  const long long J = id / ((long long)no * nv);
  double acc = 0.0;
  for (int j = 0; j < no; j++) acc += Am[(long long)j * nc * no * nv + id];
  Z[id] = acc - Hp[((long long)k * nc + J) * nv + dd];
}

// out[k][c][r] = in[k][r][c] for R x C matrices, 32x32 LDS tiles
__global__ void k_transpose(const double *__restrict__ in, double *__restrict__ out, int R, int C) {
  __shared__ double t[32][33];
  const long long base = (long long)blockIdx.z * R * C;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    t[y][tx] = (r < R && c < C) ? in[base + (long long)r * C + c] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (r < R && c < C) out[base + (long long)c * R + r] = t[tx][y];
  }
}

// ------------------------------------------------------------- host launchers
#define L1D(kern, n, ...) \
  do { if (!g_dry && (n) > 0) hipLaunchKernelGGL(kern, dim3(nblk(n)), dim3(256), 0, s, __VA_ARGS__); } while (0)

// dst[r][k] = src[r][k] for k < nk of rows of length ld
__global__ void k_pack_cols(const double *src, long long rows, int ld, int nk, double *dst) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= rows * nk) return;
  const long long r = id / nk;
  dst[id] = src[r * ld + (id - r * nk)];
}

// C[k][D][b][c] = T[(b*NV + D)][(c*no + k)]
__global__ void k_vvvo_permute(const double *T, int no, int nv, int NV, double *C) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long nv2 = (long long)nv * nv;
  if (id >= (long long)no * NV * nv2) return;
  const int c = id % nv, b = (id / nv) % nv;
  const long long kD = id / nv2;
  const int D = kD % NV, k = kD / NV;
  C[id] = T[((long long)b * NV + D) * ((long long)nv * no) + (long long)c * no + k];
}

void launch_pack_cols(const double *src, long long rows, int ld, int nk, double *dst, hipStream_t s) {
  L1D(k_pack_cols, rows * nk, src, rows, ld, nk, dst);
}

void launch_vvvo_permute(const double *T, int no, int nv, int NV, double *C, hipStream_t s) {
  L1D(k_vvvo_permute, (long long)no * NV * nv * nv, T, no, nv, NV, C);
}

void launch_lhat_vO_init(const double *LOV, int nc, int NO, int NV, int nv, double *LhvO, hipStream_t s) {
  L1D(k_lhat_vO_init, (long long)nc * nv * NO, LOV, nc, NO, NV, nv, LhvO);
}

void launch_fock_s(const double *LOV, const double *x, int nc, int NO, int NV, double *tmp_xT, double *tmp_s,
                   hipStream_t s) {
  if (g_dry || nc <= 0) return;
  launch_transpose(x, tmp_xT, 1, NV, NO, s);
  hipLaunchKernelGGL(k_fock_s, dim3(nc), dim3(256), 0, s, LOV, tmp_xT, nc, NO, NV, tmp_s);
}

void launch_fock_finish(const double *LOV, const double *tmp_s, const double *tmp_y, int nc, int NO, int NV, int no,
                        int nv, double *tmp_z, double *out, hipStream_t s) {
  L1D(k_fock_z, (long long)nc * no * nv, LOV, tmp_s, tmp_y, nc, NO, NV, no, nv, tmp_z);
  L1D(k_sum_rows, (long long)no * nv, tmp_z, (long long)nc, (long long)no * nv, out);
}

void launch_pack_vVoo(const double *x, int no, int nv, int NV, int rbar, double *xA, hipStream_t s) {
  L1D(k_pack_vVoo, (long long)no * no * nv * NV, x, no, nv, NV, rbar, xA);
}
void launch_rbar_vvoO(const double *x, int no, int nv, int NO, double *xB, hipStream_t s) {
  L1D(k_rbar_vvoO, (long long)nv * nv * no * NO, x, no, nv, NO, xB);
}
void launch_pack_vvoo(const double *x, int no, int nv, int NV, int mode, double *xV, hipStream_t s) {
  L1D(k_pack_vvoo, (long long)no * no * nv * nv, x, no, nv, NV, mode, xV);
}

void launch_dot(const double *a, const double *b, long long n, double scale, double *part, double *out,
                hipStream_t s) {
  if (g_dry) return;
  hipLaunchKernelGGL(k_dot_partial, dim3(512), dim3(256), 0, s, a, b, n, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, s, part, 512, scale, out);
}

void launch_strengths(const double *A, int N, int ncomp, int nstate, const double *Dm0, const double *D0m,
                      const double *D00, const double *sv, const double *om, double *Tm0, double *T0m, double *f,
                      hipStream_t s) {
  if (g_dry || N <= 0 || ncomp <= 0 || nstate <= 0) return;
  hipLaunchKernelGGL(k_moments, dim3(ncomp, nstate), dim3(256), 0, s, A, (long long)N * N, ncomp, Dm0, D0m, D00, sv,
                     Tm0, T0m);
  hipLaunchKernelGGL(k_strength, dim3((nstate + 63) / 64), dim3(64), 0, s, Tm0, T0m, om, ncomp, nstate, f);
}

void launch_add_diag(double *D, int NO, int N, const double *sv, double f, hipStream_t s) {
  L1D(k_add_diag, (long long)NO, D, NO, N, sv, f);
}

void launch_add_vo(double *D, int NO, int N, int no, int nv, const double *Y, double f, hipStream_t s) {
  L1D(k_add_vo, (long long)no * nv, D, NO, N, no, nv, Y, f);
}

void launch_sym_denom(const double *W, double *Xu, const UniqueTriple *ut, int nu, int no, int nv, const double *eps_o,
                      const double *eps_v, const VecBatch &vb, long long tb, long long te, const LocalTerms &lt,
                      const OccTerm &ot, hipStream_t s) {
  if (nu <= 0 || nv <= 0 || vb.nvec <= 0 || g_dry) return;
  const int nt = (nv + TT - 1) / TT;
  LocalTerms l = lt;
  if (!l.L1) l.L1v = l.LVv = 0;
  const int nw = vb.tl ? vb.ntl : nu;  // triples visited
  if (nw <= 0) return;
  const dim3 grid((unsigned)((long long)vb.nvec * nw * nt * nt * nt));
  if (ot.nseg > 0 && ot.xs[0])
    hipLaunchKernelGGL(k_sym_denom<true>, grid, dim3(256), 0, s, W, Xu, ut, no, nv, eps_o, eps_v, vb, tb, te, l, ot,
                       nu);
  else
    hipLaunchKernelGGL(k_sym_denom<false>, grid, dim3(256), 0, s, W, Xu, ut, no, nv, eps_o, eps_v, vb, tb, te, l, ot,
                       nu);
}

__global__ void k_zero(double *dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = 0.0;
}

void launch_zero(double *dst, long long n, hipStream_t s) {
  if (n <= 0 || g_dry) return;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, n);
}

void launch_contra(const double *Xu, void *Xt, double *Xc, const UniqueTriple *ut, int nu, int no, int nv,
                   const VecBatch &vb, int contra_form, hipStream_t s, bool xt_f32) {
  if (nu <= 0 || nv <= 0 || vb.nvec <= 0 || g_dry) return;
  const int nt = (nv + TT - 1) / TT;
  const int sp0 = vb.p0, sp1 = vb.np > 0 ? vb.p0 + vb.np : no;
  const int nw = vb.tl ? vb.ntl : nu;  // triples visited
  if (nw <= 0) return;
  const dim3 grid((unsigned)((long long)vb.nvec * nw * nt * nt * nt));
  if (contra_form == 2 || (contra_form == 0 && (nv % TT == 0 || nv > 4 * TT))) {
    // one workgroup per orbit of tiles reads each sub-cube of X_u once (measured 2.3 -> 1.8 ms
    // per launch at n_v = 80, right + left transform 174.6 -> 168.3 ms at n_v = 136; at n_v = 60
    // the per-tile kernel is as fast, its neighbouring tiles share the partial lines of a row in
    // L2).  Ragged tiles are exact: a member tile loads zeros past n_v, a permuted read of an
    // output inside n_v stays inside n_v, and writes stop at n_v.
    const int norb = nt * (nt + 1) * (nt + 2) / 6;
    const dim3 og((unsigned)((long long)vb.nvec * nw * norb));
    if (xt_f32)
      hipLaunchKernelGGL(k_contra_orbit<float>, og, dim3(256), 0, s, Xu, (float *)Xt, ut, no, nv, nw, vb.nvec, vb.xu,
                         vb.xt, sp0, sp1, vb.tl);
    else
      hipLaunchKernelGGL(k_contra_orbit<double>, og, dim3(256), 0, s, Xu, (double *)Xt, ut, no, nv, nw, vb.nvec, vb.xu,
                         vb.xt, sp0, sp1, vb.tl);
  } else if (xt_f32) {
    hipLaunchKernelGGL(k_contra_scatter<float>, grid, dim3(256), 0, s, Xu, (float *)Xt, ut, no, nv, 0, nw, vb.nvec,
                       vb.xu, vb.xt, sp0, sp1, vb.tl);
  } else {
    hipLaunchKernelGGL(k_contra_scatter<double>, grid, dim3(256), 0, s, Xu, (double *)Xt, ut, no, nv, 0, nw, vb.nvec,
                       vb.xu, vb.xt, sp0, sp1, vb.tl);
  }
  if (Xc)
    hipLaunchKernelGGL(k_contra_scatter<double>, grid, dim3(256), 0, s, Xu, Xc, ut, no, nv, 1, nw, vb.nvec, vb.xu,
                       vb.w, sp0, sp1, vb.tl);
}

void launch_permute_denom(const double *W, double *Xu, void *Xt, double *Xc, const UniqueTriple *ut, int nu,
                          int no, int nv, const double *eps_o, const double *eps_v, const VecBatch &vb,
                          long long tb, long long te, const LocalTerms &lt, const OccTerm &ot, int contra_form,
                          hipStream_t s, bool xt_f32) {
  launch_sym_denom(W, Xu, ut, nu, no, nv, eps_o, eps_v, vb, tb, te, lt, ot, s);
  launch_contra(Xu, Xt, Xc, ut, nu, no, nv, vb, contra_form, s, xt_f32);
}

void launch_small_right(const void *X, const void *T, const double *gov, const double *F, const double *U,
                        int no, int nv, double *part1, double *Yvv, hipStream_t s, bool x_f32, int p0, int np,
                        bool yacc) {
  if (no <= 0 || nv <= 0 || g_dry) return;
  if (np <= 0) np = no;
  part1 += (long long)p0 * no * nv;  // rows of the slab (the blocks hold p - p0)
  Yvv += (long long)p0 * no * nv * nv;
  const int ya = yacc ? 1 : 0;
  if (x_f32) {  // one value of a per workgroup
    const dim3 grid((unsigned)(np * no * nv));
    if (T)
      hipLaunchKernelGGL((k_small_right<true, float, 1>), grid, dim3(256), 0, s, (const float *)X, (const float *)T,
                         gov, F, U, no, nv, part1, Yvv, ya);
    else
      hipLaunchKernelGGL((k_small_right<false, float, 1>), grid, dim3(256), 0, s, (const float *)X,
                         (const float *)nullptr, gov, F, U, no, nv, part1, Yvv, ya);
    return;
  }
  const dim3 grid((unsigned)(np * no * ((nv + 3) / 4)));  // four values of a per workgroup
  if (T)
    hipLaunchKernelGGL((k_small_right<true, double, 4>), grid, dim3(256), 0, s, (const double *)X, (const double *)T,
                       gov, F, U, no, nv, part1, Yvv, ya);
  else
    hipLaunchKernelGGL((k_small_right<false, double, 4>), grid, dim3(256), 0, s, (const double *)X,
                       (const double *)nullptr, gov, F, U, no, nv, part1, Yvv, ya);
}

void launch_vec_map(const double *A2, const double *B2, int no, int nv, int NO, int NV, int mode, double *oA,
                    double *oB, hipStream_t s) {
  L1D(k_vec_map, (long long)nv * NV * no * no + (long long)nv * nv * no * NO, A2, B2, no, nv, NO, NV, mode, oA, oB);
}

void launch_cvs_project(const double *x1, const double *x2a, const double *x2b, double *y1, double *y2a, double *y2b,
                        const unsigned char *core, int no, int nv, int NO, int NV, hipStream_t s) {
  const long long n = (long long)NV * NO + (long long)nv * NV * no * no + (long long)nv * nv * no * NO;
  L1D(k_cvs_project, n, x1, x2a, x2b, y1, y2a, y2b, core, no, nv, NO, NV);
}

void launch_occ_xT(const double *x, int no, int nv, int NO, double *xT, hipStream_t s) {
  L1D(k_occ_xT, (long long)no * nv * NO * occ_pitch(nv), x, no, nv, NO, xT);
}

__global__ void k_to_f32(const double *__restrict__ src, long long n, float *__restrict__ dst) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

void launch_to_f32(const double *src, long long n, float *dst, hipStream_t s) { L1D(k_to_f32, n, src, n, dst); }

__global__ void k_swap01(const double *__restrict__ src, int n, long long inner, double *__restrict__ dst) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)n * n * inner) return;
  const long long pq = i / inner, x = i - pq * inner;
  const int p = (int)(pq / n), q = (int)(pq - (long long)p * n);
  dst[((long long)q * n + p) * inner + x] = src[i];
}

void launch_swap01(const double *src, int n, long long inner, double *dst, hipStream_t s) {
  L1D(k_swap01, (long long)n * n * inner, src, n, inner, dst);
}

void launch_transpose(const double *in, double *out, int batch, int R, int C, hipStream_t s) {
  if (g_dry || batch <= 0 || R <= 0 || C <= 0) return;
  hipLaunchKernelGGL(k_transpose, dim3((C + 31) / 32, (R + 31) / 32, batch), dim3(256), 0, s, in, out, R, C);
}

void gram_kl_shape(int no, long long ne, int &nch, long long &chunk) {
  const int nij = no * no;
  nch = std::max(1, (3072 + nij - 1) / nij);
  chunk = (ne + nch - 1) / nch;
  chunk = (chunk + 63) / 64 * 64;
  nch = (int)((ne + chunk - 1) / chunk);
}

void launch_gram_kl(const double *X1, const double *X2, int no, long long ne, double *P, double alpha, double beta,
                    double *C, long long ldc, hipStream_t s) {
  if (g_dry || no <= 0 || ne <= 0) return;
  int nch;
  long long chunk;
  gram_kl_shape(no, ne, nch, chunk);
  const int nw = no * no * nch;
  hipLaunchKernelGGL(k_gram_kl, dim3((unsigned)nw), dim3(256), 0, s, X1, X2, no, ne, chunk, nch, P);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(no * no)), dim3(256), 0, s, P, nw, no, alpha, beta, C, ldc);
}

int gram_cd_chunks(long long nrows) {
  const long long nslab = (nrows + 15) / 16;
  return (int)std::max(1LL, std::min(512LL, nslab / 4));
}

void launch_gram_cd(const double *X1, const double *X2, int n, long long nrows, double *P, double alpha, double beta,
                    double *C, long long ldc, hipStream_t s) {
  if (g_dry || n <= 0 || nrows <= 0) return;
  const int nw = gram_cd_chunks(nrows);
  long long chunk = (nrows + nw - 1) / nw;
  chunk = (chunk + 15) / 16 * 16;
  const int nwu = (int)((nrows + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_gram_cd, dim3((unsigned)nwu), dim3(512), 0, s, X1, X2, n, nrows, chunk, P);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(n * n)), dim3(256), 0, s, P, nwu, n, alpha, beta, C, ldc);
}

void launch_sum_rows(const double *P, long long rows, long long n, double *out, hipStream_t s) {
  L1D(k_sum_rows, n, P, rows, n, out);
}

void launch_diag_sum(const double *Q, int no, int nv, int NO, double *V, hipStream_t s) {
  L1D(k_diag_sum, (long long)no * nv, Q, no, nv, NO, V);
}

void launch_left_Z(const double *Am, const double *Hp, int nc, int no, int nv, double *Z, hipStream_t s) {
  L1D(k_left_Z, (long long)nc * no * nv, Am, Hp, nc, no, nv, Z);
}

void launch_singles_out(const double *part1, int no, int nv, int NO, int NV, double *x1, hipStream_t s) {
  L1D(k_singles_out, (long long)NV * NO, part1, no, nv, NO, NV, x1);
}

void launch_doubles_out(const DoublesRaw &y, double *out_a, double *out_b, hipStream_t s) {
  const long long n = (long long)y.nv * y.NV * y.no * y.no + (long long)y.nv * y.nv * y.no * y.NO;
  L1D(k_doubles_out, n, y, out_a, out_b);
}

}  // namespace mlcc3
