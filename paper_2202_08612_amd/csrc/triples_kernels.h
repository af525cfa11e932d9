// Launchers of the element-wise / reduction kernels of the triples path.
#pragma once
#include <hip/hip_runtime.h>

namespace mlcc3 {

// One unique active occupied triple i>=j>=k; mask bit s set when the pair
// permutation s gives an ordering not produced by an earlier s; canon is the index
// in the canonical list of triples that are not all equal (-1 for i=j=k).
struct UniqueTriple {
  int i, j, k, mask;
  long long canon;
};

// Extra local terms of the left triples (SI L3): L^a_i g_jbkc + L^{ab}_{ij} F_kc.
struct LocalTerms {
  const double *L1 = nullptr;   // [N_V][N_O]  (vector v at + v*L1v)
  const double *gov = nullptr;  // g_jbkc as [j][k][b][c]
  const double *LV = nullptr;   // L^{ab}_{ij} as [i][j][a][b]  (vector v at + v*LVv)
  long long L1v = 0, LVv = 0;
  const double *F = nullptr;    // F_kc as [k][c]
  int NO = 0;
};

// Occupied (N_O-sized) term of W, applied inside the permutation pass:
//   W[p][q][r][x][y][z] -= sum_seg sum_L x_seg(x, y, p, L) G_seg[L][q][r][z]
// with x stored transposed as xT[p][x][L][y] (launch_occ_xT) so that the MFMA operand
// loads run along y, and G stored [L][q][r][z].
struct OccTerm {
  const double *x[2] = {nullptr, nullptr};
  const double *G[2] = {nullptr, nullptr};
  long long xv[2] = {0, 0}, gv[2] = {0, 0};  // per-vector strides (0: shared by all vectors)
  int nseg = 0, NO = 0;
  // reduced-precision forms: FP32 copies of every segment's x and G (same layouts, per-vector
  // strides xsv/gsv); when set, the term is formed from them with FP32 MFMA products (FP32 sums
  // over the N_O values of L of one segment, added into the FP64 sub-cube)
  const float *xs[2] = {nullptr, nullptr};
  const float *Gs[2] = {nullptr, nullptr};
  long long xsv[2] = {0, 0}, gsv[2] = {0, 0};
};

// Raw (pre-symmetrisation) doubles blocks; delta=1 applies Delta^{-1}.
struct DoublesRaw {
  const double *YvV = nullptr;  // [i][j][a][D]
  const double *YvO = nullptr;  // [i][a][b][L]
  const double *Yvv = nullptr;  // [i][j][a][b]
  int no = 0, nv = 0, NO = 0, NV = 0, delta = 0;
};

// dst[r][k] = src[r*ld + k] for k < nk (packs the first nk columns of each row)
void launch_pack_cols(const double *src, long long rows, int ld, int nk, double *dst, hipStream_t s);
// C[k][D][b][c] = T[(b*NV + D)][(c*no + k)]
void launch_vvvo_permute(const double *T, int no, int nv, int NV, double *C, hipStream_t s);
// LhvO[J][c][K] = L_OV[J][K][c] (first term of the T1-transformed vO block)
void launch_lhat_vO_init(const double *LOV, int nc, int NO, int NV, int nv, double *LhvO, hipStream_t s);
// s_J = sum_LD L^J_LD x^D_L
// s_J = sum_LD L^J_LD x^D_L (x as [N_V][N_O]; tmp_xT holds its [N_O][N_V] transpose)
void launch_fock_s(const double *LOV, const double *x, int nc, int NO, int NV, double *tmp_xT, double *tmp_s,
                   hipStream_t s);
// X_kc = sum_J (2 L^J_kc s_J - sum_L y^J_kL L^J_Lc) (fixed order over J)
void launch_fock_finish(const double *LOV, const double *tmp_s, const double *tmp_y, int nc, int NO, int NV, int no,
                        int nv, double *tmp_z, double *out, hipStream_t s);
void launch_pack_vVoo(const double *x, int no, int nv, int NV, int rbar, double *xA, hipStream_t s);
void launch_rbar_vvoO(const double *x, int no, int nv, int NO, double *xB, hipStream_t s);
void launch_pack_vvoo(const double *x, int no, int nv, int NV, int mode, double *xV, hipStream_t s);
// out[0] = scale * sum a[i] b[i]; part holds 512 doubles of scratch
void launch_dot(const double *a, const double *b, long long n, double scale, double *part, double *out,
                hipStream_t s);
void launch_add_diag(double *D, int NO, int N, const double *sv, double f, hipStream_t s);
// transition moments and oscillator strengths (om: device omegas)
void launch_strengths(const double *A, int N, int ncomp, int nstate, const double *Dm0, const double *D0m,
                      const double *D00, const double *sv, const double *om, double *Tm0, double *T0m, double *f,
                      hipStream_t s);
void launch_add_vo(double *D, int NO, int N, int no, int nv, const double *Y, double f, hipStream_t s);
// Several trial vectors in one launch: vector v < nvec reads W + v*w, writes Xu + v*xu,
// Xt + v*xt (Xc likewise) and uses omega[v].
constexpr int kMaxVecBatch = 32;
// cvs != 0: core-valence separation, unique triples without a core occupied index (bit of
// core_bits) are skipped.
struct VecBatch {
  int nvec = 1;
  long long w = 0, xu = 0, xt = 0;
  double omega[kMaxVecBatch] = {0.0};
  int cvs = 0;
  unsigned long long core_bits = 0;
  // occupied slab (np > 0): the ordered blocks in W and Xt are those with first index
  // p0 <= p < p0 + np, stored at [p - p0][q][r]; the symmetrisation adds the slab's orderings
  // into Xu (writes them when p0 == 0) and the contravariant pass writes the slab's orderings
  int p0 = 0, np = 0;
  // the unique triples the passes visit: tl[0..ntl) (indices into the triple list), NULL = all
  // (a slab's passes visit only the triples with an index in the slab)
  const int *tl = nullptr;
  int ntl = 0;
};

// W -> Xu (covariant unique-triple blocks [u][a][b][c], rows of pitch occ_pitch(n_v)) -> Xt
// (contravariant, all orderings)
// (and, if Xc is not NULL, the covariant X to every ordering); contravariant pass per
// sub-cube (contra_form 1), per orbit of sub-cubes (2), or by the size rule (0: per orbit
// when 16 divides n_v or n_v > 64)
// (xt_f32: Xt holds float elements; the covariant copy Xc is always double)
// launch_sym_denom and launch_contra are its two passes on their own (for occupied slabs)
void launch_sym_denom(const double *W, double *Xu, const UniqueTriple *ut, int nu, int no, int nv, const double *eps_o,
                      const double *eps_v, const VecBatch &vb, long long tb, long long te, const LocalTerms &lt,
                      const OccTerm &ot, hipStream_t s);
void launch_contra(const double *Xu, void *Xt, double *Xc, const UniqueTriple *ut, int nu, int no, int nv,
                   const VecBatch &vb, int contra_form, hipStream_t s, bool xt_f32);
// dst[0..n) = 0
void launch_zero(double *dst, long long n, hipStream_t s);
void launch_permute_denom(const double *W, double *Xu, void *Xt, double *Xc, const UniqueTriple *ut, int nu,
                          int no, int nv, const double *eps_o, const double *eps_v, const VecBatch &vb,
                          long long tb, long long te, const LocalTerms &lt, const OccTerm &ot, int contra_form,
                          hipStream_t s, bool xt_f32 = false);
// X, T: ordered blocks of double, or of float when x_f32; with np > 0 the blocks hold the
// occupied slab p0 <= p < p0 + np ([p - p0][q][r]) and the outputs are written for its rows
// (part1 + p0 n_o n_v, Yvv + p0 n_o n_v^2); yacc adds into Yvv instead of writing it
void launch_small_right(const void *X, const void *T, const double *gov, const double *F, const double *U,
                        int no, int nv, double *part1, double *Yvv, hipStream_t s, bool x_f32 = false, int p0 = 0,
                        int np = 0, bool yacc = false);
// pairing maps of the doubles blocks (mode 0 symmetrise, 1 gradient -> left vector, 2 left
// vector -> gradient representer); outputs must not alias inputs
void launch_vec_map(const double *A2, const double *B2, int no, int nv, int NO, int NV, int mode, double *oA,
                    double *oB, hipStream_t s);
// CVS projection y = P x of a vector (may be in place): singles keep core I, doubles keep the
// elements with a core occupied index; core: device flags [N_O]
void launch_cvs_project(const double *x1, const double *x2a, const double *x2b, double *y1, double *y2a, double *y2b,
                        const unsigned char *core, int no, int nv, int NO, int NV, hipStream_t s);
// xT[p][a][L][b] = x[a][b][p][L]  (x: [n_v][n_v][n_o][N_O]); the b rows have the pitch
// occ_pitch(n_v) (padding zero), so that the 16-wide segments the MFMA operand loads read
// are whole 128-byte lines
__host__ __device__ inline int occ_pitch(int nv) { return (nv + 15) / 16 * 16; }
void launch_occ_xT(const double *x, int no, int nv, int NO, double *xT, hipStream_t s);
// dst[i] = FP32 of src[i] (rounded to nearest), i < n
void launch_to_f32(const double *src, long long n, float *dst, hipStream_t s);
// dst[q][p][x] = src[p][q][x] (p, q < n, x < inner); dst must not alias src
void launch_swap01(const double *src, int n, long long inner, double *dst, hipStream_t s);
// out[z][c][r] = in[z][r][c], z < batch
void launch_transpose(const double *in, double *out, int batch, int R, int C, hipStream_t s);
// out[i] = sum_r P[r][i], r = 0..rows-1 (fixed order)
// C[k][l] = alpha sum_{(i,j),e} X1[i][j][k][e] X2[i][j][l][e] + beta C[k][l] for ordered-triple
// buffers with ne = n_v^3 values per triple, n_o <= 16; P holds the per-workgroup partials
// (gram_kl_shape gives their count: no * no * nch blocks of no * no doubles)
void gram_kl_shape(int no, long long ne, int &nch, long long &chunk);
void launch_gram_kl(const double *X1, const double *X2, int no, long long ne, double *P, double alpha, double beta,
                    double *C, long long ldc, hipStream_t s);
// C[c][d] = alpha sum_k X1[k][c] X2[k][d] + beta C[c][d] over nrows rows of n contiguous values,
// for 64 < n <= 160; P holds gram_cd_chunks(nrows) partial n x n blocks
int gram_cd_chunks(long long nrows);
void launch_gram_cd(const double *X1, const double *X2, int n, long long nrows, double *P, double alpha, double beta,
                    double *C, long long ldc, hipStream_t s);
void launch_sum_rows(const double *P, long long rows, long long n, double *out, hipStream_t s);
void launch_diag_sum(const double *Q, int no, int nv, int NO, double *V, hipStream_t s);
void launch_left_Z(const double *Am, const double *Hp, int nc, int no, int nv, double *Z, hipStream_t s);
void launch_singles_out(const double *part1, int no, int nv, int NO, int NV, double *x1, hipStream_t s);
void launch_doubles_out(const DoublesRaw &y, double *out_a, double *out_b, hipStream_t s);

}  // namespace mlcc3
