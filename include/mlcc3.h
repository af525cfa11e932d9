/* libmlcc3: MI355X (gfx950) implementation of the CC3 triples hot path of
 * equation-of-motion MLCC3 (Paul, Folkestad, Myhre, Koch: "Oscillator strengths
 * from equation-of-motion multilevel CC3", Implementation section and the
 * Supporting Information equations).
 *
 * The library computes, on one GPU, the triples contributions of the active
 * orbital space to
 *   - the ground-state residual Omega (SI: contributions to the contravariant
 *     ground-state residual; eq. tau3 for the triples amplitudes),
 *   - the right Jacobian transformation rho = J R (SI: Jacobian transformation
 *     of a trial vector R; eqs. R3, ups_v, ups_o),
 *   - the left (transpose) transformation sigma = L^T J (SI: transformation with
 *     the transpose of the Jacobian).
 * For every unique active occupied triple i>=j>=k the triples amplitudes are
 * built from the doubles and the T1-transformed Cholesky integrals, summed over
 * the six pair permutations P^{abc}_{ijk}, divided by the orbital-energy
 * denominators, converted to contravariant form and contracted back.
 *
 * Conventions (all arrays FP64, C row-major, last index fastest):
 *   orbitals: occupied (N_O) then virtual (N_V); the first n_o occupied and the
 *   first n_v virtual orbitals are active.  Capital indices run over the full
 *   spaces, lower-case ones over the active spaces.
 *   eps_o [N_O], eps_v [N_V]          orbital energies (canonical reference)
 *   L_OO  [n_chol][N_O][N_O]           bare MO Cholesky vectors, g_pqrs = sum_J L^J_pq L^J_rs,
 *   L_OV  [n_chol][N_O][N_V]           symmetric in pq (L_VO is the transpose of L_OV)
 *   L_vV  [n_chol][n_v][N_V]           active-virtual rows of the virtual-virtual block
 *   t1    [N_V][N_O]                   t^A_I
 *   t2_vVoo [n_v][N_V][n_o][n_o]       t^{aD}_{ij}   (two blocks of the symmetric doubles,
 *   t2_vvoO [n_v][n_v][n_o][N_O]       t^{ab}_{iL}    Implementation section after eq. tau3)
 *   vector blocks x1 [N_V][N_O], x2_vVoo, x2_vvoO as the t-blocks; inputs must be
 *   pair-symmetric (X^{AB}_{IJ} = X^{BA}_{JI}) and agree where the blocks overlap.
 *
 * Outputs are the triples contribution only (the caller adds its CCSD part) and
 * are overwritten.  Output doubles are covariant values of the full symmetric
 * doubles array on the two blocks; singles are [N_V][N_O] and zero outside the
 * active block.  The contravariant -> covariant map is
 * X^{AB}_{IJ} = (2 X~^{AB}_{IJ} + X~^{BA}_{IJ}) / 3 (Implementation section);
 * rho_2 additionally carries Delta^{-1}, Delta_{ai,bj} = 1 + delta_ij delta_ab (SI).
 *
 * Pointers in mlcc3_ground / mlcc3_vec / mlcc3_out are DEVICE pointers on the
 * device the workspace was created for; omega arrays are HOST arrays.  Every array must
 * hold at least the element count its layout and the sizes imply: the library checks
 * pointers for NULL but cannot see allocation sizes, and reads past a short array.  The
 * caller owns all buffers; the library never frees or retains them beyond the
 * call.  Work is enqueued on `stream` (a hipStream_t, NULL = default stream)
 * and the call returns after enqueue; outputs are valid once the stream has
 * synchronised.  Inputs are read-only; outputs must not alias inputs.  One
 * workspace must not be used by two calls at the same time.
 *
 * Return value: MLCC3_OK or a negative status (mlcc3_status_string).  No C++
 * exception crosses this interface and the library never aborts the process.
 */
#ifndef MLCC3_H
#define MLCC3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MLCC3_OK = 0,
  MLCC3_EINVAL = -1,       /* bad sizes, NULL pointers, nvec < 1, bad options          */
  MLCC3_ESINGULAR = -2,    /* |eps^{abc}_{ijk} - omega| < opts.guard for an active triple */
  MLCC3_ENOMEM = -3,       /* device allocation failed                                  */
  MLCC3_EHIP = -4,         /* HIP runtime error (text in mlcc3_status_string / last_error) */
  MLCC3_ENONFINITE = -5,   /* NaN/Inf found in an input (only with opts.check_finite)   */
  MLCC3_ESTATE = -6,       /* reuse_ground: the ground-state inputs changed since the workspace
                              prepared its blocks (no work enqueued)                      */
  MLCC3_EUNSUPPORTED = -7  /* requested precision or device not supported               */
};

/* Arithmetic of the O(N_V n_v^3 n_o^3) GEMMs of the Implementation section: the d-contractions
   that build the triples intermediates in every reduced form, and also the N_V-wide
   back-contractions of the contravariant triples (rho^{aD}_{ij}, sigma^{aD}_{ij},
   Omega^{aD}_{ij}: FP32 MFMA in the FP32 form; split-bf16 in the split-bf16 forms, which also
   run the left transform's Bq product so, the triples operand split while it is staged).  In the reduced forms
   of the ground residual and the right and left transforms, the contravariant triples blocks
   (tau~, R~, L~; formed in FP64) are stored in FP32 and widened to FP64 where they are read
   (about 6e-8 relative per element), and the occupied (N_O-sized) term of each intermediate,
   sum_L x^{ab}_{pL} G_{Lqrc}, runs as FP32 MFMA products on FP32 copies of its operands (FP32
   sums over the N_O values of L, added in FP64), and the N_O-wide back-contractions of the
   FP32 blocks run as FP32 MFMA products (FP32 sums over 16-deep K slabs, added in FP64); the
   densities keep all of these in FP64.  The permutations, denominators and every output stay
   FP64 in all forms.
   MLCC3_FP32:   FP32 MFMA on operands rounded to FP32, FP32 sums over 32-deep K slabs, FP64
                 across slabs (about 1e-7 relative).
   MLCC3_BF16X3: split-bf16 products (Henry, Tang and Heinecke, ARITH 2019): each operand is
                 hi + lo in bf16, products hi*hi + hi*lo + lo*hi in bf16 MFMA with FP32 sums
                 over 64-deep K steps, FP64 across steps (about 2^-16 = 1.5e-5 relative per
                 product; expected to miss 1e-6 on random-sign data).
   MLCC3_BF16X6: the same with a three-way split hi + mid + lo and the six products whose plane
                 indices sum to at most 2 (about 2^-24 relative per product). */
enum { MLCC3_FP64 = 0, MLCC3_FP32 = 1, MLCC3_BF16X3 = 2, MLCC3_BF16X6 = 3 };

typedef struct {
  int32_t n_o, n_v, N_O, N_V, n_chol; /* 0 <= n_o <= N_O, 0 <= n_v <= N_V, n_chol >= 1 */
  const double *eps_o, *eps_v;
  const double *L_OO, *L_OV, *L_vV;
  const double *t1, *t2_vVoo, *t2_vvoO;
} mlcc3_ground;

typedef struct { const double *x1, *x2_vVoo, *x2_vvoO; } mlcc3_vec;
typedef struct { double *x1, *x2_vVoo, *x2_vvoO; } mlcc3_out;

typedef struct {
  int32_t precision;      /* MLCC3_FP64 (default), MLCC3_FP32, MLCC3_BF16X3, MLCC3_BF16X6:
                             arithmetic of the d-contraction GEMMs and of the N_V-wide
                             back-contractions; in the reduced forms
                             also FP32 storage of the contravariant triples blocks and FP32
                             MFMA for the occupied term and the N_O-wide products (not in the
                             densities); denominators and accumulation stay FP64 */
  int32_t reuse_ground;   /* nonzero: the ground-state inputs (same pointers) are unchanged
                             since the last call on this workspace; reuse its prepared blocks.
                             The call checks that: a 64-bit fingerprint of the inputs' contents
                             (one read of them and one wait for the stream) must equal the one
                             taken when the blocks were prepared, else MLCC3_ESTATE */
  int64_t triple_begin;   /* half-open range over the canonical list of unique occupied     */
  int64_t triple_end;     /* triples (i>=j>=k, not all equal; i outer, k inner); end < 0 = all.
                             Outputs are the partial sums over that range.                 */
  double guard;           /* minimum |eps^{abc}_{ijk} - omega| (0 disables the check)       */
  int32_t check_finite;   /* nonzero: scan inputs for NaN/Inf first                          */
  const uint8_t *cvs_core; /* core-valence separation for core excited states (Implementation
                             section): NULL = off, else a HOST array of N_O flags (nonzero = core
                             orbital).  The right and left transforms then skip the unique
                             triples whose three occupied indices are all valence (tau3 terms
                             included) and project their input and output vectors onto the
                             elements with at least one core occupied index; the d-contraction
                             skips its all-valence tiles.  Needs n_o <= 64.  The ground residual
                             and the densities reject it (MLCC3_EINVAL). */
  int32_t reuse_tau;      /* nonzero (with reuse_ground): the ground residual and the right and
                             left transforms reuse the tau~ blocks (ground-state triples
                             amplitudes, contravariant, all ordered triples, kept in the
                             workspace) that an earlier call on this workspace formed for the same
                             ground state, triple range, core-valence setting and precision,
                             instead of forming them again (the tau3 d-contraction and
                             permutation passes are skipped; results are unchanged).  Any
                             preparation of a new ground state discards them. */
} mlcc3_opts;

typedef struct mlcc3_ws_s *mlcc3_ws;

/* Workspace: device scratch and the cached ground-state blocks, bound to `device`.  Every
 * compute entry point also accepts ws = NULL: the call then runs on a temporary workspace on
 * the current device, prepares the ground-state blocks itself (reuse_ground has no effect) and
 * waits for the device to finish before it returns and frees that workspace. */
int mlcc3_ws_create(mlcc3_ws *ws, int device);
int mlcc3_ws_destroy(mlcc3_ws ws);
/* Bytes of device memory currently held by the workspace. */
int64_t mlcc3_ws_bytes(mlcc3_ws ws);

/* Optional phase timer: when enabled, HIP events are recorded on the call's stream around
 * every d-contraction GEMM launch (phase 0: the W = sum_D x^{aD}_{ij} G_{bDck} GEMMs of
 * tau3, R3 and L3).  Enabling (or re-enabling) clears the recorded marks.
 * mlcc3_ws_phase_stats waits for the recorded events and returns the number of launches,
 * their summed device time in ms and the FLOPs executed by those launches. */
int mlcc3_ws_timing(mlcc3_ws ws, int32_t enable);
int mlcc3_ws_phase_stats(mlcc3_ws ws, int32_t phase, int64_t *launches, double *total_ms, double *flops);

/* Launch-shape choices of a workspace (the knobs an autotuner times; none changes what is
 * computed, only the launch shape, so results agree to rounding).  0 in a field = the
 * library's size-based default.
 *   dc_wg_per_cu: workgroups per CU of the persistent d-contraction grid (1..8), or -1 for one
 *                 workgroup per tile;
 *   back_ksplit:  K parts of the single-vector N_V-wide back-contraction GEMMs (1..8);
 *   narrow_tile:  block tile of the generic FP64 GEMM in the N_O-wide back-contractions,
 *                 10*TM + TN for a (32 TM) x (32 TN) tile, TM and TN in {1, 2, 4};
 *   contra_form:  contravariant pass: 1 = one workgroup per 16^3 sub-cube, 2 = one per orbit
 *                 of sub-cubes under the virtual permutations (any n_v); the default takes the
 *                 orbit pass when 16 divides n_v or n_v > 64;
 *   vec_group:    cap on the vectors that share one launch in the right and left transforms;
 *   occ_slab:     ground residual and right and left transforms in occupied slabs: the
 *                 ordered-triple buffers hold the triples whose first index p lies in a slab
 *                 of at most occ_slab values (the unique-triple blocks are accumulated slab by
 *                 slab, the back-contractions take the slab's rows or sum over slabs); 0 = the
 *                 whole occupied range in one slab when its buffers fit in the device memory,
 *                 else the widest slab that fits (results agree with the one-slab call to
 *                 rounding; the densities always use one slab).
 * mlcc3_ws_set_tuning(ws, NULL) restores the defaults; out-of-range values give MLCC3_EINVAL. */
typedef struct {
  int32_t dc_wg_per_cu, back_ksplit, narrow_tile, contra_form, vec_group, occ_slab;
} mlcc3_tuning;
int mlcc3_ws_set_tuning(mlcc3_ws ws, const mlcc3_tuning *t);
int mlcc3_ws_get_tuning(mlcc3_ws ws, mlcc3_tuning *t);

void mlcc3_opts_default(mlcc3_opts *o);

/* Number of unique active occupied triples i>=j>=k, not all equal: C(n_o+2,3) - n_o. */
int64_t mlcc3_num_triples(int32_t n_o);

/* Triples contribution to the ground-state residual (SI ground-state residual
 * equations): Omega^a_i = sum tau~ g_jbkc, Omega^{ab}_{ij} from P sum tau~ F_kc,
 * Omega^{ab}_{iL} = -P sum tau~ g_jLkc, Omega^{aD}_{ij} = P sum tau~ g_Dbkc. */
int mlcc3_ground_residual(mlcc3_ws ws, const mlcc3_ground *g, const mlcc3_opts *opts,
                          mlcc3_out *omega_T, void *stream);

/* The ground residual without any device allocation, for callers that cannot allocate (code
 * that runs under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same inputs, outputs and results as mlcc3_ground_residual with a fresh workspace (opts may
 * be NULL; reuse_ground and reuse_tau must be 0, there is no workspace to reuse), but every
 * intermediate lives in one fixed scratch array in device memory, linked into the library:
 * mlcc3_noalloc_scratch_bytes() bytes (128 MiB) on each device the call runs on, held until the
 * process ends.  The call first sizes the intermediates on the host without touching the
 * device; a problem that needs more scratch than that returns MLCC3_EINVAL (the text names the
 * bytes needed) with no work enqueued.  It never calls hipMalloc or hipFree.  Runs on the
 * current device.  All calls on one device share that device's scratch: calls that overlap in
 * time on one device (different streams or host threads) race and give wrong results; calls
 * ordered on one stream are safe.  The scratch keeps the previous call's contents; everything
 * the call reads from it is written first within the call.  Like the other entry points it
 * returns after enqueue, except that preparing the integral blocks waits for the stream once. */
int mlcc3_ground_residual_noalloc(const mlcc3_ground *g, const mlcc3_opts *opts, mlcc3_out *omega_T,
                                  void *stream);
int64_t mlcc3_noalloc_scratch_bytes(void);

/* Triples contribution to rho_m = J(omega_m) R_m for nvec trial vectors (eq. R3 and
 * the SI right-transformation terms).  R and rho are host arrays of nvec descriptors
 * holding device pointers; omega[nvec] is a host array. */
int mlcc3_right_transform(mlcc3_ws ws, const mlcc3_ground *g, int32_t nvec, const double *omega,
                          const mlcc3_vec *R, mlcc3_out *rho, const mlcc3_opts *opts, void *stream);

/* Triples contribution to sigma_m = L_m^T J(omega_m) (SI transpose transformation:
 * L3, sigma^D_L, sigma^D_l, sigma^d_L, sigma^{aD}_{ij}, sigma^{ab}_{iL}). */
int mlcc3_left_transform(mlcc3_ws ws, const mlcc3_ground *g, int32_t nvec, const double *omega,
                         const mlcc3_vec *L, mlcc3_out *sigma, const mlcc3_opts *opts, void *stream);

/* Triples terms of the transition densities of nstate excited states (SI left and right
 * density equations, Implementation section: occupied and virtual loops).
 *   D_m0[m][N][N]: left transition density D^{m-0} of state m from the left vector L[m]
 *                  (L3 at omega[m]) and tau3;
 *   D_0m[m][N][N]: right transition density D^{0-m} from R[m] (R3 at omega[m]), the
 *                  ground-state multipliers `lambda` (lambda3 from the L3 recipe at omega = 0)
 *                  and tau3; the doubles of R enter as Rbar = (1 + delta_{ai,bj}) R;
 *   s[m]         = (1/6) sum lambda~3 R3; 2 s[m] is already added to the occupied diagonal
 *                  of D_0m, the term -s D^{0-0} is left to the caller.
 * N = N_O + N_V, occupied orbitals first; element [p][q] multiplies A_pq.  D and s are
 * device arrays, overwritten.  t2_vVoO[n_v][N_V][n_o][N_O] = t^{cD}_{kL} and
 * t2_vVOo[n_v][N_V][N_O][n_o] = t^{cD}_{Lk} are the extra doubles blocks of the right
 * density (device).  With a triple range only the unique triples in the range carry
 * triples amplitudes (terms coupling two occupied triples are then not additive over
 * ranges). */
int mlcc3_triples_densities(mlcc3_ws ws, const mlcc3_ground *g, const double *t2_vVoO, const double *t2_vVOo,
                            int32_t nstate, const double *omega, const mlcc3_vec *L, const mlcc3_vec *R,
                            const mlcc3_vec *lambda, double *D_m0, double *D_0m, double *s,
                            const mlcc3_opts *opts, void *stream);

/* Transition moments and oscillator strengths from transition densities (Theory section: a
 * density contracted with a one-electron operator, sum_pq D_pq A_pq; the triples terms of the
 * densities come from mlcc3_triples_densities, the ground-state density D^{0-0} from the same
 * call with L = lambda and omega = 0).  For state m and operator component x (e.g. the three
 * dipole components):
 *   T_m0[m][x] = sum_pq D_m0[m][p][q] A[x][p][q]
 *   T_0m[m][x] = sum_pq (D_0m[m][p][q] - s[m] D_00[p][q]) A[x][p][q]
 *   f[m]       = (2/3) omega[m] sum_x T_0m[m][x] T_m0[m][x]
 * (the EOM-CC oscillator strength; the paper uses it without printing it).  The caller adds the
 * CCSD parts of the densities before the call when full moments are wanted.  A [ncomp][N][N],
 * D_m0 and D_0m [nstate][N][N], D_00 [N][N], s [nstate], outputs T_m0, T_0m [nstate][ncomp]
 * and f [nstate] are device arrays; omega [nstate] is a host array.  Returns after the stream
 * has finished the work. */
int mlcc3_oscillator_strengths(mlcc3_ws ws, int32_t N, int32_t ncomp, const double *A, int32_t nstate,
                               const double *omega, const double *D_m0, const double *D_0m, const double *D_00,
                               const double *s, double *T_m0, double *T_0m, double *f, void *stream);

/* Pairing maps of trial vectors, for gradients through the transforms.
 * The left and right vectors are paired by G(L, R) = sum L1 R1 + sum_{(AI)>=(BJ)} L~ R with
 * L~^{AB}_{IJ} = 2 L^{AB}_{IJ} - L^{BA}_{IJ} (the contravariant form of the doubles,
 * Implementation section; the left transform is the adjoint of the right one under G).  An
 * amplitude X^{AB}_{IJ} = X^{BA}_{JI} is stored at up to four positions of the two blocks.
 *   MLCC3_MAP_SYMMETRIZE:    out = the mean over the positions of each amplitude (makes any
 *                            block pair consistent and pair-symmetric);
 *   MLCC3_MAP_GRAD_TO_LEFT:  in = an elementwise (Euclidean) gradient g over the block arrays;
 *                            out = the left vector L with G(L, y) = <g, y> for every consistent y:
 *                            L = (2 s + s^{BA}_{IJ}) / 3, s = the sum of g over the positions;
 *   MLCC3_MAP_LEFT_TO_GRAD:  in = a consistent vector S; out = the elementwise representer h of
 *                            G(S, .) on consistent vectors, spread evenly over the positions:
 *                            h = (2 S - S^{BA}_{IJ}) / (number of positions).
 * With rho = J R (right transform of the symmetrised R), the gradient of a loss with elementwise
 * gradient g over rho is LEFT_TO_GRAD(sigma) with sigma the left transform of GRAD_TO_LEFT(g).
 * Singles are copied.  Only the dimensions of g are read; in/out are nvec device vectors,
 * outputs must not alias inputs.  Enqueued on stream. */
enum { MLCC3_MAP_SYMMETRIZE = 0, MLCC3_MAP_GRAD_TO_LEFT = 1, MLCC3_MAP_LEFT_TO_GRAD = 2 };
int mlcc3_vec_map(mlcc3_ws ws, const mlcc3_ground *g, int32_t mode, int32_t nvec, const mlcc3_vec *in,
                  mlcc3_out *out, void *stream);

/* Algorithmic FLOPs of one call (which: 0 ground residual, 1 right, 2 left) for nvec
 * vectors over the full triple list: U = 2 N_V n_v^3 (n_o^3 - n_o); ground 2U,
 * right/left (1 + 3 nvec) U (Implementation section cost model with the exact
 * number of ordered triples). */
double mlcc3_flops(const mlcc3_ground *g, int32_t which, int32_t nvec);

const char *mlcc3_status_string(int status);
/* Text of the last error on the calling thread ("" if none). */
const char *mlcc3_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLCC3_H */
