/* FP64 CPU oracle for the MLCC3 triples hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no source, header or helper with the HIP path.
 *
 * The restricted occupied loop i>=j>=k over n_v^3 blocks (Implementation
 * section) written as plain loops.  All arrays are host pointers in the layouts
 * of the public C-ABI (occupied orbitals first, active orbitals first inside
 * each space; last index fastest):
 *   eps_o[N_O] eps_v[N_V] L_OO[nc][N_O][N_O] L_OV[nc][N_O][N_V] L_vV[nc][n_v][N_V]
 *   t1[N_V][N_O] t2_vVoo[n_v][N_V][n_o][n_o] t2_vvoO[n_v][n_v][n_o][N_O]
 *   vectors: x1[N_V][N_O], x2_vVoo, x2_vvoO as the t2 blocks.
 * Outputs are overwritten with the triples contribution summed over the unique
 * occupied triples with canonical index in [tb, te) (i>=j>=k, not all equal,
 * enumerated i outer, k inner).  te < 0 means "to the end".
 */
#ifndef MLCC3_ORACLE_H
#define MLCC3_ORACLE_H
#include <stdint.h>

typedef struct {
  int n_o, n_v, N_O, N_V, n_chol;
  const double *eps_o, *eps_v, *L_OO, *L_OV, *L_vV, *t1, *t2_vVoo, *t2_vvoO;
  /* core-valence separation (Implementation section, core excited states): NULL = off, else
   * N_O flags (nonzero = core orbital).  The right and left transforms then skip the unique
   * triples whose three occupied indices are all valence, and project their input and output
   * vectors onto the elements with at least one core occupied index. */
  const unsigned char *cvs_core;
} orc_problem;

int orc_num_threads(void);
int64_t orc_num_triples(int n_o);

int orc_ground_residual(const orc_problem *P, int64_t tb, int64_t te,
                        double *om1, double *om2_vVoo, double *om2_vvoO);
int orc_right_transform(const orc_problem *P, double omega, const double *R1,
                        const double *R2_vVoo, const double *R2_vvoO, int64_t tb, int64_t te,
                        double *rho1, double *rho2_vVoo, double *rho2_vvoO);
int orc_left_transform(const orc_problem *P, double omega, const double *L1,
                       const double *L2_vVoo, const double *L2_vvoO, int64_t tb, int64_t te,
                       double *sig1, double *sig2_vVoo, double *sig2_vvoO);
/* Triples terms of the transition densities for one excited state (SI left and right
 * density equations).  Dm0 and D0m are [N][N] (N = N_O + N_V, occupied first), element
 * [p][q] multiplies A_pq.  lam* is the ground-state multiplier vector (lambda3 from the L3
 * recipe at omega = 0), t2_vVoO[n_v][N_V][n_o][N_O] = t^{cD}_{kL} and
 * t2_vVOo[n_v][N_V][N_O][n_o] = t^{cD}_{Lk}.  *s = (1/6) sum lambda~3 R3; 2s is added to the
 * occupied diagonal of D0m.  Only unique triples in [tb, te) carry triples amplitudes. */
int orc_densities(const orc_problem *P, const double *t2_vVoO, const double *t2_vVOo, double omega,
                  const double *L1, const double *L2a, const double *L2b, const double *R1,
                  const double *R2a, const double *R2b, const double *l1, const double *l2a,
                  const double *l2b, int64_t tb, int64_t te, double *Dm0, double *D0m, double *s);
/* The covariant n_v^3 block X^{abc}_{ijk} of one unique triple (kind 0 = tau3,
 * 1 = R3, 2 = L3), for symmetry and closed-form checks. */
int orc_triples_block(const orc_problem *P, int kind, double omega, const double *x1,
                      const double *x2_vVoo, const double *x2_vvoO, int i, int j, int k,
                      double *out);
#endif
