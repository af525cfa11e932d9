/* FP64 CPU oracle for the MLCC3 triples hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, deterministic reference written from the paper (Paul, Folkestad,
 * Myhre, Koch: EOM oscillator strengths for MLCC3), Implementation section and
 * the Supporting Information equations.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; it shares nothing with the HIP path.
 *
 * Structure (Implementation section): the triples of one unique occupied triple
 * i>=j>=k are built as an n_v^3 block, X = -(eps^{abc}_{ijk} - omega)^{-1} P W,
 * where P sums the six simultaneous permutations of the pairs (ai),(bj),(ck)
 * (eq. tau3) and W is the doubles-times-integral term of eq. tau3 / eq. R3 /
 * the SI L3 equation.  The contravariant block X~ (virtual indices permuted at
 * fixed ijk; see DESIGN notes on eq. contra_3) is then contracted for every
 * distinct ordering (p,q,r) of (i,j,k), each ordering exactly once, which
 * reproduces the unrestricted sums over j,k of the SI.
 *
 * Readings where the text is silent or garbled (pinned by the brute-force,
 * finite-difference and adjoint tests):
 *  - T1 transform Lhat = (1-T) L (1+T); ghat_pqrs = sum_J Lhat^J_pq Lhat^J_rs;
 *  - F_kc = sum_LD (2 g_kcLD - g_kDLc) t^D_L (canonical HF reference);
 *  - Upsilon from dLhat = Lhat R - R Lhat (eqs. ups_v, ups_o);
 *  - Rbar = (1 + delta_{ai,bj}) R on the inputs, Delta^{-1} on rho_2 only;
 *  - L3 couples L^{aD}_{ij} g_Dbkc and L^{ab}_{iL} g_jLkc (exact transpose);
 *  - sigma^D_L: (2 g_kcLD - g_kDLc), minus on its 2nd and 3rd terms;
 *  - contravariant->covariant: X = (2 X~^{AB}_{IJ} + X~^{BA}_{IJ}) / 3.
 */
#include "mlcc3_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int no, nv, NO, NV, nc;
  const orc_problem *P;
  double *LhOO;  /* [nc][NO][NO]  Lhat_IK                         */
  double *Lh_vV; /* [nc][nv][NV]  Lhat_aB  (active virtual row)    */
  double *Lh_Vv; /* [nc][NV][nv]  Lhat_Db  (active virtual column) */
  double *Lh_vO; /* [nc][nv][NO]  Lhat_cK                          */
  double *G1;    /* [no][NV][nv][nv]  ghat_bDck   G1[k][D][b][c]   */
  double *Go;    /* [no][no][NO][nv]  ghat_Ljck   Go[j][k][L][c]   */
  double *gov;   /* [no][no][nv][nv]  g_jbkc      gov[j][k][b][c]  */
  double *gOL;   /* [no][no][nv][NO]  ghat_jLkc   gOL[j][k][c][L]  */
  double *gVb;   /* [no][nv][nv][NV]  ghat_Dbkc   gVb[k][b][c][D]  */
  double *gLb;   /* [no][nv][nv][NO]  g_Lbkc      gLb[k][b][c][L]  */
  double *F;     /* [no][nv]          F_kc                          */
  double *tD;    /* [no][no][nv][NV]  t^{aD}_{ij} tD[i][j][a][D]    */
  double *tL;    /* [no][nv][nv][NO]  t^{ab}_{iL} tL[i][a][b][L]    */
} ctx;

#define IDX4(a, b, c, d, nb, nc_, nd) ((((size_t)(a) * (nb) + (b)) * (nc_) + (c)) * (nd) + (d))

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

int orc_num_threads(void) { return omp_get_max_threads(); }

int64_t orc_num_triples(int n_o) {
  int64_t n = n_o;
  return n * (n + 1) * (n + 2) / 6 - n;
}

/* canonical unique triples i>=j>=k, not all equal; i outermost, k innermost */
static int64_t triple_list(int no, int *T) {
  int64_t t = 0;
  for (int i = 0; i < no; i++)
    for (int j = 0; j <= i; j++)
      for (int k = 0; k <= j; k++) {
        if (i == j && j == k) continue;
        T[3 * t] = i; T[3 * t + 1] = j; T[3 * t + 2] = k;
        t++;
      }
  return t;
}

static const int PERM[6][3] = {{0, 1, 2}, {1, 0, 2}, {2, 1, 0}, {0, 2, 1}, {2, 0, 1}, {1, 2, 0}};

/* ---------------------------------------------------------------- prep -- */
static void ctx_free(ctx *c) {
  free(c->LhOO); free(c->Lh_vV); free(c->Lh_Vv); free(c->Lh_vO);
  free(c->G1); free(c->Go); free(c->gov); free(c->gOL); free(c->gVb); free(c->gLb);
  free(c->F); free(c->tD); free(c->tL);
}

/* X_kc = sum_{LD} (2 g_kcLD - g_kDLc) x^D_L over the bare (ov|ov) integrals,
   evaluated as sum_J [2 L_kc (sum_LD L_LD x^D_L) - sum_D L_kD (sum_L L_Lc x^D_L)] */
static void ov_fock_like(const ctx *c, const double *x, double *out) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV, nc = c->nc;
  const double *LOV = c->P->L_OV;
  memset(out, 0, sizeof(double) * no * nv);
  double *sJ = zalloc(nc); /* s_J = sum_LD L_LD x^D_L */
#pragma omp parallel for schedule(static)
  for (int J = 0; J < nc; J++) {
    const double *Lov = LOV + (size_t)J * NO * NV;
    double s = 0.0;
    for (int L = 0; L < NO; L++)
      for (int D = 0; D < NV; D++) s += Lov[L * NV + D] * x[D * NO + L];
    sJ[J] = s;
  }
#pragma omp parallel for schedule(static)
  for (int cc = 0; cc < nv; cc++) {
    double *u = zalloc(NV); /* u_D = sum_L L_Lc x^D_L */
    for (int J = 0; J < nc; J++) {
      const double *Lov = LOV + (size_t)J * NO * NV;
      memset(u, 0, sizeof(double) * NV);
      for (int D = 0; D < NV; D++)
        for (int L = 0; L < NO; L++) u[D] += Lov[L * NV + cc] * x[D * NO + L];
      for (int k = 0; k < no; k++) {
        double e = 0.0;
        for (int D = 0; D < NV; D++) e += Lov[k * NV + D] * u[D];
        out[k * nv + cc] += 2.0 * Lov[k * NV + cc] * sJ[J] - e;
      }
    }
    free(u);
  }
  free(sJ);
}

static void ctx_init(ctx *c, const orc_problem *P) {
  const int no = P->n_o, nv = P->n_v, NO = P->N_O, NV = P->N_V, nc = P->n_chol;
  c->no = no; c->nv = nv; c->NO = NO; c->NV = NV; c->nc = nc; c->P = P;
  const double *LOO = P->L_OO, *LOV = P->L_OV, *LvV = P->L_vV, *t1 = P->t1;
  c->LhOO = zalloc((size_t)nc * NO * NO);
  c->Lh_vV = zalloc((size_t)nc * nv * NV);
  c->Lh_Vv = zalloc((size_t)nc * NV * nv);
  c->Lh_vO = zalloc((size_t)nc * nv * NO);
  /* T1 transformation Lhat = (1 - T) L (1 + T), T[V,O] = t1, blockwise */
#pragma omp parallel for schedule(static)
  for (int J = 0; J < nc; J++) {
    const double *Loo = LOO + (size_t)J * NO * NO, *Lov = LOV + (size_t)J * NO * NV,
                 *Lvv = LvV + (size_t)J * nv * NV;
    double *hOO = c->LhOO + (size_t)J * NO * NO;
    for (int I = 0; I < NO; I++)
      for (int K = 0; K < NO; K++) {
        double s = Loo[I * NO + K];
        for (int B = 0; B < NV; B++) s += Lov[I * NV + B] * t1[B * NO + K];
        hOO[I * NO + K] = s;
      }
    for (int a = 0; a < nv; a++)
      for (int B = 0; B < NV; B++) {
        double s = Lvv[a * NV + B];
        for (int I = 0; I < NO; I++) s -= t1[a * NO + I] * Lov[I * NV + B];
        c->Lh_vV[((size_t)J * nv + a) * NV + B] = s;
      }
    for (int D = 0; D < NV; D++)
      for (int b = 0; b < nv; b++) {
        double s = Lvv[b * NV + D]; /* L_Db = L_bD */
        for (int I = 0; I < NO; I++) s -= t1[D * NO + I] * Lov[I * NV + b];
        c->Lh_Vv[((size_t)J * NV + D) * nv + b] = s;
      }
    /* Lhat_cK = [(1 - T) M]_cK with M = L (1 + T): M_cK = L_cK + sum_B L_cB t_BK, and the
       occupied rows of M are M_IK = hOO[I][K] (formed above) */
    for (int cc = 0; cc < nv; cc++)
      for (int K = 0; K < NO; K++) {
        double s = Lov[K * NV + cc]; /* L_cK = L_Kc */
        for (int B = 0; B < NV; B++) s += Lvv[cc * NV + B] * t1[B * NO + K];
        for (int I = 0; I < NO; I++) s -= t1[cc * NO + I] * hOO[I * NO + K];
        c->Lh_vO[((size_t)J * nv + cc) * NO + K] = s;
      }
  }
  /* integral blocks, ghat_pqrs = sum_J Lhat^J_pq Lhat^J_rs */
  /* ghat_bDck and ghat_Ljck: accumulate over J with c innermost */
  c->G1 = zalloc((size_t)no * NV * nv * nv);
  c->Go = zalloc((size_t)no * no * NO * nv);
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < no; k++)
    for (int D = 0; D < NV; D++) {
      double *w = zalloc(nv);
      for (int J = 0; J < nc; J++) {
        for (int cc = 0; cc < nv; cc++) w[cc] = c->Lh_vO[((size_t)J * nv + cc) * NO + k];
        for (int b = 0; b < nv; b++) {
          const double f = c->Lh_vV[((size_t)J * nv + b) * NV + D];
          double *g = c->G1 + IDX4(k, D, b, 0, NV, nv, nv);
          for (int cc = 0; cc < nv; cc++) g[cc] += f * w[cc];
        }
      }
      free(w);
    }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < no; k++)
    for (int j = 0; j < no; j++) {
      double *w = zalloc(nv);
      for (int J = 0; J < nc; J++) {
        for (int cc = 0; cc < nv; cc++) w[cc] = c->Lh_vO[((size_t)J * nv + cc) * NO + k];
        for (int L = 0; L < NO; L++) {
          const double f = c->LhOO[((size_t)J * NO + L) * NO + j];
          double *g = c->Go + IDX4(j, k, L, 0, no, NO, nv);
          for (int cc = 0; cc < nv; cc++) g[cc] += f * w[cc];
        }
      }
      free(w);
    }
  c->gov = zalloc((size_t)no * no * nv * nv);
  c->gOL = zalloc((size_t)no * no * nv * NO);
#pragma omp parallel for collapse(2) schedule(static)
  for (int j = 0; j < no; j++)
    for (int k = 0; k < no; k++) {
      for (int b = 0; b < nv; b++)
        for (int cc = 0; cc < nv; cc++) {
          double s = 0.0;
          for (int J = 0; J < nc; J++)
            s += LOV[((size_t)J * NO + j) * NV + b] * LOV[((size_t)J * NO + k) * NV + cc];
          c->gov[IDX4(j, k, b, cc, no, nv, nv)] = s;
        }
      for (int cc = 0; cc < nv; cc++)
        for (int L = 0; L < NO; L++) {
          double s = 0.0;
          for (int J = 0; J < nc; J++)
            s += c->LhOO[((size_t)J * NO + j) * NO + L] * LOV[((size_t)J * NO + k) * NV + cc];
          c->gOL[IDX4(j, k, cc, L, no, nv, NO)] = s;
        }
    }
  /* ghat_Dbkc and g_Lbkc: accumulate over J with the full-space index innermost */
  c->gVb = zalloc((size_t)no * nv * nv * NV);
  c->gLb = zalloc((size_t)no * nv * nv * NO);
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < no; k++)
    for (int b = 0; b < nv; b++) {
      double *wD = zalloc(NV), *wL = zalloc(NO);
      for (int J = 0; J < nc; J++) {
        for (int D = 0; D < NV; D++) wD[D] = c->Lh_Vv[((size_t)J * NV + D) * nv + b];
        for (int L = 0; L < NO; L++) wL[L] = LOV[((size_t)J * NO + L) * NV + b];
        for (int cc = 0; cc < nv; cc++) {
          const double f = LOV[((size_t)J * NO + k) * NV + cc];
          double *g = c->gVb + IDX4(k, b, cc, 0, nv, nv, NV), *g2 = c->gLb + IDX4(k, b, cc, 0, nv, nv, NO);
          for (int D = 0; D < NV; D++) g[D] += f * wD[D];
          for (int L = 0; L < NO; L++) g2[L] += f * wL[L];
        }
      }
      free(wD); free(wL);
    }
  /* F_kc = sum_{LD} (2 g_kcLD - g_kDLc) t^D_L with bare (ov|ov) */
  c->F = zalloc((size_t)no * nv);
  ov_fock_like(c, t1, c->F);
  /* amplitudes repacked with the summation index last */
  c->tD = zalloc((size_t)no * no * nv * NV);
  c->tL = zalloc((size_t)no * nv * nv * NO);
  for (int a = 0; a < nv; a++)
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++)
          c->tD[IDX4(i, j, a, D, no, nv, NV)] = P->t2_vVoo[IDX4(a, D, i, j, NV, no, no)];
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int i = 0; i < no; i++)
        for (int L = 0; L < NO; L++)
          c->tL[IDX4(i, a, b, L, nv, nv, NO)] = P->t2_vvoO[IDX4(a, b, i, L, nv, no, NO)];
}

/* ------------------------------------------------------- vector prep -- */
typedef struct {
  double *xD, *xL;   /* Rbar repacked as tD/tL                          */
  double *U1, *Uo;   /* Upsilon_bDck [k][D][b][c], Upsilon_Ljck [j][k][L][c] */
  double *Ukc;       /* Upsilon_kc [k][c]                               */
  double *Xi;        /* sum_D g_jDkc R^D_L  as Xi[j][k][c][L]           */
} rvec;

static void rvec_free(rvec *v) { free(v->xD); free(v->xL); free(v->U1); free(v->Uo); free(v->Ukc); free(v->Xi); }

static void rvec_init(const ctx *c, rvec *v, const double *R1, const double *R2a, const double *R2b) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV, nc = c->nc;
  const double *LOV = c->P->L_OV;
  v->xD = zalloc((size_t)no * no * nv * NV);
  v->xL = zalloc((size_t)no * nv * nv * NO);
  for (int a = 0; a < nv; a++)
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) {
          double f = (a == D && i == j) ? 2.0 : 1.0; /* Rbar = (1 + delta_{ai,bj}) R */
          v->xD[IDX4(i, j, a, D, no, nv, NV)] = f * R2a[IDX4(a, D, i, j, NV, no, no)];
        }
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int i = 0; i < no; i++)
        for (int L = 0; L < NO; L++) {
          double f = (a == b && i == L) ? 2.0 : 1.0;
          v->xL[IDX4(i, a, b, L, nv, nv, NO)] = f * R2b[IDX4(a, b, i, L, nv, no, NO)];
        }
  /* one-index transformed Cholesky blocks, dLhat = Lhat R - R Lhat */
  double *dOO = zalloc((size_t)nc * NO * NO), *dvV = zalloc((size_t)nc * nv * NV),
         *dvO = zalloc((size_t)nc * nv * NO);
#pragma omp parallel for schedule(static)
  for (int J = 0; J < nc; J++) {
    const double *Lov = LOV + (size_t)J * NO * NV;
    for (int I = 0; I < NO; I++)
      for (int K = 0; K < NO; K++) {
        double s = 0.0;
        for (int A = 0; A < NV; A++) s += Lov[I * NV + A] * R1[A * NO + K];
        dOO[((size_t)J * NO + I) * NO + K] = s;
      }
    for (int a = 0; a < nv; a++)
      for (int B = 0; B < NV; B++) {
        double s = 0.0;
        for (int I = 0; I < NO; I++) s -= R1[a * NO + I] * Lov[I * NV + B];
        dvV[((size_t)J * nv + a) * NV + B] = s;
      }
    for (int cc = 0; cc < nv; cc++)
      for (int K = 0; K < NO; K++) {
        double s = 0.0;
        for (int B = 0; B < NV; B++) s += c->Lh_vV[((size_t)J * nv + cc) * NV + B] * R1[B * NO + K];
        for (int I = 0; I < NO; I++) s -= R1[cc * NO + I] * c->LhOO[((size_t)J * NO + I) * NO + K];
        dvO[((size_t)J * nv + cc) * NO + K] = s;
      }
  }
  /* Upsilon_bDck = sum_J (dL_bD Lh_ck + Lh_bD dL_ck), Upsilon_Ljck likewise */
  v->U1 = zalloc((size_t)no * NV * nv * nv);
  v->Uo = zalloc((size_t)no * no * NO * nv);
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < no; k++)
    for (int D = 0; D < NV; D++) {
      double *w = zalloc(nv), *dw = zalloc(nv);
      for (int J = 0; J < nc; J++) {
        for (int cc = 0; cc < nv; cc++) {
          w[cc] = c->Lh_vO[((size_t)J * nv + cc) * NO + k];
          dw[cc] = dvO[((size_t)J * nv + cc) * NO + k];
        }
        for (int b = 0; b < nv; b++) {
          const double f = dvV[((size_t)J * nv + b) * NV + D], h = c->Lh_vV[((size_t)J * nv + b) * NV + D];
          double *g = v->U1 + IDX4(k, D, b, 0, NV, nv, nv);
          for (int cc = 0; cc < nv; cc++) g[cc] += f * w[cc] + h * dw[cc];
        }
      }
      free(w); free(dw);
    }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < no; k++)
    for (int j = 0; j < no; j++) {
      double *w = zalloc(nv), *dw = zalloc(nv);
      for (int J = 0; J < nc; J++) {
        for (int cc = 0; cc < nv; cc++) {
          w[cc] = c->Lh_vO[((size_t)J * nv + cc) * NO + k];
          dw[cc] = dvO[((size_t)J * nv + cc) * NO + k];
        }
        for (int L = 0; L < NO; L++) {
          const double f = dOO[((size_t)J * NO + L) * NO + j], h = c->LhOO[((size_t)J * NO + L) * NO + j];
          double *g = v->Uo + IDX4(j, k, L, 0, no, NO, nv);
          for (int cc = 0; cc < nv; cc++) g[cc] += f * w[cc] + h * dw[cc];
        }
      }
      free(w); free(dw);
    }
  v->Ukc = zalloc((size_t)no * nv);
  ov_fock_like(c, R1, v->Ukc);
  /* Xi_jLkc = sum_D g_jDkc R^D_L with g_jDkc = sum_J L_jD L_kc (bare) */
  v->Xi = zalloc((size_t)no * no * nv * NO);
#pragma omp parallel for collapse(2) schedule(static)
  for (int j = 0; j < no; j++)
    for (int k = 0; k < no; k++) {
      double *g = zalloc(NV);
      for (int cc = 0; cc < nv; cc++) {
        memset(g, 0, NV * sizeof(double));
        for (int J = 0; J < nc; J++) {
          const double f = LOV[((size_t)J * NO + k) * NV + cc];
          const double *lj = LOV + ((size_t)J * NO + j) * NV;
          for (int D = 0; D < NV; D++) g[D] += lj[D] * f;
        }
        for (int L = 0; L < NO; L++) {
          double s = 0.0;
          for (int D = 0; D < NV; D++) s += g[D] * R1[D * NO + L];
          v->Xi[IDX4(j, k, cc, L, no, nv, NO)] = s;
        }
      }
      free(g);
    }
  free(dOO); free(dvV); free(dvO);
}

/* ------------------------------------------------------ triples block -- */
/* W[x][y][z] += sum_D xD[p][q][x][D] GD[r][D][y][z] - sum_L xL[p][x][y][L] GL[q][r][L][z] */
static void add_W(const ctx *c, int p, int q, int r, const double *xD, const double *xL,
                  const double *GD, const double *GL, double *W) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV;
  const size_t nv2 = (size_t)nv * nv;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < nv; x++) {
    double *Wx = W + (size_t)x * nv2;
    const double *xr = xD + IDX4(p, q, x, 0, no, nv, NV);
    for (int D = 0; D < NV; D++) {
      const double f = xr[D];
      const double *g = GD + IDX4(r, D, 0, 0, NV, nv, nv);
      for (size_t yz = 0; yz < nv2; yz++) Wx[yz] += f * g[yz];
    }
    for (int y = 0; y < nv; y++) {
      const double *xl = xL + IDX4(p, x, y, 0, nv, nv, NO);
      for (int L = 0; L < NO; L++) {
        const double f = xl[L];
        const double *g = GL + IDX4(q, r, L, 0, no, NO, nv);
        for (int z = 0; z < nv; z++) Wx[(size_t)y * nv + z] -= f * g[z];
      }
    }
  }
}

/* Z[x][y][z] += L^x_p g_qyrz + L^{xy}_{pq} F_rz  (the two local terms of the SI L3) */
static void add_Z_local(const ctx *c, int p, int q, int r, const double *L1, const double *L2a,
                        double *Z) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < nv; x++)
    for (int y = 0; y < nv; y++)
      for (int z = 0; z < nv; z++)
        Z[((size_t)x * nv + y) * nv + z] += L1[x * NO + p] * c->gov[IDX4(q, r, y, z, no, nv, nv)] +
                                            L2a[IDX4(x, y, p, q, NV, no, no)] * c->F[r * nv + z];
}

/* Z[x][y][z] += sum_D L^{xD}_{pq} g_Dyrz - sum_L L^{xy}_{pL} g_qLrz */
static void add_Z_contr(const ctx *c, int p, int q, int r, const double *lD, const double *lL,
                        double *Z) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < nv; x++)
    for (int y = 0; y < nv; y++)
      for (int z = 0; z < nv; z++) {
        double s = 0.0;
        const double *l = lD + IDX4(p, q, x, 0, no, nv, NV), *g = c->gVb + IDX4(r, y, z, 0, nv, nv, NV);
        for (int D = 0; D < NV; D++) s += l[D] * g[D];
        const double *l2 = lL + IDX4(p, x, y, 0, nv, nv, NO), *g2 = c->gOL + IDX4(q, r, z, 0, no, nv, NO);
        for (int L = 0; L < NO; L++) s -= l2[L] * g2[L];
        Z[((size_t)x * nv + y) * nv + z] += s;
      }
}

typedef struct {
  int kind;                     /* 0 tau3, 1 R3, 2 L3 */
  double omega;
  const rvec *rv;               /* R3 */
  const double *L1, *L2a;       /* L3 local terms */
  const double *lD, *lL;        /* L3 contractions (L2 repacked, no Delta) */
} bsrc;

/* covariant block X^{abc}_{ijk} = -(eps - omega)^{-1} sum_s W_{o.s}[v.s] */
static void build_block(const ctx *c, const bsrc *s, const int o[3], double *X, double *Wt) {
  const int nv = c->nv;
  const size_t n3 = (size_t)nv * nv * nv;
  memset(X, 0, n3 * sizeof(double));
  for (int ps = 0; ps < 6; ps++) {
    const int *S = PERM[ps];
    const int p = o[S[0]], q = o[S[1]], r = o[S[2]];
    memset(Wt, 0, n3 * sizeof(double));
    if (s->kind == 0) {
      add_W(c, p, q, r, c->tD, c->tL, c->G1, c->Go, Wt);
    } else if (s->kind == 1) {
      add_W(c, p, q, r, s->rv->xD, s->rv->xL, c->G1, c->Go, Wt);
      add_W(c, p, q, r, c->tD, c->tL, s->rv->U1, s->rv->Uo, Wt);
    } else {
      add_Z_local(c, p, q, r, s->L1, s->L2a, Wt);
      add_Z_contr(c, p, q, r, s->lD, s->lL, Wt);
    }
#pragma omp parallel for schedule(static)
    for (int v0 = 0; v0 < nv; v0++) {
      int v[3];
      v[0] = v0;
      for (v[1] = 0; v[1] < nv; v[1]++)
        for (v[2] = 0; v[2] < nv; v[2]++)
          X[((size_t)v[0] * nv + v[1]) * nv + v[2]] += Wt[((size_t)v[S[0]] * nv + v[S[1]]) * nv + v[S[2]]];
    }
  }
  const double *eo = c->P->eps_o, *ev = c->P->eps_v;
  const double eocc = eo[o[0]] + eo[o[1]] + eo[o[2]];
#pragma omp parallel for schedule(static)
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int cc = 0; cc < nv; cc++)
        X[((size_t)a * nv + b) * nv + cc] *= -1.0 / (ev[a] + ev[b] + ev[cc] - eocc - s->omega);
}

/* X~ = 4X - 2X^{bac} - 2X^{cba} - 2X^{acb} + X^{cab} + X^{bca} at fixed ijk */
static void contravariant(int nv, const double *X, double *Xt) {
#pragma omp parallel for schedule(static)
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int cc = 0; cc < nv; cc++) {
#define E(x, y, z) X[((size_t)(x) * nv + (y)) * nv + (z)]
        Xt[((size_t)a * nv + b) * nv + cc] = 4.0 * E(a, b, cc) - 2.0 * E(b, a, cc) - 2.0 * E(cc, b, a) -
                                             2.0 * E(a, cc, b) + E(cc, a, b) + E(b, cc, a);
#undef E
      }
}

/* block of the ordering (o[S0],o[S1],o[S2]): Y[w] = X[u] with u[S_n] = w_n */
static void reorder(int nv, const int S[3], const double *X, double *Y) {
#pragma omp parallel for schedule(static)
  for (int w0 = 0; w0 < nv; w0++) {
    int w[3], u[3];
    w[0] = w0;
    for (w[1] = 0; w[1] < nv; w[1]++)
      for (w[2] = 0; w[2] < nv; w[2]++) {
        u[S[0]] = w[0]; u[S[1]] = w[1]; u[S[2]] = w[2];
        Y[((size_t)w[0] * nv + w[1]) * nv + w[2]] = X[((size_t)u[0] * nv + u[1]) * nv + u[2]];
      }
  }
}

/* distinct orderings of a unique triple: returns count, fills perm ids */
static int orderings(const int o[3], int ids[6]) {
  int n = 0, seen[6][3];
  for (int ps = 0; ps < 6; ps++) {
    int p = o[PERM[ps][0]], q = o[PERM[ps][1]], r = o[PERM[ps][2]], dup = 0;
    for (int m = 0; m < n; m++)
      if (seen[m][0] == p && seen[m][1] == q && seen[m][2] == r) dup = 1;
    if (dup) continue;
    seen[n][0] = p; seen[n][1] = q; seen[n][2] = r;
    ids[n++] = ps;
  }
  return n;
}

/* CVS: is the unique triple o skipped (no core occupied index)? */
static int cvs_skip(const orc_problem *P, const int *o) {
  if (!P->cvs_core) return 0;
  return !(P->cvs_core[o[0]] || P->cvs_core[o[1]] || P->cvs_core[o[2]]);
}

/* CVS projection of a vector in place: singles x1[A][I] keep core I; doubles keep the elements
 * with a core index among the two occupied ones. */
static void cvs_project(const orc_problem *P, double *x1, double *x2a, double *x2b) {
  if (!P->cvs_core) return;
  const unsigned char *c = P->cvs_core;
  const int no = P->n_o, nv = P->n_v, NO = P->N_O, NV = P->N_V;
  for (int A = 0; A < NV; A++)
    for (int I = 0; I < NO; I++)
      if (!c[I]) x1[A * NO + I] = 0.0;
  for (int a = 0; a < nv; a++)
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++)
          if (!c[i] && !c[j]) x2a[(((size_t)a * NV + D) * no + i) * no + j] = 0.0;
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int i = 0; i < no; i++)
        for (int L = 0; L < NO; L++)
          if (!c[i] && !c[L]) x2b[(((size_t)a * nv + b) * no + i) * NO + L] = 0.0;
}

/* projected copies of a CVS input vector (plain copies when CVS is off) */
static void cvs_copy(const orc_problem *P, const double *x1, const double *x2a, const double *x2b, double **y1,
                     double **y2a, double **y2b) {
  const size_t n1 = (size_t)P->N_V * P->N_O, na = (size_t)P->n_v * P->N_V * P->n_o * P->n_o,
               nb = (size_t)P->n_v * P->n_v * P->n_o * P->N_O;
  *y1 = (double *)malloc(sizeof(double) * (n1 ? n1 : 1));
  *y2a = (double *)malloc(sizeof(double) * (na ? na : 1));
  *y2b = (double *)malloc(sizeof(double) * (nb ? nb : 1));
  memcpy(*y1, x1, sizeof(double) * n1);
  if (na) memcpy(*y2a, x2a, sizeof(double) * na);
  if (nb) memcpy(*y2b, x2b, sizeof(double) * nb);
  cvs_project(P, *y1, *y2a, *y2b);
}

static int range_ok(int64_t *tb, int64_t *te, int64_t nt) {
  if (*te < 0 || *te > nt) *te = nt;
  if (*tb < 0) *tb = 0;
  if (*tb > *te) *tb = *te;
  return 1;
}

/* --------------------------------------------- shared right/ground part -- */
/* rho1[x][p] += sum X~ g_qyrz ; Yvv(F)+ ; YvO- ; YvV+  (SI Omega / rho terms) */
static void contract_right(const ctx *c, int p, int q, int r, const double *Xt, double *rho1,
                           double *YvV, double *YvO, double *Ytmp) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV;
  const size_t nv2 = (size_t)nv * nv;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < nv; x++) {
    const double *X = Xt + (size_t)x * nv2;
    double s = 0.0;
    const double *g = c->gov + IDX4(q, r, 0, 0, no, nv, nv);
    for (size_t yz = 0; yz < nv2; yz++) s += X[yz] * g[yz];
    rho1[x * no + p] += s;
    for (int y = 0; y < nv; y++) {
      double f = 0.0;
      for (int z = 0; z < nv; z++) f += X[y * nv + z] * c->F[r * nv + z];
      YvV[IDX4(x, y, p, q, NV, no, no)] += f;
      for (int L = 0; L < NO; L++) {
        double sL = 0.0;
        for (int z = 0; z < nv; z++) sL += X[y * nv + z] * c->gOL[IDX4(q, r, z, L, no, nv, NO)];
        YvO[IDX4(x, y, p, L, nv, no, NO)] -= sL;
      }
    }
    double *yt = Ytmp + (size_t)x * NV;
    memset(yt, 0, NV * sizeof(double));
    for (size_t yz = 0; yz < nv2; yz++) {
      const double f = X[yz];
      const double *g2 = c->gVb + ((size_t)r * nv2 + yz) * NV;
      for (int D = 0; D < NV; D++) yt[D] += f * g2[D];
    }
    for (int D = 0; D < NV; D++) YvV[IDX4(x, D, p, q, NV, no, no)] += yt[D];
  }
}

/* covariant doubles from the raw blocks: X~ = Delta^-1 (Y + Y^T), X = (2X~ + X~^{BA}_{IJ})/3 */
static double Yfull(const ctx *c, const double *YvV, const double *YvO, int A, int B, int I, int J) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV;
  double s = 0.0;
  if (A < nv && I < no && J < no) s += YvV[IDX4(A, B, I, J, NV, no, no)];
  if (A < nv && B < nv && I < no) s += YvO[IDX4(A, B, I, J, nv, no, NO)];
  return s;
}
static double Xcontra(const ctx *c, const double *YvV, const double *YvO, int A, int B, int I, int J,
                      int with_delta) {
  double s = Yfull(c, YvV, YvO, A, B, I, J) + Yfull(c, YvV, YvO, B, A, J, I);
  if (with_delta && A == B && I == J) s *= 0.5;
  return s;
}
static double Xcov(const ctx *c, const double *YvV, const double *YvO, int A, int B, int I, int J, int wd) {
  return (2.0 * Xcontra(c, YvV, YvO, A, B, I, J, wd) + Xcontra(c, YvV, YvO, B, A, I, J, wd)) / 3.0;
}
static void write_doubles(const ctx *c, const double *YvV, const double *YvO, int wd, double *out_a,
                          double *out_b) {
  const int no = c->no, nv = c->nv, NO = c->NO, NV = c->NV;
#pragma omp parallel for schedule(static)
  for (int a = 0; a < nv; a++) {
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) out_a[IDX4(a, D, i, j, NV, no, no)] = Xcov(c, YvV, YvO, a, D, i, j, wd);
    for (int b = 0; b < nv; b++)
      for (int i = 0; i < no; i++)
        for (int L = 0; L < NO; L++) out_b[IDX4(a, b, i, L, nv, no, NO)] = Xcov(c, YvV, YvO, a, b, i, L, wd);
  }
}

/* ------------------------------------------------------------ entries -- */
int orc_ground_residual(const orc_problem *P, int64_t tb, int64_t te, double *om1, double *om2a,
                        double *om2b) {
  ctx c;
  ctx_init(&c, P);
  const int no = c.no, nv = c.nv, NO = c.NO, NV = c.NV;
  const size_t n3 = (size_t)nv * nv * nv;
  int64_t nt = orc_num_triples(no);
  range_ok(&tb, &te, nt);
  int *T = (int *)malloc(sizeof(int) * 3 * (nt + 1));
  triple_list(no, T);
  double *X = zalloc(n3), *Xt = zalloc(n3), *Xo = zalloc(n3), *Wt = zalloc(n3);
  double *rho = zalloc((size_t)nv * no), *YvV = zalloc((size_t)nv * NV * no * no),
         *YvO = zalloc((size_t)nv * nv * no * NO), *Ytmp = zalloc((size_t)nv * NV);
  bsrc s = {0};
  s.kind = 0;
  for (int64_t t = tb; t < te; t++) {
    const int o[3] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
    build_block(&c, &s, o, X, Wt);
    contravariant(nv, X, Xt);
    int ids[6], n = orderings(o, ids);
    for (int m = 0; m < n; m++) {
      const int *S = PERM[ids[m]];
      reorder(nv, S, Xt, Xo);
      contract_right(&c, o[S[0]], o[S[1]], o[S[2]], Xo, rho, YvV, YvO, Ytmp);
    }
  }
  memset(om1, 0, sizeof(double) * NV * NO);
  for (int a = 0; a < nv; a++)
    for (int i = 0; i < no; i++) om1[a * NO + i] = rho[a * no + i];
  write_doubles(&c, YvV, YvO, 0, om2a, om2b);
  free(T); free(X); free(Xt); free(Xo); free(Wt); free(rho); free(YvV); free(YvO); free(Ytmp);
  ctx_free(&c);
  return 0;
}

int orc_right_transform(const orc_problem *P, double omega, const double *R1, const double *R2a,
                        const double *R2b, int64_t tb, int64_t te, double *rho1, double *rho2a,
                        double *rho2b) {
  ctx c;
  ctx_init(&c, P);
  double *R1p, *R2ap, *R2bp;
  cvs_copy(P, R1, R2a, R2b, &R1p, &R2ap, &R2bp);
  R1 = R1p;
  R2a = R2ap;
  R2b = R2bp;
  rvec rv;
  rvec_init(&c, &rv, R1, R2a, R2b);
  const int no = c.no, nv = c.nv, NO = c.NO, NV = c.NV;
  const size_t n3 = (size_t)nv * nv * nv, nv2 = (size_t)nv * nv;
  int64_t nt = orc_num_triples(no);
  range_ok(&tb, &te, nt);
  int *T = (int *)malloc(sizeof(int) * 3 * (nt + 1));
  triple_list(no, T);
  double *X = zalloc(n3), *Rt = zalloc(n3), *Tt = zalloc(n3), *Ro = zalloc(n3), *To = zalloc(n3),
         *Wt = zalloc(n3);
  double *rho = zalloc((size_t)nv * no), *YvV = zalloc((size_t)nv * NV * no * no),
         *YvO = zalloc((size_t)nv * nv * no * NO), *Ytmp = zalloc((size_t)nv * NV),
         *Xtau = zalloc((size_t)no * no * nv * NO);
  bsrc st = {0}, sr = {0};
  st.kind = 0;
  sr.kind = 1; sr.omega = omega; sr.rv = &rv;
  for (int64_t t = tb; t < te; t++) {
    const int o[3] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
    if (cvs_skip(P, o)) continue;
    build_block(&c, &st, o, X, Wt);
    contravariant(nv, X, Tt);
    build_block(&c, &sr, o, X, Wt);
    contravariant(nv, X, Rt);
    int ids[6], n = orderings(o, ids);
    for (int m = 0; m < n; m++) {
      const int *S = PERM[ids[m]];
      const int p = o[S[0]], q = o[S[1]], r = o[S[2]];
      reorder(nv, S, Rt, Ro);
      reorder(nv, S, Tt, To);
      contract_right(&c, p, q, r, Ro, rho, YvV, YvO, Ytmp);
      /* tau~ terms: + tau~ Upsilon_kc ; - tau~ g_jDkc R^D_L ; Xtau = tau~ g_Lbkc */
#pragma omp parallel for schedule(static)
      for (int x = 0; x < nv; x++) {
        const double *Xx = To + (size_t)x * nv2;
        for (int y = 0; y < nv; y++) {
          double f = 0.0;
          for (int z = 0; z < nv; z++) f += Xx[y * nv + z] * rv.Ukc[r * nv + z];
          YvV[IDX4(x, y, p, q, NV, no, no)] += f;
          for (int L = 0; L < NO; L++) {
            double sL = 0.0;
            for (int z = 0; z < nv; z++) sL += Xx[y * nv + z] * rv.Xi[IDX4(q, r, z, L, no, nv, NO)];
            YvO[IDX4(x, y, p, L, nv, no, NO)] -= sL;
          }
        }
        for (int L = 0; L < NO; L++) {
          double sL = 0.0;
          for (size_t yz = 0; yz < nv2; yz++) sL += Xx[yz] * c.gLb[((size_t)r * nv2 + yz) * NO + L];
          Xtau[IDX4(p, q, x, L, no, nv, NO)] += sL;
        }
      }
    }
  }
  /* Y^{aD}_{ij} -= sum_L Xtau_ij[a][L] R^D_L */
#pragma omp parallel for schedule(static)
  for (int a = 0; a < nv; a++)
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) {
          double s = 0.0;
          for (int L = 0; L < NO; L++) s += Xtau[IDX4(i, j, a, L, no, nv, NO)] * R1[D * NO + L];
          YvV[IDX4(a, D, i, j, NV, no, no)] -= s;
        }
  memset(rho1, 0, sizeof(double) * NV * NO);
  for (int a = 0; a < nv; a++)
    for (int i = 0; i < no; i++) rho1[a * NO + i] = rho[a * no + i];
  write_doubles(&c, YvV, YvO, 1, rho2a, rho2b);
  cvs_project(P, rho1, rho2a, rho2b);
  free(T); free(X); free(Rt); free(Tt); free(Ro); free(To); free(Wt); free(rho); free(YvV); free(YvO);
  free(Ytmp); free(Xtau);
  free(R1p); free(R2ap); free(R2bp);
  rvec_free(&rv);
  ctx_free(&c);
  return 0;
}

int orc_left_transform(const orc_problem *P, double omega, const double *L1, const double *L2a,
                       const double *L2b, int64_t tb, int64_t te, double *sig1, double *sig2a,
                       double *sig2b) {
  ctx c;
  ctx_init(&c, P);
  double *L1p, *L2ap, *L2bp;
  cvs_copy(P, L1, L2a, L2b, &L1p, &L2ap, &L2bp);
  L1 = L1p;
  L2a = L2ap;
  L2b = L2bp;
  const int no = c.no, nv = c.nv, NO = c.NO, NV = c.NV, nc = c.nc;
  const size_t n3 = (size_t)nv * nv * nv, nv2 = (size_t)nv * nv;
  const double *LOV = P->L_OV;
  int64_t nt = orc_num_triples(no);
  range_ok(&tb, &te, nt);
  int *T = (int *)malloc(sizeof(int) * 3 * (nt + 1));
  triple_list(no, T);
  /* L2 repacked with the summation index last (plain, no Delta) */
  double *lD = zalloc((size_t)no * no * nv * NV), *lL = zalloc((size_t)no * nv * nv * NO);
  for (int a = 0; a < nv; a++)
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) lD[IDX4(i, j, a, D, no, nv, NV)] = L2a[IDX4(a, D, i, j, NV, no, no)];
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int i = 0; i < no; i++)
        for (int L = 0; L < NO; L++) lL[IDX4(i, a, b, L, nv, nv, NO)] = L2b[IDX4(a, b, i, L, nv, no, NO)];
  double *X = zalloc(n3), *Lt = zalloc(n3), *Tt = zalloc(n3), *Lo = zalloc(n3), *To = zalloc(n3),
         *Wt = zalloc(n3);
  double *QvV = zalloc((size_t)nv * NV * no * no), *QvO = zalloc((size_t)nv * nv * no * NO);
  double *Bq = zalloc((size_t)no * nv * nv * NV);        /* B_r[b][c][E] = sum L~ t^{aE}_{pq}  */
  double *Aq = zalloc((size_t)no * no * nv * NO);        /* A_qr[c][M] = sum L~ t^{ab}_{pM}    */
  double *V = zalloc((size_t)no * nv);                   /* V_kc = sum tau~ L^{ab}_{ij}        */
  double *Xtau = zalloc((size_t)no * no * nv * NO);      /* sum tau~ g_Lbkc                    */
  double *Qtau = zalloc((size_t)no * no * nv * NO);      /* Qtau_jk[c][L] = sum tau~ L^{ab}_{iL} */
  bsrc st = {0}, sl = {0};
  st.kind = 0;
  sl.kind = 2; sl.omega = omega; sl.L1 = L1; sl.L2a = L2a; sl.lD = lD; sl.lL = lL;
  for (int64_t t = tb; t < te; t++) {
    const int o[3] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
    if (cvs_skip(P, o)) continue;
    build_block(&c, &st, o, X, Wt);
    contravariant(nv, X, Tt);
    build_block(&c, &sl, o, X, Wt);
    contravariant(nv, X, Lt);
    int ids[6], n = orderings(o, ids);
    for (int m = 0; m < n; m++) {
      const int *S = PERM[ids[m]];
      const int p = o[S[0]], q = o[S[1]], r = o[S[2]];
      reorder(nv, S, Lt, Lo);
      reorder(nv, S, Tt, To);
      /* sigma^{aD}_{ij} += sum L~ g_bDck ; sigma^{ab}_{iL} -= sum L~ g_Ljck ; Xtau */
#pragma omp parallel for schedule(static)
      for (int x = 0; x < nv; x++) {
        const double *Xx = Lo + (size_t)x * nv2, *Tx = To + (size_t)x * nv2;
        for (int D = 0; D < NV; D++) {
          double s = 0.0;
          const double *g = c.G1 + IDX4(r, D, 0, 0, NV, nv, nv);
          for (size_t yz = 0; yz < nv2; yz++) s += Xx[yz] * g[yz];
          QvV[IDX4(x, D, p, q, NV, no, no)] += s;
        }
        for (int y = 0; y < nv; y++)
          for (int L = 0; L < NO; L++) {
            double s = 0.0;
            const double *g = c.Go + IDX4(q, r, L, 0, no, NO, nv);
            for (int z = 0; z < nv; z++) s += Xx[y * nv + z] * g[z];
            QvO[IDX4(x, y, p, L, nv, no, NO)] -= s;
          }
        for (int L = 0; L < NO; L++) {
          double s = 0.0;
          for (size_t yz = 0; yz < nv2; yz++) s += Tx[yz] * c.gLb[((size_t)r * nv2 + yz) * NO + L];
          Xtau[IDX4(p, q, x, L, no, nv, NO)] += s;
        }
      }
      /* B_r[y][z][E] += sum_x L~^{xyz}_{pqr} t^{xE}_{pq} */
#pragma omp parallel for schedule(static)
      for (int y = 0; y < nv; y++)
        for (int z = 0; z < nv; z++) {
          double *b = Bq + IDX4(r, y, z, 0, nv, nv, NV);
          for (int x = 0; x < nv; x++) {
            const double f = Lo[((size_t)x * nv + y) * nv + z];
            const double *tt = c.tD + IDX4(p, q, x, 0, no, nv, NV);
            for (int E = 0; E < NV; E++) b[E] += f * tt[E];
          }
        }
      /* A_qr[z][M] += sum_xy L~ t^{xy}_{pM};  V_rz += sum_xy tau~ L^{xy}_{pq};
         Qtau_qr[z][L] += sum_xy tau~ L^{xy}_{pL} */
#pragma omp parallel for schedule(static)
      for (int z = 0; z < nv; z++) {
        double *A = Aq + IDX4(q, r, z, 0, no, nv, NO), *Qt = Qtau + IDX4(q, r, z, 0, no, nv, NO);
        double vs = 0.0;
        for (int x = 0; x < nv; x++)
          for (int y = 0; y < nv; y++) {
            const double fl = Lo[((size_t)x * nv + y) * nv + z], ft = To[((size_t)x * nv + y) * nv + z];
            const double *tt = c.tL + IDX4(p, x, y, 0, nv, nv, NO), *ll = lL + IDX4(p, x, y, 0, nv, nv, NO);
            for (int M = 0; M < NO; M++) { A[M] += fl * tt[M]; Qt[M] += ft * ll[M]; }
            vs += ft * L2a[IDX4(x, y, p, q, NV, no, no)];
          }
        V[r * nv + z] += vs;
      }
    }
  }
  /* ---- singles: sigma1[D][L] -------------------------------------------- */
  memset(sig1, 0, sizeof(double) * NV * NO);
  /* sum_kc V_kc (2 g_kcLD - g_kDLc) is the same contraction as F_kc, transposed */
  for (int J = 0; J < nc; J++) {
    const double *Lov = LOV + (size_t)J * NO * NV;
    double a2 = 0.0;
    for (int k = 0; k < no; k++)
      for (int cc = 0; cc < nv; cc++) a2 += V[k * nv + cc] * Lov[k * NV + cc];
#pragma omp parallel for schedule(static)
    for (int L = 0; L < NO; L++) {
      double *u = zalloc(no), *w = zalloc(no);
      for (int k = 0; k < no; k++)
        for (int cc = 0; cc < nv; cc++) u[k] += V[k * nv + cc] * Lov[L * NV + cc]; /* sum_c V_kc L_Lc */
      for (int j = 0; j < no; j++)                                                 /* sum_kc L_kc Qtau_jk[c][L] */
        for (int k = 0; k < no; k++)
          for (int cc = 0; cc < nv; cc++) w[j] += Lov[k * NV + cc] * Qtau[IDX4(j, k, cc, L, no, nv, NO)];
      for (int D = 0; D < NV; D++) {
        double s = 2.0 * a2 * Lov[L * NV + D];
        for (int k = 0; k < no; k++) s -= Lov[k * NV + D] * u[k];
        for (int j = 0; j < no; j++) s -= Lov[j * NV + D] * w[j];
        sig1[D * NO + L] += s;
      }
      free(u); free(w);
    }
  }
  /* - sum_{ija} L^{aD}_{ij} Xtau_ij[a][L] */
#pragma omp parallel for schedule(static)
  for (int D = 0; D < NV; D++)
    for (int L = 0; L < NO; L++) {
      double s = 0.0;
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++)
          for (int a = 0; a < nv; a++) s -= L2a[IDX4(a, D, i, j, NV, no, no)] * Xtau[IDX4(i, j, a, L, no, nv, NO)];
      sig1[D * NO + L] += s;
    }
  /* sigma^D_l += sum B_l[b][c][E] g_bEcD - sum A_jl[c][M] g_MjcD - sum A_lk[c][M] g_MDck */
  double *H = zalloc((size_t)no * nc * nv), *H3 = zalloc((size_t)no * nc * NO);
#pragma omp parallel for collapse(2) schedule(static)
  for (int l = 0; l < no; l++)
    for (int J = 0; J < nc; J++) {
      for (int cc = 0; cc < nv; cc++) {
        double s = 0.0;
        for (int b = 0; b < nv; b++)
          for (int E = 0; E < NV; E++)
            s += Bq[IDX4(l, b, cc, E, nv, nv, NV)] * c.Lh_vV[((size_t)J * nv + b) * NV + E];
        for (int j = 0; j < no; j++)
          for (int M = 0; M < NO; M++)
            s -= Aq[IDX4(j, l, cc, M, no, nv, NO)] * c.LhOO[((size_t)J * NO + M) * NO + j];
        H[((size_t)l * nc + J) * nv + cc] = s;
      }
      for (int M = 0; M < NO; M++) {
        double s = 0.0;
        for (int k = 0; k < no; k++)
          for (int cc = 0; cc < nv; cc++)
            s += Aq[IDX4(l, k, cc, M, no, nv, NO)] * c.Lh_vO[((size_t)J * nv + cc) * NO + k];
        H3[((size_t)l * nc + J) * NO + M] = s;
      }
    }
#pragma omp parallel for schedule(static)
  for (int D = 0; D < NV; D++)
    for (int l = 0; l < no; l++) {
      double s = 0.0;
      for (int J = 0; J < nc; J++) {
        for (int cc = 0; cc < nv; cc++) s += H[((size_t)l * nc + J) * nv + cc] * c.Lh_vV[((size_t)J * nv + cc) * NV + D];
        for (int M = 0; M < NO; M++) s -= H3[((size_t)l * nc + J) * NO + M] * LOV[((size_t)J * NO + M) * NV + D];
      }
      sig1[D * NO + l] += s;
    }
  /* sigma^d_L += sum A_jk[d][M] g_MjLk - sum B_k[b][d][E] g_LkbE - sum B_k[d][c][E] g_LEck,
     with the L-independent factors sum_M A Lh_Mj, sum_bE B Lh_bE and sum_kc B Lh_ck first */
  double *Am = zalloc((size_t)nc * no * no * nv), *Hb = zalloc((size_t)nc * no * nv),
         *He = zalloc((size_t)nc * nv * NV);
#pragma omp parallel for schedule(static)
  for (int J = 0; J < nc; J++) {
    const double *hOO = c.LhOO + (size_t)J * NO * NO;
    for (int j = 0; j < no; j++)
      for (int k = 0; k < no; k++)
        for (int d = 0; d < nv; d++) {
          double s = 0.0;
          for (int M = 0; M < NO; M++) s += Aq[IDX4(j, k, d, M, no, nv, NO)] * hOO[M * NO + j];
          Am[IDX4(J, j, k, d, no, no, nv)] = s;
        }
    for (int k = 0; k < no; k++)
      for (int d = 0; d < nv; d++) {
        double s = 0.0;
        for (int b = 0; b < nv; b++)
          for (int E = 0; E < NV; E++) s += Bq[IDX4(k, b, d, E, nv, nv, NV)] * c.Lh_vV[((size_t)J * nv + b) * NV + E];
        Hb[((size_t)J * no + k) * nv + d] = s;
      }
    for (int d = 0; d < nv; d++) {
      double *he = He + ((size_t)J * nv + d) * NV;
      for (int k = 0; k < no; k++)
        for (int cc = 0; cc < nv; cc++) {
          const double f = c.Lh_vO[((size_t)J * nv + cc) * NO + k];
          const double *bb = Bq + IDX4(k, d, cc, 0, nv, nv, NV);
          for (int E = 0; E < NV; E++) he[E] += bb[E] * f;
        }
    }
  }
#pragma omp parallel for schedule(static)
  for (int d = 0; d < nv; d++)
    for (int L = 0; L < NO; L++) {
      double s = 0.0;
      for (int J = 0; J < nc; J++) {
        const double *hOO = c.LhOO + (size_t)J * NO * NO;
        for (int j = 0; j < no; j++)
          for (int k = 0; k < no; k++) s += Am[IDX4(J, j, k, d, no, no, nv)] * hOO[L * NO + k];
        for (int k = 0; k < no; k++) s -= hOO[L * NO + k] * Hb[((size_t)J * no + k) * nv + d];
        const double *he = He + ((size_t)J * nv + d) * NV, *lL = LOV + ((size_t)J * NO + L) * NV;
        for (int E = 0; E < NV; E++) s -= lL[E] * he[E];
      }
      sig1[d * NO + L] += s;
    }
  free(Am); free(Hb); free(He);
  write_doubles(&c, QvV, QvO, 0, sig2a, sig2b);
  cvs_project(P, sig1, sig2a, sig2b);
  free(L1p); free(L2ap); free(L2bp);
  free(T); free(lD); free(lL); free(X); free(Lt); free(Tt); free(Lo); free(To); free(Wt);
  free(QvV); free(QvO); free(Bq); free(Aq); free(V); free(Xtau); free(Qtau); free(H); free(H3);
  ctx_free(&c);
  return 0;
}

int orc_triples_block(const orc_problem *P, int kind, double omega, const double *x1,
                      const double *x2a, const double *x2b, int i, int j, int k, double *out) {
  if (kind < 0 || kind > 2) return -1;
  ctx c;
  ctx_init(&c, P);
  const int no = c.no, nv = c.nv, NO = c.NO, NV = c.NV;
  const size_t n3 = (size_t)nv * nv * nv;
  double *Wt = zalloc(n3);
  bsrc s = {0};
  s.kind = kind; s.omega = omega;
  rvec rv = {0};
  double *lD = NULL, *lL = NULL;
  if (kind == 1) {
    rvec_init(&c, &rv, x1, x2a, x2b);
    s.rv = &rv;
  } else if (kind == 2) {
    lD = zalloc((size_t)no * no * nv * NV);
    lL = zalloc((size_t)no * nv * nv * NO);
    for (int a = 0; a < nv; a++)
      for (int D = 0; D < NV; D++)
        for (int p = 0; p < no; p++)
          for (int q = 0; q < no; q++) lD[IDX4(p, q, a, D, no, nv, NV)] = x2a[IDX4(a, D, p, q, NV, no, no)];
    for (int a = 0; a < nv; a++)
      for (int b = 0; b < nv; b++)
        for (int p = 0; p < no; p++)
          for (int L = 0; L < NO; L++) lL[IDX4(p, a, b, L, nv, nv, NO)] = x2b[IDX4(a, b, p, L, nv, no, NO)];
    s.L1 = x1; s.L2a = x2a; s.lD = lD; s.lL = lL;
  }
  const int o[3] = {i, j, k};
  build_block(&c, &s, o, out, Wt);
  if (kind == 1) rvec_free(&rv);
  free(lD); free(lL); free(Wt);
  ctx_free(&c);
  return 0;
}

/* ------------------------------------------------------------ densities -- */
/* store the block X (of unique triple o) for every distinct ordering into Y[p][q][r][abc] */
static void store_orderings(const ctx *c, const int o[3], const double *X, double *Y, double *tmp) {
  const int no = c->no, nv = c->nv;
  const size_t n3 = (size_t)nv * nv * nv;
  int ids[6], n = orderings(o, ids);
  for (int m = 0; m < n; m++) {
    const int *S = PERM[ids[m]];
    reorder(nv, S, X, tmp);
    memcpy(Y + ((size_t)(o[S[0]] * no + o[S[1]]) * no + o[S[2]]) * n3, tmp, n3 * sizeof(double));
  }
}

int orc_densities(const orc_problem *P, const double *t2_vVoO, const double *t2_vVOo, double omega,
                  const double *L1, const double *L2a, const double *L2b, const double *R1,
                  const double *R2a, const double *R2b, const double *l1, const double *l2a,
                  const double *l2b, int64_t tb, int64_t te, double *Dm0, double *D0m, double *sout) {
  ctx c;
  ctx_init(&c, P);
  const int no = c.no, nv = c.nv, NO = c.NO, NV = c.NV, N = NO + NV;
  const size_t n3 = (size_t)nv * nv * nv, nord = (size_t)no * no * no;
  int64_t nt = orc_num_triples(no);
  range_ok(&tb, &te, nt);
  int *T = (int *)malloc(sizeof(int) * 3 * (nt + 1));
  triple_list(no, T);
  rvec rv;
  rvec_init(&c, &rv, R1, R2a, R2b);
  /* left vectors repacked (no Delta) for the L3 recipe */
  double *lDL = zalloc((size_t)no * no * nv * NV), *lLL = zalloc((size_t)no * nv * nv * NO);
  double *lDl = zalloc((size_t)no * no * nv * NV), *lLl = zalloc((size_t)no * nv * nv * NO);
  for (int a = 0; a < nv; a++)
    for (int D = 0; D < NV; D++)
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) {
          lDL[IDX4(i, j, a, D, no, nv, NV)] = L2a[IDX4(a, D, i, j, NV, no, no)];
          lDl[IDX4(i, j, a, D, no, nv, NV)] = l2a[IDX4(a, D, i, j, NV, no, no)];
        }
  for (int a = 0; a < nv; a++)
    for (int b = 0; b < nv; b++)
      for (int i = 0; i < no; i++)
        for (int L = 0; L < NO; L++) {
          lLL[IDX4(i, a, b, L, nv, nv, NO)] = L2b[IDX4(a, b, i, L, nv, no, NO)];
          lLl[IDX4(i, a, b, L, nv, nv, NO)] = l2b[IDX4(a, b, i, L, nv, no, NO)];
        }
  /* all-ordering storage of tau, tau~, L~, lambda~, R3, R3~ */
  double *Tau = zalloc(nord * n3), *TauT = zalloc(nord * n3), *Lt = zalloc(nord * n3),
         *Lam = zalloc(nord * n3), *R3 = zalloc(nord * n3), *R3t = zalloc(nord * n3);
  double *X = zalloc(n3), *Xt = zalloc(n3), *Wt = zalloc(n3), *tmp = zalloc(n3);
  bsrc st = {0}, sl = {0}, sa = {0}, sr = {0};
  st.kind = 0;
  sl.kind = 2; sl.omega = omega; sl.L1 = L1; sl.L2a = L2a; sl.lD = lDL; sl.lL = lLL;
  sa.kind = 2; sa.omega = 0.0; sa.L1 = l1; sa.L2a = l2a; sa.lD = lDl; sa.lL = lLl;
  sr.kind = 1; sr.omega = omega; sr.rv = &rv;
  for (int64_t t = tb; t < te; t++) {
    const int o[3] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
    build_block(&c, &st, o, X, Wt);
    store_orderings(&c, o, X, Tau, tmp);
    contravariant(nv, X, Xt);
    store_orderings(&c, o, Xt, TauT, tmp);
    build_block(&c, &sl, o, X, Wt);
    contravariant(nv, X, Xt);
    store_orderings(&c, o, Xt, Lt, tmp);
    build_block(&c, &sa, o, X, Wt);
    contravariant(nv, X, Xt);
    store_orderings(&c, o, Xt, Lam, tmp);
    build_block(&c, &sr, o, X, Wt);
    store_orderings(&c, o, X, R3, tmp);
    contravariant(nv, X, Xt);
    store_orderings(&c, o, Xt, R3t, tmp);
  }
#define BLK(A, p, q, r) ((A) + ((size_t)((p) * no + (q)) * no + (r)) * n3)
#define E3(x, y, z) (((size_t)(x) * nv + (y)) * nv + (z))
  const double *t2a = P->t2_vVoo, *t2b = P->t2_vvoO;
  /* amplitude accessors on the blocks */
#define TA(a, D, i, j) t2a[IDX4(a, D, i, j, NV, no, no)]            /* t^{aD}_{ij}   */
#define TB(a, b, i, L) t2b[IDX4(a, b, i, L, nv, no, NO)]            /* t^{ab}_{iL}   */
  memset(Dm0, 0, sizeof(double) * N * N);
  memset(D0m, 0, sizeof(double) * N * N);
  /* ---- D^{m-0} ---- */
  /* D_kl -= 1/2 sum L~^{abc}_{ijl} tau^{abc}_{ijk} ;  D_cd += 1/2 sum L~^{abc}_{ijk} tau^{abd}_{ijk} */
  for (int k = 0; k < no; k++)
    for (int l = 0; l < no; l++) {
      double acc = 0.0;
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) {
          const double *A = BLK(Lt, i, j, l), *B = BLK(Tau, i, j, k);
          for (size_t e = 0; e < n3; e++) acc += A[e] * B[e];
        }
      Dm0[k * N + l] -= 0.5 * acc;
    }
#pragma omp parallel for collapse(2) schedule(static)
  for (int cc = 0; cc < nv; cc++)
    for (int d = 0; d < nv; d++) {
      double acc = 0.0;
      for (size_t q = 0; q < nord; q++)
        for (int a = 0; a < nv; a++)
          for (int b = 0; b < nv; b++) acc += Lt[q * n3 + E3(a, b, cc)] * Tau[q * n3 + E3(a, b, d)];
      Dm0[(NO + cc) * N + NO + d] += 0.5 * acc;
    }
  /* D_ld += sum L^{ab}_{ij} tau~^{abd}_{ijl} */
  for (int l = 0; l < no; l++)
    for (int d = 0; d < nv; d++) {
      double acc = 0.0;
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++)
          for (int a = 0; a < nv; a++)
            for (int b = 0; b < nv; b++) acc += L2a[IDX4(a, b, i, j, NV, no, no)] * BLK(TauT, i, j, l)[E3(a, b, d)];
      Dm0[l * N + NO + d] += acc;
    }
  /* D_LD -= sum L~^{abc}_{ijk} t^{ac}_{iL} t^{bD}_{jk}, through V_jkbL = sum_{iac} L~ t^{ac}_{iL} */
  double *V = zalloc((size_t)no * no * nv * NO);
#pragma omp parallel for collapse(2) schedule(static)
  for (int j = 0; j < no; j++)
    for (int k = 0; k < no; k++)
      for (int b = 0; b < nv; b++)
        for (int L = 0; L < NO; L++) {
          double acc = 0.0;
          for (int i = 0; i < no; i++) {
            const double *A = BLK(Lt, i, j, k);
            for (int a = 0; a < nv; a++)
              for (int cc = 0; cc < nv; cc++) acc += A[E3(a, b, cc)] * TB(a, cc, i, L);
          }
          V[IDX4(j, k, b, L, no, nv, NO)] = acc;
        }
#pragma omp parallel for collapse(2) schedule(static)
  for (int L = 0; L < NO; L++)
    for (int D = 0; D < NV; D++) {
      double acc = 0.0;
      for (int j = 0; j < no; j++)
        for (int k = 0; k < no; k++)
          for (int b = 0; b < nv; b++) acc += V[IDX4(j, k, b, L, no, nv, NO)] * TA(b, D, j, k);
      Dm0[L * N + NO + D] -= acc;
    }
  /* ---- D^{0-m} ---- */
  /* X^{bc}_{jk} = sum_{ai} lambda~^{abc}_{ijk} R^a_i */
  double *Xl = zalloc((size_t)no * no * nv * nv);
  for (int j = 0; j < no; j++)
    for (int k = 0; k < no; k++)
      for (int b = 0; b < nv; b++)
        for (int cc = 0; cc < nv; cc++) {
          double acc = 0.0;
          for (int i = 0; i < no; i++)
            for (int a = 0; a < nv; a++) acc += BLK(Lam, i, j, k)[E3(a, b, cc)] * R1[a * NO + i];
          Xl[IDX4(j, k, b, cc, no, nv, nv)] = acc;
        }
  /* D_Kl -= sum lambda~^{abc}_{ijl} R^a_i t^{bc}_{jK} */
  for (int K = 0; K < NO; K++)
    for (int l = 0; l < no; l++) {
      double acc = 0.0;
      for (int j = 0; j < no; j++)
        for (int b = 0; b < nv; b++)
          for (int cc = 0; cc < nv; cc++) acc += Xl[IDX4(j, l, b, cc, no, nv, nv)] * TB(b, cc, j, K);
      D0m[K * N + l] -= acc;
    }
  /* D_kl -= 1/2 sum lambda~^{abc}_{ijl} R^{abc}_{ijk};  Z_kl = sum lambda~_{ijk} tau_{ijl} */
  double *Zt = zalloc((size_t)no * no);
  for (int k = 0; k < no; k++)
    for (int l = 0; l < no; l++) {
      double acc = 0.0, z = 0.0;
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++) {
          const double *A = BLK(Lam, i, j, l), *B = BLK(R3, i, j, k);
          const double *A2 = BLK(Lam, i, j, k), *B2 = BLK(Tau, i, j, l);
          for (size_t e = 0; e < n3; e++) { acc += A[e] * B[e]; z += A2[e] * B2[e]; }
        }
      D0m[k * N + l] -= 0.5 * acc;
      Zt[k * no + l] = z;
    }
  /* D_ld += sum X^{bc}_{jk} (tau^{bcd}_{jkl} - tau^{bcd}_{jlk}) + sum lambda^{ab}_{ij} R~^{abd}_{ijl}
     (the SI prints the doubles multipliers with a tilde; read as the plain lambda^{ab}_{ij}, the
     multiplier analog of the left density's L^{ab}_{ij} tau~^{abd}_{ijl}) */
  for (int l = 0; l < no; l++)
    for (int d = 0; d < nv; d++) {
      double acc = 0.0;
      for (int j = 0; j < no; j++)
        for (int k = 0; k < no; k++)
          for (int b = 0; b < nv; b++)
            for (int cc = 0; cc < nv; cc++)
              acc += Xl[IDX4(j, k, b, cc, no, nv, nv)] *
                     (BLK(Tau, j, k, l)[E3(b, cc, d)] - BLK(Tau, j, l, k)[E3(b, cc, d)]);
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++)
          for (int a = 0; a < nv; a++)
            for (int b = 0; b < nv; b++) {
              acc += l2a[IDX4(a, b, i, j, NV, no, no)] * BLK(R3t, i, j, l)[E3(a, b, d)];
            }
      D0m[l * N + NO + d] += acc;
    }
  /* Rbar accessors */
#define RBA(a, D, i, j) (((a) == (D) && (i) == (j) ? 2.0 : 1.0) * R2a[IDX4(a, D, i, j, NV, no, no)])
#define RBB(a, b, i, L) (((a) == (b) && (i) == (L) ? 2.0 : 1.0) * R2b[IDX4(a, b, i, L, nv, no, NO)])
  /* Y_kc = sum lambda~^{abc}_{ijk} Rbar^{ab}_{ij} */
  double *Yc = zalloc((size_t)no * nv);
  for (int k = 0; k < no; k++)
    for (int cc = 0; cc < nv; cc++) {
      double acc = 0.0;
      for (int i = 0; i < no; i++)
        for (int j = 0; j < no; j++)
          for (int a = 0; a < nv; a++)
            for (int b = 0; b < nv; b++) acc += BLK(Lam, i, j, k)[E3(a, b, cc)] * RBA(a, b, i, j);
      Yc[k * nv + cc] = acc;
    }
  /* D_LD += 1/2 sum Y_kc (2 t^{cD}_{kL} - t^{cD}_{Lk})
           - sum lambda~^{abc}_{ijk} (Rbar^{ac}_{iL} t^{bD}_{jk} + Rbar^{aD}_{ik} t^{bc}_{jL})
     D_lD -= 1/2 sum Z_kl R^D_k ;  D_Ld -= 1/2 sum Zv_cd R^c_L */
  double *Zv = zalloc((size_t)nv * nv);
#pragma omp parallel for collapse(2) schedule(static)
  for (int cc = 0; cc < nv; cc++)
    for (int d = 0; d < nv; d++) {
      double z = 0.0, r = 0.0;
      for (size_t q = 0; q < nord; q++)
        for (int a = 0; a < nv; a++)
          for (int b = 0; b < nv; b++) {
            z += Lam[q * n3 + E3(a, b, cc)] * Tau[q * n3 + E3(a, b, d)];
            r += Lam[q * n3 + E3(a, b, cc)] * R3[q * n3 + E3(a, b, d)];
          }
      Zv[cc * nv + d] = z;
      D0m[(NO + cc) * N + NO + d] += 0.5 * r;   /* D_cd += 1/2 sum lambda~^{abc} R^{abd} */
    }
  /* V2_jkbL = sum_{iac} lambda~^{abc}_{ijk} Rbar^{ac}_{iL};  V3_ikaL = sum_{jbc} lambda~^{abc}_{ijk} t^{bc}_{jL} */
  double *V2 = zalloc((size_t)no * no * nv * NO), *V3 = zalloc((size_t)no * no * nv * NO);
#pragma omp parallel for collapse(2) schedule(static)
  for (int p = 0; p < no; p++)
    for (int q = 0; q < no; q++)
      for (int x = 0; x < nv; x++)
        for (int L = 0; L < NO; L++) {
          double a2 = 0.0, a3 = 0.0;
          for (int r = 0; r < no; r++) {
            /* V2 with (j,k,b) = (p,q,x), i = r */
            const double *A = BLK(Lam, r, p, q);
            for (int a = 0; a < nv; a++)
              for (int cc = 0; cc < nv; cc++) a2 += A[E3(a, x, cc)] * RBB(a, cc, r, L);
            /* V3 with (i,k,a) = (p,q,x), j = r */
            const double *B = BLK(Lam, p, r, q);
            for (int b = 0; b < nv; b++)
              for (int cc = 0; cc < nv; cc++) a3 += B[E3(x, b, cc)] * TB(b, cc, r, L);
          }
          V2[IDX4(p, q, x, L, no, nv, NO)] = a2;
          V3[IDX4(p, q, x, L, no, nv, NO)] = a3;
        }
#pragma omp parallel for collapse(2) schedule(static)
  for (int L = 0; L < NO; L++)
    for (int D = 0; D < NV; D++) {
      double acc = 0.0;
      for (int k = 0; k < no; k++)
        for (int cc = 0; cc < nv; cc++)
          acc += 0.5 * Yc[k * nv + cc] *
                 (2.0 * t2_vVoO[IDX4(cc, D, k, L, NV, no, NO)] - t2_vVOo[IDX4(cc, D, L, k, NV, NO, no)]);
      for (int p = 0; p < no; p++)
        for (int q = 0; q < no; q++)
          for (int x = 0; x < nv; x++)
            acc -= V2[IDX4(p, q, x, L, no, nv, NO)] * TA(x, D, p, q) + V3[IDX4(p, q, x, L, no, nv, NO)] * RBA(x, D, p, q);
      if (L < no)
        for (int k = 0; k < no; k++) acc -= 0.5 * Zt[k * no + L] * R1[D * NO + k];
      if (D < nv)
        for (int cc = 0; cc < nv; cc++) acc -= 0.5 * Zv[cc * nv + D] * R1[cc * NO + L];
      D0m[L * N + NO + D] += acc;
    }
  /* D_ck += 1/2 Y_kc ;  D_cD += sum X^{bc}_{jk} t^{bD}_{jk} */
  for (int cc = 0; cc < nv; cc++) {
    for (int k = 0; k < no; k++) D0m[(NO + cc) * N + k] += 0.5 * Yc[k * nv + cc];
    for (int D = 0; D < NV; D++) {
      double acc = 0.0;
      for (int j = 0; j < no; j++)
        for (int k = 0; k < no; k++)
          for (int b = 0; b < nv; b++) acc += Xl[IDX4(j, k, b, cc, no, nv, nv)] * TA(b, D, j, k);
      D0m[(NO + cc) * N + NO + D] += acc;
    }
  }
  /* s = 1/6 sum lambda~ R3 ; D_LL += 2 s */
  double sdot = 0.0;
  for (size_t e = 0; e < nord * n3; e++) sdot += Lam[e] * R3[e];
  const double sv = sdot / 6.0;
  for (int L = 0; L < NO; L++) D0m[L * N + L] += 2.0 * sv;
  *sout = sv;
#undef BLK
#undef E3
#undef TA
#undef TB
#undef RBA
#undef RBB
  free(T); free(lDL); free(lLL); free(lDl); free(lLl);
  free(Tau); free(TauT); free(Lt); free(Lam); free(R3); free(R3t);
  free(X); free(Xt); free(Wt); free(tmp); free(Xl); free(Zt); free(Yc); free(Zv); free(V); free(V2); free(V3);
  rvec_free(&rv);
  ctx_free(&c);
  return 0;
}
