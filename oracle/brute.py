"""Brute-force FP64 reference for the MLCC3 triples terms (TEST INFRASTRUCTURE).

Part of the oracle: only tests, the smoke check and the benchmark's CPU
baseline may import it.  It shares no code with the HIP path.

Every triples quantity is stored for *all* (A,B,C,I,J,K) of the full orbital
space and multiplied by the active mask M = [A,B,C < n_v][I,J,K < n_o]
(two-level MLCC3 cluster operator, Theory section, eq. T_op: T3 acts in the
active space only, summation indices run over the full space, Implementation
section after eq. tau3).  Each formula is then one full-range einsum, written
in the paper's index order, with no restricted loop, no blocking and no
reuse of intermediates between different outputs.  Mask = 1 is full CC3,
mask = 0 is CCSD.  Only tiny sizes are practical (memory ~ (N_V N_O)^3).

Conventions (readings where the text is silent or garbled):
* orbitals: occupied [0,N_O) then virtual [N_O,N); active = first n_o / n_v;
* T1 transform: Lhat = (1-T) L (1+T), T[N_O+A, I] = t^A_I (Theory: T1-transformed
  Hamiltonian); ghat_pqrs = sum_J Lhat^J_pq Lhat^J_rs (SI, Cholesky paragraph);
* F_kc = sum_{LD} (2 g_kcLD - g_kDLc) t^D_L with F(0) = diag(eps) (canonical HF);
* Upsilon = d ghat / d t1 along R1, i.e. dLhat = Lhat R - R Lhat (eqs. ups_v,
  ups_o; SI Upsilon_kc);
* P^{abc}_{ijk}: all 6 simultaneous permutations of the pairs (ai),(bj),(ck)
  (eq. tau3);
* contravariant triples: 4X - 2X^{bac} - 2X^{cba} - 2X^{acb} + X^{cab} + X^{bca},
  virtual indices permuted at fixed ijk (eq. contra_3 as printed permutes whole
  pairs, which would vanish identically for pair-symmetric X);
* L3 uses the exact transpose of the right-transform couplings
  (sum_D L^{aD}_{ij} g_Dbkc - sum_L L^{ab}_{iL} g_jLkc);
* sigma^D_L uses (2 g_kcLD - g_kDLc) and minus signs on its 2nd/3rd terms;
* rho^{ab}_{iL} second term uses the contravariant tau~.
"""
from __future__ import annotations

import numpy as np

PAIR_PERMS = ("abcijk", "bacjik", "cbakji", "acbikj", "cabkij", "bcajki")


def _perm(X, labels):
    return np.einsum(labels + "->abcijk", X)


def P3(X):
    """Sum over the six simultaneous pair permutations (eq. tau3)."""
    return sum(_perm(X, p) for p in PAIR_PERMS)


def tilde3(X):
    """Contravariant triples, virtual permutations at fixed occupied indices."""
    return (4.0 * X - 2.0 * _perm(X, "bacijk") - 2.0 * _perm(X, "cbaijk")
            - 2.0 * _perm(X, "acbijk") + _perm(X, "cabijk") + _perm(X, "bcaijk"))


def transpose_pairs2(X):
    """X^{BA}_{JI} for a full doubles array X[A,B,I,J]."""
    return np.einsum("baji->abij", X)


def to_covariant2(Xt):
    """Omega^{AB}_{IJ} = (2 Omega~^{AB}_{IJ} + Omega~^{BA}_{IJ}) / 3 (Implementation section)."""
    return (2.0 * Xt + np.einsum("baij->abij", Xt)) / 3.0


def delta2(NV, NO):
    """Delta_{AI,BJ} = 1 + delta_AB delta_IJ (SI definitions)."""
    D = np.ones((NV, NV, NO, NO))
    for A in range(NV):
        for I in range(NO):
            D[A, A, I, I] = 2.0
    return D


class Brute:
    """Full-space brute force for one ground state (t1, t2, integrals)."""

    def __init__(self, n_o, n_v, eps_o, eps_v, L_full, t1, t2):
        self.n_o, self.n_v = n_o, n_v
        self.NO, self.NV = eps_o.size, eps_v.size
        NO, NV = self.NO, self.NV
        self.N = NO + NV
        self.eps_o, self.eps_v = eps_o, eps_v
        self.L = L_full
        self.t1, self.t2 = t1, t2
        self.o = slice(0, NO)
        self.v = slice(NO, self.N)
        # active mask on triples
        mo = (np.arange(NO) < n_o).astype(float)
        mv = (np.arange(NV) < n_v).astype(float)
        self.mask = np.einsum("a,b,c,i,j,k->abcijk", mv, mv, mv, mo, mo, mo)
        # orbital-energy denominators eps^{abc}_{ijk}
        ev, eo = eps_v, eps_o
        self.eps3 = (ev[:, None, None, None, None, None] + ev[None, :, None, None, None, None]
                     + ev[None, None, :, None, None, None] - eo[None, None, None, :, None, None]
                     - eo[None, None, None, None, :, None] - eo[None, None, None, None, None, :])
        self.Lh = self.t1_transform(L_full, t1)
        self.g = np.einsum("Jpq,Jrs->pqrs", self.Lh, self.Lh)        # T1-transformed
        self.g0 = np.einsum("Jpq,Jrs->pqrs", L_full, L_full)         # bare
        self.F = self.fock_ov(t1)
        self.Delta = delta2(NV, NO)
        self.cvs = None

    def set_cvs(self, core):
        """Core-valence separation (Implementation section, core excited states): triples
        without a core occupied index are dropped, and the right and left transforms project
        their input and output vectors onto the elements with at least one core occupied index."""
        c = np.asarray(core, dtype=bool)
        self.cvs = c
        anycore = (c[:, None, None] | c[None, :, None] | c[None, None, :]).astype(float)
        self.mask = self.mask * anycore[None, None, None]

    def cvs_project(self, X1, X2):
        if self.cvs is None:
            return X1, X2
        c = self.cvs
        return X1 * c[None, :], X2 * (c[:, None] | c[None, :])[None, None]

    # -- building blocks ----------------------------------------------------
    def embed1(self, x1):
        M = np.zeros((self.N, self.N))
        M[self.v, self.o] = x1
        return M

    def t1_transform(self, L, t1):
        T = self.embed1(t1)
        one = np.eye(self.N)
        return np.einsum("pr,Jrs,sq->Jpq", one - T, L, one + T)

    def fock_ov(self, t1):
        o, v = self.o, self.v
        gov = self.g0[o, v, o, v]                   # g_kcLD (bare = T1-invariant ov|ov)
        return 2.0 * np.einsum("kcld,dl->kc", gov, t1) - np.einsum("kdlc,dl->kc", gov, t1)

    def upsilon(self, R1):
        R = self.embed1(R1)
        dL = np.einsum("Jpr,rq->Jpq", self.Lh, R) - np.einsum("pr,Jrq->Jpq", R, self.Lh)
        return np.einsum("Jpq,Jrs->pqrs", dL, self.Lh) + np.einsum("Jpq,Jrs->pqrs", self.Lh, dL)

    def upsilon_kc(self, R1):
        o, v = self.o, self.v
        gov = self.g0[o, v, o, v]
        return 2.0 * np.einsum("kcld,dl->kc", gov, R1) - np.einsum("kdlc,dl->kc", gov, R1)

    def W(self, x2, G):
        """sum_D x^{aD}_{ij} G_bDck - sum_L x^{ab}_{iL} G_Ljck, full space, unmasked."""
        o, v = self.o, self.v
        return (np.einsum("adij,bdck->abcijk", x2, G[v, v, v, o])
                - np.einsum("abil,ljck->abcijk", x2, G[o, o, v, o]))

    def triples(self, Wsum, omega):
        """-(eps - omega)^{-1} P(W), restricted to the active space."""
        return -P3(Wsum) / (self.eps3 - omega) * self.mask

    # -- ground state ---------------------------------------------------------
    def tau3(self):
        return self.triples(self.W(self.t2, self.g), 0.0)

    def ground_residual(self, tau=None):
        """Triples contributions to Omega_1 and Omega_2 (SI ground-state residual).
        Test hook: `tau` replaces the triples amplitudes (the residual is linear in them), and
        the attribute F (the occupied-virtual Fock block F_kc) may be overwritten."""
        o, v = self.o, self.v
        g = self.g
        tt = tilde3(self.tau3() if tau is None else tau)
        om1 = np.einsum("abcijk,jbkc->ai", tt, g[o, v, o, v])
        Y = (np.einsum("abcijk,kc->abij", tt, self.F)
             - np.einsum("abcijk,jlkc->abil", tt, g[o, o, o, v])
             + np.einsum("abcijk,dbkc->adij", tt, g[v, v, o, v]))
        om2 = to_covariant2(Y + transpose_pairs2(Y))
        return om1, om2

    def ground_residual_at(self, t1, t2):
        """Omega^(T) at other amplitudes (finite-difference checks)."""
        b = Brute(self.n_o, self.n_v, self.eps_o, self.eps_v, self.L, t1, t2)
        return b.ground_residual()

    # -- right transform ------------------------------------------------------
    def R3(self, R1, R2, omega):
        Rb = self.Delta * R2
        return self.triples(self.W(Rb, self.g) + self.W(self.t2, self.upsilon(R1)), omega)

    def right_transform(self, R1, R2, omega, R3=None):
        """Triples contributions to rho = J R (SI right Jacobian transformation).  Test hook:
        `R3` replaces the right triples amplitudes (rho is linear in them)."""
        if self.cvs is not None:
            R1, R2 = self.cvs_project(R1, R2)
            return self.cvs_project(*self._right(R1, R2, omega, R3))
        return self._right(R1, R2, omega, R3)

    def _right(self, R1, R2, omega, R3=None):
        o, v = self.o, self.v
        g = self.g
        tt = tilde3(self.tau3())
        Rt = tilde3(self.R3(R1, R2, omega) if R3 is None else R3)
        rho1 = np.einsum("abcijk,jbkc->ai", Rt, g[o, v, o, v])
        Y = (np.einsum("abcijk,kc->abij", Rt, self.F)
             + np.einsum("abcijk,kc->abij", tt, self.upsilon_kc(R1))
             - np.einsum("abcijk,jlkc->abil", Rt, g[o, o, o, v])
             - np.einsum("abcijk,jdkc,dl->abil", tt, g[o, v, o, v], R1)
             + np.einsum("abcijk,dbkc->adij", Rt, g[v, v, o, v])
             - np.einsum("abcijk,lbkc,dl->adij", tt, g[o, v, o, v], R1))
        rho2 = to_covariant2((Y + transpose_pairs2(Y)) / self.Delta)
        return rho1, rho2

    # -- left transform -------------------------------------------------------
    def L3(self, L1, L2, omega):
        o, v = self.o, self.v
        g = self.g
        Z = (np.einsum("ai,jbkc->abcijk", L1, g[o, v, o, v])
             + np.einsum("abij,kc->abcijk", L2, self.F)
             + np.einsum("adij,dbkc->abcijk", L2, g[v, v, o, v])
             - np.einsum("abil,jlkc->abcijk", L2, g[o, o, o, v]))
        return self.triples(Z, omega)

    def left_transform(self, L1, L2, omega):
        """Triples contributions to sigma = L^T J (SI transpose Jacobian transformation)."""
        if self.cvs is not None:
            L1, L2 = self.cvs_project(L1, L2)
            return self.cvs_project(*self._left(L1, L2, omega))
        return self._left(L1, L2, omega)

    def _left(self, L1, L2, omega):
        o, v = self.o, self.v
        g, t2 = self.g, self.t2
        tt = tilde3(self.tau3())
        Lt = tilde3(self.L3(L1, L2, omega))
        gov = g[o, v, o, v]
        s1 = (2.0 * np.einsum("abcijk,abij,kcld->dl", tt, L2, gov)
              - np.einsum("abcijk,abij,kdlc->dl", tt, L2, gov)
              - np.einsum("abcijk,lbkc,adij->dl", tt, gov, L2)
              - np.einsum("abcijk,jdkc,abil->dl", tt, gov, L2))
        s1 += (np.einsum("abcijl,aeij,becd->dl", Lt, t2, g[v, v, v, v])
               - np.einsum("abcijl,abim,mjcd->dl", Lt, t2, g[o, o, v, v])
               - np.einsum("abcilk,abim,mdck->dl", Lt, t2, g[o, v, v, o]))
        s1 += (np.einsum("abdijk,abim,mjlk->dl", Lt, t2, g[o, o, o, o])
               - np.einsum("abdijk,aeij,lkbe->dl", Lt, t2, g[o, o, v, v])
               - np.einsum("adcijk,aeij,leck->dl", Lt, t2, g[o, v, v, o]))
        Q = (np.einsum("abcijk,bdck->adij", Lt, g[v, v, v, o])
             - np.einsum("abcijk,ljck->abil", Lt, g[o, o, v, o]))
        s2 = to_covariant2(Q + transpose_pairs2(Q))
        return s1, s2


    # -- transition densities ---------------------------------------------------
    def lambda3(self, lam1, lam2):
        """lambda3 from the L3 recipe with (lambda1, lambda2) at omega = 0 (ground-state multipliers)."""
        return self.L3(lam1, lam2, 0.0)

    def density_m0(self, L1, L2, omega, terms=False):
        """Triples terms of the left transition density D^{m-0} (SI left density), D[p][q]
        multiplies A_pq; occupied orbitals first.  terms=True returns the N x N contribution of
        each printed term by name instead of their sum."""
        o, v = self.o, self.v
        t2 = self.t2
        tau = self.tau3()
        tt = tilde3(tau)
        Lt = tilde3(self.L3(L1, L2, omega))
        T = {k: np.zeros((self.N, self.N)) for k in ("kl", "ld", "LD", "cd")}
        T["kl"][o, o] -= 0.5 * np.einsum("abcijl,abcijk->kl", Lt, tau)
        T["ld"][o, v] += np.einsum("abij,abdijl->ld", L2, tt)
        T["LD"][o, v] -= np.einsum("abcijk,acil,bdjk->ld", Lt, t2, t2)
        T["cd"][v, v] += 0.5 * np.einsum("abcijk,abdijk->cd", Lt, tau)
        if terms:
            return T
        return T["kl"] + T["ld"] + T["LD"] + T["cd"]

    def density_0m(self, lam1, lam2, R1, R2, omega, terms=False):
        """Triples terms of the right transition density D^{0-m} (SI right density) and the
        triples overlap s = (1/6) sum lambda~3 R3.  The occupied diagonal carries 2s; the
        -s D^{0-0} term is left to the caller.  Doubles of R enter as Rbar = Delta R; the doubles
        multipliers of the D_ld term enter plain (printed with a tilde).
        terms=True returns ({name: N x N contribution of each printed term}, s)."""
        o, v = self.o, self.v
        t2 = self.t2
        tau = self.tau3()
        lt = tilde3(self.lambda3(lam1, lam2))
        R3 = self.R3(R1, R2, omega)
        Rt = tilde3(R3)
        Rb = self.Delta * R2
        names = ("Kl", "kl", "ld_R1tau", "ld_l2Rt", "LD_Rbt", "LD_Rbt2", "lD", "Ld", "ck", "cD", "cd", "LL")
        T = {k: np.zeros((self.N, self.N)) for k in names}
        T["Kl"][o, o] -= np.einsum("abcijl,ai,bcjk->kl", lt, R1, t2)
        T["kl"][o, o] -= 0.5 * np.einsum("abcijl,abcijk->kl", lt, R3)
        T["ld_R1tau"][o, v] += (np.einsum("abcijk,ai,bcdjkl->ld", lt, R1, tau)
                                - np.einsum("abcijk,ai,bcdjlk->ld", lt, R1, tau))
        # the printed lambda~^{ab}_{ij} read as the plain multipliers lambda^{ab}_{ij}: the term is
        # the multiplier analog of the left density's L^{ab}_{ij} tau~^{abd}_{ijl} term
        T["ld_l2Rt"][o, v] += np.einsum("abij,abdijl->ld", lam2, Rt)
        T["LD_Rbt"][o, v] += 0.5 * (2.0 * np.einsum("abcijk,abij,cdkl->ld", lt, Rb, t2)
                                    - np.einsum("abcijk,abij,cdlk->ld", lt, Rb, t2))
        T["LD_Rbt2"][o, v] -= (np.einsum("abcijk,acil,bdjk->ld", lt, Rb, t2)
                               + np.einsum("abcijk,adik,bcjl->ld", lt, Rb, t2))
        T["lD"][o, v] -= 0.5 * np.einsum("abcijk,abcijl,dk->ld", lt, tau, R1)
        T["Ld"][o, v] -= 0.5 * np.einsum("abcijk,abdijk,cl->ld", lt, tau, R1)
        T["ck"][v, o] += 0.5 * np.einsum("abcijk,abij->ck", lt, Rb)
        T["cD"][v, v] += np.einsum("abcijk,ai,bdjk->cd", lt, R1, t2)
        T["cd"][v, v] += 0.5 * np.einsum("abcijk,abdijk->cd", lt, R3)
        s = float(np.sum(lt * R3)) / 6.0
        T["LL"][o, o] += 2.0 * s * np.eye(self.NO)
        if terms:
            return T, s
        D = np.zeros((self.N, self.N))
        for k in names:
            D += T[k]
        return D, s


# ----------------------------------------------------------------------------
# block views matching the C-ABI layouts
def blocks2(X, n_o, n_v):
    return {"x2_vVoo": np.ascontiguousarray(X[:n_v, :, :n_o, :n_o]),
            "x2_vvoO": np.ascontiguousarray(X[:n_v, :n_v, :n_o, :])}


def pair_form(d, L1, L2, R1, R2):
    """G(L,R) = sum L1 R1 + sum_{(AI)>=(BJ)} L~2 R2 over full arrays."""
    NV, NO = R1.shape
    Lt = 2.0 * L2 - np.einsum("baij->abij", L2)
    prod = Lt * R2
    tot = np.sum(prod) + np.einsum("aaii->", prod)
    return float(np.sum(L1 * R1) + 0.5 * tot)
