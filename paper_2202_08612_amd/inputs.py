"""Seeded synthetic inputs for the MLCC3 triples hot path.

This module only *produces inputs*; it contains none of the method's
arithmetic.  Both the CPU oracle (``oracle/``) and the HIP path read the same
arrays from here, and nothing else is shared between them.

Every number is drawn from a counter-based generator: SplitMix64 (Steele, Lea
and Flood, OOPSLA 2014) hashed over (seed, tensor id, canonical multi-index),
followed by the Box-Muller transform for normal deviates.  Because a value
depends only on its key, any block of a tensor can be generated without
materialising the full tensor, and symmetric partners share one draw:

* Cholesky vectors  L^J_pq = L^J_qp   keyed on (J, min(p,q), max(p,q)),
  with p, q full orbital indices (occupied first, then virtual);
* doubles arrays     X^{AB}_{IJ} = X^{BA}_{JI}  keyed on the unordered pair of
  compound indices {A*N_O+I, B*N_O+J}.

Distributions (paper's workload recipe as fixed for this synthetic stand-in):
occupied energies U[-2.0,-0.3], virtual energies U[0.1,3.0], L ~ N(0, 0.05^2),
t1 ~ N(0, 0.01^2), t2 ~ N(0, 0.02^2), trial vectors N(0,1) then normalised
over the packed block support, lambda ~ N(0,0.01^2) / N(0,0.02^2).  The
core-like configuration moves occupied orbital 0 to U[-15.5,-14.5].

Array layouts (C order, last index fastest), matching ``include/mlcc3.h``:

  eps_o   [N_O]                     eps_v   [N_V]
  L_OO    [n_chol][N_O][N_O]        L_OV    [n_chol][N_O][N_V]
  L_vV    [n_chol][n_v][N_V]        t1      [N_V][N_O]        (t^A_I)
  t2_vVoo [n_v][N_V][n_o][n_o]      (t^{aD}_{ij})
  t2_vvoO [n_v][n_v][n_o][N_O]      (t^{ab}_{iL})
  t2_vVoO [n_v][N_V][n_o][N_O]      (t^{cD}_{kL}, densities only)
  t2_vVOo [n_v][N_V][N_O][n_o]      (t^{cD}_{Lk}, densities only)
  vector: x1 [N_V][N_O], x2_vVoo, x2_vvoO  (same shapes as the t2 blocks)
"""
from __future__ import annotations

import dataclasses
import concurrent.futures
import os

import numpy as np

_U64 = np.uint64
_GOLD = _U64(0x9E3779B97F4A7C15)
_M1 = _U64(0xBF58476D1CE4E5B9)
_M2 = _U64(0x94D049BB133111EB)

# tensor ids (part of every key)
TID_EPS_O, TID_EPS_V, TID_L, TID_T1, TID_T2 = 1, 2, 3, 4, 5
TID_VEC1, TID_VEC2 = 16, 17          # + 2*vector_slot


def _splitmix64(x):
    x = (x + _GOLD).astype(_U64, copy=False)
    z = (x ^ (x >> _U64(30))) * _M1
    z = (z ^ (z >> _U64(27))) * _M2
    return z ^ (z >> _U64(31))


def _key(seed: int, tid: int, *idx):
    h = _splitmix64(np.asarray([seed], dtype=_U64) * _U64(0x100000001B3) + _U64(tid))
    for ix in idx:
        h = _splitmix64(h ^ (np.asarray(ix).astype(_U64) * _U64(0xD1B54A32D192ED03)))
    return h


def _uniform(h):
    return (_splitmix64(h ^ _U64(0x5851F42D4C957F2D)) >> _U64(11)).astype(np.float64) * (2.0 ** -53)


def _normal(h):
    u1 = ((_splitmix64(h ^ _U64(0x14057B7EF767814F)) >> _U64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)
    u2 = (_splitmix64(h ^ _U64(0x2545F4914F6CDD1D)) >> _U64(11)).astype(np.float64) * (2.0 ** -53)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Dims:
    n_o: int
    n_v: int
    N_O: int
    N_V: int
    n_chol: int

    @property
    def N(self):
        return self.N_O + self.N_V


# The five workloads (active n_o/n_v, total N_O/N_V, Cholesky rank).
CONFIGS = {
    0: dict(dims=Dims(4, 12, 6, 20, 60), nvec=1, core=False),
    1: dict(dims=Dims(12, 60, 30, 250, 600), nvec=1, core=False),
    2: dict(dims=Dims(12, 60, 30, 250, 600), nvec=1, core=False),
    3: dict(dims=Dims(16, 80, 40, 400, 1000), nvec=4, core=False),
    4: dict(dims=Dims(8, 60, 90, 1100, 2500), nvec=8, core=True),
}


# Inactive-space sweep at a fixed active space (n_o = 8, n_v = 136), with the occupied and
# virtual counts of the formaldehyde + 1..6 water series (Results section, table of system
# sizes); Cholesky rank 3 (N_O + N_V).
SWEEP_NV = [(13, 217), (18, 304), (23, 391), (28, 478), (33, 565), (38, 652)]


def sweep_dims(k: int) -> Dims:
    NO, NV = SWEEP_NV[k]
    return Dims(8, 136, NO, NV, 3 * (NO + NV))


def config_seed(cfg: int) -> int:
    return 20220217 + int(cfg)


def omegas(cfg_or_core, nvec: int):
    """Per-vector excitation energies: 0.40+0.10m (valence), 15.20+0.01m (core)."""
    core = cfg_or_core if isinstance(cfg_or_core, bool) else CONFIGS[cfg_or_core]["core"]
    m = np.arange(nvec, dtype=np.float64)
    return (15.20 + 0.01 * m) if core else (0.40 + 0.10 * m)


# ----------------------------------------------------------------------------
def orbital_energies(seed, d: Dims, core=False):
    eo = -2.0 + 1.7 * _uniform(_key(seed, TID_EPS_O, np.arange(d.N_O)))
    ev = 0.1 + 2.9 * _uniform(_key(seed, TID_EPS_V, np.arange(d.N_V)))
    if core and d.N_O > 0:
        eo[0] = -15.5 + _uniform(_key(seed, TID_EPS_O, np.array([1 << 40])))[0]
    return eo, ev


def cholesky_block(seed, d: Dims, rows, cols, sigma=0.05, chunk=64):
    """L^J_{pq} for full orbital index arrays rows (p) and cols (q): [n_chol][len(rows)][len(cols)]."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    p = rows[:, None]
    q = cols[None, :]
    lo = np.minimum(p, q)
    hi = np.maximum(p, q)
    out = np.empty((d.n_chol, rows.size, cols.size), dtype=np.float64)

    def fill(j0):
        j1 = min(d.n_chol, j0 + chunk)
        J = np.arange(j0, j1, dtype=np.int64)[:, None, None]
        out[j0:j1] = sigma * _normal(_key(seed, TID_L, J, lo[None], hi[None]))

    _parallel(fill, range(0, d.n_chol, chunk))
    return out


def _parallel(fn, items):
    """Run fn over items on a few threads (numpy releases the GIL in the element-wise work);
    every item writes a disjoint slice, so the result does not depend on the schedule."""
    items = list(items)
    nthr = min(len(items), max(1, min(16, os.cpu_count() or 1)))
    if nthr <= 1:
        for it in items:
            fn(it)
        return
    with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
        for _ in ex.map(fn, items):
            pass


def singles(seed, tid, d: Dims, sigma):
    A = np.arange(d.N_V)[:, None]
    I = np.arange(d.N_O)[None, :]
    return sigma * _normal(_key(seed, tid, A, I))


def doubles_block(seed, tid, d: Dims, A, B, I, J, sigma):
    """X^{AB}_{IJ} on the outer grid A x B x I x J (index arrays, full ranges)."""
    A = np.asarray(A, dtype=np.int64)[:, None, None, None]
    B = np.asarray(B, dtype=np.int64)[None, :, None, None]
    I = np.asarray(I, dtype=np.int64)[None, None, :, None]
    J = np.asarray(J, dtype=np.int64)[None, None, None, :]
    out = np.empty((A.shape[0], B.shape[1], I.shape[2], J.shape[3]), dtype=np.float64)

    def fill(a):
        u = A[a:a + 1] * d.N_O + I
        v = B * d.N_O + J
        out[a:a + 1] = sigma * _normal(_key(seed, tid, np.minimum(u, v), np.maximum(u, v)))

    _parallel(fill, range(A.shape[0]))
    return out


def doubles_blocks(seed, tid, d: Dims, sigma, with_density_blocks=False):
    o, v = np.arange(d.n_o), np.arange(d.n_v)
    O, V = np.arange(d.N_O), np.arange(d.N_V)
    out = {
        "x2_vVoo": doubles_block(seed, tid, d, v, V, o, o, sigma),
        "x2_vvoO": doubles_block(seed, tid, d, v, v, o, O, sigma),
    }
    if with_density_blocks:
        out["x2_vVoO"] = doubles_block(seed, tid, d, v, V, o, O, sigma)
        out["x2_vVOo"] = doubles_block(seed, tid, d, v, V, O, o, sigma)
    return out


def packed_norm2(d: Dims, x1, x2_vVoo, x2_vvoO):
    """Sum of squares over singles plus the packed (non-redundant) block-union doubles."""
    a = np.arange(d.n_v)[:, None, None, None]
    D = np.arange(d.N_V)[None, :, None, None]
    i = np.arange(d.n_o)[None, None, :, None]
    j = np.arange(d.n_o)[None, None, None, :]
    keep = (D >= d.n_v) | (a * d.N_O + i >= D * d.N_O + j)
    L = np.arange(d.N_O)[None, None, None, :]
    keep2 = np.broadcast_to(L >= d.n_o, x2_vvoO.shape)
    return float(np.sum(x1 ** 2) + np.sum(np.where(keep, x2_vVoo, 0.0) ** 2)
                 + np.sum(np.where(keep2, x2_vvoO, 0.0) ** 2))


def trial_vector(seed, d: Dims, slot: int, normalise=True, sigma1=1.0, sigma2=1.0):
    tid1, tid2 = TID_VEC1 + 2 * slot, TID_VEC2 + 2 * slot
    vec = {"x1": singles(seed, tid1, d, sigma1)}
    vec.update(doubles_blocks(seed, tid2, d, sigma2))
    if normalise:
        s = 1.0 / np.sqrt(packed_norm2(d, vec["x1"], vec["x2_vVoo"], vec["x2_vvoO"]))
        vec = {k: v * s for k, v in vec.items()}
    return vec


# vector slots: right vectors 0..63, left vectors 64..127, lambda 128
SLOT_R, SLOT_L, SLOT_LAMBDA = 0, 64, 128


@dataclasses.dataclass
class Problem:
    dims: Dims
    seed: int
    eps_o: np.ndarray
    eps_v: np.ndarray
    L_OO: np.ndarray
    L_OV: np.ndarray
    L_vV: np.ndarray
    t1: np.ndarray
    t2_vVoo: np.ndarray
    t2_vvoO: np.ndarray
    t2_vVoO: np.ndarray | None = None
    t2_vVOo: np.ndarray | None = None

    def arrays(self):
        return {k: getattr(self, k) for k in
                ("eps_o", "eps_v", "L_OO", "L_OV", "L_vV", "t1", "t2_vVoo", "t2_vvoO",
                 "t2_vVoO", "t2_vVOo")}


def make_problem(d: Dims, seed: int, core=False, with_density_blocks=False) -> Problem:
    eo, ev = orbital_energies(seed, d, core)
    O = np.arange(d.N_O)
    Vfull = d.N_O + np.arange(d.N_V)
    vact = d.N_O + np.arange(d.n_v)
    t2 = doubles_blocks(seed, TID_T2, d, 0.02, with_density_blocks)
    return Problem(
        dims=d, seed=seed, eps_o=eo, eps_v=ev,
        L_OO=cholesky_block(seed, d, O, O),
        L_OV=cholesky_block(seed, d, O, Vfull),
        L_vV=cholesky_block(seed, d, vact, Vfull),
        t1=singles(seed, TID_T1, d, 0.01),
        t2_vVoo=t2["x2_vVoo"], t2_vvoO=t2["x2_vvoO"],
        t2_vVoO=t2.get("x2_vVoO"), t2_vVOo=t2.get("x2_vVOo"),
    )


def right_vectors(p: Problem, nvec: int):
    return [trial_vector(p.seed, p.dims, SLOT_R + m) for m in range(nvec)]


def left_vectors(p: Problem, nvec: int):
    return [trial_vector(p.seed, p.dims, SLOT_L + m) for m in range(nvec)]


def lambda_vector(p: Problem):
    return trial_vector(p.seed, p.dims, SLOT_LAMBDA, normalise=False, sigma1=0.01, sigma2=0.02)


def make_config(cfg: int, with_density_blocks=None):
    c = CONFIGS[cfg]
    wd = (cfg == 4) if with_density_blocks is None else with_density_blocks
    p = make_problem(c["dims"], config_seed(cfg), core=c["core"], with_density_blocks=wd)
    return p


# ----------------------------------------------------------------------------
# Full tensors (tiny sizes only): the blocks above are slices of these.
def full_cholesky(seed, d: Dims):
    allp = np.arange(d.N)
    return cholesky_block(seed, d, allp, allp)


def full_doubles(seed, tid, d: Dims, sigma):
    V, O = np.arange(d.N_V), np.arange(d.N_O)
    return doubles_block(seed, tid, d, V, V, O, O, sigma)


def full_vector(seed, d: Dims, slot: int, normalise=True, sigma1=1.0, sigma2=1.0):
    """The trial vector as full arrays x1 [N_V][N_O], x2 [N_V][N_V][N_O][N_O]; same
    scale factor as ``trial_vector`` so the block slices agree exactly."""
    tid1, tid2 = TID_VEC1 + 2 * slot, TID_VEC2 + 2 * slot
    x1 = singles(seed, tid1, d, sigma1)
    x2 = full_doubles(seed, tid2, d, sigma2)
    if normalise:
        blk = trial_vector(seed, d, slot, normalise=False, sigma1=sigma1, sigma2=sigma2)
        s = 1.0 / np.sqrt(packed_norm2(d, blk["x1"], blk["x2_vVoo"], blk["x2_vvoO"]))
        x1, x2 = x1 * s, x2 * s
    return x1, x2
