"""ctypes binding of the FP64 restricted-loop oracle ``libmlcc3_oracle.so`` (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmlcc3_oracle.so")
_lib = None


_SO_SANITIZE = os.path.join(_HERE, "libmlcc3_oracle_san.so")


def build(verbose=False, sanitize=False):
    """Compile the oracle with gcc (plain C, OpenMP, no BLAS).  sanitize=True builds
    libmlcc3_oracle_san.so with AddressSanitizer and UndefinedBehaviorSanitizer (load it with
    gcc's libasan preloaded)."""
    so = _SO_SANITIZE if sanitize else _SO
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wno-unused-variable", *san, "-o", so + ".tmp",
           os.path.join(_HERE, "mlcc3_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(so + ".tmp", so)
    return so


class _Problem(ctypes.Structure):
    _fields_ = [("n_o", ctypes.c_int), ("n_v", ctypes.c_int), ("N_O", ctypes.c_int),
                ("N_V", ctypes.c_int), ("n_chol", ctypes.c_int)] + \
               [(k, ctypes.POINTER(ctypes.c_double)) for k in
                ("eps_o", "eps_v", "L_OO", "L_OV", "L_vV", "t1", "t2_vVoo", "t2_vvoO")] + \
               [("cvs_core", ctypes.POINTER(ctypes.c_ubyte))]


def lib():
    global _lib
    if _lib is None:
        so = os.environ.get("MLCC3_ORACLE_SO", _SO)   # the sanitizer build, under the CPU checks
        if so == _SO and not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(so)
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_triples.restype = ctypes.c_int64
        L.orc_num_triples.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Holds the problem arrays (kept alive for the C side)."""

    def __init__(self, prob, cvs_core=None):
        """cvs_core: None, or N_O flags (nonzero = core orbital) for core-valence separation in
        the right and left transforms."""
        d = prob.dims
        self.d = d
        self._keep = {k: _c(getattr(prob, k)) for k in
                      ("eps_o", "eps_v", "L_OO", "L_OV", "L_vV", "t1", "t2_vVoo", "t2_vvoO")}
        self.P = _Problem(d.n_o, d.n_v, d.N_O, d.N_V, d.n_chol,
                          *[_ptr(self._keep[k]) for k in
                            ("eps_o", "eps_v", "L_OO", "L_OV", "L_vV", "t1", "t2_vVoo", "t2_vvoO")])
        if cvs_core is not None:
            self._core = np.ascontiguousarray(np.asarray(cvs_core) != 0, dtype=np.uint8)
            assert self._core.size == d.N_O
            self.P.cvs_core = self._core.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))

    def _outs(self):
        d = self.d
        return (np.zeros((d.N_V, d.N_O)), np.zeros((d.n_v, d.N_V, d.n_o, d.n_o)),
                np.zeros((d.n_v, d.n_v, d.n_o, d.N_O)))

    def num_triples(self):
        return lib().orc_num_triples(self.d.n_o)

    def ground_residual(self, tb=0, te=-1):
        o = self._outs()
        lib().orc_ground_residual(ctypes.byref(self.P), ctypes.c_int64(tb), ctypes.c_int64(te),
                                  *[_ptr(x) for x in o])
        return {"x1": o[0], "x2_vVoo": o[1], "x2_vvoO": o[2]}

    def _vec_call(self, fn, omega, vec, tb, te):
        v = [_c(vec[k]) for k in ("x1", "x2_vVoo", "x2_vvoO")]
        o = self._outs()
        fn(ctypes.byref(self.P), ctypes.c_double(omega), *[_ptr(x) for x in v],
           ctypes.c_int64(tb), ctypes.c_int64(te), *[_ptr(x) for x in o])
        return {"x1": o[0], "x2_vVoo": o[1], "x2_vvoO": o[2]}

    def right_transform(self, omega, vec, tb=0, te=-1):
        return self._vec_call(lib().orc_right_transform, omega, vec, tb, te)

    def left_transform(self, omega, vec, tb=0, te=-1):
        return self._vec_call(lib().orc_left_transform, omega, vec, tb, te)

    def densities(self, omega, Lvec, Rvec, lam, t2_vVoO, t2_vVOo, tb=0, te=-1):
        """(D^{m-0}, D^{0-m}, s) triples terms for one state (see mlcc3_oracle.h)."""
        d = self.d
        N = d.N_O + d.N_V
        Dm0, D0m = np.zeros((N, N)), np.zeros((N, N))
        s = ctypes.c_double()
        args = [_c(t2_vVoO), _c(t2_vVOo)]
        vecs = [_c(v[k]) for v in (Lvec, Rvec, lam) for k in ("x1", "x2_vVoo", "x2_vvoO")]
        lib().orc_densities(ctypes.byref(self.P), _ptr(args[0]), _ptr(args[1]), ctypes.c_double(omega),
                            *[_ptr(x) for x in vecs], ctypes.c_int64(tb), ctypes.c_int64(te),
                            _ptr(Dm0), _ptr(D0m), ctypes.byref(s))
        return Dm0, D0m, float(s.value)

    def triples_block(self, kind, i, j, k, omega=0.0, vec=None):
        d = self.d
        out = np.zeros((d.n_v, d.n_v, d.n_v))
        if vec is None:
            v = [np.zeros(1)] * 3
        else:
            v = [_c(vec[kk]) for kk in ("x1", "x2_vVoo", "x2_vvoO")]
        lib().orc_triples_block(ctypes.byref(self.P), ctypes.c_int(kind), ctypes.c_double(omega),
                                *[_ptr(x) for x in v], i, j, k, _ptr(out))
        return out


def num_threads():
    return lib().orc_num_threads()


def oscillator_strengths(A, omega, Dm0, D0m, D00, s):
    """Transition moments and oscillator strengths of states m (plain definition):
    T^{m0}_x = sum_pq D^{m-0}_pq A^x_pq (Theory section: densities contracted with a one-electron
    operator), T^{0m}_x = sum_pq (D^{0-m} - s D^{0-0})_pq A^x_pq (the -s D^{0-0} term the SI right
    density leaves out), f = (2/3) omega sum_x T^{0m}_x T^{m0}_x (the length-gauge EOM-CC oscillator
    strength, Stanton and Bartlett, J. Chem. Phys. 98, 7029 (1993); used but not printed in the
    paper).  A [ncomp][N][N], Dm0/D0m [nstate][N][N], D00 [N][N]."""
    A = np.asarray(A, dtype=np.float64)
    Dm0 = np.asarray(Dm0, dtype=np.float64)
    D0m = np.asarray(D0m, dtype=np.float64)
    nstate, ncomp = Dm0.shape[0], A.shape[0]
    Tm0 = np.zeros((nstate, ncomp))
    T0m = np.zeros((nstate, ncomp))
    f = np.zeros(nstate)
    for m in range(nstate):
        for x in range(ncomp):
            Tm0[m, x] = np.sum(Dm0[m] * A[x])
            T0m[m, x] = np.sum((D0m[m] - s[m] * D00) * A[x])
        f[m] = 2.0 / 3.0 * omega[m] * np.sum(T0m[m] * Tm0[m])
    return Tm0, T0m, f
