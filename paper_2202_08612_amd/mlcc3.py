"""Thin ctypes binding of ``libmlcc3.so`` (the C-ABI in ``include/mlcc3.h``).

Argument marshalling only: every step of the triples path runs in the HIP
library.  torch provides device memory and the current stream.  Importing this
module raises if the library has not been built (``python -m
paper_2202_08612_amd.build``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlcc3.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_08612_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ESINGULAR, ENOMEM, EHIP, ENONFINITE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6}

_dp = ctypes.POINTER(ctypes.c_double)


class _Ground(ctypes.Structure):
    _fields_ = [("n_o", ctypes.c_int32), ("n_v", ctypes.c_int32), ("N_O", ctypes.c_int32),
                ("N_V", ctypes.c_int32), ("n_chol", ctypes.c_int32)] + \
               [(k, ctypes.c_void_p) for k in ("eps_o", "eps_v", "L_OO", "L_OV", "L_vV", "t1",
                                                "t2_vVoo", "t2_vvoO")]


class _Vec(ctypes.Structure):
    _fields_ = [("x1", ctypes.c_void_p), ("x2_vVoo", ctypes.c_void_p), ("x2_vvoO", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("reuse_ground", ctypes.c_int32),
                ("triple_begin", ctypes.c_int64), ("triple_end", ctypes.c_int64),
                ("guard", ctypes.c_double), ("check_finite", ctypes.c_int32),
                ("cvs_core", ctypes.c_void_p), ("reuse_tau", ctypes.c_int32)]


TUNING_FIELDS = ("dc_wg_per_cu", "back_ksplit", "narrow_tile", "contra_form", "vec_group", "occ_slab")


class _Tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in TUNING_FIELDS]


_lib.mlcc3_ws_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
_lib.mlcc3_ws_set_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tuning)]
_lib.mlcc3_ws_get_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tuning)]
_lib.mlcc3_ws_destroy.argtypes = [ctypes.c_void_p]
_lib.mlcc3_ws_bytes.argtypes = [ctypes.c_void_p]
_lib.mlcc3_ws_bytes.restype = ctypes.c_int64
_lib.mlcc3_ws_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.mlcc3_ws_phase_stats.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.mlcc3_num_triples.argtypes = [ctypes.c_int32]
_lib.mlcc3_num_triples.restype = ctypes.c_int64
_lib.mlcc3_opts_default.argtypes = [ctypes.POINTER(_Opts)]
_lib.mlcc3_ground_residual.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Ground), ctypes.POINTER(_Opts),
                                       ctypes.POINTER(_Vec), ctypes.c_void_p]
_lib.mlcc3_ground_residual_noalloc.argtypes = [ctypes.POINTER(_Ground), ctypes.POINTER(_Opts), ctypes.POINTER(_Vec),
                                               ctypes.c_void_p]
_lib.mlcc3_noalloc_scratch_bytes.restype = ctypes.c_int64
for _fn in ("mlcc3_right_transform", "mlcc3_left_transform"):
    getattr(_lib, _fn).argtypes = [ctypes.c_void_p, ctypes.POINTER(_Ground), ctypes.c_int32, _dp,
                                   ctypes.POINTER(_Vec), ctypes.POINTER(_Vec), ctypes.POINTER(_Opts),
                                   ctypes.c_void_p]
_lib.mlcc3_triples_densities.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Ground), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, _dp, ctypes.POINTER(_Vec), ctypes.POINTER(_Vec),
                                         ctypes.POINTER(_Vec), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(_Opts), ctypes.c_void_p]
_lib.mlcc3_vec_map.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Ground), ctypes.c_int32, ctypes.c_int32,
                               ctypes.POINTER(_Vec), ctypes.POINTER(_Vec), ctypes.c_void_p]
_lib.mlcc3_oscillator_strengths.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_int32, _dp] + [ctypes.c_void_p] * 7 + [ctypes.c_void_p]
_lib.mlcc3_flops.argtypes = [ctypes.POINTER(_Ground), ctypes.c_int32, ctypes.c_int32]
_lib.mlcc3_flops.restype = ctypes.c_double
_lib.mlcc3_status_string.argtypes = [ctypes.c_int]
_lib.mlcc3_status_string.restype = ctypes.c_char_p
_lib.mlcc3_last_error.restype = ctypes.c_char_p

EXPORTED = ["mlcc3_ws_create", "mlcc3_ws_destroy", "mlcc3_ws_bytes", "mlcc3_ws_timing", "mlcc3_ws_phase_stats",
            "mlcc3_ws_set_tuning", "mlcc3_ws_get_tuning", "mlcc3_opts_default",
            "mlcc3_num_triples", "mlcc3_ground_residual", "mlcc3_right_transform",
            "mlcc3_left_transform", "mlcc3_triples_densities", "mlcc3_vec_map", "mlcc3_oscillator_strengths", "mlcc3_flops",
            "mlcc3_status_string", "mlcc3_last_error"]
MAP_SYMMETRIZE, MAP_GRAD_TO_LEFT, MAP_LEFT_TO_GRAD = 0, 1, 2


class MLCC3Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _check(rc):
    if rc != OK:
        msg = _lib.mlcc3_last_error().decode() or _lib.mlcc3_status_string(rc).decode()
        raise MLCC3Error(rc, msg)


def num_triples(n_o):
    return int(_lib.mlcc3_num_triples(n_o))


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Workspace:
    """Device scratch and cached ground-state blocks on one GPU."""

    def __init__(self, device=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        _check(_lib.mlcc3_ws_create(ctypes.byref(h), self.device.index or 0))
        self.h = h

    def bytes(self):
        return int(_lib.mlcc3_ws_bytes(self.h))

    def timing(self, enable=True):
        _check(_lib.mlcc3_ws_timing(self.h, 1 if enable else 0))

    def phase_stats(self, phase=0):
        n, ms, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.mlcc3_ws_phase_stats(self.h, phase, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)))
        return {"launches": int(n.value), "ms": float(ms.value), "flops": float(fl.value)}

    def set_tuning(self, tuning=None):
        """Launch-shape choices of this workspace (dict over TUNING_FIELDS, missing keys = 0 =
        the library default); None restores all defaults."""
        if tuning is None:
            _check(_lib.mlcc3_ws_set_tuning(self.h, None))
            return
        bad = set(tuning) - set(TUNING_FIELDS)
        if bad:
            raise KeyError(f"unknown tuning fields {sorted(bad)}")
        t = _Tuning(*[int(tuning.get(k, 0)) for k in TUNING_FIELDS])
        _check(_lib.mlcc3_ws_set_tuning(self.h, ctypes.byref(t)))

    def get_tuning(self):
        t = _Tuning()
        _check(_lib.mlcc3_ws_get_tuning(self.h, ctypes.byref(t)))
        return {k: int(getattr(t, k)) for k in TUNING_FIELDS}

    def close(self):
        if self.h:
            _check(_lib.mlcc3_ws_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GROUND_KEYS = ("eps_o", "eps_v", "L_OO", "L_OV", "L_vV", "t1", "t2_vVoo", "t2_vvoO")
VEC_KEYS = ("x1", "x2_vVoo", "x2_vvoO")


def ground_sizes(d):
    """Element counts of the ground-state arrays (layouts in include/mlcc3.h)."""
    no, nv, NO, NV, nc = d.n_o, d.n_v, d.N_O, d.N_V, d.n_chol
    return {"eps_o": NO, "eps_v": NV, "L_OO": nc * NO * NO, "L_OV": nc * NO * NV, "L_vV": nc * nv * NV,
            "t1": NV * NO, "t2_vVoo": nv * NV * no * no, "t2_vvoO": nv * nv * no * NO}


def vec_sizes(d):
    """Element counts of the blocks of a trial vector or output."""
    no, nv, NO, NV = d.n_o, d.n_v, d.N_O, d.N_V
    return {"x1": NV * NO, "x2_vVoo": nv * NV * no * no, "x2_vvoO": nv * nv * no * NO}


def _dev(x, device, n=None, what="array"):
    """FP64 contiguous copy (or view) of x on device.  The library takes bare pointers and reads
    the element counts its sizes imply, so every array is checked here: a missing one or one of
    the wrong size would be read out of bounds on the device."""
    if x is None:
        raise ValueError(f"{what}: missing")
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.float64)
    else:
        t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device)
    if n is not None and t.numel() != n:
        raise ValueError(f"{what}: {t.numel()} elements, expected {n}")
    return t.contiguous()


class Ground:
    """Ground-state inputs resident on the device (see include/mlcc3.h for layouts)."""

    def __init__(self, prob, device="cuda"):
        d = prob.dims
        self.dims = d
        n = ground_sizes(d)
        self.t = {k: _dev(getattr(prob, k), device, n[k], k) for k in GROUND_KEYS}
        self.c = _Ground(d.n_o, d.n_v, d.N_O, d.N_V, d.n_chol,
                         *[self.t[k].data_ptr() for k in GROUND_KEYS])

    def flops(self, which, nvec=1):
        return float(_lib.mlcc3_flops(ctypes.byref(self.c), which, nvec))


def vec_to_device(vec, device="cuda"):
    return {k: _dev(vec[k], device) for k in VEC_KEYS}


def empty_out(d, device="cuda"):
    return {"x1": torch.empty((d.N_V, d.N_O), dtype=torch.float64, device=device),
            "x2_vVoo": torch.empty((d.n_v, d.N_V, d.n_o, d.n_o), dtype=torch.float64, device=device),
            "x2_vvoO": torch.empty((d.n_v, d.n_v, d.n_o, d.N_O), dtype=torch.float64, device=device)}


def _vecs(lst, d, device):
    """C array of vector descriptors; every block must be a contiguous FP64 tensor of the size
    the dimensions give, on the workspace's device."""
    n = vec_sizes(d)
    dev = torch.device(device)
    arr = (_Vec * len(lst))()
    for m, v in enumerate(lst):
        for k in VEC_KEYS:
            t = v[k]
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError(f"vector {m} block {k}: not a contiguous float64 tensor")
            if t.device.type != dev.type or (dev.index is not None and t.device.index != dev.index):
                raise ValueError(f"vector {m} block {k}: on {t.device}, expected {dev}")
            if t.numel() != n[k]:
                raise ValueError(f"vector {m} block {k}: {t.numel()} elements, expected {n[k]}")
        arr[m] = _Vec(v["x1"].data_ptr(), v["x2_vVoo"].data_ptr(), v["x2_vvoO"].data_ptr())
    return arr


def _check_ground(ws, ground):
    dev = torch.device(ws.device)
    for k, t in ground.t.items():
        if t.device.type != dev.type or (dev.index is not None and t.device.index != dev.index):
            raise ValueError(f"ground array {k}: on {t.device}, expected {dev}")


def make_opts(precision="fp64", reuse_ground=False, triple_range=None, guard=0.0, check_finite=False,
              cvs_core=None, reuse_tau=False):
    o = _Opts()
    _lib.mlcc3_opts_default(ctypes.byref(o))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.reuse_ground = 1 if reuse_ground else 0
    o.reuse_tau = 1 if reuse_tau else 0
    if triple_range is not None:
        o.triple_begin, o.triple_end = int(triple_range[0]), int(triple_range[1])
    o.guard = float(guard)
    o.check_finite = 1 if check_finite else 0
    if cvs_core is not None:
        o._cvs = np.ascontiguousarray(np.asarray(cvs_core) != 0, dtype=np.uint8)  # kept alive with o
        o.cvs_core = o._cvs.ctypes.data
    return o


def ground_residual(ws, ground, out=None, **kw):
    out = empty_out(ground.dims, ws.device) if out is None else out
    o = make_opts(**kw)
    _check_ground(ws, ground)
    arr = _vecs([out], ground.dims, ws.device)
    _check(_lib.mlcc3_ground_residual(ws.h, ctypes.byref(ground.c), ctypes.byref(o), arr, _stream(ws.device)))
    return out


def noalloc_scratch_bytes():
    return int(_lib.mlcc3_noalloc_scratch_bytes())


def ground_residual_noalloc(ground, out, device="cuda", **kw):
    """mlcc3_ground_residual_noalloc on `device` (made current for the call): no device allocation
    inside the library; `out` (e.g. from empty_out) is filled."""
    dev = torch.device(device)
    o = make_opts(**kw)
    for k, t in ground.t.items():
        if t.device.type != dev.type or (dev.index is not None and t.device.index != dev.index):
            raise ValueError(f"ground array {k}: on {t.device}, expected {dev}")
    arr = _vecs([out], ground.dims, dev)
    with torch.cuda.device(dev):
        _check(_lib.mlcc3_ground_residual_noalloc(ctypes.byref(ground.c), ctypes.byref(o), arr, _stream(dev)))
    return out


def _transform(fn, ws, ground, omegas, vecs, outs=None, **kw):
    n = len(vecs)
    outs = [empty_out(ground.dims, ws.device) for _ in range(n)] if outs is None else outs
    om = (ctypes.c_double * n)(*[float(w) for w in omegas])
    o = make_opts(**kw)
    _check_ground(ws, ground)
    vin, vout = _vecs(vecs, ground.dims, ws.device), _vecs(outs, ground.dims, ws.device)
    _check(fn(ws.h, ctypes.byref(ground.c), n, om, vin, vout, ctypes.byref(o), _stream(ws.device)))
    return outs


def oscillator_strengths(ws, A, omegas, D_m0, D_0m, D_00, s):
    """Transition moments T_m0, T_0m ([nstate][ncomp]) and oscillator strengths f ([nstate]) from
    densities D_m0, D_0m ([nstate][N][N]), D_00 ([N][N]), s ([nstate]) and operator A ([ncomp][N][N])."""
    dev = ws.device
    A = _dev(A, dev, what="A")
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError(f"A: shape {tuple(A.shape)}, expected [ncomp][N][N]")
    ncomp, N = A.shape[0], A.shape[1]
    D_m0, D_0m = _dev(D_m0, dev, what="D_m0"), _dev(D_0m, dev, what="D_0m")
    n = D_m0.shape[0] if D_m0.dim() == 3 else -1
    D_m0, D_0m = _dev(D_m0, dev, n * N * N, "D_m0"), _dev(D_0m, dev, n * N * N, "D_0m")
    D_00, sv = _dev(D_00, dev, N * N, "D_00"), _dev(s, dev, n, "s")
    if len(omegas) != n:
        raise ValueError(f"{len(omegas)} omegas for {n} states")
    Tm0 = torch.empty((n, ncomp), dtype=torch.float64, device=dev)
    T0m = torch.empty((n, ncomp), dtype=torch.float64, device=dev)
    f = torch.empty((n,), dtype=torch.float64, device=dev)
    om = (ctypes.c_double * n)(*[float(w) for w in omegas])
    _check(_lib.mlcc3_oscillator_strengths(ws.h, N, ncomp, A.data_ptr(), n, om, D_m0.data_ptr(), D_0m.data_ptr(),
                                           D_00.data_ptr(), sv.data_ptr(), Tm0.data_ptr(), T0m.data_ptr(),
                                           f.data_ptr(), _stream(dev)))
    return Tm0, T0m, f


def vec_map(ws, ground, mode, vecs, outs=None):
    """Pairing maps of trial vectors (MAP_SYMMETRIZE, MAP_GRAD_TO_LEFT, MAP_LEFT_TO_GRAD)."""
    n = len(vecs)
    outs = [empty_out(ground.dims, ws.device) for _ in range(n)] if outs is None else outs
    vin, vout = _vecs(vecs, ground.dims, ws.device), _vecs(outs, ground.dims, ws.device)
    _check(_lib.mlcc3_vec_map(ws.h, ctypes.byref(ground.c), int(mode), n, vin, vout, _stream(ws.device)))
    return outs


def right_transform(ws, ground, omegas, vecs, outs=None, **kw):
    return _transform(_lib.mlcc3_right_transform, ws, ground, omegas, vecs, outs, **kw)


def left_transform(ws, ground, omegas, vecs, outs=None, **kw):
    return _transform(_lib.mlcc3_left_transform, ws, ground, omegas, vecs, outs, **kw)


def to_numpy(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def triples_densities(ws, ground, omegas, Lvecs, Rvecs, lam, t2_vVoO, t2_vVOo, **kw):
    """Triples terms of D^{m-0}, D^{0-m} ([nstate][N][N]) and s ([nstate]) on the device."""
    d = ground.dims
    n = len(Lvecs)
    if len(Rvecs) != n:
        raise ValueError(f"{n} left and {len(Rvecs)} right vectors")
    N = d.N_O + d.N_V
    nt2 = d.n_v * d.N_V * d.n_o * d.N_O
    a = _dev(t2_vVoO, ws.device, nt2, "t2_vVoO")
    b = _dev(t2_vVOo, ws.device, nt2, "t2_vVOo")
    _check_ground(ws, ground)
    vl, vr, vlam = _vecs(Lvecs, d, ws.device), _vecs(Rvecs, d, ws.device), _vecs([lam], d, ws.device)
    Dm0 = torch.empty((n, N, N), dtype=torch.float64, device=ws.device)
    D0m = torch.empty((n, N, N), dtype=torch.float64, device=ws.device)
    sv = torch.empty((n,), dtype=torch.float64, device=ws.device)
    om = (ctypes.c_double * n)(*[float(w) for w in omegas])
    o = make_opts(**kw)
    _check(_lib.mlcc3_triples_densities(ws.h, ctypes.byref(ground.c), a.data_ptr(), b.data_ptr(), n, om,
                                        vl, vr, vlam, Dm0.data_ptr(), D0m.data_ptr(), sv.data_ptr(),
                                        ctypes.byref(o), _stream(ws.device)))
    return Dm0, D0m, sv
