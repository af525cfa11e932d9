"""Occupied slabs: the ground residual and the right and left transforms with the ordered-triple
buffers restricted to the triples whose first index lies in a slab (workspace tuning occ_slab),
against the same calls in one slab (to rounding: the unique-triple blocks are summed slab by slab)
and against the FP64 oracle."""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, rel

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_08612_amd import mlcc3
    return mlcc3


def _np(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def _same(a, b, tol, what):
    for k in b:
        assert np.all(np.isfinite(a[k])), (what, k)
        assert rel(a[k], b[k]) <= tol, (what, k, rel(a[k], b[k]))


def _calls(lib, ws, g, om, R, L, prec, **kw):
    Om = _np(lib.ground_residual(ws, g, precision=prec, **{k: v for k, v in kw.items() if k != "cvs_core"}))
    rho = [_np(x) for x in lib.right_transform(ws, g, om, R, reuse_ground=True, precision=prec, **kw)]
    sig = [_np(x) for x in lib.left_transform(ws, g, om, L, reuse_ground=True, precision=prec, **kw)]
    return Om, rho, sig


CASES = [(I.Dims(4, 12, 6, 20, 60), 1), (I.Dims(4, 12, 6, 20, 60), 3), (I.Dims(5, 17, 7, 37, 23), 2),
         (I.Dims(6, 9, 6, 140, 33), 4), (I.Dims(3, 32, 4, 41, 11), 2), (I.Dims(4, 12, 5, 100, 24), 1)]


@pytest.mark.parametrize("prec", ["fp64", "bf16x6", "fp32"])
@pytest.mark.parametrize("d,w", CASES, ids=lambda x: str(x))
def test_slabs_equal_one_slab_and_oracle(lib, d, w, prec):
    p = I.make_problem(d, 61)
    g = lib.Ground(p)
    om = I.omegas(False, 2)
    Rh, Lh = I.right_vectors(p, 2), I.left_vectors(p, 2)
    R = [lib.vec_to_device(v) for v in Rh]
    L = [lib.vec_to_device(v) for v in Lh]
    ws1, wss = lib.Workspace(0), lib.Workspace(0)
    try:
        wss.set_tuning({"occ_slab": w})
        one = _calls(lib, ws1, g, om, R, L, prec)
        sl = _calls(lib, wss, g, om, R, L, prec)
    finally:
        ws1.close()
        wss.close()
    tol = 1e-13 if prec == "fp64" else 1e-11
    _same(sl[0], one[0], tol, "ground")
    for m in range(2):
        _same(sl[1][m], one[1][m], tol, ("right", m))
        _same(sl[2][m], one[2][m], tol, ("left", m))
    if prec != "fp64":
        return
    from oracle.oracle import Oracle
    orc = Oracle(p)
    _same(sl[0], orc.ground_residual(), TOL, "ground vs oracle")
    for m in range(2):
        _same(sl[1][m], orc.right_transform(om[m], Rh[m]), TOL, ("right vs oracle", m))
        _same(sl[2][m], orc.left_transform(om[m], Lh[m]), TOL, ("left vs oracle", m))


@pytest.mark.parametrize("w", [1, 2])
def test_slabs_with_core_valence_separation_and_range(lib, w):
    """Core orbital 0, a range of unique triples that holds core and all-valence triples."""
    from oracle.oracle import Oracle
    d = I.Dims(5, 14, 7, 30, 21)
    p = I.make_problem(d, 63, core=True)
    g = lib.Ground(p)
    core = [1] + [0] * (d.N_O - 1)
    rng = (2, 9)
    om = I.omegas(True, 2)
    Rh, Lh = I.right_vectors(p, 2), I.left_vectors(p, 2)
    R = [lib.vec_to_device(v) for v in Rh]
    L = [lib.vec_to_device(v) for v in Lh]
    ws1, wss = lib.Workspace(0), lib.Workspace(0)
    try:
        wss.set_tuning({"occ_slab": w})
        one = _calls(lib, ws1, g, om, R, L, "fp64", triple_range=rng, cvs_core=core)
        sl = _calls(lib, wss, g, om, R, L, "fp64", triple_range=rng, cvs_core=core)
    finally:
        ws1.close()
        wss.close()
    _same(sl[0], one[0], 1e-13, "ground")
    orc = Oracle(p, cvs_core=core)
    for m in range(2):
        _same(sl[1][m], one[1][m], 1e-13, ("right", m))
        _same(sl[2][m], one[2][m], 1e-13, ("left", m))
        _same(sl[1][m], orc.right_transform(om[m], Rh[m], *rng), TOL, ("right vs oracle", m))
        _same(sl[2][m], orc.left_transform(om[m], Lh[m], *rng), TOL, ("left vs oracle", m))
    _same(sl[0], Oracle(p).ground_residual(*rng), TOL, "ground vs oracle")
