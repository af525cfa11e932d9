"""Mixed-precision path (precision="fp32"): the d-contractions run as FP32 MFMA with FP32
accumulation on rounded copies of the FP64 operands; the occupied term, the permutations,
the denominators, the back-contractions and every output stay FP64.  Every result is checked
against the FP64 oracle at 1e-6 relative (norm-wise and max-abs over max-abs), and against
the FP64 GPU path to show that the rounded path really ran.
"""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, pair_form_blocks, rel

pytestmark = pytest.mark.gpu
MIXTOL = 1e-6
SHAPES = [I.CONFIGS[0]["dims"], I.Dims(5, 17, 7, 37, 23), I.Dims(6, 9, 6, 140, 33)]


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_08612_amd import mlcc3
    return mlcc3


@pytest.fixture(scope="module")
def ws(lib):
    w = lib.Workspace(0)
    yield w
    w.close()


def _np(x):
    return x.detach().cpu().numpy() if hasattr(x, "detach") else x


def _check_mixed(mixed, ref, fp64):
    for k in ("x1", "x2_vVoo", "x2_vvoO"):
        m, r, f = _np(mixed[k]), ref[k], _np(fp64[k])
        assert np.all(np.isfinite(m)), k
        assert rel(m, r) <= MIXTOL, (k, rel(m, r))
        assert maxrel(m, r) <= MIXTOL, (k, maxrel(m, r))
        if np.linalg.norm(r) > 0:
            assert rel(m, f) > 1e-13, (k, "mixed result equals the FP64 one")


def _setup(lib, d, seed):
    from oracle.oracle import Oracle
    p = I.make_problem(d, seed)
    return p, Oracle(p), lib.Ground(p)


@pytest.mark.parametrize("d", SHAPES, ids=lambda d: f"{d.n_o}-{d.n_v}-{d.N_O}-{d.N_V}-{d.n_chol}")
def test_mixed_ground_right_left(lib, ws, d):
    p, orc, g = _setup(lib, d, 31)
    _check_mixed(lib.ground_residual(ws, g, precision="fp32"), orc.ground_residual(), lib.ground_residual(ws, g))
    R = I.right_vectors(p, 2)
    L = I.left_vectors(p, 2)
    om = I.omegas(False, 2)
    Rd = [lib.vec_to_device(r) for r in R]
    Ld = [lib.vec_to_device(v) for v in L]
    rm = lib.right_transform(ws, g, om, Rd, precision="fp32")
    r64 = lib.right_transform(ws, g, om, Rd)
    lm = lib.left_transform(ws, g, om, Ld, precision="fp32")
    l64 = lib.left_transform(ws, g, om, Ld)
    for m in range(2):
        _check_mixed(rm[m], orc.right_transform(om[m], R[m]), r64[m])
        _check_mixed(lm[m], orc.left_transform(om[m], L[m]), l64[m])


@pytest.mark.parametrize("rng", [(0, 4), (347, 352)])
def test_mixed_full_shape_subsets(lib, ws, rng):
    from oracle.oracle import Oracle
    p = I.make_config(1)
    orc = Oracle(p)
    g = lib.Ground(p)
    R = I.right_vectors(p, 1)[0]
    L = I.left_vectors(p, 1)[0]
    w = I.omegas(1, 1)[0]
    rm = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, precision="fp32")[0]
    r64 = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, reuse_ground=True)[0]
    _check_mixed(rm, orc.right_transform(w, R, *rng), r64)
    lm = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], triple_range=rng, reuse_ground=True,
                            precision="fp32")[0]
    l64 = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], triple_range=rng, reuse_ground=True)[0]
    _check_mixed(lm, orc.left_transform(w, L, *rng), l64)


def test_mixed_pairing_full_config1(lib, ws):
    """<L|A R> with the mixed right transform against the FP64 path (itself within 1e-10 of the
    oracle), config 1, all triples."""
    p = I.make_config(1)
    d = p.dims
    g = lib.Ground(p)
    R = I.right_vectors(p, 1)[0]
    L = I.left_vectors(p, 1)[0]
    w = I.omegas(1, 1)[0]
    r64 = lib.to_numpy(lib.right_transform(ws, g, [w], [lib.vec_to_device(R)])[0])
    rmx = lib.to_numpy(lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], reuse_ground=True,
                                           precision="fp32")[0])
    a, b = pair_form_blocks(d, L, r64), pair_form_blocks(d, L, rmx)
    assert abs(a - b) <= MIXTOL * abs(a), (a, b)
    for k in r64:
        assert rel(rmx[k], r64[k]) <= MIXTOL, (k, rel(rmx[k], r64[k]))


def test_mixed_densities(lib, ws):
    from oracle.oracle import Oracle
    d = I.Dims(4, 6, 5, 11, 13)
    p = I.make_problem(d, 8, with_density_blocks=True)
    orc = Oracle(p)
    g = lib.Ground(p)
    L = I.left_vectors(p, 1)
    R = I.right_vectors(p, 1)
    lam = I.lambda_vector(p)
    om = I.omegas(False, 1)
    got = lib.triples_densities(ws, g, om, [lib.vec_to_device(v) for v in L], [lib.vec_to_device(v) for v in R],
                                lib.vec_to_device(lam), p.t2_vVoO, p.t2_vVOo, precision="fp32")
    ref = orc.densities(om[0], L[0], R[0], lam, p.t2_vVoO, p.t2_vVOo)
    for a, b in ((got[0][0], ref[0]), (got[1][0], ref[1])):
        a = _np(a)
        assert rel(a, b) <= MIXTOL and maxrel(a, b) <= MIXTOL, (rel(a, b), maxrel(a, b))
    assert abs(float(got[2][0]) - ref[2]) <= MIXTOL * abs(ref[2])
