"""Mixed-precision paths: the d-contractions run as FP32 MFMA on rounded copies of the FP64
operands (precision="fp32"), or as split-bf16 MFMA products (precision="bf16x6": three bf16
planes per operand, six products; "bf16x3": two planes, three products).  In the reduced forms
the contravariant triples blocks are stored in FP32, the occupied term of each intermediate and
the N_O-wide back-contractions run as FP32 MFMA products, and the split-bf16 forms also run the
N_V-wide back-contractions (and the Bq intermediate of the left transform) in split-bf16
products; the permutations, the denominators and every output stay FP64.  Every result is
checked against the FP64 oracle, norm-wise and max-abs over max-abs, and against the FP64 GPU
path to show that the reduced-precision path really ran.

Tolerances: fp32 and bf16x6 at 1e-6.  bf16x3 drops the lo*lo product and the remainder beyond
two bf16 planes: per product about 3 * 2^-18 = 1.1e-5 relative to |x y| (each plane keeps 8
significant bits, so |x - hi - lo| <= 2^-18 |x|).  The outputs are linear in the
d-contraction results, whose sums of random-sign products lose up to about one more order of
magnitude against their norms, so bf16x3 is held to 2e-4 and expected NOT to meet 1e-6.
"""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, pair_form_blocks, rel

pytestmark = pytest.mark.gpu
MIXTOL = 1e-6
TOL = {"fp32": MIXTOL, "bf16x6": MIXTOL, "bf16x3": 2e-4}
PRECS = list(TOL)
# N_V >= 96 takes the split-bf16 N_V-wide products (n_v = 9: element loads of the staged operand;
# n_v = 12: its 16-byte loads)
SHAPES = [I.CONFIGS[0]["dims"], I.Dims(5, 17, 7, 37, 23), I.Dims(6, 9, 6, 140, 33), I.Dims(4, 12, 5, 100, 24)]


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


def _check_mixed(mixed, ref, fp64, tol=MIXTOL):
    for k in ("x1", "x2_vVoo", "x2_vvoO"):
        m, r, f = _np(mixed[k]), ref[k], _np(fp64[k])
        assert np.all(np.isfinite(m)), k
        assert rel(m, r) <= tol, (k, rel(m, r))
        assert maxrel(m, r) <= tol, (k, maxrel(m, r))
        if np.linalg.norm(r) > 0:
            assert rel(m, f) > 1e-13, (k, "mixed result equals the FP64 one")


def _setup(lib, d, seed):
    from oracle.oracle import Oracle
    p = I.make_problem(d, seed)
    return p, Oracle(p), lib.Ground(p)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d", SHAPES, ids=lambda d: f"{d.n_o}-{d.n_v}-{d.N_O}-{d.N_V}-{d.n_chol}")
def test_mixed_ground_right_left(lib, ws, d, prec):
    tol = TOL[prec]
    p, orc, g = _setup(lib, d, 31)
    _check_mixed(lib.ground_residual(ws, g, precision=prec), orc.ground_residual(), lib.ground_residual(ws, g), tol)
    R = I.right_vectors(p, 2)
    L = I.left_vectors(p, 2)
    om = I.omegas(False, 2)
    Rd = [lib.vec_to_device(r) for r in R]
    Ld = [lib.vec_to_device(v) for v in L]
    rm = lib.right_transform(ws, g, om, Rd, precision=prec)
    r64 = lib.right_transform(ws, g, om, Rd)
    lm = lib.left_transform(ws, g, om, Ld, precision=prec)
    l64 = lib.left_transform(ws, g, om, Ld)
    for m in range(2):
        _check_mixed(rm[m], orc.right_transform(om[m], R[m]), r64[m], tol)
        _check_mixed(lm[m], orc.left_transform(om[m], L[m]), l64[m], tol)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("rng", [(0, 4), (347, 352)])
def test_mixed_full_shape_subsets(lib, ws, rng, prec):
    from oracle.oracle import Oracle
    p = I.make_config(1)
    orc = Oracle(p)
    g = lib.Ground(p)
    R = I.right_vectors(p, 1)[0]
    L = I.left_vectors(p, 1)[0]
    w = I.omegas(1, 1)[0]
    rm = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, precision=prec)[0]
    r64 = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, reuse_ground=True)[0]
    _check_mixed(rm, orc.right_transform(w, R, *rng), r64, TOL[prec])
    lm = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], triple_range=rng, reuse_ground=True,
                            precision=prec)[0]
    l64 = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], triple_range=rng, reuse_ground=True)[0]
    _check_mixed(lm, orc.left_transform(w, L, *rng), l64, TOL[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_pairing_full_config1(lib, ws, prec):
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
                                           precision=prec)[0])
    a, b = pair_form_blocks(d, L, r64), pair_form_blocks(d, L, rmx)
    assert abs(a - b) <= TOL[prec] * abs(a), (a, b)
    for k in r64:
        assert rel(rmx[k], r64[k]) <= TOL[prec], (k, rel(rmx[k], r64[k]))


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_densities(lib, ws, prec):
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
                                lib.vec_to_device(lam), p.t2_vVoO, p.t2_vVOo, precision=prec)
    ref = orc.densities(om[0], L[0], R[0], lam, p.t2_vVoO, p.t2_vVOo)
    tol = TOL[prec]
    for a, b in ((got[0][0], ref[0]), (got[1][0], ref[1])):
        a = _np(a)
        assert rel(a, b) <= tol and maxrel(a, b) <= tol, (rel(a, b), maxrel(a, b))
    assert abs(float(got[2][0]) - ref[2]) <= tol * abs(ref[2])
