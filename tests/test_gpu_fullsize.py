"""HIP path vs the FP64 oracle at the full workload sizes, element by element, through the C-ABI.

* Config 1 (n_o=12, n_v=60, N_O=30, N_V=250, rank 600) over ALL 352 unique triples with no triple
  range, i.e. exactly the launch configuration the benchmark times (no triple filter): ground
  residual, right and left transform in FP64 (<= 1e-10) and in the reduced-precision forms
  (FP32 MFMA and six-product split-bf16 <= 1e-6, three-product split-bf16 <= 2e-4, see
  test_gpu_mixed.py for the error model), plus <L|A R> against the oracle's.
* Config 4 (core-shaped: n_o=8 with the core-like orbital 0, n_v=60, N_O=90, N_V=1100, rank 2500)
  on a range of unique triples that holds core-containing triples (degenerate and not) and
  all-valence ones: right and left transform with and without core-valence separation (two
  vectors per launch), and the transition densities.
* Config 3 (n_o=16, n_v=80, N_O=40, N_V=400, rank 1000): the right transform of four vectors in one
  launch (the differentiable forward) on the first and the last triples, and the left transform
  (its backward) on the last triples.
* The inactive-space sweep's first point (n_o=8, n_v=136, N_O=13, N_V=217, rank 690) on a range of
  unique triples: ground residual, right and left transform, densities.

The oracle's outputs for the config-1 all-triples case are computed once per session.
"""
import time

import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, pair_form_blocks, rel

pytestmark = pytest.mark.gpu
TOL = 1e-10
MIXTOL = {"fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 2e-4}


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
    return x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)


def _check(gpu, ref, tol=TOL, what=""):
    for k in ("x1", "x2_vVoo", "x2_vvoO"):
        g = _np(gpu[k])
        assert np.all(np.isfinite(g)), (what, k)
        assert rel(g, ref[k]) <= tol, (what, k, rel(g, ref[k]))
        assert maxrel(g, ref[k]) <= tol, (what, k, maxrel(g, ref[k]))


def _check_dens(got, ref, tol=TOL, what=""):
    Dm0, D0m, s = got
    for name, a, b in (("D_m0", Dm0, ref[0]), ("D_0m", D0m, ref[1])):
        a = _np(a)
        assert np.all(np.isfinite(a)), (what, name)
        assert rel(a, b) <= tol, (what, name, rel(a, b))
        assert maxrel(a, b) <= tol, (what, name, maxrel(a, b))
    assert abs(float(s) - ref[2]) <= tol * abs(ref[2]), (what, float(s), ref[2])


def _say(msg):
    print(msg, flush=True)


# --------------------------------------------------------------------- config 1, all triples
@pytest.fixture(scope="module")
def cfg1(lib):
    from oracle.oracle import Oracle
    p = I.make_config(1)
    orc = Oracle(p)
    R = I.right_vectors(p, 1)[0]
    L = I.left_vectors(p, 1)[0]
    w = float(I.omegas(1, 1)[0])
    t0 = time.time()
    ref = {"ground": orc.ground_residual(), "right": orc.right_transform(w, R), "left": orc.left_transform(w, L)}
    _say(f"config-1 oracle over all {orc.num_triples()} triples: {time.time() - t0:.1f} s")
    return p, lib.Ground(p), w, R, L, ref


def _cfg1_calls(lib, ws, g, w, R, L, prec):
    return {
        "ground": lib.ground_residual(ws, g, precision=prec),
        "right": lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], reuse_ground=True, precision=prec)[0],
        "left": lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], reuse_ground=True, precision=prec)[0],
    }


def test_config1_all_triples_fp64(lib, ws, cfg1):
    p, g, w, R, L, ref = cfg1
    _say("config 1, all triples, fp64")
    got = _cfg1_calls(lib, ws, g, w, R, L, "fp64")
    for k in got:
        _check(got[k], ref[k], TOL, f"config 1 {k}")


@pytest.mark.parametrize("prec", list(MIXTOL))
def test_config1_all_triples_mixed(lib, ws, cfg1, prec):
    p, g, w, R, L, ref = cfg1
    tol = MIXTOL[prec]
    _say(f"config 1, all triples, {prec}")
    got = _cfg1_calls(lib, ws, g, w, R, L, prec)
    for k in got:
        _check(got[k], ref[k], tol, f"config 1 {k} {prec}")
    # the scalar <L|A R> = G(L, rho) against the oracle's
    a = pair_form_blocks(p.dims, L, {k: _np(v) for k, v in got["right"].items()})
    b = pair_form_blocks(p.dims, L, ref["right"])
    assert abs(a - b) <= tol * abs(b), (prec, a, b)


# ------------------------------------------------------------------- config 4, core triples
def _canon(n_o):
    out = []
    for i in range(n_o):
        for j in range(i + 1):
            for k in range(j + 1):
                if not (i == j == k):
                    out.append((i, j, k))
    return out


CFG4_RANGE = (2, 7)  # (2,0,0) (2,1,0) (2,1,1) (2,2,0) (2,2,1): core orbital 0 in three of them


def test_config4_range_holds_core_and_valence_triples():
    t = _canon(8)[CFG4_RANGE[0]:CFG4_RANGE[1]]
    assert sum(1 for x in t if 0 in x) == 3 and sum(1 for x in t if 0 not in x) == 2, t
    assert any(len(set(x)) == 3 for x in t if 0 in x), t


@pytest.fixture(scope="module")
def cfg4(lib):
    p = I.make_config(4, with_density_blocks=True)
    return p, lib.Ground(p)


@pytest.mark.parametrize("cvs", [False, True], ids=["plain", "cvs"])
def test_config4_core_range_transforms(lib, ws, cfg4, cvs):
    """Two vectors per launch; vector 0 (plain) or vector 1 (CVS) against the oracle (batched
    launches equal single calls bit for bit, tested separately)."""
    from oracle.oracle import Oracle
    p, g = cfg4
    d = p.dims
    core = [1] + [0] * (d.N_O - 1)
    om = [float(x) for x in I.omegas(4, 2)]
    Rs, Ls = I.right_vectors(p, 2), I.left_vectors(p, 2)
    kw = dict(triple_range=CFG4_RANGE)
    if cvs:
        kw["cvs_core"] = core
    _say(f"config 4, triples {CFG4_RANGE}, cvs={cvs}")
    rho = lib.right_transform(ws, g, om, [lib.vec_to_device(v) for v in Rs], **kw)
    sig = lib.left_transform(ws, g, om, [lib.vec_to_device(v) for v in Ls], reuse_ground=True, **kw)
    m = 1 if cvs else 0
    orc = Oracle(p, cvs_core=core if cvs else None)
    t0 = time.time()
    _check(rho[m], orc.right_transform(om[m], Rs[m], *CFG4_RANGE), TOL, f"config 4 right cvs={cvs}")
    _check(sig[m], orc.left_transform(om[m], Ls[m], *CFG4_RANGE), TOL, f"config 4 left cvs={cvs}")
    _say(f"  oracle {time.time() - t0:.1f} s")


def test_config4_core_range_densities(lib, ws, cfg4):
    from oracle.oracle import Oracle
    p, g = cfg4
    om = [float(I.omegas(4, 1)[0])]
    L, R, lam = I.left_vectors(p, 1)[0], I.right_vectors(p, 1)[0], I.lambda_vector(p)
    _say(f"config 4 densities, triples {CFG4_RANGE}")
    got = lib.triples_densities(ws, g, om, [lib.vec_to_device(L)], [lib.vec_to_device(R)], lib.vec_to_device(lam),
                                p.t2_vVoO, p.t2_vVOo, triple_range=CFG4_RANGE)
    t0 = time.time()
    ref = Oracle(p).densities(om[0], L, R, lam, p.t2_vVoO, p.t2_vVOo, *CFG4_RANGE)
    _say(f"  oracle {time.time() - t0:.1f} s")
    _check_dens((got[0][0], got[1][0], got[2][0]), ref, TOL, "config 4 densities")


# --------------------------------------------------------------------- config 3, forward
@pytest.fixture(scope="module")
def cfg3(lib):
    from oracle.oracle import Oracle
    p = I.make_config(3)
    return p, lib.Ground(p), Oracle(p)


@pytest.mark.parametrize("rng", [(0, 3), (797, 800)])
def test_config3_forward_four_vectors(lib, ws, cfg3, rng):
    p, g, orc = cfg3
    assert orc.num_triples() == 800
    om = [float(x) for x in I.omegas(3, 4)]
    Rs = I.right_vectors(p, 4)
    _say(f"config 3 right transform, 4 vectors, triples {rng}")
    rho = lib.right_transform(ws, g, om, [lib.vec_to_device(v) for v in Rs], triple_range=rng)
    for m in (0, 3):
        _check(rho[m], orc.right_transform(om[m], Rs[m], *rng), TOL, f"config 3 right v{m} {rng}")


def test_config3_backward_last_triples(lib, ws, cfg3):
    p, g, orc = cfg3
    rng = (797, 800)
    om = [float(x) for x in I.omegas(3, 4)]
    Ls = I.left_vectors(p, 4)
    _say(f"config 3 left transform, 4 vectors, triples {rng}")
    sig = lib.left_transform(ws, g, om, [lib.vec_to_device(v) for v in Ls], triple_range=rng)
    _check(sig[2], orc.left_transform(om[2], Ls[2], *rng), TOL, "config 3 left v2")


# ------------------------------------------------------------------ inactive-space sweep point
def test_sweep_point_no8_nv136(lib, ws):
    from oracle.oracle import Oracle
    d = I.sweep_dims(0)
    assert (d.n_o, d.n_v, d.N_O, d.N_V) == (8, 136, 13, 217)
    rng = (77, 81)  # (7,0,0) (7,1,0) (7,1,1) (7,2,0)
    p = I.make_problem(d, I.config_seed(1), with_density_blocks=True)
    orc = Oracle(p)
    g = lib.Ground(p)
    w = 0.4
    R, L, lam = I.right_vectors(p, 1)[0], I.left_vectors(p, 1)[0], I.lambda_vector(p)
    _say(f"sweep point {d}, triples {rng}")
    _check(lib.ground_residual(ws, g, triple_range=rng), orc.ground_residual(*rng), TOL, "sweep ground")
    _check(lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, reuse_ground=True)[0],
           orc.right_transform(w, R, *rng), TOL, "sweep right")
    _check(lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], triple_range=rng, reuse_ground=True)[0],
           orc.left_transform(w, L, *rng), TOL, "sweep left")
    got = lib.triples_densities(ws, g, [w], [lib.vec_to_device(L)], [lib.vec_to_device(R)], lib.vec_to_device(lam),
                                p.t2_vVoO, p.t2_vVOo, triple_range=rng, reuse_ground=True)
    _check_dens((got[0][0], got[1][0], got[2][0]), orc.densities(w, L, R, lam, p.t2_vVoO, p.t2_vVOo, *rng), TOL,
                "sweep densities")


@pytest.mark.parametrize("d", [I.Dims(2, 136, 3, 140, 9), I.Dims(2, 160, 3, 163, 9)], ids=str)
def test_wide_virtual_space_transforms(lib, ws, d):
    """n_v = 136 and 160 (ragged 16-wide sub-cube grids, orbit form of the contravariant pass):
    right and left transform of every triple against the oracle."""
    from oracle.oracle import Oracle
    p = I.make_problem(d, 41)
    orc = Oracle(p)
    g = lib.Ground(p)
    R, L = I.right_vectors(p, 1)[0], I.left_vectors(p, 1)[0]
    _say(f"wide virtual space {d}")
    _check(lib.right_transform(ws, g, [0.45], [lib.vec_to_device(R)])[0], orc.right_transform(0.45, R), TOL,
           "wide right")
    _check(lib.left_transform(ws, g, [0.45], [lib.vec_to_device(L)], reuse_ground=True)[0],
           orc.left_transform(0.45, L), TOL, "wide left")

