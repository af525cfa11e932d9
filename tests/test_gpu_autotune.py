"""Launch-shape tuning of the triples path.

Every value of every knob of the workspace tuning (d-contraction grid, split-K of the N_V-wide
back-contractions, tile of the N_O-wide back-contractions, contravariant pass form, vector
group size) must give the default's results to rounding; the autotuner must pick, apply and
cache a setting whose transforms still match the oracle at the FP64 bar.
"""
import json

import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import rel

pytestmark = pytest.mark.gpu
TOL = 1e-10
# 16 divides n_v: the default is the orbit form, contra_form 1 the per-sub-cube one
D = I.Dims(4, 32, 6, 47, 19)


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


def _host(lib, outs):
    return [lib.to_numpy(o) for o in outs]


def _same(a, b, tol, what):
    for m in range(len(b)):
        for k in b[m]:
            assert rel(a[m][k], b[m][k]) <= tol, (what, m, k, rel(a[m][k], b[m][k]))


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_every_knob_value_gives_the_default_result(lib, ws, prec):
    from paper_2202_08612_amd.autotune import CANDIDATES
    p = I.make_problem(D, 5)
    g = lib.Ground(p)
    R = [lib.vec_to_device(v) for v in I.right_vectors(p, 3)]
    L = [lib.vec_to_device(v) for v in I.left_vectors(p, 3)]
    om = I.omegas(False, 3)
    ws.set_tuning(None)
    r0 = _host(lib, lib.right_transform(ws, g, om, R, precision=prec))
    l0 = _host(lib, lib.left_transform(ws, g, om, L, reuse_ground=True, precision=prec))
    try:
        for knob, vals in CANDIDATES.items():
            for v in vals:
                if v == 0:
                    continue
                ws.set_tuning({knob: v})
                assert ws.get_tuning()[knob] == v
                r = _host(lib, lib.right_transform(ws, g, om, R, reuse_ground=True, precision=prec))
                l = _host(lib, lib.left_transform(ws, g, om, L, reuse_ground=True, precision=prec))
                _same(r, r0, 1e-12, f"right {knob}={v}")
                _same(l, l0, 1e-12, f"left {knob}={v}")
    finally:
        ws.set_tuning(None)


def test_autotune_picks_caches_and_matches_oracle(lib, tmp_path):
    from oracle.oracle import Oracle
    from paper_2202_08612_amd.autotune import autotune
    p = I.make_problem(D, 6)
    orc = Oracle(p)
    g = lib.Ground(p)
    Rh, Lh = I.right_vectors(p, 2), I.left_vectors(p, 2)
    R = [lib.vec_to_device(v) for v in Rh]
    L = [lib.vec_to_device(v) for v in Lh]
    om = I.omegas(False, 2)
    cache = str(tmp_path / "autotune.json")
    w1 = lib.Workspace(0)
    try:
        tuning, rep = autotune(w1, g, om, R, L, cache=cache, reps=1)
        assert not rep["cached"]
        assert set(tuning) == set(lib.TUNING_FIELDS)
        assert w1.get_tuning() == tuning
        assert len(rep["trials"]) >= 10 and rep["ms"] <= rep["default_ms"]
        with open(cache) as f:
            db = json.load(f)
        assert db[rep["key"]]["tuning"] == tuning
    finally:
        w1.close()
    w2 = lib.Workspace(0)
    try:
        tuning2, rep2 = autotune(w2, g, om, R, L, cache=cache)
        assert rep2["cached"] and tuning2 == tuning and w2.get_tuning() == tuning
        r = _host(lib, lib.right_transform(w2, g, om, R))
        l = _host(lib, lib.left_transform(w2, g, om, L, reuse_ground=True))
        for m in range(2):
            ref_r = orc.right_transform(om[m], Rh[m])
            ref_l = orc.left_transform(om[m], Lh[m])
            for k in ref_r:
                assert rel(r[m][k], ref_r[k]) <= TOL, ("right", m, k, rel(r[m][k], ref_r[k]))
                assert rel(l[m][k], ref_l[k]) <= TOL, ("left", m, k, rel(l[m][k], ref_l[k]))
    finally:
        w2.close()


@pytest.mark.parametrize("dims", [I.Dims(3, 20, 5, 30, 11), I.Dims(5, 17, 7, 37, 23)], ids=str)
def test_orbit_pass_on_ragged_sub_cubes(lib, ws, dims):
    """The orbit form of the contravariant pass (contra_form 2) on a virtual space that 16 does
    not divide: the oracle's results at the FP64 bar, and the per-sub-cube form's to rounding."""
    from oracle.oracle import Oracle
    p = I.make_problem(dims, 9)
    orc = Oracle(p)
    g = lib.Ground(p)
    Rh, Lh = I.right_vectors(p, 2), I.left_vectors(p, 2)
    R = [lib.vec_to_device(v) for v in Rh]
    L = [lib.vec_to_device(v) for v in Lh]
    om = I.omegas(False, 2)
    out = {}
    try:
        for form in (1, 2):
            ws.set_tuning({"contra_form": form})
            out[form] = (_host(lib, lib.right_transform(ws, g, om, R)),
                         _host(lib, lib.left_transform(ws, g, om, L, reuse_ground=True)),
                         lib.to_numpy(lib.ground_residual(ws, g, reuse_ground=True)))
    finally:
        ws.set_tuning(None)
    _same(out[2][0], out[1][0], 1e-12, "right")
    _same(out[2][1], out[1][1], 1e-12, "left")
    _same([out[2][2]], [out[1][2]], 1e-12, "ground")
    for m in range(2):
        ref_r = orc.right_transform(om[m], Rh[m])
        ref_l = orc.left_transform(om[m], Lh[m])
        for k in ref_r:
            assert rel(out[2][0][m][k], ref_r[k]) <= TOL, ("right", m, k)
            assert rel(out[2][1][m][k], ref_l[k]) <= TOL, ("left", m, k)
