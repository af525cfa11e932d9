"""The paper's guanine 15/150 active space (Results section, Table t:Gua_1state) on one GPU.

N_O=39, N_V=263, rank 906, n_o=15, n_v=150: each ordered-triple buffer holds n_o^3 n_v^3 doubles
(91 GB; element offsets beyond 2^31), and a transform's workspace is about 196 GiB.  Three unique
triples, (2,1,0) (2,1,1) (2,2,0): ground residual, and right and left transform with core-valence
separation (core orbital 0), against the FP64 oracle at 1e-10.  In a module of its own so that
the earlier modules' workspaces are released before it allocates.
"""
import gc
import time

import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, rel

pytestmark = pytest.mark.gpu
TOL = 1e-10
NEED = 200 * 2**30


def _canon(n_o):
    return [(i, j, k) for i in range(n_o) for j in range(i + 1) for k in range(j + 1) if not (i == j == k)]


def _check(got, ref, what):
    for k in ("x1", "x2_vVoo", "x2_vvoO"):
        g = got[k]
        assert np.all(np.isfinite(g)), (what, k)
        assert rel(g, ref[k]) <= TOL, (what, k, rel(g, ref[k]))
        assert maxrel(g, ref[k]) <= TOL, (what, k, maxrel(g, ref[k]))


def test_guanine_15_150_core_range():
    import torch
    assert torch.cuda.is_available()
    from oracle.oracle import Oracle
    from paper_2202_08612_amd import mlcc3 as lib
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info(0)
    if total < NEED:
        pytest.skip(f"device memory {total / 2**30:.0f} GiB < {NEED / 2**30:.0f} GiB")
    assert free >= NEED, f"only {free / 2**30:.0f} GiB free of {total / 2**30:.0f} GiB before the 15/150 case"
    d = I.Dims(15, 150, 39, 263, 906)
    rng = (3, 6)
    assert _canon(15)[rng[0]:rng[1]] == [(2, 1, 0), (2, 1, 1), (2, 2, 0)]
    p = I.make_problem(d, 20220217 + 200 + 15, core=True)
    core = [1] + [0] * (d.N_O - 1)
    w = float(I.omegas(True, 1)[0])
    R, L = I.right_vectors(p, 1)[0], I.left_vectors(p, 1)[0]
    ws = lib.Workspace(0)
    try:
        g = lib.Ground(p)
        print(f"guanine 15/150, triples {rng}", flush=True)
        om = lib.ground_residual(ws, g, triple_range=rng)
        rho = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, reuse_ground=True,
                                  cvs_core=core)[0]
        sig = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], triple_range=rng, reuse_ground=True,
                                 cvs_core=core)[0]
        got = [{k: x[k].detach().cpu().numpy() for k in x} for x in (om, rho, sig)]
        print(f"  workspace {ws.bytes() / 2**30:.1f} GiB", flush=True)
    finally:
        ws.close()
    t0 = time.time()
    _check(got[0], Oracle(p).ground_residual(*rng), "15/150 ground")
    orc = Oracle(p, cvs_core=core)
    _check(got[1], orc.right_transform(w, R, *rng), "15/150 right cvs")
    _check(got[2], orc.left_transform(w, L, *rng), "15/150 left cvs")
    print(f"  oracle {time.time() - t0:.1f} s", flush=True)


def test_guanine_20_200_occupied_slabs():
    """20/200 (512 GB per ordered-triple buffer): the calls run in occupied slabs chosen from the
    device memory; ground residual and right transform with core-valence separation on two
    unique triples, (2,1,0) (2,1,1), against the oracle."""
    import torch
    from oracle.oracle import Oracle
    from paper_2202_08612_amd import mlcc3 as lib
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info(0)
    if total < NEED:
        pytest.skip(f"device memory {total / 2**30:.0f} GiB < {NEED / 2**30:.0f} GiB")
    d = I.Dims(20, 200, 39, 263, 906)
    rng = (3, 5)
    assert _canon(20)[rng[0]:rng[1]] == [(2, 1, 0), (2, 1, 1)]
    p = I.make_problem(d, 20220217 + 200 + 20, core=True)
    core = [1] + [0] * (d.N_O - 1)
    w = float(I.omegas(True, 1)[0])
    R = I.right_vectors(p, 1)[0]
    ws = lib.Workspace(0)
    try:
        g = lib.Ground(p)
        print(f"guanine 20/200, triples {rng}", flush=True)
        om = lib.ground_residual(ws, g, triple_range=rng)
        rho = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], triple_range=rng, reuse_ground=True,
                                  cvs_core=core)[0]
        got = [{k: x[k].detach().cpu().numpy() for k in x} for x in (om, rho)]
        used = ws.bytes()
        print(f"  workspace {used / 2**30:.1f} GiB of {total / 2**30:.0f} GiB", flush=True)
    finally:
        ws.close()
    assert used < 0.9 * total
    t0 = time.time()
    _check(got[0], Oracle(p).ground_residual(*rng), "20/200 ground")
    _check(got[1], Oracle(p, cvs_core=core).right_transform(w, R, *rng), "20/200 right cvs")
    print(f"  oracle {time.time() - t0:.1f} s", flush=True)
