"""The ground residual entry point that allocates nothing (mlcc3_ground_residual_noalloc) against
the workspace entry point mlcc3_ground_residual and the FP64 oracle, through the C-ABI: two calls
in a row on the fixed scratch, the second with a smaller problem (the scratch then holds the
first call's larger contents), plus a triple range and the size rejection."""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_08612_amd import mlcc3
    return mlcc3


def _np(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def _poison(out):
    for v in out.values():
        v.fill_(float("nan"))
    return out


@pytest.mark.parametrize("rng", [None, (3, 11)], ids=["all", "range"])
def test_noalloc_equals_workspace_call_twice(lib, rng):
    from oracle.oracle import Oracle
    ws = lib.Workspace(0)
    kw = {} if rng is None else {"triple_range": rng}
    # larger problem first, then a smaller one on the same scratch
    for d, seed in ((I.Dims(6, 24, 10, 48, 120), 71), (I.Dims(4, 12, 6, 20, 60), 72)):
        print(f"noalloc ground residual {d} range={rng}", flush=True)
        p = I.make_problem(d, seed)
        g = lib.Ground(p)
        ref = _np(lib.ground_residual(ws, g, **kw))
        got = _np(lib.ground_residual_noalloc(g, _poison(lib.empty_out(d)), **kw))
        orc = Oracle(p).ground_residual(*(rng if rng else (0, -1)))
        for k in ref:
            assert np.all(np.isfinite(got[k])), k
            assert rel(got[k], ref[k]) <= 1e-13 and maxrel(got[k], ref[k]) <= 1e-13, (k, rel(got[k], ref[k]))
            assert rel(got[k], orc[k]) <= 1e-10 and maxrel(got[k], orc[k]) <= 1e-10, (k, rel(got[k], orc[k]))
    ws.close()


def test_noalloc_rejects_problems_beyond_its_scratch(lib):
    d = I.CONFIGS[1]["dims"]
    p = I.make_problem(d, 5)
    g = lib.Ground(p)
    out = lib.empty_out(d)
    with pytest.raises(lib.MLCC3Error) as e:
        lib.ground_residual_noalloc(g, out)
    assert e.value.code == -1 and "bytes of scratch" in str(e.value)
    assert lib.noalloc_scratch_bytes() == 128 << 20
