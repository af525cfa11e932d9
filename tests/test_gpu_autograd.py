"""Differentiation: paper_2202_08612_amd.autograd.RightTransform (forward: right transform of the
symmetrised R; backward: the left transform through the pairing maps).  Checked by
  * the library maps against their numpy definitions (tests/helpers.py, pinned on the CPU),
  * the vector-Jacobian identity <g, J R> = <grad_R, R> (the adjoint identity in elementwise form),
  * central finite differences with step 1e-6 in FP64 along inconsistent directions,
  * the oracle: grad_R = LEFT_TO_GRAD(oracle left transform of GRAD_TO_LEFT(g)),
at small shapes and at the full config-3 shape (n_o=16, n_v=80, N_O=40, N_V=400, rank 1000),
where the 4 trial vectors also go through one right-transform call.
"""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import euclid, map_grad_to_left, map_left_to_grad, map_symmetrize, maxrel, rel

pytestmark = pytest.mark.gpu
SHAPES = [I.Dims(3, 4, 4, 6, 10), I.Dims(5, 17, 7, 37, 23)]


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


def _rand(d, rng, scale=1.0):
    return {"x1": scale * rng.standard_normal((d.N_V, d.N_O)),
            "x2_vVoo": scale * rng.standard_normal((d.n_v, d.N_V, d.n_o, d.n_o)),
            "x2_vvoO": scale * rng.standard_normal((d.n_v, d.n_v, d.n_o, d.N_O))}


def _np(v):
    return {k: x.detach().cpu().numpy() for k, x in v.items()}


def _leaf(lib, v):
    import torch
    return {k: x.clone().requires_grad_(True) for k, x in lib.vec_to_device(v).items()}


def _fwd_bwd(lib, ws, g_dev, omega, R, gout, precision="fp64"):
    from paper_2202_08612_amd import autograd as AD
    import torch
    x = _leaf(lib, R)
    rho = AD.right_transform(ws, g_dev, omega, x["x1"], x["x2_vVoo"], x["x2_vvoO"], precision=precision)
    go = lib.vec_to_device(gout)
    loss = sum((r * go[k]).sum() for r, k in zip(rho, ("x1", "x2_vVoo", "x2_vvoO")))
    loss.backward()
    grad = {k: x[k].grad.detach().cpu().numpy() for k in x}
    return float(loss), {k: r.detach().cpu().numpy() for r, k in zip(rho, ("x1", "x2_vVoo", "x2_vvoO"))}, grad


@pytest.mark.parametrize("d", SHAPES, ids=str)
def test_vec_map_matches_numpy(lib, ws, d):
    p = I.make_problem(d, 5)
    g = lib.Ground(p)
    rng = np.random.default_rng(4)
    x = _rand(d, rng)
    S = I.trial_vector(9, d, 64)
    for mode, fn, inp in ((lib.MAP_SYMMETRIZE, map_symmetrize, x), (lib.MAP_GRAD_TO_LEFT, map_grad_to_left, x),
                          (lib.MAP_LEFT_TO_GRAD, map_left_to_grad, S)):
        got = _np(lib.vec_map(ws, g, mode, [lib.vec_to_device(inp)])[0])
        ref = fn(d, inp)
        for k in ref:
            assert np.allclose(got[k], ref[k], rtol=1e-14, atol=1e-14), (mode, k)


@pytest.mark.parametrize("d", SHAPES, ids=str)
def test_autograd_vjp_fd_and_oracle(lib, ws, d):
    from oracle.oracle import Oracle
    p = I.make_problem(d, 21)
    g = lib.Ground(p)
    rng = np.random.default_rng(8)
    R = I.trial_vector(21, d, 0)
    gout = _rand(d, rng)
    w = 0.45
    loss, rho, grad = _fwd_bwd(lib, ws, g, w, R, gout)
    # vector-Jacobian identity (R consistent, rho linear in R)
    assert abs(euclid(grad, R) - loss) <= 1e-11 * abs(loss), (euclid(grad, R), loss)
    # finite differences along an inconsistent direction, step 1e-6
    dR = _rand(d, rng)
    h = 1e-6
    lp, _, _ = _fwd_bwd(lib, ws, g, w, {k: R[k] + h * dR[k] for k in R}, gout)
    lm, _, _ = _fwd_bwd(lib, ws, g, w, {k: R[k] - h * dR[k] for k in R}, gout)
    fd = (lp - lm) / (2 * h)
    an = euclid(grad, dR)
    assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-300), (fd, an)
    # oracle
    orc = Oracle(p)
    ref_rho = orc.right_transform(w, R)
    for k in rho:
        assert rel(rho[k], ref_rho[k]) <= 1e-10
    ref_grad = map_left_to_grad(d, orc.left_transform(w, map_grad_to_left(d, gout)))
    for k in grad:
        assert rel(grad[k], ref_grad[k]) <= 1e-10, (k, rel(grad[k], ref_grad[k]))
        assert maxrel(grad[k], ref_grad[k]) <= 1e-10, (k, maxrel(grad[k], ref_grad[k]))


def test_config3_batched_vectors_adjoint_fd_oracle(lib, ws):
    """Config 3 at full size: 4 right vectors in one call equal 4 single calls; for each vector the
    vector-Jacobian identity holds; FD (step 1e-6) for one vector; the mixed form beside FP64;
    backward against the oracle on the first two unique triples."""
    from paper_2202_08612_amd import autograd as AD
    from oracle.oracle import Oracle
    import torch
    p = I.make_config(3)
    d = p.dims
    g = lib.Ground(p)
    Rs = I.right_vectors(p, 4)
    om = [float(x) for x in I.omegas(3, 4)]
    Rd = [lib.vec_to_device(r) for r in Rs]
    batched = lib.right_transform(ws, g, om, Rd)
    for m in range(4):
        single = lib.right_transform(ws, g, [om[m]], [Rd[m]], reuse_ground=True)[0]
        for k in single:
            assert torch.equal(single[k], batched[m][k]), (m, k)
    rng = np.random.default_rng(3)
    gout = _rand(d, rng, 1e-3)
    for m in range(4):
        loss, _, grad = _fwd_bwd(lib, ws, g, om[m], Rs[m], gout)
        assert abs(euclid(grad, Rs[m]) - loss) <= 1e-10 * abs(loss), (m, euclid(grad, Rs[m]), loss)
    dR = _rand(d, rng, 1e-2)
    h = 1e-6
    lp, _, _ = _fwd_bwd(lib, ws, g, om[0], {k: Rs[0][k] + h * dR[k] for k in dR}, gout)
    lm, _, _ = _fwd_bwd(lib, ws, g, om[0], {k: Rs[0][k] - h * dR[k] for k in dR}, gout)
    loss, _, grad = _fwd_bwd(lib, ws, g, om[0], Rs[0], gout)
    an = euclid(grad, dR)
    assert abs((lp - lm) / (2 * h) - an) <= 1e-6 * abs(an)
    # mixed beside FP64
    lmx, rmx, gmx = _fwd_bwd(lib, ws, g, om[0], Rs[0], gout, precision="fp32")
    assert abs(lmx - loss) <= 1e-6 * abs(loss)
    for k in gmx:
        assert rel(gmx[k], grad[k]) <= 1e-6, (k, rel(gmx[k], grad[k]))
    # backward against the oracle on a triple range
    rng_t = (0, 2)
    gl = lib.vec_to_device(map_grad_to_left(d, gout))
    sig = _np(lib.left_transform(ws, g, [om[0]], [gl], triple_range=rng_t, reuse_ground=True)[0])
    ref = Oracle(p).left_transform(om[0], map_grad_to_left(d, gout), *rng_t)
    for k in sig:
        assert rel(sig[k], ref[k]) <= 1e-10, (k, rel(sig[k], ref[k]))


@pytest.mark.parametrize("case", ["tiny-full", "config0-fast"])
def test_gradcheck(lib, ws, case):
    """torch.autograd.gradcheck of the right transform: the full numerical Jacobian (central
    differences, FP64) against the backward at a tiny shape, and torch's fast mode (random
    projections) at the config-0 shape."""
    import torch
    from paper_2202_08612_amd import autograd as AD
    d = I.Dims(2, 3, 3, 4, 5) if case == "tiny-full" else I.CONFIGS[0]["dims"]
    p = I.make_problem(d, 41)
    g = lib.Ground(p)
    lib.ground_residual(ws, g)  # prepares the ground-state blocks that the forward reuses
    R = _leaf(lib, _rand(d, np.random.default_rng(3)))

    def f(x1, x2a, x2b):
        return AD.right_transform(ws, g, 0.43, x1, x2a, x2b)

    assert torch.autograd.gradcheck(f, (R["x1"], R["x2_vVoo"], R["x2_vvoO"]), eps=1e-6, atol=1e-7, rtol=1e-5,
                                    fast_mode=(case != "tiny-full"))
