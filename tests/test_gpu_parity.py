"""HIP path vs the FP64 oracle, element by element, through the C-ABI (FP64: <= 1e-10 relative).

Sizes span several GEMM tiles and ragged tails; the full config-1 shape is checked
on subsets of the triple list (partial sums are part of the ABI) and by properties
that hold at any size (range additivity, adjoint identity, linearity).
"""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import maxrel, pair_form_blocks, rel

pytestmark = pytest.mark.gpu
TOL = 1e-10

SMALL = [I.Dims(3, 4, 4, 6, 10), I.Dims(4, 5, 5, 7, 12), I.CONFIGS[0]["dims"], I.Dims(4, 6, 4, 6, 9),
         I.Dims(2, 3, 4, 5, 8), I.Dims(5, 17, 7, 37, 23), I.Dims(6, 9, 6, 140, 33), I.Dims(4, 16, 5, 23, 17),
         I.Dims(3, 32, 4, 41, 11), I.Dims(17, 3, 18, 5, 7)]  # the last: n_o > 16 (generic occupied Gram blocks)


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


def _check(gpu, ref, tol=TOL):
    for k in ("x1", "x2_vVoo", "x2_vvoO"):
        g = gpu[k].detach().cpu().numpy() if hasattr(gpu[k], "detach") else gpu[k]
        assert np.all(np.isfinite(g)), k
        assert rel(g, ref[k]) <= tol, (k, rel(g, ref[k]))
        assert maxrel(g, ref[k]) <= tol, (k, maxrel(g, ref[k]))


def _setup(lib, d, seed):
    from oracle.oracle import Oracle
    p = I.make_problem(d, seed)
    return p, Oracle(p), lib.Ground(p)


@pytest.mark.parametrize("d", SMALL, ids=lambda d: f"{d.n_o}-{d.n_v}-{d.N_O}-{d.N_V}-{d.n_chol}")
def test_ground_residual(lib, ws, d):
    p, orc, g = _setup(lib, d, 1234)
    _check(lib.ground_residual(ws, g), orc.ground_residual())


@pytest.mark.parametrize("d", SMALL, ids=lambda d: f"{d.n_o}-{d.n_v}-{d.N_O}-{d.N_V}-{d.n_chol}")
def test_right_transform(lib, ws, d):
    p, orc, g = _setup(lib, d, 99)
    R = I.right_vectors(p, 2)
    om = I.omegas(False, 2)
    out = lib.right_transform(ws, g, om, [lib.vec_to_device(r) for r in R])
    for m in range(2):
        _check(out[m], orc.right_transform(om[m], R[m]))


def test_triple_range_and_reuse(lib, ws):
    d = I.Dims(5, 7, 6, 15, 11)
    p, orc, g = _setup(lib, d, 5)
    R = I.right_vectors(p, 1)[0]
    nt = lib.num_triples(d.n_o)
    for (a, b) in ((0, 1), (3, 9), (9, nt), (4, 4)):
        out = lib.right_transform(ws, g, [0.45], [lib.vec_to_device(R)], triple_range=(a, b),
                                  reuse_ground=True)[0]
        _check(out, orc.right_transform(0.45, R, a, b))


def test_ccsd_reductions_give_zero(lib, ws):
    for d in (I.Dims(1, 5, 4, 9, 7), I.Dims(4, 1, 5, 9, 7), I.Dims(0, 3, 3, 5, 4)):
        p = I.make_problem(d, 3)
        g = lib.Ground(p)
        out = lib.ground_residual(ws, g)
        assert all(v.numel() == 0 or float(v.abs().max()) == 0.0 for v in out.values())
        R = lib.vec_to_device(I.right_vectors(p, 1)[0])
        out = lib.right_transform(ws, g, [0.5], [R])[0]
        assert all(v.numel() == 0 or float(v.abs().max()) == 0.0 for v in out.values())


@pytest.mark.parametrize("cfg", [1])
@pytest.mark.parametrize("rng", [(0, 5), (140, 143), (347, 352)])
def test_full_shape_subsets(lib, ws, cfg, rng):
    """Full config shapes (N_V, N_O, rank), a subset of the triple list (degenerate ones included)."""
    from oracle.oracle import Oracle
    p = I.make_config(cfg)
    orc = Oracle(p)
    g = lib.Ground(p)
    R = I.right_vectors(p, 1)[0]
    om = I.omegas(cfg, 1)[0]
    _check(lib.ground_residual(ws, g, triple_range=rng), orc.ground_residual(*rng))
    out = lib.right_transform(ws, g, [om], [lib.vec_to_device(R)], triple_range=rng, reuse_ground=True)[0]
    _check(out, orc.right_transform(om, R, *rng))


def test_full_shape_range_additivity(lib, ws):
    """Config 1, every triple: the full call equals the sum of disjoint ranges."""
    import torch
    p = I.make_config(1)
    g = lib.Ground(p)
    R = lib.vec_to_device(I.right_vectors(p, 1)[0])
    nt = lib.num_triples(p.dims.n_o)
    full = lib.right_transform(ws, g, [0.4], [R])[0]
    parts = [lib.right_transform(ws, g, [0.4], [R], triple_range=r, reuse_ground=True)[0]
             for r in ((0, 100), (100, 251), (251, nt))]
    for k in full:
        tot = sum(x[k] for x in parts)
        assert float((tot - full[k]).norm() / full[k].norm()) < 1e-13
        assert torch.isfinite(full[k]).all()


def test_errors(lib, ws):
    d = I.Dims(3, 4, 4, 6, 10)
    p = I.make_problem(d, 1)
    g = lib.Ground(p)
    R = lib.vec_to_device(I.right_vectors(p, 1)[0])
    with pytest.raises(lib.MLCC3Error) as e:
        lib.right_transform(ws, g, [0.4], [R], triple_range=(5, 2))
    assert e.value.code == lib.EINVAL
    # omega placed on a denominator: rejected by the guard check
    eo, ev = p.eps_o, p.eps_v
    w = ev[0] + ev[1] + ev[2] - eo[0] - eo[1] - eo[2]
    with pytest.raises(lib.MLCC3Error) as e:
        lib.right_transform(ws, g, [w], [R], guard=1e-3)
    assert e.value.code == lib.ESINGULAR
    bad = I.make_problem(d, 1)
    bad.t1 = bad.t1.copy()
    bad.t1[0, 0] = np.nan
    with pytest.raises(lib.MLCC3Error) as e:
        lib.ground_residual(ws, lib.Ground(bad), check_finite=True)
    assert e.value.code == lib.ENONFINITE
    # the workspace is still usable afterwards
    _ = lib.ground_residual(ws, g)


@pytest.mark.parametrize("d", SMALL, ids=lambda d: f"{d.n_o}-{d.n_v}-{d.N_O}-{d.N_V}-{d.n_chol}")
def test_left_transform(lib, ws, d):
    p, orc, g = _setup(lib, d, 77)
    L = I.left_vectors(p, 2)
    om = I.omegas(False, 2)
    out = lib.left_transform(ws, g, om, [lib.vec_to_device(v) for v in L])
    for m in range(2):
        _check(out[m], orc.left_transform(om[m], L[m]))


@pytest.mark.parametrize("rng", [(0, 4), (347, 352)])
def test_left_full_shape_subsets(lib, ws, rng):
    from oracle.oracle import Oracle
    p = I.make_config(1)
    orc = Oracle(p)
    g = lib.Ground(p)
    L = I.left_vectors(p, 1)[0]
    out = lib.left_transform(ws, g, [0.4], [lib.vec_to_device(L)], triple_range=rng)[0]
    _check(out, orc.left_transform(0.4, L, *rng))


def test_adjoint_identity_full_config1(lib, ws):
    """<L, J R>_G = <J^T L, R>_G at the full config-1 size, GPU only, per block pairing."""
    p = I.make_config(1)
    d = p.dims
    g = lib.Ground(p)
    R = I.right_vectors(p, 1)[0]
    L = I.left_vectors(p, 1)[0]
    for Lpart in ("x1", "x2"):
        Lp = {k: (v if k.startswith(Lpart) else 0 * v) for k, v in L.items()}
        sig = lib.to_numpy(lib.left_transform(ws, g, [0.4], [lib.vec_to_device(Lp)], reuse_ground=True)[0])
        for Rpart in ("x1", "x2"):
            Rp = {k: (v if k.startswith(Rpart) else 0 * v) for k, v in R.items()}
            rho = lib.to_numpy(lib.right_transform(ws, g, [0.4], [lib.vec_to_device(Rp)], reuse_ground=True)[0])
            lhs = pair_form_blocks(d, Lp, rho)
            rhs = pair_form_blocks(d, sig, Rp)
            assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (Lpart, Rpart, lhs, rhs)


# ------------------------------------------------------------------ densities
def _dens_case(lib, d, seed, cfg=None):
    from oracle.oracle import Oracle
    p = I.make_config(cfg, with_density_blocks=True) if cfg is not None else \
        I.make_problem(d, seed, with_density_blocks=True)
    return p, Oracle(p), lib.Ground(p)


def _check_dens(got, ref, tol=TOL):
    Dm0, D0m, s = got
    for a, b in ((Dm0, ref[0]), (D0m, ref[1])):
        a = a.detach().cpu().numpy()
        assert np.all(np.isfinite(a))
        assert rel(a, b) <= tol, rel(a, b)
        assert maxrel(a, b) <= tol, maxrel(a, b)
    assert abs(float(s) - ref[2]) <= tol * abs(ref[2])


@pytest.mark.parametrize("d", SMALL, ids=lambda d: f"{d.n_o}-{d.n_v}-{d.N_O}-{d.N_V}-{d.n_chol}")
def test_densities(lib, ws, d):
    p, orc, g = _dens_case(lib, d, 31)
    Ls, Rs = I.left_vectors(p, 2), I.right_vectors(p, 2)
    lam = I.lambda_vector(p)
    om = I.omegas(False, 2)
    Dm0, D0m, s = lib.triples_densities(ws, g, om, [lib.vec_to_device(v) for v in Ls],
                                        [lib.vec_to_device(v) for v in Rs], lib.vec_to_device(lam),
                                        p.t2_vVoO, p.t2_vVOo)
    for m in range(2):
        ref = orc.densities(om[m], Ls[m], Rs[m], lam, p.t2_vVoO, p.t2_vVOo)
        _check_dens((Dm0[m], D0m[m], s[m]), ref)


@pytest.mark.parametrize("rng", [(0, 6), (340, 352)])
def test_densities_full_shape_subsets(lib, ws, rng):
    p, orc, g = _dens_case(lib, None, None, cfg=1)
    L, R, lam = I.left_vectors(p, 1)[0], I.right_vectors(p, 1)[0], I.lambda_vector(p)
    got = lib.triples_densities(ws, g, [0.4], [lib.vec_to_device(L)], [lib.vec_to_device(R)],
                                lib.vec_to_device(lam), p.t2_vVoO, p.t2_vVOo, triple_range=rng)
    ref = orc.densities(0.4, L, R, lam, p.t2_vVoO, p.t2_vVOo, *rng)
    _check_dens((got[0][0], got[1][0], got[2][0]), ref)


def test_density_traces_full_config1(lib, ws):
    """tr D^{m-0} = 0 and tr D^{0-m} = 2 N_O s over every triple at the full config-1 size."""
    p, orc, g = _dens_case(lib, None, None, cfg=1)
    d = p.dims
    Ls, Rs = I.left_vectors(p, 2), I.right_vectors(p, 2)
    Dm0, D0m, s = lib.triples_densities(ws, g, [0.4, 0.5], [lib.vec_to_device(v) for v in Ls],
                                        [lib.vec_to_device(v) for v in Rs], lib.vec_to_device(I.lambda_vector(p)),
                                        p.t2_vVoO, p.t2_vVOo)
    for m in range(2):
        A, B = Dm0[m].cpu().numpy(), D0m[m].cpu().numpy()
        assert np.all(np.isfinite(A)) and np.all(np.isfinite(B))
        assert abs(np.trace(A)) <= 1e-11 * np.abs(A).max()
        assert abs(np.trace(B) - 2 * d.N_O * float(s[m])) <= 1e-11 * np.abs(B).max()


def test_vector_groups_equal_single_calls(lib, ws, monkeypatch):
    """Several vectors share one persistent d-contraction launch and one launch per permutation
    pass; groups of 2 (environment cap), of 3 and single calls give identical results."""
    import torch
    d = I.Dims(5, 17, 7, 37, 23)
    p = I.make_problem(d, 12)
    g = lib.Ground(p)
    om = [0.41, 0.47, 0.53]
    R = [lib.vec_to_device(v) for v in I.right_vectors(p, 3)]
    L = [lib.vec_to_device(v) for v in I.left_vectors(p, 3)]
    for fn, vecs in ((lib.right_transform, R), (lib.left_transform, L)):
        for prec in ("fp64", "fp32"):
            monkeypatch.delenv("MLCC3_VEC_BATCH", raising=False)
            full = fn(ws, g, om, vecs, precision=prec)
            monkeypatch.setenv("MLCC3_VEC_BATCH", "2")
            pairs = fn(ws, g, om, vecs, reuse_ground=True, precision=prec)
            monkeypatch.delenv("MLCC3_VEC_BATCH", raising=False)
            singles = [fn(ws, g, [om[m]], [vecs[m]], reuse_ground=True, precision=prec)[0] for m in range(3)]
            for m in range(3):
                for k in full[m]:
                    assert torch.equal(full[m][k], pairs[m][k]), (fn.__name__, prec, m, k)
                    assert torch.equal(full[m][k], singles[m][k]), (fn.__name__, prec, m, k)


def test_oscillator_strengths(lib, ws):
    """D^{m-0}, D^{0-m}, s and D^{0-0} (densities with L -> lambda, omega = 0) on the GPU, then the
    moments and strengths with three symmetric operator components, against the oracle."""
    from oracle.oracle import Oracle, oscillator_strengths
    d = I.Dims(4, 6, 5, 11, 13)
    p = I.make_problem(d, 19, with_density_blocks=True)
    orc = Oracle(p)
    g = lib.Ground(p)
    Ls, Rs, lam = I.left_vectors(p, 2), I.right_vectors(p, 2), I.lambda_vector(p)
    om = [0.43, 0.61]
    dv = lambda v: lib.vec_to_device(v)
    Dm0, D0m, s = lib.triples_densities(ws, g, om, [dv(v) for v in Ls], [dv(v) for v in Rs], dv(lam),
                                        p.t2_vVoO, p.t2_vVOo)
    D00 = lib.triples_densities(ws, g, [0.0], [dv(lam)], [dv(Rs[0])], dv(lam), p.t2_vVoO, p.t2_vVOo,
                                reuse_ground=True)[0][0]
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, d.N, d.N))
    A = A + A.transpose(0, 2, 1)
    Tm0, T0m, f = lib.oscillator_strengths(ws, A, om, Dm0, D0m, D00, s)
    rD = [orc.densities(om[m], Ls[m], Rs[m], lam, p.t2_vVoO, p.t2_vVOo) for m in range(2)]
    rD00 = orc.densities(0.0, lam, Rs[0], lam, p.t2_vVoO, p.t2_vVOo)[0]
    eT, eT0, ef = oscillator_strengths(A, om, np.stack([x[0] for x in rD]), np.stack([x[1] for x in rD]), rD00,
                                       [x[2] for x in rD])
    for a, b in ((Tm0, eT), (T0m, eT0), (f, ef)):
        a = a.cpu().numpy()
        assert rel(a, b) <= 1e-10 and maxrel(a, b) <= 1e-10, (rel(a, b), maxrel(a, b))


# ------------------------------------------------------- core-valence separation (CVS)
CVS_SHAPES = [(I.Dims(4, 5, 5, 7, 12), [0, 1, 0, 0, 0]), (I.Dims(5, 17, 7, 37, 23), [1, 0, 0, 0, 0, 0, 0])]


@pytest.mark.parametrize("d,core", CVS_SHAPES, ids=lambda x: str(x))
def test_cvs_right_left(lib, ws, d, core):
    from oracle.oracle import Oracle
    p = I.make_problem(d, 71, core=True)
    orc = Oracle(p, cvs_core=core)
    g = lib.Ground(p)
    R, L = I.right_vectors(p, 2), I.left_vectors(p, 2)
    om = [15.2, 15.21]
    rho = lib.right_transform(ws, g, om, [lib.vec_to_device(v) for v in R], cvs_core=core)
    sig = lib.left_transform(ws, g, om, [lib.vec_to_device(v) for v in L], cvs_core=core, reuse_ground=True)
    for m in range(2):
        _check(rho[m], orc.right_transform(om[m], R[m]))
        _check(sig[m], orc.left_transform(om[m], L[m]))
    with pytest.raises(lib.MLCC3Error) as e:
        lib.ground_residual(ws, g, cvs_core=core)
    assert e.value.code == lib.EINVAL


def test_reuse_tau(lib):
    """opts.reuse_tau: transforms after a ground-residual call on the same workspace reuse its
    tau~ blocks and give exactly the results of fresh calls; a different ground state, triple
    range or precision forms them again, and so does a densities call in between."""
    import torch
    d = I.Dims(5, 17, 7, 37, 23)
    p1, p2 = I.make_problem(d, 81), I.make_problem(d, 82, with_density_blocks=True)
    g1, g2 = lib.Ground(p1), lib.Ground(p2)
    R = [lib.vec_to_device(v) for v in I.right_vectors(p1, 2)]
    L = [lib.vec_to_device(v) for v in I.left_vectors(p1, 2)]
    om = I.omegas(False, 2)
    wf, wt = lib.Workspace(0), lib.Workspace(0)
    try:
        ref_r1 = lib.right_transform(wf, g1, om, R)
        ref_l1 = lib.left_transform(wf, g1, om, L, reuse_ground=True)
        ref_rng = lib.right_transform(wf, g1, om, R, reuse_ground=True, triple_range=(3, 17))
        ref_r2 = lib.right_transform(wf, g2, om, R)
        ref_mx = lib.right_transform(wf, g2, om, R, reuse_ground=True, precision="fp32")
        ref_l2 = lib.left_transform(wf, g2, om, L, reuse_ground=True)

        def same(a, b):
            for m in range(len(b)):
                for k in b[m]:
                    assert torch.equal(a[m][k], b[m][k]), (m, k)

        lib.ground_residual(wt, g1)
        same(lib.right_transform(wt, g1, om, R, reuse_ground=True, reuse_tau=True), ref_r1)
        same(lib.left_transform(wt, g1, om, L, reuse_ground=True, reuse_tau=True), ref_l1)
        same(lib.right_transform(wt, g1, om, R, reuse_ground=True, reuse_tau=True, triple_range=(3, 17)), ref_rng)
        same(lib.right_transform(wt, g1, om, R, reuse_ground=True, reuse_tau=True), ref_r1)
        same(lib.right_transform(wt, g2, om, R, reuse_ground=True, reuse_tau=True), ref_r2)
        same(lib.right_transform(wt, g2, om, R, reuse_ground=True, reuse_tau=True, precision="fp32"), ref_mx)
        # the densities form tau~ (with its covariant form) again on this workspace
        lam = lib.vec_to_device(I.lambda_vector(p2))
        lib.triples_densities(wt, g2, om, L, R, lam, p2.t2_vVoO, p2.t2_vVOo, reuse_ground=True)
        same(lib.left_transform(wt, g2, om, L, reuse_ground=True, reuse_tau=True), ref_l2)
        same(lib.right_transform(wt, g2, om, R, reuse_ground=True, reuse_tau=True), ref_r2)
    finally:
        wf.close()
        wt.close()


def test_null_workspace(lib, ws):
    """A call without a workspace (NULL through the C-ABI) gives the same results as one with."""
    import torch

    class NoWorkspace:
        h = None
        device = torch.device("cuda", 0)

    d = I.Dims(5, 17, 7, 37, 23)
    p = I.make_problem(d, 77)
    g = lib.Ground(p)
    R = [lib.vec_to_device(v) for v in I.right_vectors(p, 2)]
    om = I.omegas(False, 2)
    a = lib.right_transform(ws, g, om, R)
    b = lib.right_transform(NoWorkspace(), g, om, R)
    c = lib.ground_residual(NoWorkspace(), g)
    e = lib.ground_residual(ws, g, reuse_ground=True)
    for m in range(2):
        for k in a[m]:
            assert torch.equal(a[m][k], b[m][k]), (m, k)
    for k in c:
        assert torch.equal(c[k], e[k]), k


def test_cvs_with_triple_ranges(lib, ws):
    """Core-valence separation combined with triple ranges (the d-contraction and N_V-wide
    back-contraction tiles of unneeded ordered triples are skipped): each range against the
    oracle over the same range, and the ranges add up to the whole CVS transform."""
    from oracle.oracle import Oracle
    d = I.Dims(5, 48, 7, 61, 19)
    core = [0, 1, 0, 0, 0, 0, 0]
    p = I.make_problem(d, 73, core=True)
    orc = Oracle(p, cvs_core=core)
    g = lib.Ground(p)
    R, L = I.right_vectors(p, 1)[0], I.left_vectors(p, 1)[0]
    w = 15.2
    nt = lib.num_triples(d.n_o)
    full_r = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], cvs_core=core)[0]
    full_l = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], cvs_core=core, reuse_ground=True)[0]
    parts_r, parts_l = [], []
    for rng in ((0, 9), (9, 24), (24, nt)):
        r = lib.right_transform(ws, g, [w], [lib.vec_to_device(R)], cvs_core=core, triple_range=rng,
                                reuse_ground=True)[0]
        l = lib.left_transform(ws, g, [w], [lib.vec_to_device(L)], cvs_core=core, triple_range=rng,
                               reuse_ground=True)[0]
        _check(r, orc.right_transform(w, R, *rng))
        _check(l, orc.left_transform(w, L, *rng))
        parts_r.append(r)
        parts_l.append(l)
    for full, parts in ((full_r, parts_r), (full_l, parts_l)):
        for k in full:
            tot = sum(x[k] for x in parts)
            assert float((tot - full[k]).norm() / full[k].norm()) < 1e-12, k


def test_cvs_full_config4(lib, ws):
    """Core-shaped workload at full size with its core orbital as the CVS core: the adjoint identity
    inside the CVS space, outputs in the CVS space, the mixed form within 1e-6."""
    p = I.make_config(4)
    d = p.dims
    g = lib.Ground(p)
    core = [1] + [0] * (d.N_O - 1)
    R, L = I.right_vectors(p, 2), I.left_vectors(p, 2)
    om = [float(x) for x in I.omegas(4, 2)]
    rho = lib.right_transform(ws, g, om, [lib.vec_to_device(v) for v in R], cvs_core=core)
    sig = lib.left_transform(ws, g, om, [lib.vec_to_device(v) for v in L], cvs_core=core, reuse_ground=True)
    for m in range(2):
        a = pair_form_blocks(d, L[m], lib.to_numpy(rho[m]))
        b = pair_form_blocks(d, lib.to_numpy(sig[m]), R[m])
        assert abs(a - b) <= 1e-10 * abs(a), (m, a, b)
        r = lib.to_numpy(rho[m])
        assert np.all(r["x1"][:, 1:] == 0) and np.all(r["x2_vVoo"][:, :, 1:, 1:] == 0)
    rmx = lib.right_transform(ws, g, om, [lib.vec_to_device(v) for v in R], cvs_core=core, reuse_ground=True,
                              precision="fp32")
    for k in rho[0]:
        assert rel(rmx[0][k].cpu().numpy(), rho[0][k].cpu().numpy()) <= 1e-6, k


def test_executed_dcontract_flops_match_the_cost_model(lib, ws):
    """The d-contraction launches execute exactly the model's O(N_V n_v^3 n_o^3) work: per product
    term 2 N_V n_v^3 over all n_o^3 ordered triples (the n_o diagonal ones are formed and left
    out of the algorithmic count U = 2 N_V n_v^3 (n_o^3 - n_o)); tau3 once per call, two terms
    per right vector, one per left vector."""
    d = I.Dims(5, 17, 7, 37, 23)
    p = I.make_problem(d, 5)
    g = lib.Ground(p)
    R = [lib.vec_to_device(v) for v in I.right_vectors(p, 3)]
    L = [lib.vec_to_device(v) for v in I.left_vectors(p, 3)]
    om = I.omegas(False, 3)
    T = 2.0 * d.N_V * d.n_v ** 3 * d.n_o ** 3
    U = 2.0 * d.N_V * d.n_v ** 3 * (d.n_o ** 3 - d.n_o)
    for name, call, terms, model in (
            ("ground", lambda: lib.ground_residual(ws, g), 1, 2 * U),
            ("right", lambda: lib.right_transform(ws, g, om, R, reuse_ground=True), 1 + 2 * 3, (1 + 3 * 3) * U),
            ("left", lambda: lib.left_transform(ws, g, om, L, reuse_ground=True), 1 + 3, (1 + 3 * 3) * U)):
        lib.right_transform(ws, g, om[:1], R[:1])  # prepared ground, warm buffers
        ws.timing(True)
        call()
        st = ws.phase_stats(0)
        ws.timing(False)
        assert st["flops"] == terms * T, (name, st["flops"], terms * T)
        fl = g.flops({"ground": 0, "right": 1, "left": 2}[name], 3)
        assert fl == model, (name, fl, model)


@pytest.mark.parametrize("d", [I.Dims(2, 70, 3, 75, 10), I.Dims(3, 66, 4, 71, 9), I.Dims(2, 136, 3, 140, 9),
                               I.Dims(2, 160, 3, 163, 9)], ids=str)
def test_densities_wide_virtual_space(lib, ws, d):
    """64 < n_v <= 160: the virtual Gram blocks (D_cd) take the whole-output MFMA kernel."""
    p, orc, g = _dens_case(lib, d, 37)
    Ls, Rs = I.left_vectors(p, 1), I.right_vectors(p, 1)
    lam = I.lambda_vector(p)
    om = I.omegas(False, 1)
    got = lib.triples_densities(ws, g, om, [lib.vec_to_device(v) for v in Ls], [lib.vec_to_device(v) for v in Rs],
                                lib.vec_to_device(lam), p.t2_vVoO, p.t2_vVOo)
    ref = orc.densities(om[0], Ls[0], Rs[0], lam, p.t2_vVoO, p.t2_vVOo)
    _check_dens((got[0][0], got[1][0], got[2][0]), ref)


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("d", [I.Dims(4, 12, 6, 20, 60), I.Dims(3, 32, 4, 41, 11)], ids=str)
def test_densities_every_permutation_pass_form(lib, ws, d, form):
    """Densities (covariant and contravariant blocks of every ordering) with each form of the
    contravariant pass: the oracle's results."""
    p, orc, g = _dens_case(lib, d, 37)
    Ls, Rs = I.left_vectors(p, 2), I.right_vectors(p, 2)
    lam = I.lambda_vector(p)
    om = I.omegas(False, 2)
    ws.set_tuning({"contra_form": form})
    try:
        Dm0, D0m, s = lib.triples_densities(ws, g, om, [lib.vec_to_device(v) for v in Ls],
                                            [lib.vec_to_device(v) for v in Rs], lib.vec_to_device(lam),
                                            p.t2_vVoO, p.t2_vVOo)
    finally:
        ws.set_tuning(None)
    for m in range(2):
        ref = orc.densities(om[m], Ls[m], Rs[m], lam, p.t2_vVoO, p.t2_vVOo)
        _check_dens((Dm0[m], D0m[m], s[m]), ref)
