"""The seeded generator: determinism, symmetric partners, block overlaps, recipe."""
import numpy as np

from paper_2202_08612_amd import inputs as I


def test_deterministic_and_seed_dependent():
    d = I.Dims(3, 4, 5, 7, 6)
    a, b, c = I.make_problem(d, 1), I.make_problem(d, 1), I.make_problem(d, 2)
    for k in ("eps_o", "L_OV", "t2_vVoo"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
        assert not np.array_equal(getattr(a, k), getattr(c, k))


def test_symmetries_and_overlaps():
    d = I.Dims(3, 4, 5, 7, 6)
    p = I.make_problem(d, 3, with_density_blocks=True)
    assert np.array_equal(p.L_OO, np.transpose(p.L_OO, (0, 2, 1)))
    assert np.array_equal(p.L_vV[:, :, :d.n_v], np.transpose(p.L_vV[:, :, :d.n_v], (0, 2, 1)))
    Lf = I.full_cholesky(3, d)
    assert np.array_equal(Lf[:, :d.N_O, d.N_O:], p.L_OV)
    assert np.array_equal(Lf, np.transpose(Lf, (0, 2, 1)))
    t2 = I.full_doubles(3, I.TID_T2, d, 0.02)
    assert np.array_equal(t2, np.einsum("baji->abij", t2))
    assert np.array_equal(t2[:d.n_v, :, :d.n_o, :d.n_o], p.t2_vVoo)
    assert np.array_equal(t2[:d.n_v, :d.n_v, :d.n_o, :], p.t2_vvoO)
    assert np.array_equal(t2[:d.n_v, :, :d.n_o, :], p.t2_vVoO)
    assert np.array_equal(t2[:d.n_v, :, :, :d.n_o], p.t2_vVOo)


def test_vector_normalisation_and_full_slices():
    d = I.Dims(3, 4, 5, 7, 6)
    R = I.trial_vector(9, d, 0)
    assert abs(I.packed_norm2(d, R["x1"], R["x2_vVoo"], R["x2_vvoO"]) - 1.0) < 1e-12
    R1, R2 = I.full_vector(9, d, 0)
    assert np.allclose(R1, R["x1"], rtol=0, atol=0)
    assert np.array_equal(R2[:d.n_v, :, :d.n_o, :d.n_o], R["x2_vVoo"])


def test_distribution_recipe():
    d = I.Dims(4, 6, 30, 200, 40)
    p = I.make_problem(d, 5)
    assert p.eps_o.min() >= -2.0 and p.eps_o.max() <= -0.3
    assert p.eps_v.min() >= 0.1 and p.eps_v.max() <= 3.0
    assert abs(np.std(p.L_OV) - 0.05) < 0.002 and abs(np.mean(p.L_OV)) < 0.002
    assert abs(np.std(p.t1) - 0.01) < 0.001
    core = I.make_problem(d, 5, core=True)
    assert -15.5 <= core.eps_o[0] <= -14.5
    # denominators stay away from the excitation energies used by the workloads
    ev, eo = p.eps_v, p.eps_o
    assert 3 * ev.min() - 3 * eo.max() - I.omegas(False, 4).max() >= 0.5
