"""CPU pins of the pairing maps used for gradients through the transforms: the numpy maps in
tests/helpers.py against the pairing G(L, R) = sum L1 R1 + sum_{(AI)>=(BJ)} L~ R itself."""
import numpy as np
import pytest

from paper_2202_08612_amd import inputs as I
from tests.helpers import (euclid, map_grad_to_left, map_left_to_grad, map_symmetrize, pair_form_blocks)

SHAPES = [I.Dims(3, 4, 4, 6, 10), I.Dims(2, 3, 5, 7, 4), I.Dims(4, 4, 4, 4, 5)]


def _rand(d, rng):
    return {"x1": rng.standard_normal((d.N_V, d.N_O)),
            "x2_vVoo": rng.standard_normal((d.n_v, d.N_V, d.n_o, d.n_o)),
            "x2_vvoO": rng.standard_normal((d.n_v, d.n_v, d.n_o, d.N_O))}


@pytest.mark.parametrize("d", SHAPES, ids=str)
def test_symmetrize(d):
    rng = np.random.default_rng(1)
    y = I.trial_vector(3, d, 0)           # consistent, pair-symmetric
    s = map_symmetrize(d, y)
    for k in y:
        assert np.allclose(s[k], y[k], rtol=0, atol=1e-15)
    x = map_symmetrize(d, _rand(d, rng))  # idempotent
    xx = map_symmetrize(d, x)
    for k in x:
        assert np.allclose(xx[k], x[k], rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", SHAPES, ids=str)
def test_grad_to_left_represents_the_euclidean_product(d):
    rng = np.random.default_rng(2)
    g = _rand(d, rng)
    L = map_grad_to_left(d, g)
    for slot in (0, 1, 5):
        y = I.trial_vector(11, d, slot)
        a, b = pair_form_blocks(d, L, y), euclid(g, y)
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (a, b)


@pytest.mark.parametrize("d", SHAPES, ids=str)
def test_left_to_grad_represents_the_pairing(d):
    S = I.trial_vector(7, d, 64)
    h = map_left_to_grad(d, S)
    for slot in (0, 2):
        y = I.trial_vector(13, d, slot)
        a, b = euclid(h, y), pair_form_blocks(d, S, y)
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (a, b)
    # the two maps are inverse to each other on consistent vectors
    back = map_grad_to_left(d, h)
    for k in S:
        assert np.allclose(back[k], S[k], rtol=0, atol=1e-13)
