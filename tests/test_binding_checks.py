"""The Python binding checks every array it hands to the library (CPU only, no compute call).

The C-ABI takes bare device pointers and reads the element counts that the sizes imply, so a
missing array, one of the wrong size or one on another device must be refused on the host
before any call: the library itself cannot see allocation sizes.
"""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2202_08612_amd import inputs as I

D = I.Dims(3, 5, 4, 7, 6)


@pytest.fixture(scope="module")
def lib():
    from paper_2202_08612_amd import mlcc3
    return mlcc3


class CpuWs:
    h = None
    device = torch.device("cpu")


def test_ground_sizes_checked(lib):
    p = I.make_problem(D, 3)
    g = lib.Ground(p, "cpu")
    assert all(g.t[k].numel() == n for k, n in lib.ground_sizes(D).items())
    bad = dataclasses.replace(p, L_OV=np.zeros(5))
    with pytest.raises(ValueError, match="L_OV"):
        lib.Ground(bad, "cpu")
    with pytest.raises(ValueError, match="t1: missing"):
        lib.Ground(dataclasses.replace(p, t1=None), "cpu")


def test_vector_blocks_checked(lib):
    p = I.make_problem(D, 4)
    v = lib.vec_to_device(I.right_vectors(p, 1)[0], "cpu")
    lib._vecs([v], D, "cpu")  # well formed
    short = dict(v, x2_vvoO=v["x2_vvoO"][:-1].contiguous())
    with pytest.raises(ValueError, match="x2_vvoO"):
        lib._vecs([short], D, "cpu")
    with pytest.raises(ValueError, match="expected cuda"):
        lib._vecs([v], D, torch.device("cuda", 0))
    with pytest.raises(ValueError, match="float64"):
        lib._vecs([dict(v, x1=v["x1"].float())], D, "cpu")


def test_density_blocks_checked_before_the_call(lib):
    """A problem made without the density t2 blocks (None) is refused: it once reached the
    library as a one-element array."""
    p = I.make_problem(D, 5)
    assert p.t2_vVoO is None
    g = lib.Ground(p, "cpu")
    L = [lib.vec_to_device(I.left_vectors(p, 1)[0], "cpu")]
    R = [lib.vec_to_device(I.right_vectors(p, 1)[0], "cpu")]
    lam = lib.vec_to_device(I.lambda_vector(p), "cpu")
    with pytest.raises(ValueError, match="t2_vVoO: missing"):
        lib.triples_densities(CpuWs(), g, [0.4], L, R, lam, p.t2_vVoO, p.t2_vVOo)
    pd = I.make_problem(D, 5, with_density_blocks=True)
    with pytest.raises(ValueError, match="t2_vVOo"):
        lib.triples_densities(CpuWs(), g, [0.4], L, R, lam, pd.t2_vVoO, pd.t2_vVOo[:3])
    with pytest.raises(ValueError, match="left and"):
        lib.triples_densities(CpuWs(), g, [0.4], L, R + R, lam, pd.t2_vVoO, pd.t2_vVOo)


def test_oscillator_strength_shapes_checked(lib):
    N = 6
    A = np.zeros((2, N, N))
    with pytest.raises(ValueError, match="D_00"):
        lib.oscillator_strengths(CpuWs(), A, [0.4], np.zeros((1, N, N)), np.zeros((1, N, N)), np.zeros((N, N + 1)),
                                 np.zeros(1))
    with pytest.raises(ValueError, match="omegas"):
        lib.oscillator_strengths(CpuWs(), A, [0.4, 0.5], np.zeros((1, N, N)), np.zeros((1, N, N)),
                                 np.zeros((N, N)), np.zeros(1))
