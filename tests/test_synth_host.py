"""The seeded input generator (host only): the torch evaluation of the SU(3)
exponentials draws the same field as the numpy one up to rounding, and every
link it returns is special unitary."""
import numpy as np
import pytest

from paper_2108_11989_amd import synth

pytest.importorskip("torch")


def test_torch_exponentials_match_numpy():
    rng = np.random.Generator(np.random.PCG64(11))
    r = rng.standard_normal((500, 4, 8))
    a = synth.su3_from_algebra(r, 0.3)
    b = synth.su3_from_algebra_torch(r, 0.3, device="cpu")
    assert b.shape == a.shape
    assert np.abs(a - b).max() < 1e-13
    eye = np.eye(3)
    assert np.abs(b @ np.conj(np.swapaxes(b, -1, -2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(b) - 1).max() < 1e-13


def test_make_field_backends_agree():
    a = synth.make_field(4, 4, 0.3, 5, smear_steps=2)
    b = synth.make_field(4, 4, 0.3, 5, smear_steps=2, exp_backend="torch")
    assert np.abs(a[0] - b[0]).max() < 1e-13
    assert np.array_equal(a[1], b[1])
