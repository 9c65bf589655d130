"""Pins of the Lanczos eigenvalue oracle (oracle/lanczos.py) against dense
diagonalisation, which it shares nothing with but the operator.

* On 2x4^3 (6,144 complex dimensions) the k lowest |lambda| of Q, one per
  Kramers pair, equal those of numpy's eigh of the dense Q, within the
  oracle's own residual bounds, for plain Lanczos on Q^2 and for Lanczos on a
  Chebyshev polynomial of Q^2; a dropped eigenvalue, a wrong sign or a
  misplaced pair fails it.
* The Kramers map used to close the Ritz subspace is antiunitary with
  Theta^2 = -1 and commutes with Q (sign-of-the-Pfaffian section: the
  spectrum of Q is doubly degenerate).
"""
import numpy as np
import pytest

from oracle import dense, dirac, lanczos, sign
from paper_2108_11989_amd import synth


@pytest.fixture(scope="module")
def case():
    su3, th = synth.make_field(2, 4, 0.3, 3)
    op = dirac.Operator(su3, th, 2 / 3, 1.9, 1.0)
    m0 = -0.2
    ref = dense.lowest_abs(sign.pair_spectrum(op, m0), 4)
    return op, m0, ref


@pytest.mark.parametrize("degree", [1, 8])
def test_lanczos_matches_dense(case, degree):
    op, m0, ref = case
    ev, err, applies = lanczos.lowest_q(op, m0, 4, degree=degree)
    assert np.all(err < 1e-11)
    assert np.all(np.abs(ev - ref) <= err + 1e-13)
    assert applies > 0


def test_kramers_image(case):
    op, m0, _ = case
    rng = np.random.default_rng(4)
    v = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    tv = lanczos.kramers_image(v, op.L)
    assert np.abs(lanczos.kramers_image(tv, op.L) + v).max() < 1e-14
    assert abs(np.vdot(v, tv)) < 1e-10 * np.vdot(v, v).real
    assert np.abs(op.Q(tv, m0) - lanczos.kramers_image(op.Q(v, m0), op.L)).max() < 1e-12
