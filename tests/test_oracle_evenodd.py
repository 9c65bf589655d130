"""Pins of the even-odd oracle (mass-reweighting section: D_hat, D_oo, W_eo).

* every hop changes the site parity, so D_oo (and D_ee) is block diagonal:
  the site-local term (4+m) + SW(x), Hermitian and commuting with g5, equal
  to (4+m) 1 on the free field;
* det D = det D_oo det D_hat (Schur complement), magnitude and phase -- a
  wrong sign, a transposed block or a wrong parity split fails it;
* Q_hat = g5 D_hat is Hermitian;
* the apply of D_hat equals the dense Schur complement;
* W_eo: on the free field log W_eo = 6 V_odd log|(4+m')/(4+m)| in closed form
  (V_odd odd sites of the doubled lattice, 12 components each, power 1/2);
  on a general field it equals half the difference of log|det D_oo|.
"""
import numpy as np
import pytest

from oracle import dense, dirac, evenodd
from paper_2108_11989_amd import synth

CSW, CU1 = 1.9, 1.0


@pytest.fixture(scope="module")
def tiny():
    su3, th = synth.make_field(2, 2, 0.7, 41)
    return dirac.Operator(su3, th, 2 / 3, CSW, CU1)


def test_local_term_is_the_site_diagonal_of_d(tiny):
    m0 = -0.3
    D = dense.dense_D(tiny, m0)
    loc = tiny.local_term(m0)
    n = tiny.nsites
    blocks = D.reshape(n, 12, n, 12)
    for s in range(n):
        assert np.abs(blocks[s, :, s, :] - loc[s]).max() < 1e-14
    g5 = np.diag([1.0] * 6 + [-1.0] * 6)
    for M in loc:
        assert np.abs(M - M.conj().T).max() < 1e-14
        assert np.abs(M @ g5 - g5 @ M).max() < 1e-14


def test_same_parity_blocks_are_site_local(tiny):
    m0 = 0.2
    D = dense.dense_D(tiny, m0)
    T, L = tiny.T, tiny.L
    Dee, Deo, Doe, Doo = evenodd.dense_blocks(D, T, L)
    par = evenodd.parity_sites(T, L)
    loc = tiny.local_term(m0)
    for blk, p in ((Dee, 0), (Doo, 1)):
        sites = np.nonzero(par == p)[0]
        ref = np.zeros_like(blk)
        for i, s in enumerate(sites):
            ref[12 * i:12 * i + 12, 12 * i:12 * i + 12] = loc[s]
        assert np.abs(blk - ref).max() < 1e-14


def test_free_field_local_term():
    su3, th = synth.unit_field(2, 2)
    op = dirac.Operator(su3, th, 2 / 3, CSW, CU1)
    loc = op.local_term(0.7)
    assert np.abs(loc - 4.7 * np.eye(12)).max() < 1e-15


@pytest.mark.parametrize("m0", [-0.6, 0.15])
def test_schur_determinant_identity(tiny, m0):
    D = dense.dense_D(tiny, m0)
    Dhat = evenodd.dense_dhat(D, tiny.T, tiny.L)
    _, _, _, Doo = evenodd.dense_blocks(D, tiny.T, tiny.L)
    s_d, l_d = np.linalg.slogdet(D)
    s_o, l_o = np.linalg.slogdet(Doo)
    s_h, l_h = np.linalg.slogdet(Dhat)
    assert abs(l_d - (l_o + l_h)) < 1e-10 * abs(l_d)
    assert abs(s_d - s_o * s_h) < 1e-9


def test_q_hat_is_hermitian(tiny):
    D = dense.dense_D(tiny, -0.25)
    Dhat = evenodd.dense_dhat(D, tiny.T, tiny.L)
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), Dhat.shape[0] // 12)
    Qhat = g5[:, None] * Dhat
    assert np.abs(Qhat - Qhat.conj().T).max() < 1e-13


@pytest.mark.parametrize("gamma5", [False, True])
def test_apply_dhat_equals_dense(tiny, gamma5):
    m0 = -0.1
    D = dense.dense_D(tiny, m0)
    Dhat = evenodd.dense_dhat(D, tiny.T, tiny.L)
    rng = np.random.default_rng(3)
    n = Dhat.shape[0]
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = Dhat @ v
    if gamma5:
        ref = ref.reshape(-1, 12)
        ref[:, 6:] *= -1
        ref = ref.reshape(-1)
    out = evenodd.apply_dhat(tiny, v, m0, gamma5)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_w_eo_free_field_closed_form():
    su3, th = synth.unit_field(4, 2)
    op = dirac.Operator(su3, th, 2 / 3, CSW, CU1)
    m, mp = -0.2, 0.05
    v_odd = op.nsites // 2
    assert abs(evenodd.log_w_eo(op, m, mp) - 6 * v_odd * np.log(abs((4 + mp) / (4 + m)))) < 1e-12


def test_w_eo_equals_dense_determinant_ratio(tiny):
    m, mp = -0.3, -0.27
    _, _, _, Doo_m = evenodd.dense_blocks(dense.dense_D(tiny, m), tiny.T, tiny.L)
    _, _, _, Doo_p = evenodd.dense_blocks(dense.dense_D(tiny, mp), tiny.T, tiny.L)
    ref = 0.5 * (np.linalg.slogdet(Doo_p)[1] - np.linalg.slogdet(Doo_m)[1])
    assert abs(evenodd.log_w_eo(tiny, m, mp) - ref) < 1e-12 * max(1.0, abs(ref))
