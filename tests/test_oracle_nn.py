"""Pins of the network oracle (oracle/nn.py): adjoint transports, a closed form
(the hopping operator is one network layer), gauge equivariance, identity
weights, and central finite differences of the loss gradient."""
import numpy as np
import pytest

from oracle import dirac, nn
from paper_2108_11989_amd import synth


@pytest.fixture(scope="module")
def op():
    su3, th = synth.make_field(2, 2, 0.5, 3)
    return dirac.Operator(su3, th, 2 / 3, time_bc=-1)


def _rand(op, seed):
    return synth.random_spinor(op.T, op.L, seed)


def test_transport_adjoint(op):
    a, b = _rand(op, 1), _rand(op, 2)
    for p in range(1, nn.NPATH):
        lhs = np.vdot(a, nn.transport(op, b, p))
        rhs = np.vdot(nn.transport(op, a, nn.reverse_path(p)), b)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_hopping_operator_is_one_layer():
    """D(m) without clover = layer with W^0 = (4+m), W^{+mu} = -(1-g_mu)/2, W^{-mu} = -(1+g_mu)/2."""
    su3, th = synth.make_field(4, 2, 0.4, 7)
    op = dirac.Operator(su3, th, -1 / 3, clover=False, time_bc=-1)
    g = dirac.gammas()
    m = 0.37
    W = np.zeros((1, 1, nn.NPATH, 4, 4), dtype=complex)
    W[0, 0, 0] = (4 + m) * np.eye(4)
    for mu in range(4):
        W[0, 0, 1 + 2 * mu] = -0.5 * (np.eye(4) - g[mu])
        W[0, 0, 2 + 2 * mu] = -0.5 * (np.eye(4) + g[mu])
    psi = synth.random_spinor(4, 2, 3)
    out, _ = nn.layer_forward(op, W, [psi])
    assert np.abs(out[0] - op.D(psi, m)).max() < 1e-13


def test_layer_gauge_equivariance():
    T, L = 2, 2
    su3, th = synth.make_field(T, L, 0.6, 5)
    q = 2 / 3
    op = dirac.Operator(su3, th, q)
    rng = np.random.default_rng(4)
    Om = synth.su3_from_algebra(rng.standard_normal((T, L, L, L, 8)), 1.0)
    al = rng.standard_normal((T, L, L, L))
    Om_e = np.concatenate([Om, Om.conj()], axis=1)
    al_e = np.concatenate([al, -al], axis=1)
    nb = dirac.neighbours(T, L).reshape(T, 2 * L, L, L, 4, 2)
    Omf, alf = Om_e.reshape(-1, 3, 3), al_e.reshape(-1)
    su3n, thn = np.empty_like(su3), np.empty_like(th)
    for mu in range(4):
        fwd = nb[:, :L, :, :, mu, 0]
        su3n[..., mu, :, :] = Om @ su3[..., mu, :, :] @ np.swapaxes(Omf[fwd].conj(), -1, -2)
        thn[..., mu] = th[..., mu] + al - alf[fwd]
    op2 = dirac.Operator(su3n, thn, q)
    Ws = [W * 0.3 for W in nn.identity_weights(noise=1.0, seed=2)]
    G = Om_e * np.exp(1j * q * al_e)[..., None, None]
    psi = synth.random_spinor(T, L, 8)
    gpsi = np.einsum("...ij,...aj->...ai", G, psi)
    y1, _, _ = nn.forward(op2, Ws, gpsi)
    y0, _, _ = nn.forward(op, Ws, psi)
    assert np.abs(y1 - np.einsum("...ij,...aj->...ai", G, y0)).max() < 1e-14 * np.abs(y0).max()


def test_identity_weights(op):
    psi = _rand(op, 5)
    y, _, _ = nn.forward(op, nn.identity_weights(scale=0.25), psi)
    assert np.abs(y - 0.25 * psi).max() < 1e-15
    assert nn.n_params() == 23040


def test_gradient_by_central_differences(op):
    rng = np.random.default_rng(0)
    Ws = nn.identity_weights(scale=0.5, noise=0.2, seed=1)
    xs = [_rand(op, 10), _rand(op, 11)]
    bs = [op.Q2(x, 0.3) for x in xs]
    L0, grads = nn.loss_and_grad(op, Ws, xs, bs)
    flat = nn.pack(Ws)
    gflat = nn.pack(grads)
    h = 1e-6
    for idx in rng.choice(flat.size, 24, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[idx] += h
        fm[idx] -= h
        Lp, _ = nn.loss_and_grad(op, nn.unpack(fp), xs, bs)
        Lm, _ = nn.loss_and_grad(op, nn.unpack(fm), xs, bs)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, gflat[idx])
