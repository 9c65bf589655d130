"""GPU parity of the preconditioner network (cstar_nn_* through the C ABI)
against the FP64 oracle network (oracle/nn.py).

The GPU network computes in FP32 with the FP32 links; the oracle runs in FP64
on the same FP32-rounded inputs and weights, with the links in its FP32
emulation mode (rows rounded to FP32, third row rebuilt, FP32 phase).
Forward: max |diff| <= 2e-5 max |ref| (three layers, each output entry a sum
of ~300 FP32 products; 2^-24 * sqrt(300) * a few layers is ~1e-6, with margin).
Gradient: relative 2-norm error of every layer's block <= 1e-4 (a sum over
all sites of FP32 products, accumulated per lane in FP32: ~2^-24 * number of
sites per lane * growth, well under 1e-5 here), loss relative <= 1e-5.
"""
import numpy as np
import pytest

from oracle import dirac as odirac
from oracle import nn as onn
from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [
    # T, L, eps, seed, q, time_bc
    (4, 2, 0.5, 1, 2 / 3, -1),
    (4, 4, 0.7, 2, -1 / 3, 1),
    (6, 4, 0.4, 3, 2 / 3, 1),
]


def _f32(a):
    return a.astype(np.complex64).astype(np.complex128)


def _weights(seed, scale=1.0, noise=0.3):
    """Random weights rounded to FP32: (oracle list, flat float32)."""
    flat = onn.pack(onn.identity_weights(scale=scale, noise=noise, seed=seed)).astype(np.float32)
    return onn.unpack(flat.astype(np.float64)), flat


def _native32(g, psi):
    n = psi.shape[0]
    canon = torch.from_numpy(psi).to(torch.complex64).cuda().contiguous()
    nat = g.new_native(n, cstar.FP32)
    g.pack(canon, nat, cstar.FP32, n)
    return nat


def _canon32(g, nat, shape):
    res = torch.empty(shape, dtype=torch.complex64, device="cuda")
    g.unpack(nat, res, cstar.FP32, shape[0])
    torch.cuda.synchronize()
    return res.cpu().numpy().astype(np.complex128)


def _setup(case):
    assert torch.cuda.is_available(), "GPU tests need a device"
    T, L, eps, seed, q, tbc = case
    su3, th = synth.make_field(T, L, eps, seed)
    g = cstar.Gauge(su3, th, q, time_bc=tbc)
    op = odirac.Operator(su3, th, q, time_bc=tbc, link_mode=1, clover=False)
    return g, op


@pytest.mark.parametrize("case", CASES)
def test_forward_matches_oracle(case):
    g, op = _setup(case)
    Ws, flat = _weights(case[3] + 10)
    net = cstar.Net(flat)
    psi = _f32(np.stack([synth.random_spinor(op.T, op.L, s) for s in (1, 2)]))
    b = _native32(g, psi)
    y = g.new_native(2, cstar.FP32)
    net.apply(g, b, y, nvec=2)
    out = _canon32(g, y, psi.shape)
    for j in range(2):
        ref, _, _ = onn.forward(op, Ws, psi[j])
        err = np.abs(out[j] - ref).max() / np.abs(ref).max()
        assert err < 2e-5, err
    # in place
    net.apply(g, b, b, nvec=2)
    assert np.abs(_canon32(g, b, psi.shape) - out).max() == 0.0
    net.close()
    g.close()


@pytest.mark.parametrize("case", CASES)
def test_gradient_matches_oracle(case):
    g, op = _setup(case)
    Ws, flat = _weights(case[3] + 20, scale=0.5, noise=0.2)
    net = cstar.Net(flat)
    xs = _f32(np.stack([synth.random_spinor(op.T, op.L, s) for s in (3, 4)]))
    bs = _f32(np.stack([synth.random_spinor(op.T, op.L, s) for s in (5, 6)]))
    net.zero_grad()
    loss = net.loss_grad(g, _native32(g, xs), _native32(g, bs), nvec=2)
    grad = net.grad()
    L_ref, grads = onn.loss_and_grad(op, Ws, list(xs), list(bs))
    gref = onn.pack(grads)
    assert abs(loss - L_ref) <= 1e-5 * L_ref
    off = 0
    for W in Ws:
        n = 2 * W.size
        e = np.linalg.norm(grad[off:off + n] - gref[off:off + n]) / np.linalg.norm(gref[off:off + n])
        print(f"layer block of {n} reals: relative gradient error {e:.2e}")
        assert e < 1e-4, e
        off += n
    # one Adam step from zero moments moves every weight by lr * g / (|g| + eps)
    w0 = net.weights().astype(np.float64)
    lr = 1e-3
    net.adam_step(lr)
    w1 = net.weights().astype(np.float64)
    expect = w0 - lr * grad / (np.abs(grad) + 1e-8)
    assert np.abs(w1 - expect).max() < 1e-6
    assert np.abs(net.grad()).max() == 0.0
    net.close()
    g.close()


@pytest.mark.parametrize("kappa", [0.125, 0.09])
def test_preconditioned_solver_agrees_with_plain(kappa):
    """Identity and random networks: the preconditioned solve converges to the
    plain solver's eigenvalues (the plain solver is the judge)."""
    T, L, eps, seed, q = 4, 2, 0.3, 0, 2 / 3
    su3, th = synth.make_field(T, L, eps, seed)
    g = cstar.Gauge(su3, th, q)
    m0 = 1 / (2 * kappa) - 4
    o_plain = cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=1e-10)
    e0, r0, s0 = g.lowest_eigs(m0, 4, o_plain)
    for w in (None, _weights(3, scale=0.1, noise=0.02)[1]):
        net = cstar.Net(w)
        net.attach(g)
        o_nn = cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=1e-10, use_nn=1)
        e1, r1, s1 = g.lowest_eigs(m0, 4, o_nn)
        assert s1.nn_applies > 0 and s1.nn_fallback == 0
        assert np.all(np.abs(e1 - e0) <= r0 + r1 + 1e-13)
        print(f"kappa {kappa}: plain {s0.iterations} it, preconditioned {s1.iterations} it")
        cstar.Net.detach(g)
        net.close()
    g.close()


def test_training_lowers_the_loss():
    T, L = 4, 4
    gs, xs = [], []
    for s in (31, 32):
        su3, th = synth.make_field(T, L, 0.3, s)
        g = cstar.Gauge(su3, th, 2 / 3)
        gs.append(g)
        xs.append(_native32(g, np.stack([synth.random_spinor(T, L, 100 * s + j) for j in range(4)])))
    _, flat = _weights(7, scale=1 / 16.0, noise=0.01)
    net = cstar.Net(flat)
    hist = net.train(gs, xs, 4, -0.2, 40, 2e-3)
    print("loss history", hist[0], hist[9], hist[19], hist[-1])
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.5 * hist[0]
    net.close()
    for g in gs:
        g.close()
