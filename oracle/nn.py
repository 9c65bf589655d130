"""Gauge-covariant preconditioner network, FP64 forward and backward (oracle; test infrastructure only).

The network is not in the paper; it is the learned part of this library, a
linear parallel-transport convolution in the style of published
gauge-equivariant preconditioner networks.  One layer maps Cin channels of
spinor fields to Cout channels:

    out_a(x) = sum_b sum_p W[a, b, p] (T_p in_b)(x),

with W[a, b, p] a complex 4x4 matrix acting on spin and T_p the transport
along path p: p = 0 the identity, p = 1 + 2 mu + d the hop in direction mu,
d = 0 forward (V(x,mu) psi(x+mu)), d = 1 backward (V(x-mu,mu)^H psi(x-mu)),
on the x-doubled C* lattice with the fermion time phase.  The network is
three layers with channels 1 -> 8 -> 8 -> 1.

Gradients use g = dL/dRe + i dL/dIm.  For out = W u and a real loss L:
grad W = sum g_out (x) conj(u) (summed over sites and colour), and the input
gradient is grad in_b = sum_a sum_p T_p^H W[a,b,p]^H g_out_a with
T_p^H the transport along the reversed path.

Loss on pairs (x, b = Q^2 x): L = (1/N) sum_i |M(b_i) - x_i|^2 / |x_i|^2.
"""
from __future__ import annotations

import numpy as np

NPATH = 9
CHANNELS = (1, 8, 8, 1)


def path_mu_dir(p: int):
    """(mu, direction) of path p >= 1."""
    mu, d = divmod(p - 1, 2)
    return mu, (+1 if d == 0 else -1)


def reverse_path(p: int) -> int:
    if p == 0:
        return 0
    mu, d = divmod(p - 1, 2)
    return 1 + 2 * mu + (1 - d)


def transport(op, psi, p):
    if p == 0:
        return psi.copy()
    mu, direction = path_mu_dir(p)
    return op.transport(psi, mu, direction)


def layer_shapes(channels=CHANNELS):
    return [(channels[i + 1], channels[i], NPATH, 4, 4) for i in range(len(channels) - 1)]


def n_params(channels=CHANNELS) -> int:
    """Real parameters (re and im of every complex weight)."""
    return int(sum(2 * np.prod(s) for s in layer_shapes(channels)))


def unpack(flat, channels=CHANNELS):
    """Flat float array (layers concatenated, [Cout][Cin][path][4][4] complex interleaved) -> list of W."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for s in layer_shapes(channels):
        n = int(np.prod(s))
        v = flat[o:o + 2 * n]
        out.append((v[0::2] + 1j * v[1::2]).reshape(s))
        o += 2 * n
    return out


def pack(Ws):
    parts = []
    for W in Ws:
        z = np.asarray(W, dtype=np.complex128).reshape(-1)
        v = np.empty(2 * z.size)
        v[0::2] = z.real
        v[1::2] = z.imag
        parts.append(v)
    return np.concatenate(parts)


def spin_mul(W44, psi):
    """(W psi)(x)[s][c] = sum_s' W[s][s'] psi(x)[s'][c] on canonical spinors."""
    return np.einsum("st,...tc->...sc", W44, psi)


def layer_forward(op, W, ins):
    """ins: list of Cin canonical spinors -> list of Cout spinors, plus the transported inputs."""
    Cout, Cin = W.shape[0], W.shape[1]
    tr = [[transport(op, ins[b], p) for p in range(NPATH)] for b in range(Cin)]
    outs = []
    for a in range(Cout):
        acc = np.zeros_like(ins[0])
        for b in range(Cin):
            for p in range(NPATH):
                acc += spin_mul(W[a, b, p], tr[b][p])
        outs.append(acc)
    return outs, tr


def layer_backward(op, W, tr, gouts):
    """Weight gradient and input gradient of one layer."""
    Cout, Cin = W.shape[0], W.shape[1]
    gW = np.zeros_like(W)
    for a in range(Cout):
        for b in range(Cin):
            for p in range(NPATH):
                gW[a, b, p] = np.einsum("nsc,ntc->st", gouts[a].reshape(-1, 4, 3),
                                            tr[b][p].reshape(-1, 4, 3).conj())
    gins = []
    for b in range(Cin):
        acc = np.zeros_like(gouts[0])
        for p in range(NPATH):
            h = np.zeros_like(gouts[0])
            for a in range(Cout):
                h += spin_mul(W[a, b, p].conj().T, gouts[a])
            acc += transport(op, h, reverse_path(p))
        gins.append(acc)
    return gW, gins


def forward(op, Ws, b):
    """M(b) and the stored activations."""
    acts = [[b]]
    trs = []
    for W in Ws:
        outs, tr = layer_forward(op, W, acts[-1])
        trs.append(tr)
        acts.append(outs)
    return acts[-1][0], acts, trs


def loss_and_grad(op, Ws, xs, bs):
    """L = (1/N) sum |M(b_i) - x_i|^2 / |x_i|^2 and its gradient w.r.t. every weight."""
    N = len(xs)
    L = 0.0
    grads = [np.zeros_like(W) for W in Ws]
    for x, b in zip(xs, bs):
        y, acts, trs = forward(op, Ws, b)
        r = y - x
        nx = np.vdot(x, x).real
        L += np.vdot(r, r).real / nx / N
        g = [2.0 * r / nx / N]
        for li in range(len(Ws) - 1, -1, -1):
            gW, g = layer_backward(op, Ws[li], trs[li], g)
            grads[li] += gW
    return L, grads


def identity_weights(channels=CHANNELS, scale=1.0, noise=0.0, seed=0):
    """Weights with M = scale * 1 (channel 0 carries the field through p = 0), plus optional noise."""
    rng = np.random.default_rng(seed)
    Ws = []
    for li, s in enumerate(layer_shapes(channels)):
        W = noise * (rng.standard_normal(s) + 1j * rng.standard_normal(s))
        W[0, 0, 0] += np.eye(4) * (scale if li == 0 else 1.0)
        Ws.append(W)
    return Ws
