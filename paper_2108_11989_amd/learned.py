"""Training data and training of the learned preconditioner (library calls only).

The network is not part of the paper's method.  Training recipe:
  * target vectors x: the plain solver's lowest modes of Q(m0) (n_modes per
    field) and Gaussian vectors, weight 1:1;
  * pairs (x, Q(m0)^2 x), loss (1/N) sum |M(Q^2 x) - x|^2 / |x|^2;
  * Adam on the GPU (cstar_nn_train), one step per field per pass;
  * initial weights: M = s0 * 1 through channel 0 (s0 = 1 / (4 + m0)^2, the
    inverse of Q^2's diagonal), plus small Gaussian noise on every weight so
    that the hidden channels are not stuck at the symmetric point.
The network is local and translation invariant, so its weights do not depend
on the lattice size: it can be trained on small lattices of the workload's
field distribution and used on large ones.
"""
from __future__ import annotations

import numpy as np

from . import cstar, synth

NN_CHANNELS = (1, 8, 8, 1)


def initial_weights(m0: float, noise: float = 0.01, seed: int = 0) -> np.ndarray:
    """Flat FP32 weights (layout of include/cstar.h): scaled identity plus noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = (noise * rng.standard_normal(cstar.NN_PARAMS)).astype(np.float64)
    s0 = 1.0 / (4.0 + m0) ** 2
    off = 0
    for li in range(3):
        cin, cout = NN_CHANNELS[li], NN_CHANNELS[li + 1]
        for s in range(4):
            # W[0][0][p=0][s][s], real part
            w[off + (s * 4 + s) * 2] += s0 if li == 0 else 1.0
        off += cout * cin * 9 * 32
    assert off == cstar.NN_PARAMS
    return w.astype(np.float32)


def training_vectors(g: cstar.Gauge, m0: float, n_modes: int = 4, n_gauss: int = 4, seed: int = 0,
                     tol: float = 1e-6):
    """FP32 native block of n_modes low modes of Q(m0) (plain solver) followed by n_gauss Gaussian vectors."""
    import torch
    T, L = g.T, g.L
    shape = (n_modes + n_gauss, T, 2 * L, L, L, 4, 3)
    canon = torch.empty(shape, dtype=torch.complex64, device="cuda")
    if n_modes:
        ev = g.new_native(n_modes, cstar.FP64)
        g.lowest_eigs(m0, n_modes, cstar.eig_opts(tol=tol, seed=seed + 1), evecs=ev)
        c64 = torch.empty((n_modes,) + shape[1:], dtype=torch.complex128, device="cuda")
        g.unpack(ev, c64, cstar.FP64, n_modes)
        canon[:n_modes] = c64.to(torch.complex64)
    if n_gauss:
        gs = synth.random_spinor(T, L, seed + 2, nrhs=n_gauss).astype(np.complex64)
        canon[n_modes:] = torch.from_numpy(gs).cuda()
    nat = g.new_native(n_modes + n_gauss, cstar.FP32)
    g.pack(canon.contiguous(), nat, cstar.FP32, n_modes + n_gauss)
    return nat


def train(gauges, xs, nvec: int, m0: float, epochs: int, lr: float, seed: int = 0):
    """Train a network from initial_weights on the (field, vectors) sets; returns (Net, loss history)."""
    net = cstar.Net(initial_weights(m0, seed=seed))
    hist = net.train(gauges, xs, nvec, m0, epochs, lr)
    return net, hist


def train_online(net, field_fn, n_fields: int, m0: float, steps_per_field: int, lr: float, n_modes: int = 4,
                 n_gauss: int = 4, seed: int = 0, log=None) -> np.ndarray:
    """Streaming training, for lattices whose training sets do not fit in device
    memory together: field i is drawn by field_fn(i) (a Gauge), its n_modes
    plain-solver low modes and n_gauss Gaussian vectors are formed, the network
    takes steps_per_field Adam steps on those pairs (its Adam state carries over
    from field to field), and the field is freed.  Returns the loss of every
    step, [n_fields][steps_per_field]."""
    hist = np.zeros((n_fields, steps_per_field))
    for i in range(n_fields):
        g = field_fn(i)
        x = training_vectors(g, m0, n_modes, n_gauss, seed=seed + 10 * i)
        hist[i] = net.train([g], [x], n_modes + n_gauss, m0, steps_per_field, lr)
        del x
        g.close()
        if log:
            log(i, hist[i])
    return hist
