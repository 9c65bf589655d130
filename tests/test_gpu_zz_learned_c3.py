"""What the network trained at 32^4 gains over the method without it, on a
held-out field of the batched workload's distribution (32x32^3, eps 0.3,
10 smoothing steps, q = 2/3).

The weights (`paper_2108_11989_amd/nn_c3_32x32x32x32.npy`) were trained on the
GPU by the library's kernels on 64 fields of that distribution (seeds 1000 to
1063, 4 plain-solver low modes and 4 Gaussian vectors each, 3 Adam steps per
field, streamed) with

    python3 bench.py --c3-train paper_2108_11989_amd/nn_c3_32x32x32x32.npy

On held-out field 2000 at the lightest mass of the path:
  * the trained network approximates (Q^2)^-1 better than its initial weights
    (the scaled identity 1/(4+m)^2): held-out loss below half;
  * the preconditioned eigensolve reproduces the plain solver's eigenvalues
    within their residual bounds (the plain solver is the judge), without
    falling back, and needs fewer applies of D.  Time is reported, not
    asserted: one network application costs about as much as 50 applies of D,
    which the saved applies do not repay.
"""
import os

import numpy as np
import pytest

from paper_2108_11989_amd import cstar, learned, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

T = L = 32
M0 = float(synth.kappa_to_m0(0.1365))
WEIGHTS = os.path.join(os.path.dirname(cstar.__file__), "nn_c3_32x32x32x32.npy")


def _loss(g, weights, x, nvec):
    b = g.new_native(nvec, cstar.FP32)
    tmp = g.new_native(nvec, cstar.FP32)
    g.apply(x, tmp, [M0] * nvec, cstar.FP32, True)
    g.apply(tmp, b, [M0] * nvec, cstar.FP32, True)
    net = cstar.Net(weights)
    loss = net.loss_grad(g, x, b, nvec=nvec)
    net.close()
    return loss


def test_network_trained_at_32_on_held_out_field():
    assert torch.cuda.is_available()
    w = np.load(WEIGHTS, allow_pickle=False)
    assert w.dtype == np.float32 and w.shape == (cstar.NN_PARAMS,) and np.all(np.isfinite(w))
    print("[c3 test] held-out field 2000, 32x32^3", flush=True)
    su3, th = synth.make_field(T, L, 0.3, 2000, smear_steps=10, smear_backend="torch", exp_backend="torch")
    g = cstar.Gauge(torch.from_numpy(su3).cuda(), torch.from_numpy(th).cuda(), 2 / 3)
    del su3, th

    x = learned.training_vectors(g, M0, 4, 4, seed=9000)
    l_init = _loss(g, learned.initial_weights(M0), x, 8)
    l_trained = _loss(g, w, x, 8)
    del x
    print(f"[c3 test] held-out loss: initial {l_init:.4f}, trained {l_trained:.4f}", flush=True)
    assert l_trained < 0.5 * l_init

    net = cstar.Net(w)
    opts = dict(inner=cstar.FP32_BF16LINKS, tol=1e-8, max_iter=1000)
    torch.cuda.synchronize()
    e0, r0, s0 = g.lowest_eigs(M0, 4, cstar.eig_opts(**opts))
    net.attach(g)
    e1, r1, s1 = g.lowest_eigs(M0, 4, cstar.eig_opts(**opts, use_nn=1))
    cstar.Net.detach(g)
    a0, a1 = s0.applies_inner + s0.applies_fp64, s1.applies_inner + s1.applies_fp64
    print(f"[c3 test] plain: {s0.iterations} it, {a0} applies, {s0.seconds:.2f} s; learned: {s1.iterations} it, "
          f"{a1} applies + {s1.nn_applies} network applications, {s1.seconds:.2f} s", flush=True)
    assert s1.nn_fallback == 0
    assert np.all(np.abs(e1 - e0) <= r0 + r1 + 1e-13)
    assert a1 < a0
    net.close()
    g.close()
