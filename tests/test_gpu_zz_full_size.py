"""Full-size parity of the apply at the batched 32^4 workload (32x32^3, eps 0.3,
seed 2, 10 smoothing steps, q = 2/3), in the launch configuration of the
benchmark step: one multi-RHS launch of the BF16-link form with 16
right-hand sides, each at its own mass (every other mass of the 32-point kappa
path).

* Every entry of the first and the last output equals the oracle in its
  BF16-link emulation mode on the FP32-rounded inputs, max |diff| <= 2e-6
  max |ref| (FP32 arithmetic over ~100 terms, as on the small lattices).
* A single-RHS launch of the first input gives the same output bit for bit
  (the two launches differ only in the cache policy of the clover loads).
* The FP64 form on the first input equals the exact oracle, <= 1e-13.

The paper-scale 64x32^3 launch is checked the same way, and the sign over
the 32^4 path by the driver's two orders (see the tests).

Collected near the end: these tests hold the most host memory (about 30 GB
for the paper-scale oracle) and take about three minutes, mostly in the
host-side oracle and the two signs.
"""
import numpy as np
import pytest

from oracle import dirac as odirac
from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NRHS = 16


def _relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_apply_32_4_batched_workload_multi_rhs():
    assert torch.cuda.is_available(), "GPU tests need a device"
    w = synth.WORKLOADS["batched_32^4"]
    T, L, q = w["T"], w["L"], w["q"][0]
    print("full size: 32^4 field", flush=True)
    su3, th = synth.make_field(T, L, w["eps"], w["seed"], smear_steps=w["smear"], smear_backend="torch")
    g = cstar.Gauge(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    idx = np.linspace(0, len(w["kappas"]) - 1, NRHS).round().astype(int)
    masses = [float(m) for m in synth.kappa_to_m0(w["kappas"][idx])]
    assert len(set(masses)) == NRHS
    psi = synth.random_spinor(T, L, 424242, nrhs=NRHS, dtype=np.complex64)

    print(f"full size: BF16-link launch with {NRHS} right-hand sides", flush=True)
    prec = cstar.FP32_BF16LINKS
    canon = torch.from_numpy(psi).cuda().contiguous()
    nin, nout = g.new_native(NRHS, prec), g.new_native(NRHS, prec)
    g.pack(canon, nin, prec, NRHS)
    g.apply(nin, nout, masses, prec, False)
    res = torch.empty_like(canon)
    g.unpack(nout, res, prec, NRHS)
    # the first input alone, single-RHS launch
    one_in, one_out = g.new_native(1, prec), g.new_native(1, prec)
    g.pack(canon[:1].contiguous(), one_in, prec, 1)
    g.apply(one_in, one_out, masses[:1], prec, False)
    one = torch.empty_like(canon[:1])
    g.unpack(one_out, one, prec, 1)
    torch.cuda.synchronize()
    assert torch.equal(one[0], res[0])
    picks = {j: res[j].cpu().numpy().astype(np.complex128) for j in (0, NRHS // 2, NRHS - 1)}
    del canon, res, one, nin, nout, one_in, one_out

    print("full size: oracle, BF16-link emulation", flush=True)
    opb = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1, link_mode=2)
    for j, out in picks.items():  # first, a middle and the last right-hand side
        ref = opb.apply(psi[j].astype(np.complex128), masses[j], False)
        err = _relerr(out, ref)
        print(f"  rhs {j} (m0 {masses[j]:+.4f}): max rel diff {err:.2e}", flush=True)
        assert err < 2e-6
    del opb

    print("full size: FP64 form against the exact oracle", flush=True)
    p64 = psi[0].astype(np.complex128)
    c64 = torch.from_numpy(p64[None]).cuda().contiguous()
    n64_in, n64_out = g.new_native(1, cstar.FP64), g.new_native(1, cstar.FP64)
    g.pack(c64, n64_in, cstar.FP64, 1)
    g.apply(n64_in, n64_out, masses[:1], cstar.FP64, False)
    r64 = torch.empty_like(c64)
    g.unpack(n64_out, r64, cstar.FP64, 1)
    torch.cuda.synchronize()
    out64 = r64[0].cpu().numpy()
    op = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    err = _relerr(out64, op.apply(p64, masses[0], False))
    print(f"  FP64: max rel diff {err:.2e}", flush=True)
    assert err < 1e-13
    g.close()


def test_apply_64x32_3_paper_scale_multi_rhs():
    """The paper-scale instance (64x32^3, eps 0.25, seed 4, no smoothing) at
    its second charge, q = -1/3: one BF16-link launch of 16 right-hand sides at
    16 masses of the 48-point path (the launch the sign solver issues there);
    the first and the last output against the oracle's BF16-link emulation
    (<= 2e-6), and the FP64 form of the first against the exact oracle
    (<= 1e-13)."""
    assert torch.cuda.is_available(), "GPU tests need a device"
    w = synth.WORKLOADS["paper_64x32^3"]
    T, L, q = w["T"], w["L"], w["q"][1]
    print("paper scale: 64x32^3 field", flush=True)
    su3, th = synth.make_field(T, L, w["eps"], w["seed"], smear_steps=w["smear"])
    g = cstar.Gauge(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    idx = np.linspace(0, len(w["kappas"]) - 1, NRHS).round().astype(int)
    masses = [float(m) for m in synth.kappa_to_m0(w["kappas"][idx])]
    psi = synth.random_spinor(T, L, 515151, nrhs=NRHS, dtype=np.complex64)

    print(f"paper scale: BF16-link launch with {NRHS} right-hand sides", flush=True)
    prec = cstar.FP32_BF16LINKS
    canon = torch.from_numpy(psi).cuda().contiguous()
    nin, nout = g.new_native(NRHS, prec), g.new_native(NRHS, prec)
    g.pack(canon, nin, prec, NRHS)
    g.apply(nin, nout, masses, prec, True)
    res = torch.empty_like(canon)
    g.unpack(nout, res, prec, NRHS)
    torch.cuda.synchronize()
    picks = {j: res[j].cpu().numpy().astype(np.complex128) for j in (0, NRHS - 1)}
    del canon, res, nin, nout

    opb = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1, link_mode=2)
    for j, out in picks.items():
        ref = opb.apply(psi[j].astype(np.complex128), masses[j], True)
        err = _relerr(out, ref)
        print(f"  rhs {j} (m0 {masses[j]:+.4f}): max rel diff {err:.2e}", flush=True)
        assert err < 2e-6
    del opb

    p64 = psi[0].astype(np.complex128)
    c64 = torch.from_numpy(p64[None]).cuda().contiguous()
    n64_in, n64_out = g.new_native(1, cstar.FP64), g.new_native(1, cstar.FP64)
    g.pack(c64, n64_in, cstar.FP64, 1)
    g.apply(n64_in, n64_out, masses[:1], cstar.FP64, True)
    r64 = torch.empty_like(c64)
    g.unpack(n64_out, r64, cstar.FP64, 1)
    torch.cuda.synchronize()
    op = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    err = _relerr(r64[0].cpu().numpy(), op.apply(p64, masses[0], True))
    print(f"  FP64: max rel diff {err:.2e}", flush=True)
    assert err < 1e-13
    g.close()


def test_sign_32_4_batched_workload_two_orders():
    """The sign over the batched workload's 32-point kappa path (32^4, k = 4,
    eigenvalue tolerance 1e-8, mixed precision) by the driver's two orders:
    the default one (m_max first, step A down, certified crossing counts of the
    block solver's eigenvalues) and the paper's (step A upward from the target
    with lambda_bar from the power method on Q^-2, then step B above the
    hand-over).  They decide by different means and must give the same 32
    signs; the smoothed field is nearly free and its lowest |lambda| at the
    lightest mass (about 0.336) is far from zero, so every sign is +1."""
    assert torch.cuda.is_available(), "GPU tests need a device"
    w = synth.WORKLOADS["batched_32^4"]
    T, L, q = w["T"], w["L"], w["q"][0]
    print("sign 32^4: field", flush=True)
    su3, th = synth.make_field(T, L, w["eps"], w["seed"], smear_steps=w["smear"], smear_backend="torch")
    path = np.asarray(synth.kappa_to_m0(w["kappas"]), dtype=np.float64)
    signs = {}
    for name, step_a in (("default", False), ("step_a", True)):
        g = cstar.Gauge(torch.from_numpy(su3).cuda(), torch.from_numpy(th).cuda(), q, synth.CSW_SU3, synth.CSW_U1)
        print(f"sign 32^4: {name} order", flush=True)
        sg, rep = g.pfaffian_sign(path, k=4, eig=cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=1e-8, max_iter=1000),
                                  step_a_power=step_a)
        print(f"  {name}: {rep.n_points} masses solved, {rep.seconds:.1f} s, crossings {rep.n_crossings}", flush=True)
        signs[name] = sg.copy()
        g.close()
    assert np.array_equal(signs["default"], signs["step_a"])
    assert np.all(signs["default"] == 1)
