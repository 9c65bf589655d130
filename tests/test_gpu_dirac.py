"""GPU parity of the Dirac operator (dirac_apply through the C ABI) against the oracle.

FP64: element-wise against the FP64 oracle, max |diff| <= 1e-13 * max |ref|
(the kernel and the oracle sum the same ~100 terms per entry in different
orders: a few ulp of the largest term).
FP32 / BF16-link forms: against the oracle in its link-emulation mode (the
same rounded links, FP64 arithmetic) on the FP32-rounded input, with
max |diff| <= 2e-6 * max |ref| (FP32 arithmetic over ~100 terms: about
8 * 2^-24 * sqrt(100) of the largest term, with margin); the distance to the
exact FP64 operator is reported by the precision tests.
Lattices include a partial last tile (the launch rounds up to 256 threads)
and the extent-2 directions of the smallest lattice.
"""
import numpy as np
import pytest

from oracle import dirac as odirac
from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [
    # T, L, eps, seed, q, time_bc
    (4, 2, 0.3, 0, 2 / 3, 1),
    (6, 4, 0.5, 3, -1 / 3, 1),
    (4, 4, 1.0, 7, 2 / 3, -1),
    (8, 6, 0.3, 11, 2 / 3, 1),
    (2, 2, 0.8, 5, 1.0, -1),
    # L >= 8: the time-marching kernel (one segment; T not a multiple of its 8-slice segment)
    (4, 8, 0.4, 13, 2 / 3, -1),
    (10, 8, 0.6, 17, -1 / 3, 1),
]


def _setup():
    assert torch.cuda.is_available(), "GPU tests need a device"


def gpu_apply(g, psi, masses, prec, gamma5):
    """psi: canonical numpy [nrhs, ...] -> canonical numpy result via native layout."""
    nrhs = psi.shape[0]
    cdt = torch.complex128 if prec == cstar.FP64 else torch.complex64
    canon = torch.from_numpy(psi).to(cdt).cuda().contiguous()
    nin = g.new_native(nrhs, prec)
    nout = g.new_native(nrhs, prec)
    g.pack(canon, nin, prec, nrhs)
    g.apply(nin, nout, masses, prec, gamma5)
    res = torch.empty_like(canon)
    g.unpack(nout, res, prec, nrhs)
    torch.cuda.synchronize()
    return res.cpu().numpy()


def _relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("gamma5", [False, True])
def test_fp64_apply_matches_oracle(case, gamma5):
    _setup()
    T, L, eps, seed, q, tbc = case
    print(f"fp64 apply T={T} L={L} seed={seed} g5={gamma5}", flush=True)
    su3, th = synth.make_field(T, L, eps, seed)
    g = cstar.Gauge(su3, th, q, synth.CSW_SU3, synth.CSW_U1, time_bc=tbc)
    op = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1, time_bc=tbc)
    psi = synth.random_spinor(T, L, seed + 100, nrhs=1)
    for m0 in (-0.4, 0.25):
        out = gpu_apply(g, psi, [m0], cstar.FP64, gamma5)[0]
        ref = op.apply(psi[0], m0, gamma5)
        assert _relerr(out, ref) < 1e-13
    g.close()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec,mode", [(cstar.FP32, 1), (cstar.FP32_BF16LINKS, 2)])
def test_fp32_forms_match_emulating_oracle(case, prec, mode):
    _setup()
    T, L, eps, seed, q, tbc = case
    print(f"fp32 apply prec={prec} T={T} L={L}", flush=True)
    su3, th = synth.make_field(T, L, eps, seed)
    g = cstar.Gauge(su3, th, q, synth.CSW_SU3, synth.CSW_U1, time_bc=tbc)
    op = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1, time_bc=tbc, link_mode=mode)
    ope = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1, time_bc=tbc, link_mode=0)
    psi = synth.random_spinor(T, L, seed + 200, nrhs=1).astype(np.complex64).astype(np.complex128)
    for gamma5 in (False, True):
        out = gpu_apply(g, psi, [-0.3], prec, gamma5)[0]
        ref = op.apply(psi[0], -0.3, gamma5)
        assert _relerr(out, ref) < 2e-6
        exact = ope.apply(psi[0], -0.3, gamma5)
        d = _relerr(out, exact)
        print(f"  distance to the exact FP64 operator: {d:.2e}")
        assert d < (2e-6 if mode == 1 else 2e-2)
    g.close()


@pytest.mark.parametrize("T,L", [(6, 4), (6, 8)])
@pytest.mark.parametrize("prec", [cstar.FP64, cstar.FP32_BF16LINKS])
def test_multi_rhs_matches_single(prec, T, L):
    _setup()
    su3, th = synth.make_field(T, L, 0.4, 21)
    g = cstar.Gauge(su3, th, 2 / 3)
    masses = [-0.5, -0.1, 0.0, 0.3, 1.2]
    psi = synth.random_spinor(T, L, 9, nrhs=len(masses))
    if prec != cstar.FP64:
        psi = psi.astype(np.complex64).astype(np.complex128)
    multi = gpu_apply(g, psi, masses, prec, True)
    for j, m in enumerate(masses):
        single = gpu_apply(g, psi[j:j + 1], [m], prec, True)[0]
        assert np.array_equal(single, multi[j])  # same code, same order: bitwise
    op = odirac.Operator(su3, th, 2 / 3, link_mode=0 if prec == cstar.FP64 else 2)
    for j, m in enumerate(masses):
        ref = op.apply(psi[j], m, True)
        assert _relerr(multi[j], ref) < (1e-13 if prec == cstar.FP64 else 2e-6)
    g.close()


@pytest.mark.parametrize("prec", [cstar.FP64, cstar.FP32])
def test_pack_unpack_roundtrip_is_exact(prec):
    _setup()
    T, L = 4, 4
    su3, th = synth.make_field(T, L, 0.3, 1)
    g = cstar.Gauge(su3, th, 2 / 3)
    psi = synth.random_spinor(T, L, 3, nrhs=3)
    cdt = torch.complex128 if prec == cstar.FP64 else torch.complex64
    canon = torch.from_numpy(psi).to(cdt).cuda()
    nat = g.new_native(3, prec)
    g.pack(canon, nat, prec, 3)
    back = torch.empty_like(canon)
    g.unpack(nat, back, prec, 3)
    torch.cuda.synchronize()
    assert torch.equal(back, canon)
    g.close()


def test_apply_16_4_full_lattice():
    """The single-vector workload lattice (16^4, eps 0.2, q = -1/3), every entry."""
    _setup()
    w = synth.WORKLOADS["single_16^4"]
    su3, th = synth.make_field(w["T"], w["L"], w["eps"], w["seed"])
    q = w["q"][0]
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    m0 = float(synth.kappa_to_m0(w["kappas"][0]))
    psi = synth.random_spinor(w["T"], w["L"], 77, nrhs=1)
    out = gpu_apply(g, psi, [m0], cstar.FP64, False)[0]
    assert _relerr(out, op.apply(psi[0], m0)) < 1e-13
    opb = odirac.Operator(su3, th, q, link_mode=2)
    p32 = psi.astype(np.complex64).astype(np.complex128)
    outb = gpu_apply(g, p32, [m0], cstar.FP32_BF16LINKS, True)[0]
    assert _relerr(outb, opb.apply(p32[0], m0, True)) < 2e-6
    g.close()


def test_clover_norm_bound_is_rigorous():
    """The handle's clover norm bound is >= the largest spectral norm of SW(x)."""
    _setup()
    from oracle import dense
    T, L = 2, 2
    su3, th = synth.make_field(T, L, 0.6, 4)
    g = cstar.Gauge(su3, th, 2 / 3)
    opc = odirac.Operator(su3, th, 2 / 3)
    opn = odirac.Operator(su3, th, 2 / 3, clover=False)
    SW = dense.dense_D(opc, 0.0) - dense.dense_D(opn, 0.0)
    smax = max(np.linalg.norm(SW[12 * s:12 * s + 12, 12 * s:12 * s + 12], 2) for s in range(SW.shape[0] // 12))
    b = g.clover_norm_max()
    assert smax <= b <= 3.0 * smax + 1e-12
    g.close()


def test_apply_rejects_bad_arguments_before_any_launch():
    """Empty input, a non-finite mass, aliasing blocks, an unknown precision and
    too many right-hand sides are refused with EINVAL (no kernel runs)."""
    _setup()
    su3, th = synth.make_field(4, 2, 0.3, 0)
    g = cstar.Gauge(su3, th, 2 / 3)
    a, b = g.new_native(2, cstar.FP64), g.new_native(2, cstar.FP64)
    for masses, x, y, prec in (([], a, b, cstar.FP64), ([0.1, np.nan], a, b, cstar.FP64),
                               ([0.1, np.inf], a, b, cstar.FP64), ([0.1, 0.2], a, a, cstar.FP64),
                               ([0.1], a, b, 7)):
        with pytest.raises(cstar.CstarError) as e:
            g.apply(x, y, masses, prec)
        assert e.value.status == cstar.EINVAL
    big_in, big_out = g.new_native(4097, cstar.FP64), g.new_native(4097, cstar.FP64)
    with pytest.raises(cstar.CstarError) as e:
        g.apply(big_in, big_out, np.zeros(4097), cstar.FP64)
    assert e.value.status == cstar.EINVAL
    g.close()


@pytest.mark.parametrize("prec", [cstar.FP64, cstar.FP32_BF16LINKS])
def test_apply_at_the_largest_width(prec):
    """4096 right-hand sides (the largest launch) at 4096 masses on the 4x2^3
    lattice: sampled right-hand sides, the first, the last and a ragged middle
    one, equal the single-RHS launch bit for bit and the oracle within the
    form's bound."""
    _setup()
    su3, th = synth.make_field(4, 2, 0.3, 0)
    g = cstar.Gauge(su3, th, 2 / 3)
    n = 4096
    masses = np.linspace(-0.5, 2.0, n)
    psi = synth.random_spinor(4, 2, 123, nrhs=n)
    out = gpu_apply(g, psi, masses, prec, True)
    mode = 0 if prec == cstar.FP64 else 2
    op = odirac.Operator(su3, th, 2 / 3, synth.CSW_SU3, synth.CSW_U1, link_mode=mode)
    tol = 1e-13 if prec == cstar.FP64 else 2e-6
    for j in (0, 1777, n - 1):
        single = gpu_apply(g, psi[j:j + 1], masses[j:j + 1], prec, True)[0]
        assert np.array_equal(out[j], single), j
        x = psi[j] if prec == cstar.FP64 else psi[j].astype(np.complex64).astype(np.complex128)
        ref = op.apply(x, masses[j], True)
        assert _relerr(out[j], ref) <= tol, j
    g.close()
