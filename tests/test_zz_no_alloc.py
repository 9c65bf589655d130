"""dirac_apply_noalloc (the entry point for callers that cannot allocate
device memory) against dirac_apply, through the C ABI: on two calls in a row,
the second with fewer right-hand sides (so the shared mass array holds the
first call's masses beyond the second's), every output equals dirac_apply's
bit for bit (the same kernels on the same masses).  Sizes beyond the
array's maximum are rejected."""
import numpy as np
import pytest

from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(g, fn, canon, masses, prec, gamma5):
    n = canon.shape[0]
    nin, nout = g.new_native(n, prec), g.new_native(n, prec)
    g.pack(canon, nin, prec, n)
    nout.fill_(float("nan"))
    fn(nin, nout, masses, prec, gamma5)
    res = torch.empty_like(canon)
    g.unpack(nout, res, prec, n)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("T,L,prec", [(4, 32, cstar.FP32_BF16LINKS), (4, 32, cstar.FP64), (6, 4, cstar.FP32)])
def test_noalloc_equals_dirac_apply(T, L, prec):
    assert torch.cuda.is_available(), "GPU tests need a device"
    print(f"noalloc T={T} L={L} prec={prec}", flush=True)
    su3, th = synth.make_field(T, L, 0.35, 61)
    g = cstar.Gauge(su3, th, 2 / 3, synth.CSW_SU3, synth.CSW_U1)
    cdt = torch.complex128 if prec == cstar.FP64 else torch.complex64
    for n, seed in ((12, 5), (5, 6)):
        masses = list(np.linspace(-0.5, 2.0, n) + 0.01 * seed)
        psi = synth.random_spinor(T, L, seed, nrhs=n)
        canon = torch.from_numpy(psi).to(cdt).cuda().contiguous()
        for gamma5 in (False, True):
            ref = _run(g, g.apply, canon, masses, prec, gamma5)
            out = _run(g, g.apply_noalloc, canon, masses, prec, gamma5)
            assert torch.equal(out, ref), (n, gamma5)
    g.close()


def test_noalloc_rejects_too_many_rhs():
    su3, th = synth.make_field(2, 2, 0.3, 62)
    g = cstar.Gauge(su3, th, 2 / 3)
    n = 1025
    nin, nout = g.new_native(n, cstar.FP32), g.new_native(n, cstar.FP32)
    with pytest.raises(cstar.CstarError) as e:
        g.apply_noalloc(nin, nout, np.zeros(n), cstar.FP32)
    assert e.value.status == cstar.EINVAL
    assert "CSTAR_NOALLOC_MAX_RHS" in str(e.value)
    g.close()
