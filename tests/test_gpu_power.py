"""GPU parity of q_lambda_bar_power (power method with Chebyshev acceleration
on Q^-2, the paper's lambda_bar solver for step A) through the C ABI.

Tiny lattices: lambda_bar must equal the dense oracle's min |lambda(Q)| within
the reported half-width (plus the dense solver's own rounding), the half-width
must meet the requested tolerance, and sqrt(theta) may not fall below the true
lambda_bar (a Rayleigh quotient of Q^2 bounds its lowest eigenvalue from
above).  Smoothed 8^4 field: the power method agrees with the block
eigensolver's lowest |lambda| within both bounds.  Error paths: bad options
raise EINVAL; a capped iteration returns ENOCONV with the last iterate.
"""
import numpy as np
import pytest

from oracle import sign as osign
from oracle import dirac as odirac
from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# dense eigh rounding: a small multiple of eps * ||Q|| with ||Q|| < 20 on these fields
DENSE_EPS = 64 * 2.2e-16 * 20

TINY = [
    # T, L, eps, seed, q, time_bc, masses
    (4, 2, 0.5, 1, 2 / 3, 1, (-0.3, 0.0, 0.4)),
    (4, 2, 1.0, 21, -1 / 3, -1, (-1.2, -0.5)),
    (6, 2, 0.7, 3, 2 / 3, 1, (-0.6,)),
]


@pytest.mark.parametrize("inner", [cstar.FP64, cstar.FP32_BF16LINKS])
@pytest.mark.parametrize("case", TINY)
def test_lambda_bar_power_matches_dense_oracle(case, inner):
    assert torch.cuda.is_available(), "GPU tests need a device"
    T, L, eps, seed, q, tbc, masses = case
    su3, th = synth.make_field(T, L, eps, seed)
    g = cstar.Gauge(su3, th, q, time_bc=tbc)
    op = odirac.Operator(su3, th, q, time_bc=tbc)
    for m in masses:
        print(f"lambda_bar power T={T} L={L} seed={seed} m={m}", flush=True)
        ref = float(np.min(np.abs(osign.pair_spectrum(op, m))))
        lam, bound, st = g.lambda_bar_power(m, tol=1e-10, max_outer=2000, inner=inner)
        print(f"  lambda {lam:.15f} ref {ref:.15f} bound {bound:.2e} outer {st.outer} solves {st.solves} "
              f"cg {st.cg_iterations}")
        assert bound <= 1e-10 * lam
        assert abs(lam - ref) <= bound + DENSE_EPS
        assert lam >= ref - DENSE_EPS
        # two applies per CG iteration and per outer residual; an FP32 solve adds
        # the two FP64 applies of its own residual check
        if inner == cstar.FP64:
            assert st.applies_fp64 == 2 * (st.cg_iterations + st.outer + 1) and st.applies_inner == 0
        else:
            assert st.applies_inner > 0
            assert st.applies_fp64 + st.applies_inner >= 2 * (st.cg_iterations + st.outer + 1)
    g.close()


@pytest.mark.parametrize("inner", [cstar.FP64, cstar.FP32_BF16LINKS])
def test_lambda_bar_power_agrees_with_block_solver_8_4(inner):
    """Smoothed 8^4 field of the batched workload's distribution at kappa 0.1365."""
    su3, th = synth.make_field(8, 8, 0.3, 2, smear_steps=10)
    g = cstar.Gauge(su3, th, 2 / 3)
    m = float(synth.kappa_to_m0(0.1365))
    ev, res, _ = g.lowest_eigs(m, 2, cstar.eig_opts(inner=cstar.FP64, tol=1e-10, max_iter=1000))
    lam, bound, st = g.lambda_bar_power(m, tol=1e-3, max_outer=300, inner=inner)
    print(f"8^4: power {lam:.10f} +- {bound:.2e} ({st.outer} outer, {st.solves} solves, {st.cg_iterations} CG, "
          f"{st.seconds:.2f} s); block solver {abs(ev[0]):.10f} +- {res[0]:.1e}")
    assert bound <= 1e-3 * lam
    assert abs(lam - abs(ev[0])) <= bound + res[0]
    assert lam >= abs(ev[0]) - res[0]
    g.close()


def test_lambda_bar_power_errors():
    su3, th = synth.make_field(4, 2, 0.5, 1)
    g = cstar.Gauge(su3, th, 2 / 3)
    with pytest.raises(cstar.CstarError):
        g.lambda_bar_power(0.0, degree=65)
    with pytest.raises(cstar.CstarError):
        g.lambda_bar_power(0.0, tol=-1.0)
    with pytest.raises(cstar.CstarError):
        g.lambda_bar_power(float("nan"))
    with pytest.raises(cstar.CstarError):
        g.lambda_bar_power(0.0, inner=7)
    # one outer step cannot reach 1e-14: ENOCONV, last iterate returned
    lam, bound, st = g.lambda_bar_power(0.0, tol=1e-14, max_outer=1, raise_on_noconv=False)
    assert st.outer == 1 and lam > 0.0 and bound > 1e-14 * lam
    with pytest.raises(cstar.CstarError):
        g.lambda_bar_power(0.0, tol=1e-14, max_outer=1)
    g.close()
