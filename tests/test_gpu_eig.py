"""GPU parity of q_lowest_eigs and pfaffian_sign against the oracle.

Eigenvalues: the k smallest |lambda| of Q = g5 D, one per Kramers pair, must
agree with the dense oracle spectrum to 1e-10 relative (FP64 and mixed
precision after FP64 refinement).  Signs: bit-identical to the oracle's dense
inertia (and, on the small fields, its Pfaffian).
"""
import numpy as np
import pytest

from oracle import dense, sign as osign
from oracle import dirac as odirac
from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _tiny():
    w = synth.WORKLOADS["tiny_4x2^3"]
    su3, th = synth.make_field(w["T"], w["L"], w["eps"], w["seed"])
    return w, su3, th, w["q"][0]


@pytest.mark.parametrize("inner", [cstar.FP64, cstar.FP32_BF16LINKS])
def test_lowest_eigs_tiny_all_kappas(inner):
    assert torch.cuda.is_available()
    w, su3, th, q = _tiny()
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    for kappa in w["kappas"]:
        m0 = float(synth.kappa_to_m0(kappa))
        print(f"eig tiny kappa={kappa:.4f} inner={inner}", flush=True)
        lam = osign.pair_spectrum(op, m0)
        ref = dense.lowest_abs(lam, 4)
        ev, res, st = g.lowest_eigs(m0, 4, cstar.eig_opts(inner=inner, tol=1e-12, max_iter=400))
        assert np.all(np.abs(ev - ref) <= 1e-10 * np.abs(ref)), (kappa, ev, ref)
        # reported residuals bound the true error, up to the dense oracle's own
        # rounding (LAPACK eigh: a small multiple of eps * ||Q||, ||Q|| < 20 here)
        assert np.all(np.abs(ev - ref) <= res + 64 * 2.2e-16 * 20)
    g.close()


def test_lowest_eigs_with_residual_directions_tiny():
    """opts.use_nn = 2 (the residuals of the wanted Ritz pairs appended to the
    filtered block, no network): the same eigenvalues as the dense oracle."""
    assert torch.cuda.is_available()
    w, su3, th, q = _tiny()
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    for kappa in w["kappas"][::5]:
        m0 = float(synth.kappa_to_m0(kappa))
        ref = dense.lowest_abs(osign.pair_spectrum(op, m0), 4)
        ev, res, st = g.lowest_eigs(m0, 4, cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=1e-12, max_iter=400,
                                                          use_nn=2))
        assert st.nn_applies == 0 and st.nn_fallback == 0
        assert np.all(np.abs(ev - ref) <= 1e-10 * np.abs(ref)), (kappa, ev, ref)
    g.close()


@pytest.mark.parametrize("lattice", ["tiny", "4x8^3"])
@pytest.mark.parametrize("inner", [cstar.FP64, cstar.FP32_BF16LINKS])
def test_lowest_eigs_returns_eigenvectors(lattice, inner):
    """Eigenpairs checked by the oracle's operator: ||Q v - lambda v|| within the reported bound.
    The 4x8^3 lattice runs the time-marching apply and its fused Chebyshev epilogue."""
    if lattice == "tiny":
        w, su3, th, q = _tiny()
    else:
        su3, th = synth.make_field(4, 8, 0.4, 23, smear_steps=2)
        q = 2 / 3
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    m0 = float(synth.kappa_to_m0(0.11))
    k = 3
    vec = g.new_native(k, cstar.FP64)
    ev, res, st = g.lowest_eigs(m0, k, cstar.eig_opts(inner=inner, tol=1e-12), evecs=vec)
    canon = torch.empty((k,) + op.shape, dtype=torch.complex128, device="cuda")
    g.unpack(vec, canon, cstar.FP64, k)
    torch.cuda.synchronize()
    V = canon.cpu().numpy()
    for i in range(k):
        v = V[i] / np.linalg.norm(V[i])
        r = np.linalg.norm(op.Q(v, m0) - ev[i] * v)
        assert r <= res[i] * 1.01 + 1e-13
    g.close()


def test_pfaffian_sign_tiny_path_matches_dense_inertia():
    w, su3, th, q = _tiny()
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    path = synth.kappa_to_m0(w["kappas"])
    signs, rep = g.pfaffian_sign(path, k=4, eig=cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=1e-10))
    ref = [osign.sign_inertia(op, m) for m in path]
    assert list(signs) == ref
    g.close()


@pytest.mark.parametrize("seed,eps", [(13, 1.2), (21, 1.0), (5, 1.4)])
def test_pfaffian_sign_rough_fields_with_negative_signs(seed, eps):
    """Rough fields whose flow crosses zero: GPU signs equal inertia and the Pfaffian."""
    T, L = 4, 2
    su3, th = synth.make_field(T, L, eps, seed)
    q = 2 / 3
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    path = np.linspace(-2.0, 0.4, 13)
    signs, rep = g.pfaffian_sign(path, k=6, eig=cstar.eig_opts(inner=cstar.FP64, tol=1e-10))
    ref = np.array([osign.sign_inertia(op, m) for m in path])
    refp = np.array([osign.sign_pfaffian(op, m) for m in path])
    assert np.array_equal(ref, refp)
    assert np.array_equal(signs, ref), (signs, ref)
    g.close()


def test_single_16_4_eigenvalues_fp32_vs_fp64():
    """16^4 workload (eps 0.2, q = -1/3, kappa 0.1365), k = 8: the plain FP64 form's
    eigenpairs are certified by the oracle's operator (||Q v - lambda v|| within the
    reported bound), and the mixed form (BF16/FP32 links in the filter, FP64
    Rayleigh-Ritz) agrees with them within the residual bounds at tol 1e-10."""
    w = synth.WORKLOADS["single_16^4"]
    T, L, q = w["T"], w["L"], w["q"][0]
    su3, th = synth.make_field(T, L, w["eps"], w["seed"])
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    m0 = float(synth.kappa_to_m0(w["kappas"][0]))
    k = 8
    vec = g.new_native(k, cstar.FP64)
    e64, r64, s64 = g.lowest_eigs(m0, k, cstar.eig_opts(inner=cstar.FP64, tol=1e-10, max_iter=1000), evecs=vec)
    canon = torch.empty((k,) + op.shape, dtype=torch.complex128, device="cuda")
    g.unpack(vec, canon, cstar.FP64, k)
    torch.cuda.synchronize()
    V = canon.cpu().numpy()
    for i in range(k):
        v = V[i] / np.linalg.norm(V[i])
        r = np.linalg.norm(op.Q(v, m0) - e64[i] * v)
        assert r <= r64[i] * 1.01 + 1e-12
    for inner in (cstar.FP32_BF16LINKS, cstar.FP32):
        em, rm, sm = g.lowest_eigs(m0, k, cstar.eig_opts(inner=inner, tol=1e-10, max_iter=1000))
        err = np.abs(em - e64)
        print(f"16^4 k=8 inner={inner}: |lambda - lambda_fp64| = {err}, FP64 form {s64.iterations} it / "
              f"{s64.applies_fp64} applies, mixed {sm.iterations} it / {sm.applies_inner} + {sm.applies_fp64} applies")
        assert np.all(err <= rm + r64 + 1e-13)
        assert np.all(err <= 1e-10 * np.maximum(np.abs(e64), 1e-3) + rm + r64)
    g.close()


@pytest.mark.parametrize("seed,eps", [(13, 1.2), (21, 1.0), (5, 1.4)])
def test_pfaffian_sign_step_a_power_matches_dense_inertia(seed, eps):
    """The paper's order: step A upward from the lowest path mass with lambda_bar
    from the power method on Q^-2, step B (certified counts) above where it
    stops; on the tiny workload's path and on rough fields with negative signs,
    every sign equals the dense inertia."""
    T, L = 4, 2
    su3, th = synth.make_field(T, L, eps, seed)
    q = 2 / 3
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    path = np.linspace(-2.0, 0.4, 13)
    signs, rep = g.pfaffian_sign(path, k=6, eig=cstar.eig_opts(inner=cstar.FP64, tol=1e-10), step_a_power=True)
    ref = np.array([osign.sign_inertia(op, m) for m in path])
    print(f"step A: {rep.n_points} masses, signs {signs}", flush=True)
    assert np.array_equal(signs, ref), (signs, ref)
    g.close()
    w, su3, th, q = _tiny()
    g = cstar.Gauge(su3, th, q)
    op = odirac.Operator(su3, th, q)
    path = synth.kappa_to_m0(w["kappas"])
    signs, rep = g.pfaffian_sign(path, k=4, eig=cstar.eig_opts(inner=cstar.FP32_BF16LINKS, tol=1e-10),
                                 step_a_power=True)
    assert np.array_equal(signs, [osign.sign_inertia(op, float(m)) for m in path])
    g.close()
