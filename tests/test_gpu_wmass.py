"""Mass-reweighting factor on the GPU (cstar_w_mass) against the dense oracle
(mass-reweighting section: W_mass = det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)], its
factors det(1 + R_i)^{-1} estimated by Gaussian sources on the even sites).

The sources are drawn here (seeded) and handed to both sides.  Every
exponent x_il = (eta_l, R_i eta_l) equals the oracle's dense value within
1e-7 relative (FP64 conjugate gradients to 1e-12 residual on operators of
condition ~1e4), and the estimate log W_mass = sum_i log mean_l exp(-x_il)
equals the oracle's from its exponents.  The rational function is the
library's order-(4,4) approximation of x^{-1/4} on the spectrum of Q_hat^2.
"""
import numpy as np
import pytest

from oracle import dirac as odirac
from oracle import evenodd, wmass
from paper_2108_11989_amd import cstar, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("T,L,eps,seed,q", [(4, 2, 0.4, 17, 2 / 3), (4, 4, 0.3, 23, -1 / 3)])
def test_w_mass_matches_dense_oracle(T, L, eps, seed, q):
    assert torch.cuda.is_available(), "GPU tests need a device"
    print(f"w_mass T={T} L={L}", flush=True)
    su3, th = synth.make_field(T, L, eps, seed)
    op = odirac.Operator(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    g = cstar.Gauge(su3, th, q, synth.CSW_SU3, synth.CSW_U1)
    m, mp = -0.3, -0.26
    specs = []
    for mm in (m, mp):
        Dh = wmass.dense_dhat(op, mm)
        Qh = wmass.g5_even(Dh.shape[0])[:, None] * Dh
        specs.append(np.linalg.eigvalsh(Qh @ Qh))
    A, nu2, mu2, delta = cstar.ratapprox_quartic(4, 0.9 * min(s.min() for s in specs),
                                                 1.1 * max(s.max() for s in specs))
    nsrc = 3
    ev = evenodd.parity_sites(T, L) == 0
    full = synth.random_spinor(T, L, 900 + seed, nrhs=nsrc) / np.sqrt(2.0)  # density ~ exp(-(eta, eta))
    full.reshape(nsrc, -1, 12)[:, ~ev] = 0.0
    etas = np.stack([full[l].reshape(-1, 12)[ev].reshape(-1) for l in range(nsrc)])
    canon = torch.from_numpy(full).cuda().contiguous()
    nat = g.new_native(nsrc, cstar.FP64)
    g.pack(canon, nat, cstar.FP64, nsrc)
    per = nat.numel() // nsrc
    eta_dev = torch.cat([nat[l * per: l * per + per // 2] for l in range(nsrc)]).contiguous()
    lw, expo, st = g.w_mass(m, mp, nu2, mu2, eta_dev, tol=1e-12)
    ref = wmass.exponents(op, m, mp, nu2, mu2, etas)
    print(f"  gpu {expo.ravel()}\n  ref {ref.ravel()}\n  {st.cg_iterations} CG iterations, "
          f"{st.eo_applies} applies, {st.seconds:.2f} s", flush=True)
    assert np.all(np.abs(expo - ref) <= 1e-7 * np.maximum(1.0, np.abs(ref)))
    assert abs(lw - wmass.log_estimate(ref)) <= 1e-7 * max(1.0, abs(lw))
    g.close()
