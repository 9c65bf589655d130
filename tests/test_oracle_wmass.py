"""Pins of the mass-reweighting oracle (oracle/wmass.py) and of the library's
rational approximation (cstar_ratapprox_quartic, host code).

* the product over the rational factors of det(1 + R_i)^{-1}, with S_i as the
  paper prints it, equals det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)] computed from
  its definition (the reading of the factorisation: one factor per (nu_i, mu_i),
  determinants inverted, as the Gaussian estimator delivers them);
* the Gaussian average of exp(-(eta, R eta)), density ~ exp(-(eta, eta)), is
  det(1 + R)^{-1} (Monte Carlo on a small random R, 5 standard errors);
* the rational approximation equioscillates: the attained maximum of
  |log(R(x) x^{1/4})| on a dense grid equals the returned delta, at 2n+2
  alternating extrema, poles and zeros interlace on the negative axis;
* with R covering the spectrum of Q_hat^2, log W_eo + log W_mass equals
  log|pf[C T D_m']| - log|pf[C T D_m]| within 2 N_even delta (the error
  budget of the approximation), the Pfaffian from the dense oracle.
"""
import numpy as np
import pytest

from oracle import dense, dirac, evenodd, pfaffian, sign, wmass
from paper_2108_11989_amd import cstar, synth


@pytest.fixture(scope="module")
def tiny():
    su3, th = synth.make_field(4, 2, 0.4, 17)
    return dirac.Operator(su3, th, 2 / 3, 1.9, 1.0)


def test_factorisation_reproduces_the_definition(tiny):
    m, mp = -0.25, -0.2
    nu2, mu2 = [0.09, 0.6], [0.04, 0.3]
    exact = wmass.log_w_mass_exact(tiny, m, mp, nu2, mu2)
    prod = -sum(np.linalg.slogdet(np.eye(R.shape[0]) + R)[1] for R in wmass.r_operators(tiny, m, mp, nu2, mu2))
    assert abs(prod - exact) < 1e-10 * max(1.0, abs(exact))
    assert abs(exact) > 1e-3  # the masses differ enough for the factor to matter


def test_gaussian_average_is_inverse_determinant():
    rng = np.random.default_rng(5)
    n = 4
    X = 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    R = X + X.conj().T + X.conj().T @ X  # (1 + X)^H (1 + X) - 1
    N = 400000
    eta = (rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n))) / np.sqrt(2)
    x = np.real(np.einsum("li,ij,lj->l", eta.conj(), R, eta))
    w = np.exp(-x)
    ref = 1.0 / np.real(np.linalg.det(np.eye(n) + R))
    assert abs(w.mean() - ref) < 5 * w.std() / np.sqrt(N)


@pytest.mark.parametrize("n,ra,rb", [(3, 0.05, 20.0), (6, 1e-3, 60.0), (10, 1e-4, 80.0)])
def test_rational_approximation_equioscillates(n, ra, rb):
    A, nu2, mu2, delta = cstar.ratapprox_quartic(n, ra, rb)
    x = np.exp(np.linspace(np.log(ra), np.log(rb), 400001))
    e = np.log(A * np.prod((x[:, None] + nu2) / (x[:, None] + mu2), axis=1) * x ** 0.25)
    assert abs(np.abs(e).max() - delta) < 1e-6 * delta
    # 2n+2 alternating extrema of modulus delta
    s = np.sign(e)
    ext = []
    i = 0
    while i < len(e):
        j = i
        while j < len(e) and s[j] == s[i]:
            j += 1
        ext.append(np.abs(e[i:j]).max())
        i = j
    assert len(ext) >= 2 * n + 2
    assert sum(v > delta * (1 - 1e-4) for v in ext) >= 2 * n + 2
    assert np.all(mu2 > 0) and np.all(nu2 > 0) and np.all(mu2 < nu2)
    assert np.all(nu2[:-1] < mu2[1:])


def test_w_eo_times_w_mass_approximates_the_pfaffian_ratio():
    su3, th = synth.make_field(4, 2, 0.4, 19)
    op = dirac.Operator(su3, th, 2 / 3, 1.9, 1.0)
    m, mp = -0.3, -0.22
    specs = []
    for mm in (m, mp):
        Dh = wmass.dense_dhat(op, mm)
        Q = wmass.g5_even(Dh.shape[0])[:, None] * Dh
        specs.append(np.linalg.eigvalsh(Q @ Q))
    ra, rb = 0.9 * min(s.min() for s in specs), 1.1 * max(s.max() for s in specs)
    A, nu2, mu2, delta = cstar.ratapprox_quartic(8, ra, rb)
    lwm = wmass.log_w_mass_exact(op, m, mp, nu2, mu2)
    lweo = evenodd.log_w_eo(op, m, mp)
    _, la = sign.pfaffian_normalised(op, m)
    _, lb = sign.pfaffian_normalised(op, mp)
    n_even = specs[0].size
    assert abs((lb - la) - (lweo + lwm)) <= 2 * n_even * delta
    assert abs(lb - la) > 10 * 2 * n_even * delta  # the check is not trivially satisfied
