"""Sign of the Pfaffian from its definitions (oracle; test infrastructure only).

Paper, sign-of-the-Pfaffian section:
  pf[CTD] = prod_{n=1}^{12V} lambda_n (one eigenvalue of Q = g5 D per Kramers
  pair), so W_sgn = (-1)^{N(m0)} with N the number of negative lambda_n;
  |lambda_n'(m0)| <= 1 (Feynman-Hellmann, Q'(m0) = g5), hence no eigenvalue
  crosses zero for |m - m0| < lambda_bar(m0) = min_n |lambda_n(m0)|;
  step A: m^(0) = target; stop with "step B" as soon as lambda_bar decreases,
  stop with W_sgn = 1 above m_max, else m^(n+1) = m^(n) + c lambda_bar^(n).

Normalisation of the Pfaffian: W(m) = pf[(C x 1) P_tau D(m)] / pf[(C x 1) P_tau]
(the denominator has modulus one and fixes the basis-ordering sign), so that
W(m) -> +inf as m -> +inf as the paper requires.
"""
from __future__ import annotations

import numpy as np

from . import dense, pfaffian


def pair_spectrum(op, m0: float, tol: float = 1e-9):
    """One eigenvalue per Kramers pair of Q(m0), ascending (dense)."""
    D = dense.dense_D(op, m0)
    ev = np.linalg.eigvalsh(dense.q_from_d(D))
    scale = max(1.0, np.max(np.abs(ev)))
    lam, _ = dense.kramers_pairs(ev, tol * scale)
    return lam


def sign_inertia(op, m0: float) -> int:
    """W_sgn = (-1)^N, N = number of negative eigenvalues of Q per Kramers pair."""
    lam = pair_spectrum(op, m0)
    return -1 if int(np.sum(lam < 0)) % 2 else 1


def pfaffian_normalised(op, m0: float):
    """(phase, log|W|) of W(m0) = pf[(C x 1) P_tau D] / pf[(C x 1) P_tau]."""
    D = dense.dense_D(op, m0)
    A = dense.antisymmetric_form(D, op.T, op.L)
    A0 = dense.antisymmetric_unit(op.T, op.L)
    ph, la = pfaffian.pfaffian_logphase(A)
    ph0, la0 = pfaffian.pfaffian_logphase(A0)
    return ph / ph0, la - la0


def sign_pfaffian(op, m0: float) -> int:
    ph, _ = pfaffian_normalised(op, m0)
    if abs(ph.imag) > 1e-6:
        raise ValueError(f"Pfaffian not real: phase {ph}")
    return 1 if ph.real > 0 else -1


def step_a(lambda_bar, m_target: float, c: float, m_max: float, max_steps: int = 10000):
    """The paper's step A with an eigenvalue provider lambda_bar(m) -> float.

    Returns (outcome, trace) with outcome "W=1" (m exceeded m_max without a
    decrease of lambda_bar) or "B" (lambda_bar decreased: step B needed), and
    trace the list of (m, lambda_bar).
    """
    m = m_target
    trace = []
    prev = None
    for _ in range(max_steps):
        lb = float(lambda_bar(m))
        trace.append((m, lb))
        if prev is not None and lb < prev:
            return "B", trace
        if m > m_max:
            return "W=1", trace
        prev = lb
        m = m + c * lb
    raise RuntimeError("step A did not terminate")
