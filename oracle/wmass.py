"""Mass-reweighting factor W_mass (oracle; test infrastructure only).

Paper, mass-reweighting section: |pf[C T D_m]| = |det D_m^oo|^{1/2} det[Q_hat_m^2]^{1/4},
(Q_hat^2)^{-1/4} replaced by R(Q_hat^2), R(x) = A prod_i (x + nu_i^2)/(x + mu_i^2);
W_mass = det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)] is written as a product over the
rational factors of determinants of positive Hermitian operators 1 + R_i,
R_i = (dD S_i)^H + dD S_i + (dD S_i)^H dD S_i, dD = D_hat_m' - D_hat_m, with
S_i as printed in the paper, and each is estimated by Gaussian sources on the
even sites: the average of exp(-(eta, R_i eta)) is det(1 + R_i)^{-1}.

Dense, on tiny lattices, in the order of those definitions.
"""
from __future__ import annotations

import numpy as np

from . import dense, evenodd


def dense_dhat(op, m: float) -> np.ndarray:
    return evenodd.dense_dhat(dense.dense_D(op, m), op.T, op.L)


def g5_even(n: int) -> np.ndarray:
    return np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), n // 12)


def log_w_mass_exact(op, m: float, mp: float, nu2, mu2) -> float:
    """log det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)] (A cancels)."""
    Dm, Dp = dense_dhat(op, m), dense_dhat(op, mp)
    g5 = g5_even(Dm.shape[0])
    Qm, Qp = g5[:, None] * Dm, g5[:, None] * Dp
    I = np.eye(Dm.shape[0])
    ld = lambda M: np.linalg.slogdet(M)[1]
    out = 0.0
    for a, b in zip(nu2, mu2):
        out += ld(Qm @ Qm + a * I) - ld(Qm @ Qm + b * I) - ld(Qp @ Qp + a * I) + ld(Qp @ Qp + b * I)
    return float(out)


def r_operators(op, m: float, mp: float, nu2, mu2):
    """The Hermitian R_i of every rational factor (dense)."""
    Dm, Dp = dense_dhat(op, m), dense_dhat(op, mp)
    n = Dm.shape[0]
    G5 = np.diag(g5_even(n))
    I = np.eye(n)
    dD = Dp - Dm
    out = []
    for a, b in zip(nu2, mu2):
        Ai = np.linalg.inv(Dm + 1j * np.sqrt(a) * G5)
        Bi = np.linalg.inv(Dp + 1j * np.sqrt(b) * G5)
        S = Ai - Bi - Bi @ dD @ Ai
        X = dD @ S
        out.append(X.conj().T + X + X.conj().T @ X)
    return out


def exponents(op, m: float, mp: float, nu2, mu2, etas: np.ndarray) -> np.ndarray:
    """x_il = (eta_l, R_i eta_l) for sources etas [nsrc, even dim]."""
    Rs = r_operators(op, m, mp, nu2, mu2)
    return np.array([[float(np.real(np.vdot(e, R @ e))) for e in etas] for R in Rs])


def log_estimate(expo: np.ndarray) -> float:
    """sum_i log((1/N) sum_l exp(-x_il))."""
    out = 0.0
    for x in expo:
        mn = np.min(x)
        out += -mn + np.log(np.mean(np.exp(-(x - mn))))
    return float(out)
