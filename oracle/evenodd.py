"""Even-odd decomposition of D and the factor W_eo (oracle; test infrastructure only).

Paper, mass-reweighting section (eq. detQ2 and the definition of W_eo):
with the sites of the doubled lattice split by parity p = (t+x1+x2+x3) mod 2
(every hop changes it, since L is even),

    D = [[D_ee, D_eo], [D_oe, D_oo]],   D_hat = D_ee - D_eo D_oo^{-1} D_oe  (on even sites),
    det D = det D_oo * det D_hat,        Q_hat = g5 D_hat,
    W_eo(m, m') = |det[D_oo(m') D_oo(m)^{-1}]|^{1/2},

where D_oo, the restriction of D to odd sites, keeps only the site-local term
(4+m) + SW(x).  Everything here follows those definitions: dense blocks on
tiny lattices, and an apply of D_hat from two applications of the full
operator with the local inverse in between.
"""
from __future__ import annotations

import numpy as np


def parity_sites(T: int, L: int) -> np.ndarray:
    """Parity of every doubled site, canonical order [T][2L][L][L] (x1 in [0, 2L))."""
    t, x1, x2, x3 = np.meshgrid(np.arange(T), np.arange(2 * L), np.arange(L), np.arange(L), indexing="ij")
    return ((t + x1 + x2 + x3) % 2).reshape(-1)


def eo_index(T: int, L: int):
    """Indices of the even and of the odd entries of a flat [site][spin][colour] vector."""
    par = np.repeat(parity_sites(T, L), 12)
    idx = np.arange(par.size)
    return idx[par == 0], idx[par == 1]


def dense_blocks(D: np.ndarray, T: int, L: int):
    """(D_ee, D_eo, D_oe, D_oo) of a dense D."""
    e, o = eo_index(T, L)
    return D[np.ix_(e, e)], D[np.ix_(e, o)], D[np.ix_(o, e)], D[np.ix_(o, o)]


def dense_dhat(D: np.ndarray, T: int, L: int) -> np.ndarray:
    """D_hat = D_ee - D_eo D_oo^{-1} D_oe (dense)."""
    Dee, Deo, Doe, Doo = dense_blocks(D, T, L)
    return Dee - Deo @ np.linalg.solve(Doo, Doe)


def apply_dhat(op, psi_even: np.ndarray, m0: float, gamma5: bool = False) -> np.ndarray:
    """D_hat(m0) psi on even sites (psi_even: flat [even sites][12]); g5 D_hat with gamma5.

    D (psi_e, 0) = (D_ee psi_e, D_oe psi_e);  chi_o = D_oo^{-1} D_oe psi_e;
    D (0, chi_o) = (D_eo chi_o, D_oo chi_o);  D_hat psi_e = D_ee psi_e - D_eo chi_o.
    """
    T, L = op.T, op.L
    par = parity_sites(T, L)
    ev, od = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    full = np.zeros((op.nsites, 12), dtype=np.complex128)
    full[ev] = psi_even.reshape(-1, 12)
    a = op.apply(full.reshape(op.shape), m0).reshape(op.nsites, 12)
    loc = op.local_term(m0)
    chi = np.zeros_like(full)
    chi[od] = np.linalg.solve(loc[od], a[od][..., None])[..., 0]
    b = op.apply(chi.reshape(op.shape), m0).reshape(op.nsites, 12)
    out = a[ev] - b[ev]
    if gamma5:
        out[:, 6:] *= -1.0
    return out.reshape(-1)


def log_w_eo(op, m: float, m_prime: float) -> float:
    """log W_eo = (1/2) sum over odd sites of log|det D_oo(m')(x)| - log|det D_oo(m)(x)|."""
    od = parity_sites(op.T, op.L) == 1
    _, la = np.linalg.slogdet(op.local_term(m_prime)[od])
    _, lb = np.linalg.slogdet(op.local_term(m)[od])
    return 0.5 * float(np.sum(la) - np.sum(lb))
