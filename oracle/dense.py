"""Dense forms of D and Q on tiny lattices (oracle; test infrastructure only).

Q = g5 D is Hermitian and its spectrum is doubly degenerate (paper,
sign-of-the-Pfaffian section: v and C T g5 v* are orthogonal eigenvectors with
the same eigenvalue).  The lists lambda_n, n = 1..12V, hold one eigenvalue per
Kramers pair.
"""
from __future__ import annotations

import numpy as np

from . import dirac


def dense_D(op: dirac.Operator, m0: float, gamma5: bool = False) -> np.ndarray:
    """Assemble the (24V x 24V) matrix of D(m0) (or Q) column by column."""
    n = op.dim
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = op.apply(e, m0, gamma5).reshape(-1)
        e[j] = 0.0
    return M


def gamma5_diag(nsites: int) -> np.ndarray:
    """Diagonal of g5 on [site][spin][colour]: +1 for spins 0,1 and -1 for spins 2,3."""
    g = np.array([1, 1, -1, -1], dtype=np.float64)
    return np.tile(np.repeat(g, 3), nsites)


def q_from_d(D: np.ndarray) -> np.ndarray:
    g5 = gamma5_diag(D.shape[0] // 12)
    return g5[:, None] * D


def eig_q(Q: np.ndarray):
    """All eigenvalues (ascending) and eigenvectors of the Hermitian Q."""
    return np.linalg.eigh(Q)


def kramers_pairs(evals: np.ndarray, tol: float):
    """Split an ascending spectrum into Kramers pairs.

    Returns one eigenvalue per pair (the mean of the two) and the largest
    in-pair splitting.  Raises if consecutive eigenvalues cannot be paired
    within tol.
    """
    ev = np.sort(evals)
    if ev.size % 2:
        raise ValueError("odd spectrum size")
    a, b = ev[0::2], ev[1::2]
    split = np.max(np.abs(a - b)) if ev.size else 0.0
    if split > tol:
        raise ValueError(f"spectrum not paired: max splitting {split:g} > {tol:g}")
    return 0.5 * (a + b), split


def lowest_abs(lams: np.ndarray, k: int) -> np.ndarray:
    """k smallest |lambda| (one per pair), sorted by |lambda| ascending, ties by lambda."""
    order = np.lexsort((lams, np.abs(lams)))
    return lams[order[:k]]


def tau_permutation(T: int, L: int) -> np.ndarray:
    """Index map of P_tau on the flat [site][spin][colour] vector: (P_tau psi)(x) = psi(x + L e1)."""
    idx = np.arange(2 * T * L ** 3 * 12).reshape(T, 2 * L, L, L, 4, 3)
    return np.roll(idx, -L, axis=1).reshape(-1)


def charge_conjugation() -> np.ndarray:
    """C = i g0 g2 in the oracle's chiral basis (4x4)."""
    g = dirac.gammas()
    return 1j * g[0] @ g[2]


def antisymmetric_form(D: np.ndarray, T: int, L: int) -> np.ndarray:
    """A = (C x 1_colour) P_tau D, the matrix whose Pfaffian is pf[C T D]."""
    perm = tau_permutation(T, L)
    PD = D[perm, :]
    C = charge_conjugation()
    nsites = D.shape[0] // 12
    Cfull = np.kron(np.eye(nsites), np.kron(C, np.eye(3)))
    return Cfull @ PD


def antisymmetric_unit(T: int, L: int) -> np.ndarray:
    """(C x 1) P_tau alone: the normalising matrix of the Pfaffian."""
    n = 2 * T * L ** 3 * 12
    return antisymmetric_form(np.eye(n, dtype=np.complex128), T, L)
