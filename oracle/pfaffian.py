"""Pfaffian of a complex antisymmetric matrix (oracle; test infrastructure only).

pf[M]^2 = det[M] for antisymmetric M (the algebraic relation the paper uses
to write pf[CTD] = W_sgn |det D|^{1/2}).

`pfaffian_logphase` reduces A by congruences M A M^T with unit-determinant
M (Gauss steps with pivoting on the first row), pf(M A M^T) = det(M) pf(A):
with a = A[0,1], r = A[0,2:], s = A[1,2:], B = A[2:,2:],
    pf(A) = a * pf(B + (s r^T - r s^T) / a),
and a transposition of rows/columns 1 and j changes the sign.  The value is
returned as (phase, log|pf|) because |pf| overflows a double on the smallest
lattice at large mass.

`pfaffian_bruteforce` expands along the first row,
    pf(A) = sum_j (-1)^(j+1) A[0,j] pf(A without rows/cols 0, j),
which is exact arithmetic on tiny matrices and pins the reduction.
"""
from __future__ import annotations

import numpy as np


def pfaffian_logphase(A: np.ndarray):
    """(phase, log|pf|) of an even-dimensional complex antisymmetric matrix.

    phase is a unit complex number (0 if the Pfaffian vanishes, log = -inf).
    """
    A = np.array(A, dtype=np.complex128, copy=True)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix required")
    if n % 2:
        return 0.0 + 0.0j, -np.inf
    phase = 1.0 + 0.0j
    logabs = 0.0
    while A.shape[0] > 0:
        m = A.shape[0]
        j = 1 + int(np.argmax(np.abs(A[0, 1:])))
        if A[0, j] == 0:
            return 0.0 + 0.0j, -np.inf
        if j != 1:
            A[[1, j], :] = A[[j, 1], :]
            A[:, [1, j]] = A[:, [j, 1]]
            phase = -phase
        a = A[0, 1]
        phase *= a / abs(a)
        logabs += np.log(abs(a))
        if m == 2:
            break
        r = A[0, 2:]
        s = A[1, 2:]
        A = A[2:, 2:] + (np.outer(s, r) - np.outer(r, s)) / a
    return phase, logabs


def pfaffian(A: np.ndarray) -> complex:
    ph, la = pfaffian_logphase(A)
    return ph * np.exp(la) if np.isfinite(la) else 0.0 + 0.0j


def pfaffian_bruteforce(A: np.ndarray) -> complex:
    """Row expansion of the Pfaffian; O(n!!), for n <= 12."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    if n % 2:
        return 0.0
    if n == 0:
        return 1.0
    total = 0.0 + 0.0j
    for j in range(1, n):
        keep = [k for k in range(n) if k != 0 and k != j]
        sub = A[np.ix_(keep, keep)]
        total += (-1) ** (j + 1) * A[0, j] * pfaffian_bruteforce(sub)
    return total
