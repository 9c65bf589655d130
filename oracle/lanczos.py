"""Lowest eigenvalues of Q = g5 D by Lanczos on Q^2 (oracle; test infrastructure only).

For lattices too large for dense work.  What is computed is the plain
definition behind the library's q_lowest_eigs: the k eigenvalues of the
Hermitian Q(m0) smallest in modulus, one per Kramers pair, signed (paper,
sign-of-the-Pfaffian section: the spectrum of Q is doubly degenerate, v and
its Kramers image C T g5 v^* share an eigenvalue, and pf[CTD] is the product
of one eigenvalue per pair).

Method (textbook, no acceleration):
  1. Lanczos on A = Q^2 (Hermitian, positive) in FP64 with full
     reorthogonalisation: every new basis vector is orthogonalised twice
     against the whole basis (classical Gram-Schmidt), and the projected
     matrix H = V^H A V is assembled column by column from those
     coefficients.  The basis is restarted thickly (Wu & Simon, SIAM J.
     Matrix Anal. Appl. 22 (2000) 602): when it holds m vectors, the lowest
     `keep` Ritz vectors and the last residual direction are kept.
  2. Stop when the lowest `want` Ritz values of A have Lanczos residual
     estimates |beta s_m,i| below tol * ||A||_est.
  3. Signed eigenvalues: Rayleigh-Ritz with Q on the span of the converged
     Ritz vectors and their Kramers images (a subspace closed under the
     antiunitary map, so its Q-Ritz values come in exact pairs; a Kramers
     copy that Lanczos converged twice only repeats a direction and drops
     out with the rank), then one value per pair, with the residual
     ||Q z - lambda z|| of each unit Ritz vector as a rigorous error bound.

In exact arithmetic a single Lanczos vector sees one direction of each
eigenspace of A; in floating point the Kramers partner of a converged
direction is seeded by rounding and converges later, so 2 (k + guard) Ritz
values of A are converged and the Kramers closure merges the copies.
Accidental degeneracies beyond the pairs do not occur for random fields.
"""
from __future__ import annotations

import numpy as np

from . import dense


def kramers_image(psi: np.ndarray, L: int) -> np.ndarray:
    """Theta psi = (C g5) psi(tau x)^* on canonical spinors [.., T, 2L, L, L, 4, 3]:
    antiunitary, commutes with Q, Theta^2 = -1 (so v and Theta v are orthogonal
    eigenvectors of Q with the same eigenvalue)."""
    S = dense.charge_conjugation() @ np.diag([1.0, 1.0, -1.0, -1.0])
    return np.einsum("ab,...bc->...ac", S, np.roll(psi, -L, axis=-5).conj())


def lanczos_q2(op, m0: float, want: int, basis: int = 0, keep: int = 0, tol: float = 1e-13,
               max_restarts: int = 2000, seed: int = 1, log=None):
    """Thick-restart Lanczos for the `want` lowest eigenvalues of A = Q(m0)^2.

    Returns (theta[want], X[want, dim] unit Ritz vectors, resid[want] true
    residual norms ||A x - theta x||, matvecs).  tol is relative to an upper
    bound of ||A|| from the first Ritz values."""
    n = op.dim
    shape = op.shape
    m = basis or max(3 * want, want + 40)
    kp = keep or min(m - 20, want + max(10, want // 2))
    if not (want < kp < m):
        raise ValueError("need want < keep < basis")

    def A(x):
        return op.Q(op.Q(x.reshape(shape), m0), m0).reshape(-1)

    rng = np.random.default_rng(seed)
    V = np.zeros((m + 1, n), dtype=np.complex128)
    H = np.zeros((m, m), dtype=np.complex128)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V[0] = v / np.linalg.norm(v)
    j0 = 0
    matvecs = 0
    anorm = 0.0
    for restart in range(max_restarts):
        for j in range(j0, m):
            w = A(V[j])
            matvecs += 1
            # two passes of classical Gram-Schmidt against the whole basis
            # (V^H w formed as conj(V conj(w)): no conjugated copy of the basis)
            h = (V[: j + 1] @ w.conj()).conj()
            w -= V[: j + 1].T @ h
            h2 = (V[: j + 1] @ w.conj()).conj()
            w -= V[: j + 1].T @ h2
            h += h2
            H[: j + 1, j] = h
            H[j, : j + 1] = h.conj()
            H[j, j] = h[j].real
            beta = np.linalg.norm(w)
            if j + 1 < m:
                H[j + 1, j] = H[j, j + 1] = beta
            V[j + 1] = w / beta
        theta, S = np.linalg.eigh(0.5 * (H + H.conj().T))
        anorm = max(anorm, abs(theta[-1]), abs(theta[0]))
        est = np.abs(beta * S[m - 1, :])
        if log:
            log(f"[lanczos] restart {restart}: {matvecs} matvecs, theta0 {theta[0]:.12e}, "
                f"max est (wanted) {est[:want].max():.2e}")
        if np.all(est[:want] <= tol * anorm):
            X = S[:, :want].T @ V[:m]
            res = np.array([np.linalg.norm(A(x) - t * x) for x, t in zip(X, theta[:want])])
            matvecs += want
            return theta[:want], X, res, matvecs
        # thick restart: keep the lowest kp Ritz vectors and the residual direction
        Y = S[:, :kp].T @ V[:m]
        V[:kp] = Y
        V[kp] = V[m]
        V[kp + 1:] = 0.0
        H[:] = 0.0
        H[np.arange(kp), np.arange(kp)] = theta[:kp]
        arrow = beta * S[m - 1, :kp]
        H[kp, :kp] = arrow
        H[:kp, kp] = arrow.conj()
        # the loop continues at column kp: formed against the whole basis, it
        # reproduces the arrow row above
        j0 = kp
    raise RuntimeError("lanczos_q2: no convergence")


def lowest_q(op, m0: float, k: int, guard: int = 4, tol: float = 1e-13, basis: int = 0, keep: int = 0,
             seed: int = 1, log=None):
    """The k eigenvalues of Q(m0) smallest in modulus, one per Kramers pair,
    signed, sorted by |lambda| (ties: lambda); with the residual norm of each
    (a rigorous bound on its distance to the spectrum) and the number of
    applications of Q^2."""
    # rounding seeds the Kramers partner of every converged direction and the
    # iteration amplifies it, so both copies of a low pair converge in the end:
    # ask for two Ritz values per wanted pair
    want = 2 * (k + guard)
    theta, X, res2, mv = lanczos_q2(op, m0, want, basis=basis, keep=keep, tol=tol, seed=seed, log=log)
    shape = op.shape
    Z = np.concatenate([X, kramers_image(X.reshape((want,) + shape), op.L).reshape(want, -1)])
    # orthonormal basis of the Theta-closed span (rank-revealing: a repeated
    # Kramers direction has a near-zero eigenvalue of the Gram matrix)
    G = Z.conj() @ Z.T
    g, U = np.linalg.eigh(0.5 * (G + G.conj().T))
    sel = g > 1e-8 * g.max()
    B = (U[:, sel] / np.sqrt(g[sel])).T @ Z
    QB = np.stack([op.Q(b.reshape(shape), m0).reshape(-1) for b in B])
    Hq = B.conj() @ QB.T
    lam, W = np.linalg.eigh(0.5 * (Hq + Hq.conj().T))
    Y = W.T @ B
    QY = W.T @ QB
    rq = np.linalg.norm(QY - lam[:, None] * Y, axis=1)
    # Kramers pairs: consecutive signed values agree to their residuals
    order = np.argsort(lam)
    lam, rq = lam[order], rq[order]
    if lam.size % 2:
        raise RuntimeError("odd number of Q-Ritz values in a Kramers-closed subspace")
    a, b = lam[0::2], lam[1::2]
    if np.any(np.abs(a - b) > 2 * (rq[0::2] + rq[1::2]) + 1e-13 * np.abs(lam).max()):
        raise RuntimeError("Q-Ritz values are not paired")
    pairs = 0.5 * (a + b)
    perr = np.maximum(rq[0::2], rq[1::2]) + 0.5 * np.abs(a - b)
    idx = np.lexsort((pairs, np.abs(pairs)))[:k]
    return pairs[idx], perr[idx], 2 * mv + 2 * B.shape[0]
