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
     estimates |beta s_m,i| below tol * ||A|| (||A|| bounded by
     (|4+m| + 4 + max ||SW||)^2).  Optionally the iteration runs on a
     Chebyshev polynomial of A that keeps its eigenvectors and orders the
     wanted ones first (fewer basis vectors to orthogonalise against per
     product with A); its Ritz vectors are judged by their residuals under A.
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


def clover_norm_bound(op) -> float:
    """max over sites of the spectral norm of SW(x) (the local term at m0 = -4)."""
    loc = op.local_term(-4.0)
    return float(np.max(np.linalg.norm(loc, ord=2, axis=(1, 2))))


def lanczos_q2(op, m0: float, want: int, basis: int = 0, keep: int = 0, tol: float = 1e-13,
               degree: int = 1, max_restarts: int = 2000, seed: int = 1, log=None):
    """Thick-restart Lanczos for the `want` lowest eigenvalues of A = Q(m0)^2.

    degree 1: Lanczos on A itself.  degree d > 1: Lanczos on B = p(A) with p
    the Chebyshev polynomial T_d mapped to the interval [a_cut, b], sign-fixed
    so that every eigenvalue of A below a_cut becomes an eigenvalue of B above
    1, larger the lower it is (p is monotone there), while the rest of the
    spectrum maps into [-1, 1]; b is a rigorous bound of ||A|| and a_cut the
    want-th Ritz value of a short plain Lanczos run, an upper bound of the
    want-th eigenvalue (interlacing), so the wanted eigenvalues are the
    largest of B.  The eigenvectors of B are those of A; the Ritz vectors of B
    are judged by their true residuals under A after Rayleigh-Ritz with A.

    Returns (theta[want], X[want, dim] unit Ritz vectors of A, resid[want]
    = ||A x - theta x||, matvecs of A).  tol is relative to ||A||."""
    n = op.dim
    shape = op.shape
    m = basis or max(3 * want, want + 40)
    kp = keep or min(m - 20, want + max(10, want // 2))
    if not (want < kp < m):
        raise ValueError("need want < keep < basis")
    count = [0]

    def A(x):
        count[0] += 1
        return op.Q(op.Q(x.reshape(shape), m0), m0).reshape(-1)

    qb = abs(4.0 + m0) + 4.0 + clover_norm_bound(op)
    bup = qb * qb * 1.0001
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v0 /= np.linalg.norm(v0)

    def run(apply_b, m, kp, highest, check):
        """Thick-restart Lanczos on B (apply_b); the `want` wanted Ritz values are
        the lowest (highest=False) or highest of B.  check(Y) -> done flag."""
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m, m), dtype=np.complex128)
        V[0] = v0
        j0 = 0
        for restart in range(max_restarts):
            for j in range(j0, m):
                w = apply_b(V[j])
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
            if highest:
                theta, S = theta[::-1], S[:, ::-1]
            est = np.abs(beta * S[m - 1, :])
            out = check(theta, S, V, est, restart)
            if out is not None:
                return out
            # thick restart: keep kp wanted-end Ritz vectors and the residual direction
            V[:kp] = S[:, :kp].T @ V[:m]
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

    def finish(Y):
        """Rayleigh-Ritz with A on the span of the rows of Y (orthonormal)."""
        AY = np.stack([A(y) for y in Y])
        G = Y.conj() @ AY.T
        th, Z = np.linalg.eigh(0.5 * (G + G.conj().T))
        X = Z.T @ Y
        AX = Z.T @ AY
        res = np.linalg.norm(AX - th[:, None] * X, axis=1)
        return th, X, res

    if degree <= 1:
        def check(theta, S, V, est, restart):
            if log:
                log(f"[lanczos] restart {restart}: {count[0]} matvecs, theta0 {theta[0]:.12e}, "
                    f"max est (wanted) {est[:want].max():.2e}")
            if np.all(est[:want] <= tol * bup):
                th, X, res = finish(S[:, :want].T @ V[: S.shape[0]])
                return th, X, res, count[0]
            return None

        return run(A, m, kp, False, check)

    # a_cut from a short plain run: its want-th Ritz value bounds the want-th eigenvalue from above
    npre = min(n - 1, max(2 * want, 60))
    Vp = np.zeros((npre + 1, n), dtype=np.complex128)
    Hp = np.zeros((npre, npre), dtype=np.complex128)
    Vp[0] = v0
    for j in range(npre):
        w = A(Vp[j])
        htot = np.zeros(j + 1, dtype=np.complex128)
        for _ in range(2):
            h = (Vp[: j + 1] @ w.conj()).conj()
            w -= Vp[: j + 1].T @ h
            htot += h
        Hp[: j + 1, j] = htot
        Hp[j, : j + 1] = htot.conj()
        beta = np.linalg.norm(w)
        if j + 1 < npre:
            Hp[j + 1, j] = Hp[j, j + 1] = beta
        Vp[j + 1] = w / beta
    a_cut = float(np.linalg.eigvalsh(0.5 * (Hp + Hp.conj().T))[want - 1])
    del Vp
    c0, c1 = (bup + a_cut) / 2.0, (bup - a_cut) / 2.0
    sgn = -1.0 if degree % 2 else 1.0

    def B(x):
        # p(A) x = (-1)^d T_d((A - c0)/c1) x by the three-term recurrence
        t_prev = x
        t_cur = (A(x) - c0 * x) / c1
        for _ in range(degree - 1):
            t_prev, t_cur = t_cur, 2.0 * (A(t_cur) - c0 * t_cur) / c1 - t_prev
        return sgn * t_cur

    if log:
        log(f"[lanczos] filter degree {degree} on [{a_cut:.6e}, {bup:.6e}]")

    def check_f(theta, S, V, est, restart):
        th, X, res = finish(S[:, :want].T @ V[: S.shape[0]])
        if log:
            log(f"[lanczos] restart {restart}: {count[0]} matvecs, theta0 {th[0]:.12e}, "
                f"max true residual (wanted) {res.max():.2e}")
        if np.all(res <= tol * bup) and th[-1] < a_cut:
            return th, X, res, count[0]
        return None

    return run(B, m, kp, True, check_f)


def lowest_q(op, m0: float, k: int, guard: int = 4, tol: float = 1e-13, basis: int = 0, keep: int = 0,
             degree: int = 1, seed: int = 1, log=None):
    """The k eigenvalues of Q(m0) smallest in modulus, one per Kramers pair,
    signed, sorted by |lambda| (ties: lambda); with the residual norm of each
    (a rigorous bound on its distance to the spectrum) and the number of
    applications of Q^2."""
    # rounding seeds the Kramers partner of every converged direction and the
    # iteration amplifies it, so both copies of a low pair converge in the end:
    # ask for two Ritz values per wanted pair
    want = 2 * (k + guard)
    theta, X, res2, mv = lanczos_q2(op, m0, want, basis=basis, keep=keep, tol=tol, degree=degree, seed=seed,
                                    log=log)
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
