"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module only *draws* inputs: random SU(3) x U(1) gauge fields on the
physical T x L^3 lattice, optional APE-like smoothing of those fields, random
spinors and the bare-mass paths.  It holds none of the operator's arithmetic
(no C* neighbour map, no clover, no Dirac operator): every field it returns is
a plain array that both sides read.

Layouts (host, numpy):
  su3   : complex128 [T][L][L][L][4][3][3]   (t slowest, x3 fastest, mu=0 is t)
  theta : float64    [T][L][L][L][4]         (U(1) angle; quark link phase exp(i q theta))
  spinor (x-doubled lattice, canonical): complex [T][2L][L][L][4][3]

Draw order (fixed so that a seed names one field): a PCG64 generator; first
r ~ N(0,1) of shape (V,4,8) in the order t,x1,x2,x3,mu,a, then theta =
eps * N(0,1) of shape (V,4).  U = exp(i eps sum_a r_a lambda_a / 2), built from
the eigendecomposition of the Hermitian exponent.
"""
from __future__ import annotations

import numpy as np

# Gell-Mann matrices lambda_1..lambda_8
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0] = 1
_GM[2][1, 1] = -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)


def su3_from_algebra(r: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps sum_a r_a lambda_a / 2) for r of shape (..., 8)."""
    h = eps * 0.5 * np.einsum("...a,aij->...ij", r, _GM)
    w, v = np.linalg.eigh(h)
    return np.einsum("...ik,...k,...jk->...ij", v, np.exp(1j * w), v.conj())


def su3_from_algebra_torch(r: np.ndarray, eps: float, device=None) -> np.ndarray:
    """The matrices of su3_from_algebra (equal up to rounding), evaluated with
    torch.linalg.matrix_exp (on the GPU when one is present): only a faster way
    to draw many large synthetic fields."""
    import torch
    dev = device or ("cuda" if torch.cuda.is_available() else "cpu")
    gm = torch.from_numpy(_GM.reshape(8, 9)).to(dev)
    rt = torch.from_numpy(np.ascontiguousarray(r.reshape(-1, 8))).to(dev).to(torch.complex128)
    h = ((eps * 0.5) * (rt @ gm)).reshape(-1, 3, 3)
    u = torch.linalg.matrix_exp(1j * h)
    return u.cpu().numpy().reshape(r.shape[:-1] + (3, 3))


def reunitarize(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt of rows 0,1, row 2 = conj(row0 x row1): a matrix in SU(3)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.cross(r0, r1).conj()
    return np.stack([r0, r1, r2], axis=-2)


def _roll(a: np.ndarray, mu: int, step: int) -> np.ndarray:
    """a(x + step*mu_hat) on the plain periodic torus (lattice axes 0..3)."""
    return np.roll(a, -step, axis=mu)


def ape_smooth(su3: np.ndarray, theta: np.ndarray, steps: int, alpha: float = 0.5):
    """APE-like smoothing on the physical torus with periodic wrap.

    U'(x,mu) = P[(1-alpha) U + alpha/6 * sum of the six staples]; the U(1) angle
    follows the same rule on the phases, theta' = arg[(1-alpha) e^{i theta} +
    alpha/6 * sum of staple phases].  The wrap is the plain periodic one: this
    only shapes a synthetic input and carries no boundary condition of the
    operator.
    """
    u = su3.copy()
    th = theta.copy()
    for _ in range(steps):
        new_u = np.empty_like(u)
        new_th = np.empty_like(th)
        for mu in range(4):
            stap = np.zeros(u.shape[:4] + (3, 3), dtype=np.complex128)
            zst = np.zeros(u.shape[:4], dtype=np.complex128)
            for nu in range(4):
                if nu == mu:
                    continue
                u_nu = u[..., nu, :, :]
                u_mu_xnu = _roll(u[..., mu, :, :], nu, 1)
                u_nu_xmu = _roll(u[..., nu, :, :], mu, 1)
                stap += u_nu @ u_mu_xnu @ np.swapaxes(u_nu_xmu.conj(), -1, -2)
                u_nu_m = _roll(u[..., nu, :, :], nu, -1)
                u_mu_m = _roll(u[..., mu, :, :], nu, -1)
                u_nu_mp = _roll(_roll(u[..., nu, :, :], nu, -1), mu, 1)
                stap += np.swapaxes(u_nu_m.conj(), -1, -2) @ u_mu_m @ u_nu_mp
                t_nu = th[..., nu]
                zst += np.exp(1j * (t_nu + _roll(th[..., mu], nu, 1) - _roll(th[..., nu], mu, 1)))
                zst += np.exp(1j * (-_roll(th[..., nu], nu, -1) + _roll(th[..., mu], nu, -1)
                                    + _roll(_roll(th[..., nu], nu, -1), mu, 1)))
            new_u[..., mu, :, :] = reunitarize((1 - alpha) * u[..., mu, :, :] + (alpha / 6.0) * stap)
            new_th[..., mu] = np.angle((1 - alpha) * np.exp(1j * th[..., mu]) + (alpha / 6.0) * zst)
        u, th = new_u, new_th
    return u, th


def ape_smooth_torch(su3: np.ndarray, theta: np.ndarray, steps: int, alpha: float = 0.5, device=None):
    """The same smoothing rule as ape_smooth, evaluated with torch (on the GPU
    when one is present): only a faster way to shape large synthetic inputs."""
    import torch
    dev = device or ("cuda" if torch.cuda.is_available() else "cpu")
    u = torch.from_numpy(su3).to(dev)
    th = torch.from_numpy(theta).to(dev)

    def roll(a, mu, step):
        return torch.roll(a, -step, dims=mu)

    def dag(a):
        return a.conj().transpose(-1, -2)

    def reunit(m):
        r0 = m[..., 0, :]
        r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
        r1 = m[..., 1, :]
        r1 = r1 - torch.sum(r0.conj() * r1, dim=-1, keepdim=True) * r0
        r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
        r2 = torch.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                          r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                          r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], dim=-1).conj()
        return torch.stack([r0, r1, r2], dim=-2)

    for _ in range(steps):
        new_u = torch.empty_like(u)
        new_th = torch.empty_like(th)
        for mu in range(4):
            stap = torch.zeros_like(u[..., mu, :, :])
            zst = torch.zeros(th.shape[:4], dtype=torch.complex128, device=dev)
            for nu in range(4):
                if nu == mu:
                    continue
                u_nu = u[..., nu, :, :]
                stap = stap + u_nu @ roll(u[..., mu, :, :], nu, 1) @ dag(roll(u[..., nu, :, :], mu, 1))
                u_nu_m = roll(u[..., nu, :, :], nu, -1)
                stap = stap + dag(u_nu_m) @ roll(u[..., mu, :, :], nu, -1) @ roll(u_nu_m, mu, 1)
                zst = zst + torch.exp(1j * (th[..., nu] + roll(th[..., mu], nu, 1) - roll(th[..., nu], mu, 1)))
                zst = zst + torch.exp(1j * (-roll(th[..., nu], nu, -1) + roll(th[..., mu], nu, -1)
                                            + roll(roll(th[..., nu], nu, -1), mu, 1)))
            new_u[..., mu, :, :] = reunit((1 - alpha) * u[..., mu, :, :] + (alpha / 6.0) * stap)
            new_th[..., mu] = torch.angle((1 - alpha) * torch.exp(1j * th[..., mu]) + (alpha / 6.0) * zst)
        u, th = new_u, new_th
    return np.ascontiguousarray(u.cpu().numpy()), np.ascontiguousarray(th.cpu().numpy())


def make_field(T: int, L: int, eps: float, seed: int, smear_steps: int = 0, alpha: float = 0.5,
               smear_backend: str = "numpy", exp_backend: str = "numpy"):
    """Random SU(3) x U(1) field on the physical T x L^3 lattice.

    Returns (su3 complex128 [T,L,L,L,4,3,3], theta float64 [T,L,L,L,4]).
    smear_backend "torch" evaluates the smoothing with torch (GPU if present);
    exp_backend "torch" the exponentials (same field up to rounding).
    """
    if T < 2 or L < 2 or T % 2 or L % 2:
        raise ValueError("T and L must be even and >= 2")
    rng = np.random.Generator(np.random.PCG64(seed))
    V = T * L ** 3
    r = rng.standard_normal((V, 4, 8))
    theta = eps * rng.standard_normal((V, 4))
    su3 = (su3_from_algebra_torch(r, eps) if exp_backend == "torch" else su3_from_algebra(r, eps))
    su3 = su3.reshape(T, L, L, L, 4, 3, 3)
    theta = theta.reshape(T, L, L, L, 4)
    if smear_steps:
        if smear_backend == "torch":
            su3, theta = ape_smooth_torch(su3, theta, smear_steps, alpha)
        else:
            su3, theta = ape_smooth(su3, theta, smear_steps, alpha)
    return np.ascontiguousarray(su3), np.ascontiguousarray(theta)


def unit_field(T: int, L: int):
    """Free field: U = 1, theta = 0."""
    su3 = np.zeros((T, L, L, L, 4, 3, 3), dtype=np.complex128)
    su3[..., 0, 0] = su3[..., 1, 1] = su3[..., 2, 2] = 1
    return su3, np.zeros((T, L, L, L, 4))


def random_spinor(T: int, L: int, seed: int, nrhs: int | None = None, dtype=np.complex128):
    """Gaussian spinor(s) on the x-doubled lattice, canonical [T][2L][L][L][4][3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (T, 2 * L, L, L, 4, 3) if nrhs is None else (nrhs, T, 2 * L, L, L, 4, 3)
    v = rng.standard_normal(shape + (2,))
    return (v[..., 0] + 1j * v[..., 1]).astype(dtype)


def kappa_to_m0(kappa):
    """Bare mass of the Wilson operator with unit mass coefficient: m0 = 1/(2 kappa) - 4."""
    return 1.0 / (2.0 * np.asarray(kappa, dtype=np.float64)) - 4.0


def kappa_path(k_hi: float, k_lo: float, n: int) -> np.ndarray:
    """n hopping parameters linear from k_hi down to k_lo, both ends included."""
    return np.linspace(k_hi, k_lo, n)


# Named workloads: (T, L, eps, seed, smear_steps, charges, kappa path)
WORKLOADS = {
    "tiny_4x2^3": dict(T=4, L=2, eps=0.3, seed=0, smear=0, q=(2.0 / 3.0,),
                       kappas=kappa_path(0.125, 0.05, 16)),
    "single_16^4": dict(T=16, L=16, eps=0.2, seed=1, smear=0, q=(-1.0 / 3.0,),
                        kappas=np.array([0.1365])),
    "batched_32^4": dict(T=32, L=32, eps=0.3, seed=2, smear=10, q=(2.0 / 3.0,),
                         kappas=kappa_path(0.1365, 0.05, 32)),
    "learned_32^4": dict(T=32, L=32, eps=0.3, seed=2000, smear=10, q=(2.0 / 3.0,),
                         kappas=kappa_path(0.1365, 0.05, 32)),
    "paper_64x32^3": dict(T=64, L=32, eps=0.25, seed=4, smear=0, q=(2.0 / 3.0, -1.0 / 3.0),
                          kappas=kappa_path(0.1365, 0.05, 48)),
}
CSW_SU3 = 1.9
CSW_U1 = 1.0
