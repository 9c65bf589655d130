"""ctypes wrapper of the FP64 oracle operator (dirac_oracle.c). Test infrastructure only.

The operator is the O(a)-improved Wilson-Dirac operator with SU(3) x U(1)
links and C* boundary conditions realised on the x-doubled lattice (paper,
sign-of-the-Pfaffian section and simulation setup).  Spinors are canonical
complex128 arrays [T][2L][L][L][4][3].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "dirac_oracle.c")


def build(force: bool = False) -> str:
    """Compile dirac_oracle.c with gcc (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_field_strength.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, dp]
        L.oracle_dirac.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp,
                                   dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_links.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_int, dp]
        L.oracle_dirac_tab.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double,
                                       ctypes.c_int, dp, dp]
        L.oracle_local_term.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, dp]
        L.oracle_gammas.argtypes = [dp]
        L.oracle_neighbours.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
        L.oracle_transport.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gammas() -> np.ndarray:
    """[g0, g1, g2, g3, g5, 1] as used by the oracle, complex (6,4,4)."""
    out = np.zeros((6, 4, 4), dtype=np.complex128)
    lib().oracle_gammas(_p(out))
    return out


def neighbours(T: int, L: int) -> np.ndarray:
    """C* neighbour table on the doubled lattice: int64 [2V][4][2] (mu, +1/-1)."""
    out = np.zeros((2 * T * L ** 3, 4, 2), dtype=np.int64)
    lib().oracle_neighbours(T, L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    return out


class Operator:
    """D(m0) for one gauge field and one quark charge q."""

    def __init__(self, su3, theta, q, csw_su3=1.9, csw_u1=1.0, time_bc=1, link_mode=0, clover=True):
        su3 = np.ascontiguousarray(su3, dtype=np.complex128)
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.T, self.L = su3.shape[0], su3.shape[1]
        self.su3, self.theta = su3, theta
        self.q, self.csw_su3, self.csw_u1 = float(q), float(csw_su3), float(csw_u1)
        self.time_bc, self.link_mode = int(time_bc), int(link_mode)
        self.nsites = 2 * self.T * self.L ** 3
        self._V = None
        self.F = None
        if clover:
            self.F = np.zeros((self.nsites, 6, 3, 3), dtype=np.complex128)
            lib().oracle_field_strength(self.T, self.L, _p(self.su3), _p(self.theta), self.q,
                                        self.csw_su3, self.csw_u1, _p(self.F))

    @property
    def shape(self):
        return (self.T, 2 * self.L, self.L, self.L, 4, 3)

    @property
    def dim(self):
        return self.nsites * 12

    def links(self) -> np.ndarray:
        """The quark link table the operator uses, complex [2V][4][3][3] on the
        doubled lattice (built once per operator, in its link_mode)."""
        if self._V is None:
            V = np.empty((self.nsites, 4, 3, 3), dtype=np.complex128)
            lib().oracle_links(self.T, self.L, self.q, _p(self.su3), _p(self.theta), self.link_mode, _p(V))
            self._V = V
        return self._V

    def apply(self, psi: np.ndarray, m0: float, gamma5: bool = False) -> np.ndarray:
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        if psi.size != self.dim:
            raise ValueError("spinor size mismatch")
        out = np.empty_like(psi)
        F = _p(self.F) if self.F is not None else None
        rc = lib().oracle_dirac_tab(self.T, self.L, self.time_bc, _p(self.links()), F, float(m0),
                                    int(bool(gamma5)), _p(psi), _p(out))
        if rc != 0:
            raise MemoryError("oracle_dirac failed")
        return out

    def transport(self, psi: np.ndarray, mu: int, direction: int) -> np.ndarray:
        """direction +1: V(x,mu) psi(x+mu); -1: V(x-mu,mu)^H psi(x-mu) (time phase on wrapping hops)."""
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        out = np.empty_like(psi)
        rc = lib().oracle_transport(self.T, self.L, self.time_bc, self.q, _p(self.su3), _p(self.theta), int(mu),
                                    int(direction), self.link_mode, _p(psi), _p(out))
        if rc != 0:
            raise MemoryError("oracle_transport failed")
        return out

    def local_term(self, m0: float) -> np.ndarray:
        """Site-local 12x12 part of D(m0) on every doubled site, complex [2V][12][12]
        (index 3*spin + colour): (4+m0) 1 + SW(x)."""
        out = np.empty((self.nsites, 12, 12), dtype=np.complex128)
        F = _p(self.F) if self.F is not None else None
        lib().oracle_local_term(self.T, self.L, F, float(m0), _p(out))
        return out

    def D(self, psi, m0):
        return self.apply(psi, m0, False)

    def Q(self, psi, m0):
        return self.apply(psi, m0, True)

    def Q2(self, psi, m0):
        return self.Q(self.Q(psi, m0), m0)
