"""Python binding of libcstar.so (argument marshalling only).

Every computation runs in the library's HIP kernels and host solver; this
module converts numpy / torch arguments to the C ABI of include/cstar.h and
raises on any non-OK status.  If the library has not been built the import of
`lib()` fails loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcstar.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cstar.h")

FP64, FP32, FP32_BF16LINKS = 0, 1, 2
OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EAMBIG, ESTATE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV", -5: "EAMBIG", -6: "ESTATE"}


class CstarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int), ("L", ctypes.c_int), ("time_bc", ctypes.c_int), ("q", ctypes.c_double),
                ("csw_su3", ctypes.c_double), ("csw_u1", ctypes.c_double)]


class EigOpts(ctypes.Structure):
    _fields_ = [("inner", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("block", ctypes.c_int), ("degree", ctypes.c_int), ("use_nn", ctypes.c_int),
                ("warm_start", ctypes.c_int), ("seed", ctypes.c_ulonglong)]


class EigStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("applies_fp64", ctypes.c_long), ("applies_inner", ctypes.c_long),
                ("seconds", ctypes.c_double), ("lambda_max_est", ctypes.c_double), ("nn_applies", ctypes.c_long),
                ("nn_fallback", ctypes.c_int)]


class LbarOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("degree", ctypes.c_int), ("plain_steps", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("max_cg", ctypes.c_int), ("seed", ctypes.c_ulonglong),
                ("inner", ctypes.c_int)]


class LbarStats(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int), ("solves", ctypes.c_int), ("cg_iterations", ctypes.c_long),
                ("applies_fp64", ctypes.c_long), ("beta", ctypes.c_double), ("resid_q2", ctypes.c_double),
                ("seconds", ctypes.c_double), ("applies_inner", ctypes.c_long)]


class WmassStats(ctypes.Structure):
    _fields_ = [("cg_iterations", ctypes.c_long), ("eo_applies", ctypes.c_long), ("seconds", ctypes.c_double)]


class SignOpts(ctypes.Structure):
    _fields_ = [("eig", EigOpts), ("k", ctypes.c_int), ("c", ctypes.c_double), ("m_max", ctypes.c_double),
                ("step_a_power", ctypes.c_int), ("lbar_tol", ctypes.c_double)]


class SignReport(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int), ("m", ctypes.c_double * 512), ("lambda_bar", ctypes.c_double * 512),
                ("n_crossings", ctypes.c_int), ("applies", ctypes.c_long), ("seconds", ctypes.c_double),
                ("nn_applies", ctypes.c_long), ("nn_fallbacks", ctypes.c_int)]


class ApplyTiming(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_long * 3), ("rhs", ctypes.c_long * 3), ("ms", ctypes.c_double * 3),
                ("operands", ctypes.c_long * 3)]


PROVIDER = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))
LBAR_PROVIDER = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double))

_lib = None


def lib():
    """Load libcstar.so (built in-tree by paper_2108_11989_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2108_11989_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        L.cstar_last_error.restype = ctypes.c_char_p
        L.cstar_gauge_create.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.cstar_gauge_destroy.argtypes = [vp]
        L.cstar_gauge_destroy.restype = None
        L.cstar_spinor_bytes.argtypes = [vp, ctypes.c_int]
        L.cstar_spinor_bytes.restype = ctypes.c_size_t
        L.cstar_n_sites.argtypes = [vp]
        L.cstar_n_sites.restype = ctypes.c_long
        L.cstar_spinor_pack.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
        L.cstar_spinor_unpack.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
        L.dirac_apply.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, vp, vp]
        L.dirac_apply_noalloc.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, vp, vp]
        L.cstar_even_bytes.argtypes = [vp, ctypes.c_int]
        L.cstar_even_bytes.restype = ctypes.c_size_t
        L.dirac_eo_apply.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp, vp]
        L.cstar_log_w_eo.argtypes = [vp, ctypes.c_double, ctypes.c_double, dp]
        L.q_lowest_eigs.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(EigOpts), dp, dp, vp,
                                    ctypes.POINTER(EigStats)]
        L.q_lambda_bar_power.argtypes = [vp, ctypes.c_double, ctypes.POINTER(LbarOpts), dp, dp,
                                         ctypes.POINTER(LbarStats)]
        L.pfaffian_sign.argtypes = [vp, dp, ctypes.c_int, ctypes.POINTER(SignOpts), ip, ctypes.POINTER(SignReport)]
        L.cstar_sign_driver.argtypes = [PROVIDER, vp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ip, ctypes.POINTER(SignReport)]
        L.cstar_clover_norm_max.argtypes = [vp, dp]
        L.cstar_sign_driver_a.argtypes = [LBAR_PROVIDER, PROVIDER, vp, dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, ip, ctypes.POINTER(SignReport)]
        L.cstar_w_mass.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, ctypes.c_int, vp,
                                   ctypes.c_double, dp, dp, ctypes.POINTER(WmassStats)]
        L.cstar_ratapprox_quartic.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        L.cstar_sign_ensemble.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(dp),
                                          ctypes.POINTER(dp), ctypes.c_int, ctypes.c_int, dp, dp,
                                          ctypes.POINTER(SignOpts), ip, ip, dp]
        L.cstar_timing_enable.argtypes = [vp, ctypes.c_int]
        L.cstar_timing_read.argtypes = [vp, ctypes.POINTER(ApplyTiming)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.cstar_nn_create.argtypes = [fp, ctypes.POINTER(vp)]
        L.cstar_nn_destroy.argtypes = [vp]
        L.cstar_nn_destroy.restype = None
        L.cstar_nn_get_weights.argtypes = [vp, fp]
        L.cstar_nn_set_weights.argtypes = [vp, fp]
        L.cstar_nn_get_grad.argtypes = [vp, dp]
        L.cstar_nn_zero_grad.argtypes = [vp]
        L.cstar_nn_apply.argtypes = [vp, vp, ctypes.c_int, vp, vp]
        L.cstar_nn_loss_grad.argtypes = [vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, dp]
        L.cstar_nn_adam_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.cstar_nn_train.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_double, dp]
        L.cstar_nn_attach.argtypes = [vp, vp]
        for name in ("cstar_gauge_create", "cstar_spinor_pack", "cstar_spinor_unpack", "dirac_apply",
                     "dirac_apply_noalloc", "dirac_eo_apply", "cstar_log_w_eo", "cstar_sign_ensemble",
                     "cstar_ratapprox_quartic", "cstar_w_mass", "cstar_sign_driver_a",
                     "q_lowest_eigs", "q_lambda_bar_power", "pfaffian_sign", "cstar_sign_driver", "cstar_clover_norm_max",
                     "cstar_timing_enable", "cstar_timing_read", "cstar_nn_create", "cstar_nn_get_weights",
                     "cstar_nn_set_weights", "cstar_nn_get_grad", "cstar_nn_zero_grad", "cstar_nn_apply",
                     "cstar_nn_loss_grad", "cstar_nn_adam_step", "cstar_nn_train", "cstar_nn_attach"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/cstar.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    pat = r"^\s*(?:cstar_status|void|const\s+char\s*\*|size_t|long)\s*\**\s*([A-Za-z_]\w*)\s*\("
    return re.findall(pat, txt, flags=re.M)


def _check(st):
    if st != OK:
        raise CstarError(st, lib().cstar_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def eig_opts(inner=FP32_BF16LINKS, tol=1e-10, max_iter=300, block=0, degree=0, use_nn=0, warm_start=0,
             seed=12345) -> EigOpts:
    return EigOpts(inner, tol, max_iter, block, degree, use_nn, warm_start, seed)


class Gauge:
    """One gauge field and one quark charge on the device (a cstar_gauge handle)."""

    def __init__(self, su3, theta, q, csw_su3=1.9, csw_u1=1.0, time_bc=1, stream=None):
        """su3/theta: host numpy arrays, or torch tensors on the device (complex128 / float64,
        physical-lattice layout of include/cstar.h) -- then no data crosses PCIe."""
        self.T, self.L = su3.shape[0], su3.shape[1]
        self.params = Params(self.T, self.L, int(time_bc), float(q), float(csw_su3), float(csw_u1))
        h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream)
        if hasattr(su3, "data_ptr"):
            if not (su3.is_cuda and theta.is_cuda and su3.is_contiguous() and theta.is_contiguous()):
                raise ValueError("device field tensors must be contiguous CUDA tensors")
            ps = ctypes.cast(ctypes.c_void_p(su3.data_ptr()), ctypes.POINTER(ctypes.c_double))
            pt = ctypes.cast(ctypes.c_void_p(theta.data_ptr()), ctypes.POINTER(ctypes.c_double))
            _check(lib().cstar_gauge_create(ctypes.byref(self.params), ps, pt, 1, s, ctypes.byref(h)))
        else:
            su3 = np.ascontiguousarray(su3, dtype=np.complex128)
            theta = np.ascontiguousarray(theta, dtype=np.float64)
            _check(lib().cstar_gauge_create(ctypes.byref(self.params), _dp(su3.view(np.float64)), _dp(theta), 0, s,
                                            ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().cstar_gauge_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_sites(self) -> int:
        return lib().cstar_n_sites(self.h)

    def spinor_bytes(self, prec=FP64) -> int:
        return lib().cstar_spinor_bytes(self.h, prec)

    def clover_norm_max(self) -> float:
        v = ctypes.c_double()
        _check(lib().cstar_clover_norm_max(self.h, ctypes.byref(v)))
        return v.value

    def timing(self, on=True):
        _check(lib().cstar_timing_enable(self.h, int(bool(on))))

    def read_timing(self) -> dict:
        t = ApplyTiming()
        _check(lib().cstar_timing_read(self.h, ctypes.byref(t)))
        return {p: dict(launches=t.launches[p], rhs=t.rhs[p], ms=t.ms[p], operands=t.operands[p]) for p in range(3)}

    # --- device buffers are torch tensors; the library reads/writes their memory
    def new_native(self, nrhs=1, prec=FP64):
        """Uninitialised native spinor block on the device (torch tensor)."""
        import torch
        nbytes = self.spinor_bytes(prec) * nrhs
        if prec == FP64:
            return torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
        return torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")

    def pack(self, canonical, native, prec=FP64, nrhs=1):
        _check(lib().cstar_spinor_pack(self.h, prec, nrhs, ctypes.c_void_p(canonical.data_ptr()),
                                       ctypes.c_void_p(native.data_ptr())))

    def unpack(self, native, canonical, prec=FP64, nrhs=1):
        _check(lib().cstar_spinor_unpack(self.h, prec, nrhs, ctypes.c_void_p(native.data_ptr()),
                                         ctypes.c_void_p(canonical.data_ptr())))

    def apply(self, native_in, native_out, masses, prec=FP64, gamma5=False):
        m = np.ascontiguousarray(np.atleast_1d(np.asarray(masses, dtype=np.float64)))
        _check(lib().dirac_apply(self.h, len(m), _dp(m), prec, int(bool(gamma5)),
                                 ctypes.c_void_p(native_in.data_ptr()), ctypes.c_void_p(native_out.data_ptr())))

    def apply_noalloc(self, native_in, native_out, masses, prec=FP64, gamma5=False):
        """dirac_apply_noalloc: as apply, with no device allocation (masses staged in the
        library's static device array)."""
        m = np.ascontiguousarray(np.atleast_1d(np.asarray(masses, dtype=np.float64)))
        _check(lib().dirac_apply_noalloc(self.h, len(m), _dp(m), prec, int(bool(gamma5)),
                                         ctypes.c_void_p(native_in.data_ptr()),
                                         ctypes.c_void_p(native_out.data_ptr())))

    def eo_apply(self, even_in, even_out, m0, prec=FP64, gamma5=False, nrhs=1):
        """D_hat(m0) (gamma5: Q_hat) on nrhs even vectors (the parity-0 halves of native spinors)."""
        _check(lib().dirac_eo_apply(self.h, int(nrhs), float(m0), prec, int(bool(gamma5)),
                                    ctypes.c_void_p(even_in.data_ptr()), ctypes.c_void_p(even_out.data_ptr())))

    def log_w_eo(self, m, m_prime) -> float:
        v = ctypes.c_double()
        _check(lib().cstar_log_w_eo(self.h, float(m), float(m_prime), ctypes.byref(v)))
        return v.value

    def w_mass(self, m, m_prime, nu2, mu2, eta, tol=1e-12):
        """cstar_w_mass with device sources eta (nsrc FP64 even vectors, torch):
        (log W_mass, exponents [n, nsrc], WmassStats)."""
        nu2 = np.ascontiguousarray(nu2, dtype=np.float64)
        mu2 = np.ascontiguousarray(mu2, dtype=np.float64)
        nsrc = eta.numel() * eta.element_size() // (self.spinor_bytes(FP64) // 2)
        expo = np.zeros((len(nu2), nsrc))
        lw = ctypes.c_double()
        st = WmassStats()
        _check(lib().cstar_w_mass(self.h, float(m), float(m_prime), len(nu2), _dp(nu2), _dp(mu2), int(nsrc),
                                  ctypes.c_void_p(eta.data_ptr()), float(tol), _dp(expo), ctypes.byref(lw),
                                  ctypes.byref(st)))
        return lw.value, expo, st

    def lowest_eigs(self, m0, k, opts: EigOpts | None = None, evecs=None, raise_on_noconv=True):
        ev = np.zeros(k)
        res = np.zeros(k)
        st = EigStats()
        o = opts if opts is not None else eig_opts()
        ptr = ctypes.c_void_p(evecs.data_ptr()) if evecs is not None else None
        status = lib().q_lowest_eigs(self.h, float(m0), int(k), ctypes.byref(o), _dp(ev), _dp(res), ptr,
                                     ctypes.byref(st))
        if status != OK and (raise_on_noconv or status != ENOCONV):
            _check(status)
        return ev, res, st

    def lambda_bar_power(self, m0, tol=1e-3, degree=0, plain_steps=0, max_outer=0, max_cg=0, seed=1,
                         raise_on_noconv=True, inner=FP64):
        """min |lambda(Q(m0))| by the power method with Chebyshev acceleration on Q^-2:
        (lambda_bar, half-width bound, LbarStats)."""
        o = LbarOpts(float(tol), int(degree), int(plain_steps), int(max_outer), int(max_cg), int(seed), int(inner))
        lam = ctypes.c_double(0.0)
        bound = ctypes.c_double(0.0)
        st = LbarStats()
        status = lib().q_lambda_bar_power(self.h, float(m0), ctypes.byref(o), ctypes.byref(lam), ctypes.byref(bound),
                                          ctypes.byref(st))
        if status != OK and (raise_on_noconv or status != ENOCONV):
            _check(status)
        return lam.value, bound.value, st

    def pfaffian_sign(self, m_path, k=4, c=1.9, m_max=0.0, eig: EigOpts | None = None, step_a_power=False,
                      lbar_tol=0.0):
        m = np.ascontiguousarray(np.asarray(m_path, dtype=np.float64))
        out = np.zeros(len(m), dtype=np.int32)
        rep = SignReport()
        o = SignOpts(eig if eig is not None else eig_opts(), int(k), float(c), float(m_max), int(bool(step_a_power)),
                     float(lbar_tol))
        _check(lib().pfaffian_sign(self.h, _dp(m), len(m), ctypes.byref(o),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(rep)))
        return out, rep


def ratapprox_quartic(n, ra, rb):
    """cstar_ratapprox_quartic: (A, nu2[n], mu2[n], delta) of R(x) = A prod (x+nu2)/(x+mu2) ~ x^(-1/4)."""
    A = ctypes.c_double()
    d = ctypes.c_double()
    nu2 = np.zeros(n)
    mu2 = np.zeros(n)
    _check(lib().cstar_ratapprox_quartic(int(n), float(ra), float(rb), ctypes.byref(A), _dp(nu2), _dp(mu2),
                                         ctypes.byref(d)))
    return A.value, nu2, mu2, d.value


def sign_ensemble(fields, charges, m_target, T, L, csw_su3=1.9, csw_u1=1.0, time_bc=1, k=4, c=1.9,
                  eig: EigOpts | None = None):
    """cstar_sign_ensemble over host fields [(su3, theta), ...]: (status, signs [n_cfg, n_flv],
    products [n_cfg], seconds [n_cfg])."""
    n = len(fields)
    keep = [(np.ascontiguousarray(s3, dtype=np.complex128), np.ascontiguousarray(t3, dtype=np.float64))
            for s3, t3 in fields]
    P = ctypes.POINTER(ctypes.c_double)
    su3p = (P * n)(*[_dp(s3.view(np.float64)) for s3, _ in keep])
    thp = (P * n)(*[_dp(t3) for _, t3 in keep])
    q = np.ascontiguousarray(charges, dtype=np.float64)
    m = np.ascontiguousarray(m_target, dtype=np.float64)
    signs = np.zeros((n, len(q)), dtype=np.int32)
    prods = np.zeros(n, dtype=np.int32)
    secs = np.zeros(n)
    opts = SignOpts(eig if eig is not None else eig_opts(), int(k), float(c), 0.0, 0, 0.0)
    par = Params(int(T), int(L), int(time_bc), 0.0, float(csw_su3), float(csw_u1))
    ip = ctypes.POINTER(ctypes.c_int)
    st = lib().cstar_sign_ensemble(ctypes.byref(par), n, su3p, thp, 0, len(q), _dp(q), _dp(m), ctypes.byref(opts),
                                   signs.ctypes.data_as(ip), prods.ctypes.data_as(ip), _dp(secs))
    return st, signs, prods, secs


NN_PARAMS = 23040


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


class Net:
    """The learned preconditioner network (a cstar_nn handle); weights as in include/cstar.h."""

    def __init__(self, weights=None):
        h = ctypes.c_void_p()
        if weights is None:
            _check(lib().cstar_nn_create(None, ctypes.byref(h)))
        else:
            w = np.ascontiguousarray(weights, dtype=np.float32)
            if w.size != NN_PARAMS:
                raise ValueError(f"expected {NN_PARAMS} weights")
            _check(lib().cstar_nn_create(_fp(w), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().cstar_nn_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self) -> np.ndarray:
        w = np.zeros(NN_PARAMS, dtype=np.float32)
        _check(lib().cstar_nn_get_weights(self.h, _fp(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != NN_PARAMS:
            raise ValueError(f"expected {NN_PARAMS} weights")
        _check(lib().cstar_nn_set_weights(self.h, _fp(w)))

    def grad(self) -> np.ndarray:
        g = np.zeros(NN_PARAMS)
        _check(lib().cstar_nn_get_grad(self.h, _dp(g)))
        return g

    def zero_grad(self):
        _check(lib().cstar_nn_zero_grad(self.h))

    def apply(self, gauge: "Gauge", b, y, nvec=1):
        _check(lib().cstar_nn_apply(self.h, gauge.h, int(nvec), _vp(b), _vp(y)))

    def loss_grad(self, gauge: "Gauge", x, b, nvec=1, n_total=None) -> float:
        loss = ctypes.c_double()
        _check(lib().cstar_nn_loss_grad(self.h, gauge.h, int(nvec), _vp(x), _vp(b),
                                        int(n_total if n_total else nvec), ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().cstar_nn_adam_step(self.h, float(lr), float(beta1), float(beta2), float(eps)))

    def train(self, gauges, xs, nvec, m0, epochs, lr) -> np.ndarray:
        n = len(gauges)
        hs = (ctypes.c_void_p * n)(*[g.h.value for g in gauges])
        ps = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        hist = np.zeros(epochs)
        _check(lib().cstar_nn_train(self.h, hs, n, ps, int(nvec), float(m0), int(epochs), float(lr), _dp(hist)))
        return hist

    def attach(self, gauge: "Gauge"):
        _check(lib().cstar_nn_attach(gauge.h, self.h))

    @staticmethod
    def detach(gauge: "Gauge"):
        _check(lib().cstar_nn_attach(gauge.h, None))


def sign_driver_a(lbar, provider, m_path, k, c, m_max):
    """Run the library's step-A driver over Python providers lbar(m) -> (lambda_bar, err) and
    provider(m, k) -> (evals, errs)."""
    def cb(ctx, m, kk, ev, er):
        try:
            e, r = provider(m, kk)
            for i in range(kk):
                ev[i] = float(e[i])
                er[i] = float(r[i])
            return 0
        except Exception:
            return 1

    def cbl(ctx, m, lb, er):
        try:
            a, b = lbar(m)
            lb[0] = float(a)
            er[0] = float(b)
            return 0
        except Exception:
            return 1

    cbf, cblf = PROVIDER(cb), LBAR_PROVIDER(cbl)
    m = np.ascontiguousarray(np.asarray(m_path, dtype=np.float64))
    out = np.zeros(len(m), dtype=np.int32)
    rep = SignReport()
    st = lib().cstar_sign_driver_a(cblf, cbf, None, _dp(m), len(m), int(k), float(c), float(m_max),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(rep))
    return st, out, rep


def sign_driver(provider, m_path, k, c, m_max):
    """Run the library's sign driver over a Python eigenvalue provider(m, k) -> (evals, errs)."""
    def cb(ctx, m, kk, ev, er):
        try:
            e, r = provider(m, kk)
            for i in range(kk):
                ev[i] = float(e[i])
                er[i] = float(r[i])
            return 0
        except Exception:
            return 1

    cbf = PROVIDER(cb)
    m = np.ascontiguousarray(np.asarray(m_path, dtype=np.float64))
    out = np.zeros(len(m), dtype=np.int32)
    rep = SignReport()
    st = lib().cstar_sign_driver(cbf, None, _dp(m), len(m), int(k), float(c), float(m_max),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(rep))
    return st, out, rep
