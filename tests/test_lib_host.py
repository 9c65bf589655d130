"""Host-side checks of libcstar.so that need no GPU: the library loads, exports
every function include/cstar.h declares, and its sign driver (host logic of
pfaffian_sign) gets the sign right on eigenvalue flows known in closed form.
"""
import ctypes

import numpy as np
import pytest

from paper_2108_11989_amd import cstar


def test_library_exports_every_declared_function():
    L = cstar.lib()
    names = cstar.header_functions()
    for must in ("dirac_apply", "q_lowest_eigs", "pfaffian_sign", "cstar_gauge_create", "cstar_sign_driver"):
        assert must in names
    for n in names:
        assert hasattr(L, n), n


def test_create_rejects_bad_lattice_without_gpu():
    su3 = np.zeros((3, 2, 2, 2, 4, 3, 3), dtype=np.complex128)
    th = np.zeros((3, 2, 2, 2, 4))
    with pytest.raises(cstar.CstarError) as e:
        cstar.Gauge(su3, th, 2 / 3)
    assert e.value.status == cstar.EINVAL
    su3 = np.zeros((4, 2, 2, 2, 4, 3, 3), dtype=np.complex128)
    su3[..., 0, 0] = np.nan
    th = np.zeros((4, 2, 2, 2, 4))
    with pytest.raises(cstar.CstarError) as e:
        cstar.Gauge(su3, th, 2 / 3)
    assert e.value.status == cstar.EINVAL


def _flow(seed, n=24):
    """Eigenvalue flows lambda_i(m) = a_i + s_i m, |s_i| <= 1 (the Feynman-Hellmann bound).

    Crossings m_i* = -a_i/s_i lie inside [-1, 2]; above m = 3 the count of
    negative values is even, as for Q at large mass.
    """
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.2, 1.0, n) * rng.choice([-1, 1], n)
    mstar = rng.uniform(-1.0, 2.0, n)
    a = -s * mstar
    # at m = 3 every lambda has the sign of s; make the negative count even
    if np.sum(s < 0) % 2:
        s[0] = -s[0]
        a[0] = -s[0] * mstar[0]
    return a, s


def _provider(a, s, err=1e-12):
    def prov(m, k):
        lam = a + s * m
        order = np.lexsort((lam, np.abs(lam)))[:k]
        return lam[order], np.full(k, err)
    return prov


@pytest.mark.parametrize("seed", range(12))
def test_sign_driver_on_closed_form_flows(seed):
    a, s = _flow(seed)
    path = np.linspace(-0.9, 2.5, 9)
    st, signs, rep = cstar.sign_driver(_provider(a, s), path, k=6, c=1.9, m_max=3.0)
    assert st == cstar.OK, cstar.lib().cstar_last_error()
    n_top = np.sum(a + s * 3.0 < 0)
    for m, sg in zip(path, signs):
        n = np.sum(a + s * m < 0)
        assert sg == (-1 if (n - n_top) % 2 else 1), (m, n, n_top)


def test_sign_driver_step_a_without_crossings():
    # flows rising from the target: the driver solves m_max, steps down by
    # c * lambda_bar (here past the target, so the target is solved next), and
    # certifies [target, m_max] with a few exclusion-covered points
    a = np.array([0.05, 0.3, 0.9, 1.4])
    s = np.array([0.9, 0.7, 0.5, 0.5])
    st, signs, rep = cstar.sign_driver(_provider(a, s), [0.0], k=4, c=1.9, m_max=4.0)
    assert st == cstar.OK and signs[0] == 1
    ms = np.array(rep.m[: rep.n_points])
    lb = np.array(rep.lambda_bar[: rep.n_points])
    assert np.isclose(ms[0], 4.0) and np.isclose(ms[1], 0.0)
    assert np.isclose(lb[0], np.min(a + 4.0 * s))
    # every neighbouring pair of solved masses is covered by their exclusion intervals
    order = np.argsort(ms)
    m_s, l_s = ms[order], lb[order]
    assert np.all(l_s[:-1] + l_s[1:] > np.diff(m_s))
    assert rep.n_points < 12


def test_sign_driver_skips_path_points_inside_exclusion_intervals():
    # a gapped flow: every path point lies in an exclusion interval, so far fewer
    # solves than path points are needed and every sign is +1
    a = np.array([0.8, 1.0, 1.3, 1.6])
    s = np.array([0.1, -0.1, 0.2, 0.05])
    path = np.linspace(-1.0, 1.0, 41)
    st, signs, rep = cstar.sign_driver(_provider(a, s), path, k=4, c=1.9, m_max=2.0)
    assert st == cstar.OK and np.all(signs == 1)
    assert rep.n_points < 10


def test_sign_driver_ambiguous_path_point():
    a = np.array([0.0, 0.5])
    s = np.array([1.0, 1.0])
    st, signs, rep = cstar.sign_driver(_provider(a, s, err=1e-9), [0.0, 1.0], k=2, c=1.9, m_max=2.0)
    assert st == cstar.EAMBIG
    assert signs[0] == 0


def test_sign_driver_rejects_bad_c():
    st, _, _ = cstar.sign_driver(_provider(np.ones(2), np.ones(2)), [0.0], k=2, c=2.5, m_max=1.0)
    assert st == cstar.EINVAL


def test_solvers_reject_null_handle_without_gpu():
    """Argument checks come before any device call: a null handle is EINVAL, with a message."""
    L = cstar.lib()
    lam = ctypes.c_double(0.0)
    bound = ctypes.c_double(0.0)
    st = L.q_lambda_bar_power(None, 0.0, None, ctypes.byref(lam), ctypes.byref(bound), None)
    assert st == cstar.EINVAL
    assert b"q_lambda_bar_power" in L.cstar_last_error()
    ev = np.zeros(2)
    res = np.zeros(2)
    st = L.q_lowest_eigs(None, 0.0, 2, None, ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None)
    assert st == cstar.EINVAL


def test_sign_driver_exclusion_radius_uses_every_error_bound():
    """The exclusion interval of a solved mass is min_j (|lambda_j| - err_j), not
    lambda_bar minus the error of the smallest |lambda_j|.  Flow B is a V,
    lambda_B(m) = |m - 1| - 0.1 (crossings at 0.9 and 1.1), reported 0.5 too
    high with error bound 0.5 + 1e-9 (a rigorous but loose bound); flow A is a
    constant 0.6 with a tight bound.  With the radius from A alone (0.6 at 0.6
    and at 1.5) the segment [0.6, 1.5] would count as crossing-free and the path
    point m = 1 would get the sign of m = 1.5; the rigorous radii (0.3 and 0.4)
    do not cover it, so the driver must either find the sign (-1) or report the
    point as undecidable -- never +1."""

    def prov(m, k):
        lam_b = abs(m - 1.0) - 0.1
        ev = np.array([0.6, lam_b + 0.5, 3.0 + m, -4.0 - m])
        err = np.array([1e-12, 0.5 + 1e-9, 1e-12, 1e-12])
        order = np.lexsort((ev, np.abs(ev)))[:k]
        return ev[order], err[order]

    st, signs, rep = cstar.sign_driver(prov, [0.6, 1.0, 1.4], k=4, c=1.9, m_max=1.5)
    assert st in (cstar.OK, cstar.EAMBIG)
    assert signs[1] != 1
    if st == cstar.OK:
        assert signs[1] == -1
    # the first step from m_max uses the rigorous radius: 1.5 - 1.9 * min(0.6, 0.9 - 0.5) = 0.74
    # (with the radius of flow A alone it would jump past the target to 0.6)
    ms = np.array(rep.m[: rep.n_points])
    assert np.isclose(ms[0], 1.5) and np.isclose(ms[1], 0.74)


def test_sign_ensemble_rejects_bad_arguments_without_gpu():
    L = cstar.lib()
    par = cstar.Params(4, 2, 1, 0.0, 1.9, 1.0)
    out = np.zeros(2, dtype=np.int32)
    st = L.cstar_sign_ensemble(ctypes.byref(par), 0, None, None, 0, 1, None, None, None,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), None)
    assert st == cstar.EINVAL
    assert b"cstar_sign_ensemble" in L.cstar_last_error()


def _lbar(a, s, err=1e-12):
    def lb(m):
        return float(np.min(np.abs(a + s * m))), err
    return lb


@pytest.mark.parametrize("seed", range(8))
def test_step_a_driver_on_closed_form_flows(seed):
    """Step A upward from the lowest path mass, then step B above where it stops:
    the signs equal the closed-form crossing parities."""
    a, s = _flow(seed)
    path = np.linspace(-0.9, 2.5, 9)
    st, signs, rep = cstar.sign_driver_a(_lbar(a, s), _provider(a, s), path, k=6, c=1.9, m_max=3.0)
    assert st == cstar.OK, cstar.lib().cstar_last_error()
    n_top = np.sum(a + s * 3.0 < 0)
    for m, sg in zip(path, signs):
        n = np.sum(a + s * m < 0)
        assert sg == (-1 if (n - n_top) % 2 else 1), (m, n, n_top)


def test_step_a_driver_covers_a_gapped_flow_without_eigensolves():
    """Flows that rise from the target: step A alone reaches m_max (the exclusion
    intervals cover the range), every sign is +1, and the eigensolver is never called."""
    a = np.array([0.3, 0.5, 0.9])
    s = np.array([0.9, 0.7, 0.8])
    calls = []

    def prov(m, k):
        calls.append(m)
        return _provider(a, s)(m, k)

    st, signs, rep = cstar.sign_driver_a(_lbar(a, s), prov, np.linspace(0.0, 1.0, 11), k=3, c=1.9, m_max=4.0)
    assert st == cstar.OK and np.all(signs == 1)
    assert calls == []
    ms = np.array(rep.m[: rep.n_points])
    # the step-A sequence m_{n+1} = m_n + 1.9 lambda_bar(m_n) from the lowest path mass
    lb0 = np.min(a)
    assert np.isclose(ms[0], 0.0) and np.isclose(ms[1], 1.9 * lb0)


def test_step_a_driver_hands_over_at_a_decrease():
    """lambda_bar falls after the first step (a flow crossing above the target):
    the driver hands the range above the target to step B, which finds the crossing."""
    a = np.array([-0.5, 1.2])
    s = np.array([1.0, 0.5])  # first flow crosses zero at m = 0.5
    path = [0.0, 0.3, 0.8, 1.5]
    st, signs, rep = cstar.sign_driver_a(_lbar(a, s), _provider(a, s), path, k=2, c=1.9, m_max=3.0)
    assert st == cstar.OK
    n_top = np.sum(a + s * 3.0 < 0)
    ref = [(-1 if (np.sum(a + s * m < 0) - n_top) % 2 else 1) for m in path]
    assert list(signs) == ref
    assert ref[0] == -1 and ref[-1] == 1
