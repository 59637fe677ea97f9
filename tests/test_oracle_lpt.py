"""Pins of the oracle's second-order (2LPT) initial conditions.

The second-order growth fit against the growth ODE, closed forms of the
second-order displacement for plane waves, the Hessian trace, exact finite
differences of the quadratic noise-to-s2 map, the Omega_m tangent, the
gradient of a whole 2LPT-started run by central differences, and the N-body
dynamics themselves: a run started from 2LPT carries the second-order
displacement predicted by D2(a).
"""
from dataclasses import replace

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import cosmology as C
from oracle import lpt
from oracle import mesh as M
from oracle import pm
from synthetic import Cosmology, normal, white_noise

CO = Cosmology()


# ------------------------------------------------------------ growth

def _growth_ode(omega_m):
    """D and D2 from the growth equations in a (H0 = 1):
    D'' + (3/a + E'/E) D' = 1.5 Om/(a^5 E^2) D and the same operator on D2
    equal to -1.5 Om/(a^5 E^2) D^2, from the matter-era solution at a = 1e-4."""
    E = lambda a: np.sqrt(omega_m * a ** -3 + 1 - omega_m)
    dlnE = lambda a: -1.5 * omega_m * a ** -4 / E(a) ** 2

    def rhs(a, y):
        d1, v1, d2, v2 = y
        src = 1.5 * omega_m / (a ** 5 * E(a) ** 2)
        damp = 3.0 / a + dlnE(a)
        return [v1, -damp * v1 + src * d1, v2, -damp * v2 + src * (d2 - d1 * d1)]

    a0 = 1e-4
    sol = solve_ivp(rhs, [a0, 1.0], [a0, 1.0, -3.0 / 7.0 * a0 ** 2, -6.0 / 7.0 * a0],
                    method="DOP853", rtol=1e-12, atol=1e-22, dense_output=True)
    norm = sol.sol(1.0)[0]
    return lambda a: (sol.sol(a)[2] / norm ** 2, sol.sol(a)[3] / norm ** 2)


@pytest.mark.parametrize("om", [0.3, 0.25])
def test_d2_fit_matches_growth_ode(om):
    ode = _growth_ode(om)
    for a, tol_d, tol_v in ((1 / 64, 1e-9, 1e-9), (0.1, 1e-7, 1e-7), (1.0, 3e-4, 6e-4)):
        d2, v2 = ode(a)
        assert abs(C.growth_D2(a, om) / d2 - 1) < tol_d, a
        assert abs(C.growth_dD2(a, om) / v2 - 1) < tol_v, a


def test_d2_matter_era_limit():
    a = 1e-3
    assert abs(C.growth_D2(a, 0.3) / (-3 / 7 * C.growth_D(a, 0.3) ** 2) - 1) < 1e-8


def test_g2_is_momentum_growth():
    om, h = 0.3, 1e-6
    for a in (1 / 64, 0.3, 1.0):
        dd2 = (C.growth_D2(a + h, om) - C.growth_D2(a - h, om)) / (2 * h)
        g2 = a ** 3 * C.hubble_E(a, om) * dd2
        assert abs(C.growth_G2(a, om) / g2 - 1) < 1e-8


# ------------------------------------------------- second-order field

def _grid(n, box):
    q = pm.lattice(n, box)
    return [q[:, j].reshape(n, n, n) for j in range(3)]


def test_single_plane_wave_has_no_second_order_term():
    n, box = 16, 32.0
    x, _, _ = _grid(n, box)
    delta = 0.7 * np.cos(2 * np.pi * 3 * x / box)
    hess = lpt.potential_hessian(M.rfftn(delta), n, box)
    assert np.max(np.abs(lpt.second_order_source(hess))) < 1e-15
    assert np.max(np.abs(lpt.second_order_from_density(delta, box))) < 1e-15


def test_crossed_plane_waves_closed_form():
    """delta = A cos(al x) + B cos(be y): phi_xx = A cos(al x), phi_yy = B cos(be y),
    S = A B cos(al x) cos(be y), s2 = grad phi2 with
    phi2 = -A B cos(al x) cos(be y) / (al^2 + be^2)."""
    n, box = 16, 32.0
    x, y, _ = _grid(n, box)
    al, be = 2 * np.pi * 2 / box, 2 * np.pi * 3 / box
    A, B = 0.4, -0.7
    delta = A * np.cos(al * x) + B * np.cos(be * y)
    s2 = lpt.second_order_from_density(delta, box)
    c = A * B / (al * al + be * be)
    ref0 = c * al * np.sin(al * x) * np.cos(be * y)
    ref1 = c * be * np.cos(al * x) * np.sin(be * y)
    np.testing.assert_allclose(s2[:, 0], ref0.reshape(-1), atol=1e-13)
    np.testing.assert_allclose(s2[:, 1], ref1.reshape(-1), atol=1e-13)
    assert np.max(np.abs(s2[:, 2])) < 1e-13


def test_off_axis_wave_pair_closed_form():
    """Waves along (1,1,0) and z: the mixed entries phi_xy enter S."""
    n, box = 16, 16.0
    x, y, z = _grid(n, box)
    kf = 2 * np.pi / box
    A, B = 0.5, 0.3
    delta = A * np.cos(kf * (x + y)) + B * np.cos(2 * kf * z)
    s2 = lpt.second_order_from_density(delta, box)
    # phi = -A cos(u)/(2 kf^2) - B cos(2 kf z)/(4 kf^2), u = kf (x + y):
    # phi_xx = phi_yy = phi_xy = A cos(u)/2, phi_zz = B cos(2 kf z); then
    # S = phi_xx phi_yy - phi_xy^2 + (phi_xx + phi_yy) phi_zz = A B cos(u) cos(2 kf z)
    # and phi2 = -A B cos(u) cos(2 kf z) / (6 kf^2)
    u, w = kf * (x + y), 2 * kf * z
    c = A * B / (6 * kf * kf)
    np.testing.assert_allclose(s2[:, 0], (c * kf * np.sin(u) * np.cos(w)).reshape(-1), atol=1e-13)
    np.testing.assert_allclose(s2[:, 1], (c * kf * np.sin(u) * np.cos(w)).reshape(-1), atol=1e-13)
    np.testing.assert_allclose(s2[:, 2], (c * 2 * kf * np.cos(u) * np.sin(w)).reshape(-1),
                               atol=1e-13)


def test_hessian_trace_is_linear_density():
    n, box = 16, 64.0
    dk = lpt.linear_density_k(white_noise(n, 2), box, CO)
    hess = lpt.potential_hessian(dk, n, box)
    trace = hess[0, 0] + hess[1, 1] + hess[2, 2]
    delta = M.irfftn(dk, n)
    np.testing.assert_allclose(trace, delta, atol=1e-12 * np.abs(delta).max())


def test_second_order_transpose_is_exact_gradient():
    """u . s2(w) is quadratic in w, so a central difference of any step is exact."""
    n, box = 8, 32.0
    w = white_noise(n, 11).astype(np.float64)
    u = normal((n ** 3, 3), 12)
    d = normal((n,) * 3, 13)
    f = lambda v: np.sum(u * lpt.second_order_displacement(v, box, CO))
    fd = (f(w + d) - f(w - d)) / 2.0
    g = lpt.second_order_transpose(w, u, box, CO)
    assert abs(np.sum(g * d) / fd - 1) < 1e-10


def test_second_order_omega_m_tangent():
    n, box = 8, 32.0
    w = white_noise(n, 14).astype(np.float64)
    h = 1e-5
    up = lpt.second_order_displacement(w, box, replace(CO, omega_m=CO.omega_m + h))
    dn = lpt.second_order_displacement(w, box, replace(CO, omega_m=CO.omega_m - h))
    t = lpt.second_order_tangent_omega_m(w, box, CO)
    fd = (up - dn) / (2 * h)
    assert np.linalg.norm(t - fd) < 1e-6 * np.linalg.norm(fd)


def test_second_order_scales_as_sigma8_squared():
    n, box = 8, 32.0
    w = white_noise(n, 15).astype(np.float64)
    a = lpt.second_order_displacement(w, box, CO)
    b = lpt.second_order_displacement(w, box, replace(CO, sigma8=2 * CO.sigma8))
    np.testing.assert_allclose(b, 4 * a, rtol=1e-12, atol=1e-14 * np.abs(b).max())


# ---------------------------------------------------------- dynamics

def test_2lpt_start_carries_the_second_order_growing_mode():
    """Crossed waves evolved by the PM from a = 1/64 to 0.5: the amplitude of the
    mode-coupled pattern sin(al x) cos(be y) in x-displacements should equal
    D2(0.5) A B al / (al^2 + be^2).  Started from 2LPT it does so within 5%;
    started from Zel'dovich (no second-order term at a_0) the transient leaves
    it further off."""
    n, box = 32, 32.0
    x, y, _ = _grid(n, box)
    al = be = 2 * np.pi / box
    A = B = 0.6
    delta = A * np.cos(al * x) + B * np.cos(be * y)
    s1 = pm.zeldovich_displacement(delta, box, M.poisson_radial(n, box))
    s2 = lpt.second_order_from_density(delta, box)
    pattern = (np.sin(al * x) * np.cos(be * y)).reshape(-1)
    want = C.growth_D2(0.5, CO.omega_m) * A * B * al / (al * al + be * be)
    err = {}
    for order in (1, 2):
        st = pm.Setup(n, n, box, 32, CO, 1 / 64, 0.5, order)
        run = pm.forward_from_displacement(s1, st, None, s2 if order == 2 else None)
        amp = np.sum(run.disp[-1][:, 0] * pattern) / np.sum(pattern * pattern)
        err[order] = abs(amp / want - 1)
    assert err[2] < 0.05, err
    assert err[2] < 0.6 * err[1], err


# ---------------------------------------------------- whole-run gradients

def _loss(noise, st, target, wd, wp):
    r = pm.forward(noise, st)
    return pm.mse_loss(r.dens, target)[0] + np.sum(wd * r.disp[-1]) + np.sum(wp * r.mom)


@pytest.fixture(scope="module")
def lpt2_case():
    st = pm.Setup(8, 16, 32.0, 4, CO, lpt_order=2)
    noise = white_noise(8, 3)
    target = pm.forward(white_noise(8, 4), st).dens
    wd, wp = normal((512, 3), 9), normal((512, 3), 10)
    run = pm.forward(noise, st)
    _, gd = pm.mse_loss(run.dens, target)
    g = pm.adjoint(run, noise, g_dens=gd, g_disp=wd, g_mom=wp)
    return st, noise, target, wd, wp, g


def test_lpt2_gradient_noise_fd(lpt2_case):
    st, noise, target, wd, wp, g = lpt2_case
    d = normal(noise.shape, 7)
    h = 1e-6
    fd = (_loss(noise + h * d, st, target, wd, wp) - _loss(noise - h * d, st, target, wd, wp)) / (2 * h)
    assert abs(fd / np.sum(g.noise * d) - 1) < 1e-6


@pytest.mark.parametrize("name", ["omega_m", "sigma8"])
def test_lpt2_gradient_cosmology_fd(lpt2_case, name):
    st, noise, target, wd, wp, g = lpt2_case
    h = 1e-6
    c = st.cosmo
    up = replace(st, cosmo=replace(c, **{name: getattr(c, name) + h}))
    dn = replace(st, cosmo=replace(c, **{name: getattr(c, name) - h}))
    fd = (_loss(noise, up, target, wd, wp) - _loss(noise, dn, target, wd, wp)) / (2 * h)
    assert abs(fd / getattr(g, name) - 1) < 1e-6


def test_lpt2_second_order_term_is_small_at_a0():
    """At a_0 = 1/64 the 2LPT correction is a small fraction of the Zel'dovich
    displacement (D2/D ~ -(3/7) D), but not zero."""
    st = pm.Setup(16, 32, 64.0, 1, CO, lpt_order=2)
    noise = white_noise(16, 5)
    s1 = pm.zeldovich_displacement(noise, st.box, pm.ic_radial(16, st.box, CO))
    s2 = lpt.second_order_displacement(noise, st.box, CO)
    co = C.kdk_coefficients(CO.omega_m, st.a_start, st.a_stop, 1)
    r = np.linalg.norm(co.D20 * s2) / np.linalg.norm(co.D0 * s1)
    assert 1e-5 < r < 0.05
