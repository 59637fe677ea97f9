"""Pins of the oracle's background cosmology and KDK coefficients.

Each test checks the oracle against something other than itself: a second
closed form, the Einstein-de Sitter limit, the growth ODE, or linear-theory
exactness of the integrator.
"""
import numpy as np
import pytest
from dataclasses import replace

from oracle import cosmology as C
from synthetic import Cosmology

CO = Cosmology()
A_TEST = np.array([1 / 64, 0.05, 0.1, 0.25, 0.5, 0.75, 1.0])


@pytest.mark.parametrize("om", [0.3, 0.15, 0.6])
def test_growth_hypergeometric_matches_integral(om):
    # two independent closed forms of the flat-LCDM growing mode
    d_h = C.growth_D(A_TEST, om)
    d_i = np.array([C.growth_D_integral(a, om) for a in A_TEST])
    np.testing.assert_allclose(d_h, d_i, rtol=1e-12, atol=0)


def test_growth_einstein_de_sitter_limit():
    # Omega_m = 1: D = a, G = a^3 E dD/da = a^{3/2}
    om = 1.0 - 1e-12
    np.testing.assert_allclose(C.growth_D(A_TEST, om), A_TEST, rtol=1e-9)
    np.testing.assert_allclose(C.growth_G(A_TEST, om), A_TEST ** 1.5, rtol=1e-9)


def test_growth_rate_close_to_linder_fit():
    # f = dlnD/dlna at a = 1 is within ~1% of the Omega_m^0.55 fit (Linder 2005)
    for om in (0.25, 0.3, 0.4):
        f = C.growth_dD(1.0, om) / C.growth_D(1.0, om)
        assert abs(f / om ** 0.55 - 1.0) < 0.01


def test_G_derivative_identity():
    # dG/da = 1.5 Omega_m D / (a^2 E), by a fourth-order central difference
    om = 0.3
    a = A_TEST[1:-1]
    h = 3e-3 * a
    G = lambda t: C.growth_G(t, om)
    dG = (-G(a + 2 * h) + 8 * G(a + h) - 8 * G(a - h) + G(a - 2 * h)) / (12 * h)
    rhs = 1.5 * om * C.growth_D(a, om) / (a * a * C.hubble_E(a, om))
    np.testing.assert_allclose(dG, rhs, rtol=1e-9)


def test_dD_matches_central_difference():
    om, h = 0.3, 1e-6
    a = A_TEST[1:-1]
    fd = (C.growth_D(a + h, om) - C.growth_D(a - h, om)) / (2 * h)
    np.testing.assert_allclose(C.growth_dD(a, om), fd, rtol=1e-8)


def test_sigma8_normalisation_round_trip():
    amp = C.pk_amplitude(CO)
    assert abs(C.sigma_R(CO, amp) / CO.sigma8 - 1) < 1e-10
    # an independent quadrature (dense Simpson in ln k) agrees
    assert abs(C.sigma_R(CO, amp, method="simpson") / CO.sigma8 - 1) < 1e-8


def test_transfer_function_limits():
    # T -> 1 on large scales, decreasing, ~ln(q)/(14.2 q^2) on small scales
    k = np.logspace(-5, 2, 200)
    T = C.transfer_eh_nowiggle(k, CO)
    assert abs(T[0] - 1) < 1e-4
    assert np.all(np.diff(T) < 0)
    q = k[-1] * (CO.T_cmb / 2.7) ** 2 / (CO.omega_m * CO.h)
    assert 0.02 < T[-1] * q * q / np.log(q) < 0.2


def test_tophat_window_series():
    x = np.array([1e-4, 5e-4, 2e-3])
    exact = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    np.testing.assert_allclose(C.tophat_window(x), exact, rtol=1e-6)


def _linear_kdk(co, s_amp):
    """Run the KDK scheme with the exact linear force F = D(a) s."""
    x, p = co.D0 * s_amp, co.G0 * s_amp
    D = C.growth_D(co.a, 0.3)
    out = [(x, p)]
    F = D[0] * s_amp
    for n in range(len(co.drift)):
        p = p + co.kick_a[n] * F
        x = x + co.drift[n] * p
        F = D[n + 1] * s_amp
        p = p + co.kick_b[n] * F
        out.append((x, p))
    return out


@pytest.mark.parametrize("n_steps", [1, 3, 10, 63])
def test_kdk_exact_for_linear_growth(n_steps):
    # one step of any size reproduces x = D(a) s, p = G(a) s exactly
    co = C.kdk_coefficients(0.3, 1 / 64, 1.0, n_steps)
    out = _linear_kdk(co, 1.0)
    D, G = C.growth_D(co.a, 0.3), C.growth_G(co.a, 0.3)
    for n, (x, p) in enumerate(out):
        assert abs(x - D[n]) < 1e-13 * max(1, D[n])
        assert abs(p - G[n]) < 1e-13 * max(1, G[n])


def test_kdk_time_grid():
    co = C.kdk_coefficients(0.3, 1 / 64, 1.0, 63)
    np.testing.assert_allclose(co.a, (np.arange(64) + 1) / 64, rtol=0, atol=1e-15)


def test_coefficient_derivatives_match_finer_difference():
    # central differences at two step sizes agree (smoothness in Omega_m)
    d1 = C.kdk_coefficient_derivatives(0.3, 1 / 64, 1, 10, rel_step=1e-5)
    d2 = C.kdk_coefficient_derivatives(0.3, 1 / 64, 1, 10, rel_step=1e-4)
    np.testing.assert_allclose(d1.kick_a, d2.kick_a, rtol=1e-6)
    np.testing.assert_allclose(d1.drift, d2.drift, rtol=1e-6)
    assert abs(d1.D0 / d2.D0 - 1) < 1e-6
