"""Background cosmology and growth-factor time-stepping coefficients (FP64).

Test infrastructure (see ``oracle/__init__.py``).

Units: lengths in Mpc/h, wavenumbers in h/Mpc, time unit 1/H0 (H0 = 1), scale
factor a as the time variable, canonical momentum p = a^2 dx/dt.

Passages followed
  * pmwd paper, Statement of Need: the simulation evolves N-body equations of
    motion in an expanding universe; the kick/drift integrator lineage is
    FastPM (the paper's Seljak et al. 2017 citation).
  * Flat LambdaCDM linear growth in closed hypergeometric form (Heath 1977 /
    standard result): D(a) proportional to a 2F1(1/3, 1; 11/6; -a^3 OL/Om).
  * Eisenstein & Hu 1998 no-wiggle transfer function.
  * FastPM growth-factor coefficients: each kick/drift factor is chosen so
    that one step is exact for linear (Zel'dovich) growth.
  * Second-order growth for 2LPT initial conditions: the fit
    D2 = -(3/7) D^2 Omega_m(a)^(-1/143) (Bouchet et al. 1995), with
    Omega_m(a) = Omega_m a^-3 / E^2; exactly -(3/7) D^2 in the matter era.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import integrate, special


# ---------------------------------------------------------------- background

def hubble_E(a, omega_m):
    """E(a) = H(a)/H0 for flat LambdaCDM without radiation."""
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(omega_m * a ** -3 + (1.0 - omega_m))


def _growth_unnormalised(a, omega_m):
    """Growing mode D~(a) = a 2F1(1/3, 1; 11/6; z), z = -a^3 OL/Om, and dD~/da.

    d/dz 2F1(a,b;c;z) = (ab/c) 2F1(a+1,b+1;c+1;z) gives
    dD~/da = 2F1(1/3,1;11/6;z) + (6/11) z 2F1(4/3,2;17/6;z).
    """
    a = np.asarray(a, dtype=np.float64)
    z = -a ** 3 * (1.0 - omega_m) / omega_m
    f0 = special.hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, z)
    f1 = special.hyp2f1(4.0 / 3.0, 2.0, 17.0 / 6.0, z)
    return a * f0, f0 + (6.0 / 11.0) * z * f1


def growth_D(a, omega_m):
    """Linear growth factor normalised to D(1) = 1."""
    d, _ = _growth_unnormalised(a, omega_m)
    d1, _ = _growth_unnormalised(1.0, omega_m)
    return d / d1


def growth_dD(a, omega_m):
    """dD/da with the same normalisation."""
    _, dd = _growth_unnormalised(a, omega_m)
    d1, _ = _growth_unnormalised(1.0, omega_m)
    return dd / d1


def growth_G(a, omega_m):
    """Momentum growth G(a) = a^3 E(a) dD/da, so that p = G s in linear theory."""
    a = np.asarray(a, dtype=np.float64)
    return a ** 3 * hubble_E(a, omega_m) * growth_dD(a, omega_m)


def omega_m_of_a(a, omega_m):
    """Matter density parameter at a: Omega_m a^-3 / E(a)^2."""
    a = np.asarray(a, dtype=np.float64)
    return omega_m * a ** -3 / hubble_E(a, omega_m) ** 2


def growth_D2(a, omega_m):
    """Second-order growth D2(a) = -(3/7) D(a)^2 Omega_m(a)^(-1/143)."""
    return (-3.0 / 7.0) * growth_D(a, omega_m) ** 2 * omega_m_of_a(a, omega_m) ** (-1.0 / 143.0)


def growth_dD2(a, omega_m):
    """dD2/da of the fit: D2 [2 D'/D + (3/143) (1 - Omega_m(a)) / a], using
    dln Omega_m(a)/da = -3 (1 - Omega_m(a)) / a."""
    a = np.asarray(a, dtype=np.float64)
    dlog = (2.0 * growth_dD(a, omega_m) / growth_D(a, omega_m)
            + (3.0 / 143.0) * (1.0 - omega_m_of_a(a, omega_m)) / a)
    return growth_D2(a, omega_m) * dlog


def growth_G2(a, omega_m):
    """Second-order momentum growth G2 = a^3 E dD2/da (p = G2 s2 at second order)."""
    a = np.asarray(a, dtype=np.float64)
    return a ** 3 * hubble_E(a, omega_m) * growth_dD2(a, omega_m)


def growth_D_integral(a, omega_m):
    """Integral form (5 Om / 2) E(a) int_0^a da' / (a' E(a'))^3, normalised.

    An independent route to D used only to pin the hypergeometric form.
    """
    def unnorm(x):
        val, _ = integrate.quad(lambda t: (t * hubble_E(t, omega_m)) ** -3,
                                0.0, x, epsabs=0.0, epsrel=1e-13, limit=200)
        return 2.5 * omega_m * hubble_E(x, omega_m) * val
    return unnorm(a) / unnorm(1.0)


# ------------------------------------------------- linear power spectrum

def transfer_eh_nowiggle(k, cosmo):
    """Eisenstein & Hu (1998) zero-baryon-oscillation transfer function.

    k in h/Mpc.  The sound horizon s is in Mpc, so k h s is dimensionless.
    """
    k = np.asarray(k, dtype=np.float64)
    h = cosmo.h
    om_h2 = cosmo.omega_m * h * h
    ob_h2 = cosmo.omega_b * h * h
    fb = cosmo.omega_b / cosmo.omega_m
    theta = cosmo.T_cmb / 2.7
    s = 44.5 * np.log(9.83 / om_h2) / np.sqrt(1.0 + 10.0 * ob_h2 ** 0.75)
    alpha = 1.0 - 0.328 * np.log(431.0 * om_h2) * fb + 0.38 * np.log(22.3 * om_h2) * fb * fb
    gamma_eff = cosmo.omega_m * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k * h * s) ** 4))
    q = k * theta * theta / gamma_eff
    L0 = np.log(2.0 * np.e + 1.8 * q)
    C0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return L0 / (L0 + C0 * q * q)


def tophat_window(x):
    """Fourier transform of a unit spherical top hat, 3 (sin x - x cos x) / x^3."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return np.where(small, 1.0 - x * x / 10.0, w)


def _unit_amplitude_pk(k, cosmo):
    return k ** cosmo.n_s * transfer_eh_nowiggle(k, cosmo) ** 2


def sigma_R(cosmo, amplitude, R=8.0, method="quad"):
    """RMS linear overdensity in top-hat spheres of radius R Mpc/h at a = 1.

    sigma^2 = (1 / 2 pi^2) int k^3 P(k) W(kR)^2 dln k over [1e-5, 1e2] h/Mpc.
    ``method`` picks adaptive quadrature or a dense Simpson rule (two
    independent quadratures, compared in the tests).
    """
    def integrand(lnk):
        k = np.exp(lnk)
        return k ** 3 * amplitude * _unit_amplitude_pk(k, cosmo) * tophat_window(k * R) ** 2

    lo, hi = np.log(1e-5), np.log(1e2)
    if method == "quad":
        val, _ = integrate.quad(integrand, lo, hi, epsabs=0.0, epsrel=1e-11, limit=1000)
    else:
        x = np.linspace(lo, hi, 2 ** 17 + 1)
        val = integrate.simpson(integrand(x), x=x)
    return np.sqrt(val / (2.0 * np.pi ** 2))


def pk_amplitude(cosmo):
    """A such that P(k) = A k^n_s T(k)^2 has sigma_8 equal to cosmo.sigma8."""
    return (cosmo.sigma8 / sigma_R(cosmo, 1.0)) ** 2


def linear_pk(k, cosmo, amplitude=None):
    """Linear matter power spectrum at a = 1 in (Mpc/h)^3; 0 at k = 0."""
    if amplitude is None:
        amplitude = pk_amplitude(cosmo)
    k = np.asarray(k, dtype=np.float64)
    ks = np.where(k > 0, k, 1.0)
    return np.where(k > 0, amplitude * _unit_amplitude_pk(ks, cosmo), 0.0)


# ------------------------------------------------------------- time stepping

def time_grid(a_start, a_stop, n_steps):
    """a_n for n = 0..N, linear in a."""
    return a_start + (a_stop - a_start) * np.arange(n_steps + 1, dtype=np.float64) / n_steps


@dataclass
class KDKCoefficients:
    a: np.ndarray        # a_n, n = 0..N
    kick_a: np.ndarray   # first half-kick of step n, n = 0..N-1
    drift: np.ndarray    # drift of step n
    kick_b: np.ndarray   # second half-kick of step n
    D0: float            # D(a_0), scales the Zel'dovich displacement
    G0: float            # G(a_0), scales the Zel'dovich momentum
    D20: float = 0.0     # D2(a_0), scales the second-order displacement
    G20: float = 0.0     # G2(a_0), scales the second-order momentum


def kdk_coefficients(omega_m, a_start, a_stop, n_steps):
    """FastPM-style growth-factor kick/drift factors (exact for linear growth).

    With F = -grad(phi), lap(phi) = delta, the equations of motion in a are
    dx/da = p / (a^3 E) and dp/da = 1.5 Om F / (a^2 E); linear theory gives
    x = q + D s, p = G s, F = D s, dG/da = 1.5 Om D / (a^2 E).  Hence
      kick_a_n = [G(a_{n+1/2}) - G(a_n)] / D(a_n)
      drift_n  = [D(a_{n+1}) - D(a_n)] / G(a_{n+1/2})
      kick_b_n = [G(a_{n+1}) - G(a_{n+1/2})] / D(a_{n+1})
    with a_{n+1/2} the arithmetic midpoint.
    """
    a = time_grid(a_start, a_stop, n_steps)
    ah = 0.5 * (a[:-1] + a[1:])
    D, G = growth_D(a, omega_m), growth_G(a, omega_m)
    Gh = growth_G(ah, omega_m)
    kick_a = (Gh - G[:-1]) / D[:-1]
    drift = (D[1:] - D[:-1]) / Gh
    kick_b = (G[1:] - Gh) / D[1:]
    return KDKCoefficients(a=a, kick_a=kick_a, drift=drift, kick_b=kick_b,
                           D0=float(D[0]), G0=float(G[0]),
                           D20=float(growth_D2(a[0], omega_m)),
                           G20=float(growth_G2(a[0], omega_m)))


def kdk_coefficient_derivatives(omega_m, a_start, a_stop, n_steps, rel_step=1e-5):
    """Central differences in Omega_m of every KDK factor and of D0, G0, D20, G20."""
    h = rel_step * omega_m
    up = kdk_coefficients(omega_m + h, a_start, a_stop, n_steps)
    dn = kdk_coefficients(omega_m - h, a_start, a_stop, n_steps)
    inv = 1.0 / (2.0 * h)
    return KDKCoefficients(a=up.a, kick_a=(up.kick_a - dn.kick_a) * inv,
                           drift=(up.drift - dn.drift) * inv,
                           kick_b=(up.kick_b - dn.kick_b) * inv,
                           D0=(up.D0 - dn.D0) * inv, G0=(up.G0 - dn.G0) * inv,
                           D20=(up.D20 - dn.D20) * inv, G20=(up.G20 - dn.G20) * inv)
