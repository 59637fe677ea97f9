"""Second-order Lagrangian perturbation theory (2LPT) initial conditions and
their transpose, in FP64.

Test infrastructure (see ``oracle/__init__.py``).

The pmwd paper starts its runs from first-order (Zel'dovich) initial
conditions.  This module adds the standard second-order term of Lagrangian
perturbation theory (Bouchet et al. 1995; Scoccimarro 1998), written out from
its definition:

    x = q + D s1 + D2 s2,        p = G s1 + G2 s2,

  * s1 = -grad phi1 with lap phi1 = delta_lin: the Zel'dovich displacement,
    s1_k = i k delta_lin,k / k^2 (as in ``pm.zeldovich_displacement``);
  * the second-order source is the sum over the three axis pairs i < j of
    phi1_ii phi1_jj - phi1_ij^2, where the potential's Hessian is
    phi1_ij = IDFT(k_i k_j / k^2 delta_lin,k);
  * s2 = grad phi2 with lap phi2 = S, i.e. s2_k = -i k S_k / k^2;
  * D2 = -(3/7) D^2 Omega_m(a)^(-1/143) and G2 = a^3 E dD2/da
    (``cosmology.growth_D2``, ``cosmology.growth_G2``).

Readings where the method leaves a choice:
  * Nyquist planes: a first derivative zeroes the Nyquist plane of its own
    axis (as the force does).  Hessian entries phi1_ii keep it (k_i^2 is real
    and even there, so the trace of the Hessian is delta_lin exactly);
    off-diagonal entries phi1_ij, i != j, zero the Nyquist planes of both axes.
  * The k = 0 mode of every multiplier is zero.
The transpose carries a cotangent of s2 back to the white noise through the
bilinear source; the Omega_m tangent differentiates the linear amplitude
sqrt(P(k)/V_cell) inside both Hessian factors.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import cosmology as cosmo_mod
from . import mesh as M

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def linear_amplitude(ptcl_grid, box, cosmo):
    """sqrt(P_lin(k) / V_cell) as a function of integer |n|^2 (0 at n = 0)."""
    amp = cosmo_mod.pk_amplitude(cosmo)
    vcell = (box / ptcl_grid) ** 3
    kf = 2.0 * np.pi / box

    def radial(nsq):
        k = kf * np.sqrt(nsq.astype(np.float64))
        return np.where(nsq > 0, np.sqrt(cosmo_mod.linear_pk(k, cosmo, amp) / vcell), 0.0)
    return radial


def linear_amplitude_domega_m(ptcl_grid, box, cosmo, rel_step=1e-5):
    """Central difference in Omega_m of ``linear_amplitude`` (sigma_8 fixed)."""
    h = rel_step * cosmo.omega_m
    up = linear_amplitude(ptcl_grid, box, replace(cosmo, omega_m=cosmo.omega_m + h))
    dn = linear_amplitude(ptcl_grid, box, replace(cosmo, omega_m=cosmo.omega_m - h))
    return lambda nsq: (up(nsq) - dn(nsq)) / (2.0 * h)


def hessian_multiplier(mesh, box, i, j):
    """k_i k_j / k^2 on the half spectrum (dimensionless), Nyquist rule above."""
    ns = M.wave_integers(mesh)
    nsq = ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]
    m = ns[i] * ns[j] / np.where(nsq == 0, 1, nsq).astype(np.float64)
    m = np.where(nsq == 0, 0.0, m)
    if i != j:
        for ax in (i, j):
            nyq = (ns[ax] == -mesh // 2) if ax < 2 else (ns[ax] == mesh // 2)
            m = np.where(nyq, 0.0, m)
    return m


def potential_hessian(delta_k, mesh, box):
    """{(i, j): phi1_ij} for i <= j from the half spectrum of delta_lin."""
    return {p: M.irfftn(hessian_multiplier(mesh, box, *p) * delta_k, mesh) for p in PAIRS}


def second_order_source(hess):
    """S = Sum_{i<j} (phi_ii phi_jj - phi_ij^2)."""
    h = hess
    return (h[0, 0] * h[1, 1] + h[0, 0] * h[2, 2] + h[1, 1] * h[2, 2]
            - h[0, 1] ** 2 - h[0, 2] ** 2 - h[1, 2] ** 2)


def _neg_inverse_laplacian(box):
    """Radial factor -1/k^2 of s2_k = i k (-S_k / k^2) (k = 2 pi n / box)."""
    kf = 2.0 * np.pi / box
    return lambda nsq: -1.0 / (kf * kf * np.where(nsq == 0, 1, nsq))


def displacement_from_source(source, box):
    """s2_j = IDFT(-i k_j S_k / k^2) as [N^3, 3] (gradient Nyquist rule)."""
    mesh = source.shape[0]
    sk = M.rfftn(source)
    mult = M.gradient_multipliers(mesh, box, _neg_inverse_laplacian(box))
    return np.stack([M.irfftn(m * sk, mesh).reshape(-1) for m in mult], axis=1)


def source_transpose(s2_bar, box):
    """Transpose of ``displacement_from_source``: Sum_j IDFT(conj(M_j) DFT(s2_bar_j))."""
    mesh = round(s2_bar.shape[0] ** (1.0 / 3.0))
    mult = M.gradient_multipliers(mesh, box, _neg_inverse_laplacian(box))
    acc = 0
    for j in range(3):
        acc = acc + np.conj(mult[j]) * M.rfftn(s2_bar[:, j].reshape(mesh, mesh, mesh))
    return M.irfftn(acc, mesh)


def second_order_from_density(delta_lin, box):
    """s2 [N^3, 3] of a real linear density field on an N^3 lattice."""
    mesh = delta_lin.shape[0]
    return displacement_from_source(
        second_order_source(potential_hessian(M.rfftn(delta_lin), mesh, box)), box)


def linear_density_k(noise, box, cosmo):
    """delta_lin,k = sqrt(P/V_cell) noise_k on the half spectrum."""
    npg = noise.shape[0]
    ns = M.wave_integers(npg)
    nsq = ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]
    return linear_amplitude(npg, box, cosmo)(nsq) * M.rfftn(noise)


def second_order_displacement(noise, box, cosmo):
    """s2 [Np^3, 3] of the sqrt(P/V_cell)-coloured white noise (at a = 1)."""
    npg = noise.shape[0]
    hess = potential_hessian(linear_density_k(noise, box, cosmo), npg, box)
    return displacement_from_source(second_order_source(hess), box)


def second_order_transpose(noise, s2_bar, box, cosmo):
    """dL/dnoise from the cotangent s2_bar of s2 (the noise enters twice).

    Reverse mode through S: S_bar = transpose of the source-to-displacement
    map; phi_ii_bar = S_bar (phi_jj + phi_kk) over the other two axes;
    phi_ij_bar = -2 S_bar phi_ij; each Hessian entry is the real, even Fourier
    multiplier k_i k_j / k^2 sqrt(P/V_cell) of the noise, its own transpose.
    """
    npg = noise.shape[0]
    ns = M.wave_integers(npg)
    nsq = ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]
    amp = linear_amplitude(npg, box, cosmo)(nsq)
    hess = potential_hessian(amp * M.rfftn(noise), npg, box)
    s_bar = source_transpose(s2_bar, box)
    bar = {}
    for d in range(3):
        o1, o2 = [e for e in range(3) if e != d]
        bar[d, d] = s_bar * (hess[o1, o1] + hess[o2, o2])
    for p in ((0, 1), (0, 2), (1, 2)):
        bar[p] = -2.0 * s_bar * hess[p]
    acc = 0
    for p in PAIRS:
        acc = acc + hessian_multiplier(npg, box, *p) * amp * M.rfftn(bar[p])
    return M.irfftn(acc, npg)


def second_order_tangent_omega_m(noise, box, cosmo):
    """ds2/dOmega_m through sqrt(P/V_cell) (forward mode, S bilinear)."""
    npg = noise.shape[0]
    ns = M.wave_integers(npg)
    nsq = ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]
    wk = M.rfftn(noise)
    hess = potential_hessian(linear_amplitude(npg, box, cosmo)(nsq) * wk, npg, box)
    dhess = potential_hessian(linear_amplitude_domega_m(npg, box, cosmo)(nsq) * wk, npg, box)
    dS = 0
    for i, j in ((0, 1), (0, 2), (1, 2)):
        dS = dS + dhess[i, i] * hess[j, j] + hess[i, i] * dhess[j, j] \
            - 2.0 * hess[i, j] * dhess[i, j]
    return displacement_from_source(dS, box)
