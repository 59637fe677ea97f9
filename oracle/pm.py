"""PM simulation, its discrete adjoint and the parameter gradients, in FP64.

Test infrastructure (see ``oracle/__init__.py``).

Passages followed (pmwd paper)
  * Summary: a differentiable cosmological PM simulation from initial
    conditions; gradients by the adjoint method with reverse time integration
    reconstructing the evolution history instead of storing it.
  * Statement of Need: the adjoint evolves a dual set of equations backward in
    time; discretize-then-optimize, so gradients propagate backward along the
    same discrete trajectory the forward integration took.

This oracle deliberately computes the adjoint over a STORED trajectory (every
x_n and p_{n+1/2} kept), which is the plain definition of the discrete
transpose; the GPU path reconstructs the same states by reverse-time
integration.  Agreement of the two therefore checks the reconstruction.

Initial conditions follow the Zel'dovich approximation: the linear density is
the white noise coloured by sqrt(P(k)/V_cell), the displacement is
s_k = i k delta_k / k^2, and x_0 = q + D(a_0) s, p_0 = G(a_0) s.  With
``lpt_order = 2`` the second-order term of ``lpt`` is added:
x_0 = q + D s + D2 s2, p_0 = G s + G2 s2.

Time stepping is kick-drift-kick with growth-factor coefficients
(``cosmology.kdk_coefficients``), each optionally multiplied by a per-step
scale (``Setup.step_scales``, the temporal counterpart of the learned force
filter: a correction of the time integration trained through the adjoint):
    F_0 = F(x_0)
    for n = 0 .. N-1:
        p <- p + kick_a_n F_n ;  x <- x + drift_n p ;
        F_{n+1} = F(x) ;         p <- p + kick_b_n F_{n+1}
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cosmology as cosmo_mod
from . import lpt
from . import mesh as M
from . import mlp


@dataclass
class Setup:
    ptcl_grid: int
    mesh: int
    box: float
    n_steps: int
    cosmo: object
    a_start: float = 1.0 / 64
    a_stop: float = 1.0
    lpt_order: int = 1            # 1: Zel'dovich ICs; 2: plus the 2LPT term
    step_scales: object = None    # [3, N] multipliers of kick_a, drift, kick_b (None: 1)

    @property
    def n_particles(self):
        return self.ptcl_grid ** 3

    @property
    def mass(self):
        return self.mesh ** 3 / self.n_particles


def setup_from(workload, cosmo=None):
    return Setup(workload.ptcl_grid, workload.mesh, workload.box, workload.n_steps,
                 cosmo if cosmo is not None else workload.cosmo,
                 workload.a_start, workload.a_stop)


def step_coefficients(setup):
    """KDK factors of ``setup`` with the per-step scales applied (D0, G0, D20
    and G20 unscaled)."""
    co = cosmo_mod.kdk_coefficients(setup.cosmo.omega_m, setup.a_start, setup.a_stop,
                                    setup.n_steps)
    if setup.step_scales is not None:
        sc = np.asarray(setup.step_scales, dtype=np.float64).reshape(3, setup.n_steps)
        co.kick_a, co.drift, co.kick_b = co.kick_a * sc[0], co.drift * sc[1], co.kick_b * sc[2]
    return co


def lattice(ptcl_grid, box):
    """Lagrangian positions q_j = j * box / Np, C order (last axis fastest)."""
    g = np.arange(ptcl_grid, dtype=np.float64) * (box / ptcl_grid)
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1)
    return q.reshape(-1, 3)


# ------------------------------------------------------------- ICs

def ic_radial(ptcl_grid, box, cosmo):
    """sqrt(P_lin(k) / V_cell) / k^2 as a function of integer |n|^2."""
    amp = cosmo_mod.pk_amplitude(cosmo)
    vcell = (box / ptcl_grid) ** 3
    kf = 2.0 * np.pi / box

    def radial(nsq):
        k = kf * np.sqrt(nsq.astype(np.float64))
        ks = np.where(k > 0, k, 1.0)
        return np.sqrt(cosmo_mod.linear_pk(ks, cosmo, amp) / vcell) / (ks * ks)
    return radial


def ic_radial_domega_m(ptcl_grid, box, cosmo, rel_step=1e-5):
    """Central difference in Omega_m of ``ic_radial`` (sigma_8 held fixed)."""
    from dataclasses import replace
    h = rel_step * cosmo.omega_m
    up = ic_radial(ptcl_grid, box, replace(cosmo, omega_m=cosmo.omega_m + h))
    dn = ic_radial(ptcl_grid, box, replace(cosmo, omega_m=cosmo.omega_m - h))
    return lambda nsq: (up(nsq) - dn(nsq)) / (2.0 * h)


def zeldovich_displacement(noise, box, radial):
    """s_j = IDFT(i k_j radial(|n|^2) DFT(noise)), j = 0..2, as [Np^3, 3].

    With ``radial = ic_radial`` this is the displacement field at a = 1 whose
    divergence is minus the linear density sqrt(P/V_cell)-coloured noise.
    """
    npg = noise.shape[0]
    wk = M.rfftn(noise)
    mult = M.gradient_multipliers(npg, box, radial)
    return np.stack([M.irfftn(m * wk, npg).reshape(-1) for m in mult], axis=1)


def zeldovich_transpose(s_bar, box, radial):
    """Transpose of ``zeldovich_displacement``: Sum_j IDFT(conj(M_j) DFT(s_bar_j))."""
    npg = round(s_bar.shape[0] ** (1.0 / 3.0))
    mult = M.gradient_multipliers(npg, box, radial)
    acc = 0
    for j in range(3):
        acc = acc + np.conj(mult[j]) * M.rfftn(s_bar[:, j].reshape(npg, npg, npg))
    return M.irfftn(acc, npg)


# ------------------------------------------------------------- force

def filter_at(theta, setup, a):
    """Radial filter table f(|n|^2, a) (None when the plain force is used)."""
    if theta is None:
        return None, None
    return mlp.filter_table(theta, setup.mesh, setup.box, a)


def pm_force(x, setup, filt=None):
    """Force on each particle: CIC density -> spectral F~_j -> CIC gather."""
    delta = M.density(x, setup.mesh, setup.box, setup.n_particles)
    fmesh, dk = M.force_meshes(delta, setup.box, filt)
    F = np.stack([M.gather(f, x, setup.box) for f in fmesh], axis=1)
    return F, fmesh, dk


def pm_force_vjp(x, v, setup, filt=None):
    """J_F(x)^T v for the particle force F(x) and cotangent v [P, 3].

    Three terms: (i) the gather's own position dependence, Sum_j v_j grad w . F~_j;
    (ii) the gather's transpose, a CIC scatter of v_j (no mass), pushed through
    the transposed spectral operator to a density cotangent delta_bar;
    (iii) the scatter's position dependence, m grad w . delta_bar.
    Also returns dL/df(|n|^2) for the filter table and the force F(x) itself.
    """
    F, fmesh, dk = pm_force(x, setup, filt)
    xi = np.zeros_like(x)
    for j in range(3):
        xi += v[:, j:j + 1] * M.gather_grad(fmesh[j], x, setup.box)
    gbar = [M.scatter(x, setup.mesh, setup.box, v[:, j]) for j in range(3)]
    dbar, gk = M.force_transpose(gbar, setup.box, filt)
    xi += setup.mass * M.gather_grad(dbar, x, setup.box)
    f_bar = M.filter_table_cotangent(dk, gk, setup.box) if filt is not None else None
    return xi, f_bar, F


# --------------------------------------------------------- forward run

@dataclass
class Run:
    setup: Setup
    theta: object
    s: np.ndarray                 # Zel'dovich displacement at a = 1, [P, 3]
    s2: np.ndarray = None         # second-order displacement at a = 1 (2LPT)
    disp: list = field(default_factory=list)     # x_n - q, n = 0..N
    p_half: list = field(default_factory=list)   # p_{n+1/2}, n = 0..N-1
    mom0: np.ndarray = None
    mom: np.ndarray = None        # p_N
    dens: np.ndarray = None       # delta at x_N on the mesh

    @property
    def q(self):
        return lattice(self.setup.ptcl_grid, self.setup.box)


def forward(noise, setup, theta=None):
    """Zel'dovich (or 2LPT) ICs then N KDK steps, storing the whole trajectory."""
    s = zeldovich_displacement(noise, setup.box,
                               ic_radial(setup.ptcl_grid, setup.box, setup.cosmo))
    s2 = (lpt.second_order_displacement(noise, setup.box, setup.cosmo)
          if setup.lpt_order == 2 else None)
    return forward_from_displacement(s, setup, theta, s2)


def initial_state(s, setup, s2=None):
    """(x_0 - q, p_0) = (D s + D2 s2, G s + G2 s2) at a_0 (s2 term for 2LPT)."""
    co = step_coefficients(setup)
    disp, mom = co.D0 * s, co.G0 * s
    if s2 is not None:
        disp = disp + co.D20 * s2
        mom = mom + co.G20 * s2
    return disp, mom


def forward_from_displacement(s, setup, theta=None, s2=None):
    """N KDK steps from x_0 = q + D(a_0) s (+ D2(a_0) s2), p_0 = G(a_0) s
    (+ G2(a_0) s2) for given s, s2 [P, 3]."""
    co = step_coefficients(setup)
    q = lattice(setup.ptcl_grid, setup.box)
    disp, mom = initial_state(s, setup, s2)
    run = Run(setup=setup, theta=theta, s=s, s2=s2, mom0=mom.copy())
    run.disp.append(disp.copy())
    F, _, _ = pm_force(q + disp, setup, filter_at(theta, setup, co.a[0])[0])
    for n in range(setup.n_steps):
        mom = mom + co.kick_a[n] * F
        run.p_half.append(mom.copy())
        disp = disp + co.drift[n] * mom
        run.disp.append(disp.copy())
        F, _, _ = pm_force(q + disp, setup, filter_at(theta, setup, co.a[n + 1])[0])
        mom = mom + co.kick_b[n] * F
    run.mom = mom
    run.dens = M.density(q + disp, setup.mesh, setup.box, setup.n_particles)
    return run


def reverse_reconstruct(disp_N, mom_N, setup, theta=None):
    """Reverse-time integration from (x_N, p_N) back to (x_0, p_0).

    Undoes each KDK step in reverse order, recomputing the force from the
    reconstructed positions.  Returns the list of reconstructed displacements
    (index n = 0..N) and p_0.
    """
    co = step_coefficients(setup)
    q = lattice(setup.ptcl_grid, setup.box)
    disp, mom = disp_N.copy(), mom_N.copy()
    out = [None] * (setup.n_steps + 1)
    out[-1] = disp.copy()
    for n in range(setup.n_steps - 1, -1, -1):
        F, _, _ = pm_force(q + disp, setup, filter_at(theta, setup, co.a[n + 1])[0])
        mom = mom - co.kick_b[n] * F
        disp = disp - co.drift[n] * mom
        out[n] = disp.copy()
        F, _, _ = pm_force(q + disp, setup, filter_at(theta, setup, co.a[n])[0])
        mom = mom - co.kick_a[n] * F
    return out, mom


# ---------------------------------------------------------- adjoint

@dataclass
class Gradients:
    noise: np.ndarray
    omega_m: float
    sigma8: float
    theta: object
    kick_a: np.ndarray
    kick_b: np.ndarray
    drift: np.ndarray
    D0: float
    G0: float
    xi0: np.ndarray
    pi0: np.ndarray
    D20: float = 0.0
    G20: float = 0.0
    step_scales: np.ndarray = None   # [3, N] dL/d(scale) of kick_a, drift, kick_b


def adjoint(run, noise, g_dens=None, g_disp=None, g_mom=None):
    """Exact transpose of ``forward`` over its stored trajectory.

    Cotangents xi (positions) and pi (momenta) are carried backward:
      start   xi = dL/dx_N (+ m grad w . dL/ddelta), pi = dL/dp_N
      step n  xi += J_F(x_{n+1})^T [(kick_b_n + kick_a_{n+1}) pi]   (kick_a_N = 0)
              pi += drift_n xi
      end     xi += J_F(x_0)^T [kick_a_0 pi]
    The scalar cotangents dL/dkick_a_n = Sum pi.F_n, dL/dkick_b_n = Sum pi.F_{n+1}
    and dL/ddrift_n = Sum xi.p_{n+1/2} are recorded on the way and combined
    with dcoefficient/dOmega_m; the ICs add the D0, G0 and P(k) terms.  Times
    the unscaled factors they are the gradients of the per-step scales.
    """
    st = run.setup
    N = st.n_steps
    co = step_coefficients(st)
    q = lattice(st.ptcl_grid, st.box)
    P = st.n_particles
    xN = q + run.disp[-1]
    xi = np.zeros((P, 3)) if g_disp is None else np.array(g_disp, dtype=np.float64)
    pi = np.zeros((P, 3)) if g_mom is None else np.array(g_mom, dtype=np.float64)
    if g_dens is not None:
        xi = xi + st.mass * M.gather_grad(np.asarray(g_dens, dtype=np.float64), xN, st.box)

    g_ka, g_kb, g_dr = np.zeros(N), np.zeros(N), np.zeros(N)
    g_theta = None if run.theta is None else np.zeros(mlp.N_PARAMS)

    def add_vjp(x, a, coeff):
        nonlocal xi, g_theta
        filt, cache = filter_at(run.theta, st, a)
        dxi, f_bar, F = pm_force_vjp(x, coeff * pi, st, filt)
        xi = xi + dxi
        if g_theta is not None:
            g_theta = g_theta + mlp.backward(run.theta, cache, f_bar)
        return F

    for n in range(N - 1, -1, -1):
        x1 = q + run.disp[n + 1]
        coeff = co.kick_b[n] + (co.kick_a[n + 1] if n + 1 < N else 0.0)
        F1 = add_vjp(x1, co.a[n + 1], coeff)
        dot = float(np.sum(pi * F1))
        g_kb[n] = dot
        if n + 1 < N:
            g_ka[n + 1] = dot
        g_dr[n] = float(np.sum(xi * run.p_half[n]))
        pi = pi + co.drift[n] * xi
    F0 = add_vjp(q + run.disp[0], co.a[0], co.kick_a[0])
    g_ka[0] = float(np.sum(pi * F0))

    # Zel'dovich ICs: disp_0 = D0 s, p_0 = G0 s, s = Z(noise; P(k))
    s = run.s
    s_bar = co.D0 * xi + co.G0 * pi
    gD0 = float(np.sum(xi * s))
    gG0 = float(np.sum(pi * s))
    radial = ic_radial(st.ptcl_grid, st.box, st.cosmo)
    g_noise = zeldovich_transpose(s_bar, st.box, radial)
    g_sigma8 = float(np.sum(s_bar * s)) / st.cosmo.sigma8
    dco = cosmo_mod.kdk_coefficient_derivatives(st.cosmo.omega_m, st.a_start, st.a_stop, N)
    base = cosmo_mod.kdk_coefficients(st.cosmo.omega_m, st.a_start, st.a_stop, N)
    g_scales = np.stack([g_ka * base.kick_a, g_dr * base.drift, g_kb * base.kick_b])
    if st.step_scales is not None:
        sc = np.asarray(st.step_scales, dtype=np.float64).reshape(3, N)
        dco.kick_a, dco.drift, dco.kick_b = dco.kick_a * sc[0], dco.drift * sc[1], dco.kick_b * sc[2]
    s_dom = zeldovich_displacement(noise, st.box,
                                   ic_radial_domega_m(st.ptcl_grid, st.box, st.cosmo))
    g_om = (np.dot(g_ka, dco.kick_a) + np.dot(g_kb, dco.kick_b) + np.dot(g_dr, dco.drift)
            + gD0 * dco.D0 + gG0 * dco.G0 + float(np.sum(s_bar * s_dom)))
    gD20 = gG20 = 0.0
    if run.s2 is not None:
        # 2LPT term: disp_0 += D20 s2, p_0 += G20 s2, s2 quadratic in the noise
        # (hence the factor 2 in the sigma_8 derivative, s2 ~ sigma_8^2)
        s2_bar = co.D20 * xi + co.G20 * pi
        gD20 = float(np.sum(xi * run.s2))
        gG20 = float(np.sum(pi * run.s2))
        g_noise = g_noise + lpt.second_order_transpose(np.asarray(noise, dtype=np.float64),
                                                       s2_bar, st.box, st.cosmo)
        g_sigma8 += 2.0 * float(np.sum(s2_bar * run.s2)) / st.cosmo.sigma8
        s2_dom = lpt.second_order_tangent_omega_m(np.asarray(noise, dtype=np.float64),
                                                  st.box, st.cosmo)
        g_om += gD20 * dco.D20 + gG20 * dco.G20 + float(np.sum(s2_bar * s2_dom))
    return Gradients(noise=g_noise, omega_m=float(g_om), sigma8=g_sigma8, theta=g_theta,
                     kick_a=g_ka, kick_b=g_kb, drift=g_dr, D0=gD0, G0=gG0,
                     xi0=xi, pi0=pi, D20=gD20, G20=gG20, step_scales=g_scales)


# ------------------------------------------------------------- losses

def mse_loss(dens, target):
    """L = N^-3 Sum (delta - delta_t)^2 and its cotangent 2 (delta - delta_t) / N^3."""
    d = np.asarray(dens, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    n = d.size
    return float(np.sum(d * d)) / n, 2.0 * d / n


# ------------------------------------------------------- filter-training losses
#
# The paper names no training objective for a learned force correction.  The
# reading taken: a power-spectrum term over the shells up to the Nyquist wave
# number of the coarse mesh, plus a weighted term on the final particle
# positions, both against a run of the same initial conditions on a finer mesh.

def pk_loss(dens, pk_target, box, n_bins, weight=1.0):
    """L = weight * mean_b (P_b / P_b^target - 1)^2 over shells b = 1..n_bins that
    hold modes and a nonzero target, with P measured by ``mesh.power_spectrum``;
    returns (L, dL/d dens)."""
    _, pk, cnt = M.power_spectrum(dens, box, n_bins)
    pt = np.asarray(pk_target, dtype=np.float64)
    use = (cnt > 0) & (pt != 0)
    nb = int(np.count_nonzero(use))
    r = np.where(use, pk / np.where(use, pt, 1.0) - 1.0, 0.0)
    loss = weight * float(np.sum(r * r)) / nb
    g_pk = np.where(use, weight * 2.0 * r / (np.where(use, pt, 1.0) * nb), 0.0)
    return loss, M.power_spectrum_vjp(dens, box, n_bins, g_pk)


def disp_loss(disp, disp_target, box, mesh, weight=1.0):
    """L = weight * mean_p |x_p - x_p^target|^2 / cell^2 with the periodic
    minimum-image separation (same lattice point, so x - x' = s - s' wrapped to
    [-box/2, box/2)); returns (L, dL/d disp)."""
    d = np.asarray(disp, dtype=np.float64) - np.asarray(disp_target, dtype=np.float64)
    d = d - box * np.floor(d / box + 0.5)
    cell = box / mesh
    n = d.shape[0]
    return (weight * float(np.sum(d * d)) / (n * cell * cell),
            weight * 2.0 * d / (n * cell * cell))
