"""Pins of the oracle's simulation, adjoint and gradients.

Plane-wave linear growth, IC statistics, FP64 reversibility, dot-product tests
of the whole discrete step, and central finite differences of every gradient.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import cosmology as C
from oracle import mesh as M
from oracle import mlp
from oracle import pm
from synthetic import Cosmology, Workload, mlp_init, normal, uniform, white_noise

CO = Cosmology()


def tiny(n_steps=3, np_=8, mesh=16, box=32.0):
    return pm.Setup(np_, mesh, box, n_steps, CO)


# ------------------------------------------------------------ ICs

def test_ic_mode_amplitudes():
    np_, box = 16, 64.0
    noise = white_noise(np_, 1)
    radial = pm.ic_radial(np_, box, CO)
    s = pm.zeldovich_displacement(noise, box, radial)
    # divergence of s equals minus the coloured noise (off the Nyquist planes)
    wk = M.rfftn(noise)
    n0, n1, n2 = M.wave_integers(np_)
    kf = 2 * np.pi / box
    div = sum(1j * kf * nj * M.rfftn(s[:, j].reshape(np_, np_, np_))
              for j, nj in enumerate((n0, n1, n2)))
    nsq = n0 ** 2 + n1 ** 2 + n2 ** 2
    k = kf * np.sqrt(nsq)
    pk = C.linear_pk(k, CO)
    delta_lin = wk * np.sqrt(pk / (box / np_) ** 3)
    inner = ((np.abs(n0) < np_ // 2) & (np.abs(n1) < np_ // 2) & (n2 < np_ // 2) & (nsq > 0))
    inner = np.broadcast_to(inner, wk.shape)
    np.testing.assert_allclose(div[inner], -delta_lin[inner], rtol=1e-10,
                               atol=1e-12 * np.abs(delta_lin).max())


def test_ic_nyquist_reading():
    """Each displacement component loses the Nyquist plane of its own axis and
    the k = 0 mode; the other components keep that plane (delta_lin keeps its
    Nyquist modes)."""
    np_, box = 8, 32.0
    s = pm.zeldovich_displacement(white_noise(np_, 2), box, pm.ic_radial(np_, box, CO))
    n0, n1, n2 = M.wave_integers(np_)
    nyq = [np.broadcast_to(n0 == -np_ // 2, (np_, np_, np_ // 2 + 1)),
           np.broadcast_to(n1 == -np_ // 2, (np_, np_, np_ // 2 + 1)),
           np.broadcast_to(n2 == np_ // 2, (np_, np_, np_ // 2 + 1))]
    for j in range(3):
        sk = M.rfftn(s[:, j].reshape(np_, np_, np_))
        scale = np.abs(sk).max()
        assert abs(sk[0, 0, 0]) < 1e-13 * scale
        for a in range(3):
            on = np.abs(sk[nyq[a]]).max()
            if a == j:
                assert on < 1e-13 * scale, (j, a)
            else:
                assert on > 1e-3 * scale, (j, a)


def test_ic_ensemble_power_matches_linear():
    # mean P(k) of the linear density over seeds ~ P_lin within cosmic variance
    np_, box = 16, 64.0
    radial = pm.ic_radial(np_, box, CO)
    vc = (box / np_) ** 3
    acc = 0
    nseed = 16
    for seed in range(nseed):
        wk = M.rfftn(white_noise(np_, seed))
        n0, n1, n2 = M.wave_integers(np_)
        nsq = n0 ** 2 + n1 ** 2 + n2 ** 2
        k = 2 * np.pi / box * np.sqrt(nsq)
        dl = wk * np.sqrt(C.linear_pk(k, CO) / vc)
        acc = acc + M.power_spectrum(M.irfftn(dl, np_), box, n_bins=6)[1]
    k, _, N = M.power_spectrum(white_noise(np_, 0), box, n_bins=6)
    P = acc / nseed
    # compare with the shell average of P_lin over the same modes
    n = np.fft.fftfreq(np_, 1 / np_)
    nn = np.sqrt(n[:, None, None] ** 2 + n[None, :, None] ** 2 + n[None, None, :] ** 2)
    b = np.floor(nn + 0.5)
    plin = C.linear_pk(2 * np.pi / box * nn, CO)
    for i in range(6):
        ref = plin[b == i + 1].mean()
        sig = np.sqrt(2.0 / (N[i] * nseed))
        assert abs(P[i] / ref - 1) < 5 * sig, (i, P[i] / ref, sig)


# ------------------------------------------------------------ forward

def test_plane_wave_tracks_linear_growth():
    """A small plane wave on a 64^3 lattice and 64^3 mesh grows like D(a)."""
    np_, mesh, box = 64, 64, 64.0
    st = pm.Setup(np_, mesh, box, 10, CO)
    q = pm.lattice(np_, box)
    kx = 2 * np.pi / box
    A = 0.01 / kx                      # A k D(1) = 0.01: far from shell crossing
    s = np.zeros_like(q)
    s[:, 0] = A * np.sin(kx * q[:, 0])
    run = pm.forward_from_displacement(s, st)
    co = C.kdk_coefficients(0.3, st.a_start, st.a_stop, st.n_steps)
    D = C.growth_D(co.a, 0.3)
    basis = np.sin(kx * q[:, 0])
    amp = [np.dot(d[:, 0], basis) / np.dot(basis, basis) for d in run.disp]
    ratio = np.array(amp) / amp[0]
    err = np.abs(ratio / (D / D[0]) - 1)
    assert err.max() < 5e-3, err


def test_uniform_lattice_stays_put():
    st = pm.Setup(8, 16, 16.0, 4, CO)
    run = pm.forward_from_displacement(np.zeros((512, 3)), st)
    assert np.max(np.abs(run.disp[-1])) < 1e-12
    assert np.max(np.abs(run.dens)) < 1e-12


def test_total_momentum_conserved():
    st = tiny(5)
    run = pm.forward(white_noise(8, 2), st)
    p0 = run.mom0.sum(axis=0)
    pN = run.mom.sum(axis=0)
    assert np.max(np.abs(pN - p0)) < 1e-9 * np.abs(run.mom).sum()


def test_fp64_reversibility():
    st = tiny(6)
    run = pm.forward(white_noise(8, 3), st)
    rec, mom0 = pm.reverse_reconstruct(run.disp[-1], run.mom, st)
    cell = st.box / st.mesh
    for n in range(st.n_steps + 1):
        assert np.max(np.abs(rec[n] - run.disp[n])) / cell < 1e-9
    assert np.max(np.abs(mom0 - run.mom0)) < 1e-9 * np.abs(run.mom0).max()


# ------------------------------------------------------------ adjoint

def _loss(noise, st, target, theta=None, wd=None, wp=None):
    r = pm.forward(noise, st, theta)
    L = pm.mse_loss(r.dens, target)[0]
    if wd is not None:
        L += np.sum(wd * r.disp[-1]) + np.sum(wp * r.mom)
    return L


@pytest.fixture(scope="module")
def grad_case():
    st = tiny(4)
    noise = white_noise(8, 3)
    target = pm.forward(white_noise(8, 4), st).dens
    theta = 0.5 * mlp_init(0, zero_last=False)
    wd, wp = normal((512, 3), 9), normal((512, 3), 10)
    run = pm.forward(noise, st, theta)
    _, gd = pm.mse_loss(run.dens, target)
    g = pm.adjoint(run, noise, g_dens=gd, g_disp=wd, g_mom=wp)
    return st, noise, target, theta, wd, wp, g


def test_gradient_noise_fd(grad_case):
    st, noise, target, theta, wd, wp, g = grad_case
    d = normal(noise.shape, 7)
    h = 1e-6
    fd = (_loss(noise + h * d, st, target, theta, wd, wp)
          - _loss(noise - h * d, st, target, theta, wd, wp)) / (2 * h)
    assert abs(fd / np.sum(g.noise * d) - 1) < 1e-6


@pytest.mark.parametrize("name", ["omega_m", "sigma8"])
def test_gradient_cosmology_fd(grad_case, name):
    st, noise, target, theta, wd, wp, g = grad_case
    h = 1e-6
    c = st.cosmo
    up = replace(st, cosmo=replace(c, **{name: getattr(c, name) + h}))
    dn = replace(st, cosmo=replace(c, **{name: getattr(c, name) - h}))
    fd = (_loss(noise, up, target, theta, wd, wp) - _loss(noise, dn, target, theta, wd, wp)) / (2 * h)
    assert abs(fd / getattr(g, name) - 1) < 1e-6


def test_gradient_filter_weights_fd(grad_case):
    st, noise, target, theta, wd, wp, g = grad_case
    d = normal(theta.shape, 5)
    h = 1e-6
    fd = (_loss(noise, st, target, theta + h * d, wd, wp)
          - _loss(noise, st, target, theta - h * d, wd, wp)) / (2 * h)
    assert abs(fd / np.dot(g.theta, d) - 1) < 1e-6


def test_zero_last_layer_is_plain_pm():
    st = tiny(3)
    noise = white_noise(8, 6)
    a = pm.forward(noise, st, None)
    b = pm.forward(noise, st, mlp_init(0))           # last layer zero: f == 1
    assert np.array_equal(a.disp[-1], b.disp[-1])
    assert np.array_equal(a.mom, b.mom)


def test_ic_transpose_dot_product():
    np_, box = 8, 16.0
    radial = pm.ic_radial(np_, box, CO)
    w = normal((np_,) * 3, 40)
    sb = normal((np_ ** 3, 3), 41)
    lhs = np.sum(pm.zeldovich_displacement(w, box, radial) * sb)
    rhs = np.sum(w * pm.zeldovich_transpose(sb, box, radial))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ------------------------------------------------------- filter-training losses

def test_pk_loss_gradient_matches_finite_difference():
    mesh, box, nbins = 8, 16.0, 4
    d = normal((mesh,) * 3, 51)
    target = M.power_spectrum(normal((mesh,) * 3, 52), box, nbins)[1]
    u = normal((mesh,) * 3, 53)
    L0, g = pm.pk_loss(d, target, box, nbins, weight=0.7)
    h = 1e-5
    fd = (pm.pk_loss(d + h * u, target, box, nbins, 0.7)[0]
          - pm.pk_loss(d - h * u, target, box, nbins, 0.7)[0]) / (2 * h)
    assert abs(fd - np.sum(g * u)) < 1e-7 * abs(fd)
    # zero at the target itself
    assert pm.pk_loss(d, M.power_spectrum(d, box, nbins)[1], box, nbins)[0] < 1e-28


def test_pk_loss_value_by_hand():
    """Doubling the field quadruples every P_b: loss = mean (4 - 1)^2 = 9."""
    mesh, box, nbins = 8, 16.0, 4
    d = normal((mesh,) * 3, 54)
    target = M.power_spectrum(d, box, nbins)[1]
    assert abs(pm.pk_loss(2 * d, target, box, nbins)[0] - 9.0) < 1e-12


def test_disp_loss_periodic_minimum_image():
    box, mesh, n = 32.0, 16, 50
    s = uniform((n, 3), 55, -3.0, 3.0)
    eps = normal((n, 3), 56) * 0.2
    shifts = np.round(uniform((n, 3), 57, -2.0, 2.0)) * box   # whole box periods
    L, g = pm.disp_loss(s, s + eps + shifts, box, mesh, weight=0.5)
    cell = box / mesh
    assert abs(L - 0.5 * np.sum(eps * eps) / (n * cell * cell)) < 1e-12 * L
    assert np.max(np.abs(g + 0.5 * 2 * eps / (n * cell * cell))) < 1e-12 * np.max(np.abs(g))
    # separations near half a box pick the nearer image
    a = np.array([[0.0, 0.0, 0.0]])
    b = np.array([[0.6 * box, 0.0, 0.0]])
    assert abs(pm.disp_loss(a, b, box, mesh)[0] - (0.4 * box / cell) ** 2) < 1e-9


# ------------------------------------------------- per-step coefficient scales

@pytest.fixture(scope="module")
def scale_case():
    st = tiny(4)
    scales = 1.0 + 0.1 * normal((3, 4), 60)
    st = replace(st, step_scales=scales)
    noise = white_noise(8, 3)
    target = pm.forward(white_noise(8, 4), st).dens
    theta = 0.5 * mlp_init(0, zero_last=False)
    wd, wp = normal((512, 3), 9), normal((512, 3), 10)
    run = pm.forward(noise, st, theta)
    _, gd = pm.mse_loss(run.dens, target)
    g = pm.adjoint(run, noise, g_dens=gd, g_disp=wd, g_mom=wp)
    return st, noise, target, theta, wd, wp, g


def test_step_scale_gradient_fd(scale_case):
    st, noise, target, theta, wd, wp, g = scale_case
    d = normal((3, 4), 61)
    h = 1e-6
    up = replace(st, step_scales=st.step_scales + h * d)
    dn = replace(st, step_scales=st.step_scales - h * d)
    fd = (_loss(noise, up, target, theta, wd, wp) - _loss(noise, dn, target, theta, wd, wp)) / (2 * h)
    assert abs(fd / np.sum(g.step_scales * d) - 1) < 1e-6


@pytest.mark.parametrize("row", [0, 1, 2])
def test_single_step_scale_gradient_fd(scale_case, row):
    """One coefficient at a time (kick_a, drift, kick_b of step 2)."""
    st, noise, target, theta, wd, wp, g = scale_case
    h = 1e-6
    e = np.zeros((3, 4))
    e[row, 2] = 1.0
    up = replace(st, step_scales=st.step_scales + h * e)
    dn = replace(st, step_scales=st.step_scales - h * e)
    fd = (_loss(noise, up, target, theta, wd, wp) - _loss(noise, dn, target, theta, wd, wp)) / (2 * h)
    assert abs(fd / g.step_scales[row, 2] - 1) < 1e-5


def test_omega_m_gradient_with_step_scales_fd(scale_case):
    st, noise, target, theta, wd, wp, g = scale_case
    h = 1e-6
    c = st.cosmo
    up = replace(st, cosmo=replace(c, omega_m=c.omega_m + h))
    dn = replace(st, cosmo=replace(c, omega_m=c.omega_m - h))
    fd = (_loss(noise, up, target, theta, wd, wp) - _loss(noise, dn, target, theta, wd, wp)) / (2 * h)
    assert abs(fd / g.omega_m - 1) < 1e-6


def test_unit_step_scales_are_plain_pm():
    st = tiny(3)
    noise = white_noise(8, 6)
    a = pm.forward(noise, st)
    b = pm.forward(noise, replace(st, step_scales=np.ones((3, 3))))
    assert np.array_equal(a.disp[-1], b.disp[-1]) and np.array_equal(a.mom, b.mom)


def test_scaled_drift_breaks_linear_growth_exactness():
    """The unscaled factors make one KDK step exact for linear growth (a plane
    wave grows like D); scaling the drift of that step by 1 + e moves the
    linear amplitude by about e times the step's growth increment."""
    np_, box = 16, 64.0
    q = pm.lattice(np_, box)
    kx = 2 * np.pi / box
    amp = 0.05
    s = np.zeros_like(q)
    s[:, 0] = amp * np.sin(kx * q[:, 0])
    st = pm.Setup(np_, np_, box, 1, CO, 0.02, 0.03)
    eps = 0.1
    out = []
    for sc in (None, np.array([[1.0], [1.0 + eps], [1.0]])):
        r = pm.forward_from_displacement(s, replace(st, step_scales=sc))
        out.append(np.sum(r.disp[-1][:, 0] * np.sin(kx * q[:, 0])) / np.sum(np.sin(kx * q[:, 0]) ** 2))
    D = C.growth_D(np.array([0.02, 0.03]), CO.omega_m)
    # the plain step tracks D to the force-window accuracy; the scaled one is off
    # by ~eps (D(a1) - D(a0)) amp
    assert abs(out[0] / (D[1] * amp) - 1) < 5e-3
    shift = (out[1] - out[0]) / (eps * (D[1] - D[0]) * amp)
    assert abs(shift - 1) < 0.05
