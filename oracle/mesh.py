"""Particle-mesh operators in FP64: CIC assignment, spectral force, P(k).

Test infrastructure (see ``oracle/__init__.py``).

Passages followed
  * pmwd paper, Summary: a particle-mesh (PM) simulation, i.e. particles are
    assigned to a mesh, gravity is solved with FFTs on the mesh, and forces are
    interpolated back.  Cloud-in-cell (CIC) assignment, the exact spectral
    Green's function -1/k^2 and the spectral gradient i k are the standard PM
    choices (Hockney & Eastwood); the same CIC kernel is used to assign and to
    interpolate so that the interpolation is the transpose of the assignment.
  * Conventions (readings where the paper is silent): mesh values live at cell
    centres (i + 1/2) * cell; the forward DFT is exp(-i k.x) unnormalised and
    the inverse carries 1/N; the k = 0 mode and, for each gradient component,
    the Nyquist plane of the differentiated axis are zeroed.

FFTs are library primitives (scipy.fft), pinned against brute-force DFTs.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

# Thread count handed to scipy.fft; the CPU baseline sets it to the host cores.
WORKERS = 1


def rfftn(x):
    return sfft.rfftn(x, workers=WORKERS)


def irfftn(x, n):
    return sfft.irfftn(x, s=(n, n, n), workers=WORKERS)


# ------------------------------------------------------------------ CIC

def cic_base(x, mesh, box):
    """Base node index and fractional offset of each particle, per axis.

    u = x / cell - 1/2, i = floor(u) (wrapped to [0, mesh)), t = u - floor(u).
    Node i receives weight (1 - t), node i + 1 weight t.
    """
    u = np.asarray(x, dtype=np.float64) * (mesh / box) - 0.5
    fl = np.floor(u)
    t = u - fl
    i = np.mod(fl.astype(np.int64), mesh)
    return i, t


def _corners():
    for c0 in (0, 1):
        for c1 in (0, 1):
            for c2 in (0, 1):
                yield (c0, c1, c2)


def _flat(i, c, mesh):
    j = np.mod(i + np.asarray(c), mesh)
    return (j[:, 0] * mesh + j[:, 1]) * mesh + j[:, 2]


def _weight(t, c):
    w = np.ones(t.shape[0])
    for ax in range(3):
        w = w * (t[:, ax] if c[ax] else 1.0 - t[:, ax])
    return w


def _weight_grad(t, c, axis, inv_cell):
    g = np.full(t.shape[0], inv_cell if c[axis] else -inv_cell)
    for ax in range(3):
        if ax != axis:
            g = g * (t[:, ax] if c[ax] else 1.0 - t[:, ax])
    return g


def scatter(x, mesh, box, values):
    """Sum_p values_p * w(x_p, node) onto a mesh**3 FP64 array (CIC assignment)."""
    i, t = cic_base(x, mesh, box)
    out = np.zeros(mesh ** 3)
    for c in _corners():
        out += np.bincount(_flat(i, c, mesh), weights=values * _weight(t, c),
                           minlength=mesh ** 3)
    return out.reshape(mesh, mesh, mesh)


def density(x, mesh, box, n_particles):
    """Overdensity delta = rho - 1 with particle mass (mesh^3 / n_particles)."""
    m = mesh ** 3 / n_particles
    return scatter(x, mesh, box, np.full(x.shape[0], m)) - 1.0


def gather(field, x, box):
    """Sum_nodes w(x_p, node) field(node) (CIC interpolation)."""
    mesh = field.shape[0]
    i, t = cic_base(x, mesh, box)
    flat = field.reshape(-1)
    out = np.zeros(x.shape[0])
    for c in _corners():
        out += _weight(t, c) * flat[_flat(i, c, mesh)]
    return out


def gather_grad(field, x, box):
    """d/dx_p of gather(field, x): Sum_nodes grad_x w(x_p, node) field(node).

    The CIC weight is piecewise linear; its derivative is +-1/cell along the
    axis times the other two linear factors (the right derivative where a
    particle sits exactly on a node plane).
    """
    mesh = field.shape[0]
    i, t = cic_base(x, mesh, box)
    flat = field.reshape(-1)
    inv_cell = mesh / box
    out = np.zeros(x.shape)
    for c in _corners():
        vals = flat[_flat(i, c, mesh)]
        for ax in range(3):
            out[:, ax] += _weight_grad(t, c, ax, inv_cell) * vals
    return out


# ---------------------------------------------------------------- Fourier

def wave_integers(mesh):
    """Integer wave numbers n per axis of an rfftn half spectrum.

    Returns n0, n1 in [-mesh/2, mesh/2) (broadcast shapes) and n2 in [0, mesh/2].
    """
    n = np.fft.fftfreq(mesh, d=1.0 / mesh).round().astype(np.int64)
    n_half = np.arange(mesh // 2 + 1, dtype=np.int64)
    return n[:, None, None], n[None, :, None], n_half[None, None, :]


def half_spectrum_weights(mesh):
    """Multiplicity of each rfftn mode in the full spectrum (1 on the n2 = 0
    and n2 = mesh/2 planes, 2 elsewhere)."""
    w = np.full(mesh // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return w[None, None, :]


def gradient_multipliers(mesh, box, radial):
    """M_j(k) = i k_j * radial(|n|^2) for j = 0, 1, 2 on the half spectrum.

    ``radial`` is a callable on integer |n|^2 (an array).  The k = 0 mode is
    zeroed, as is each M_j on the Nyquist plane n_j = -mesh/2 of its own axis.
    """
    n0, n1, n2 = wave_integers(mesh)
    nsq = n0 * n0 + n1 * n1 + n2 * n2
    r = radial(nsq)
    r = np.where(nsq == 0, 0.0, r)
    kf = 2.0 * np.pi / box
    out = []
    for j, nj in enumerate((n0, n1, n2)):
        # the n2 = mesh/2 column holds the Nyquist of axis 2 (n = -mesh/2)
        nyq = (nj == -mesh // 2) if j < 2 else (nj == mesh // 2)
        out.append(np.where(nyq, 0.0, 1j * kf * nj * r))
    return out


def poisson_radial(mesh, box, filt=None):
    """Radial factor of the force: f(|n|^2) / |k|^2 with k = 2 pi n / box.

    F~_k = i k f delta_k / k^2, i.e. F~ = -grad(phi) with lap(phi) = delta,
    scaled by the (optional) radial filter table ``filt`` indexed by |n|^2.
    """
    kf = 2.0 * np.pi / box

    def radial(nsq):
        nsq_safe = np.where(nsq == 0, 1, nsq)
        base = 1.0 / (kf * kf * nsq_safe)
        if filt is not None:
            base = base * filt[nsq]
        return base
    return radial


def force_meshes(delta, box, filt=None):
    """Spectral PM force F~_j = IDFT(i k_j f / k^2 DFT(delta)), j = 0, 1, 2."""
    mesh = delta.shape[0]
    dk = rfftn(delta)
    mult = gradient_multipliers(mesh, box, poisson_radial(mesh, box, filt))
    return [irfftn(m * dk, mesh) for m in mult], dk


def force_transpose(grads, box, filt=None):
    """Transpose of delta -> (F~_0, F~_1, F~_2): Sum_j IDFT(conj(M_j) DFT(G_j)).

    Also returns the DFTs of the inputs (needed for the filter gradient).
    """
    mesh = grads[0].shape[0]
    mult = gradient_multipliers(mesh, box, poisson_radial(mesh, box, filt))
    gk = [rfftn(g) for g in grads]
    acc = sum(np.conj(m) * g for m, g in zip(mult, gk))
    return irfftn(acc, mesh), gk


def filter_table_cotangent(delta_k, grads_k, box):
    """dL/df(|n|^2) for F~_j = IDFT(i k_j f(|n|^2) delta_k / k^2).

    With Gbar_j the cotangent mesh of F~_j and G_j = DFT(Gbar_j),
    dL/df(s) = N^-3 Sum_{|n|^2 = s} Sum_j Re[conj(G_j,k) i k_j delta_k / k^2]
    over the full spectrum (half-spectrum modes counted with multiplicity).
    """
    mesh = delta_k.shape[0]
    mult = gradient_multipliers(mesh, box, poisson_radial(mesh, box, None))
    n0, n1, n2 = wave_integers(mesh)
    nsq = np.broadcast_to(n0 * n0 + n1 * n1 + n2 * n2, delta_k.shape)
    wts = np.broadcast_to(half_spectrum_weights(mesh), delta_k.shape)
    contrib = sum(np.real(np.conj(g) * m * delta_k) for m, g in zip(mult, grads_k))
    table = np.bincount(nsq.reshape(-1), weights=(wts * contrib).reshape(-1),
                        minlength=3 * (mesh // 2) ** 2 + 1)
    return table / mesh ** 3


# ------------------------------------------------------------ power spectrum

def power_spectrum(delta, box, n_bins=None):
    """Shell-averaged P(k) of a real overdensity mesh.

    P(k_b) = (box^3 / N^6) <|delta_k|^2> over modes with round(|n|) = b, b >= 1,
    counting each half-spectrum mode with its full-spectrum multiplicity.
    Returns (mean |k| of the shell, P, mode count) for b = 1 .. n_bins.
    """
    mesh = delta.shape[0]
    if n_bins is None:
        n_bins = mesh // 2
    dk = rfftn(delta)
    n0, n1, n2 = wave_integers(mesh)
    nsq = np.broadcast_to(n0 * n0 + n1 * n1 + n2 * n2, dk.shape).reshape(-1)
    nabs = np.sqrt(nsq.astype(np.float64))
    b = np.floor(nabs + 0.5).astype(np.int64)
    w = np.broadcast_to(half_spectrum_weights(mesh), dk.shape).reshape(-1)
    p = (np.abs(dk) ** 2).reshape(-1)
    sel = (b >= 1) & (b <= n_bins)
    cnt = np.bincount(b[sel], weights=w[sel], minlength=n_bins + 1)[1:]
    psum = np.bincount(b[sel], weights=(w * p)[sel], minlength=n_bins + 1)[1:]
    ksum = np.bincount(b[sel], weights=(w * nabs)[sel], minlength=n_bins + 1)[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = psum / cnt * box ** 3 / mesh ** 6
        kmean = ksum / cnt * 2.0 * np.pi / box
    return kmean, pk, cnt


def power_spectrum_vjp(delta, box, n_bins, g_pk):
    """Gradient of Sum_b g_pk[b-1] P(k_b) with respect to the real mesh delta.

    From the definition P_b = (box^3 / N^6) (1/N_b) Sum_{k in shell b} |delta_k|^2
    over the FULL spectrum: d|delta_k|^2 / d delta(x) = 2 Re[conj(delta_k) e^{-ik.x}],
    so the gradient is 2 Re Sum_k t_k conj(delta_k) e^{-ik.x} with
    t_k = g_pk[b(k)-1] box^3 / (N^6 N_b), i.e. 2 N^3 Re IDFT(t delta_k) because t is
    even in k.  Computed with the full complex FFT so that no half-spectrum
    bookkeeping enters.
    """
    delta = np.asarray(delta, dtype=np.float64)
    mesh = delta.shape[0]
    _, _, cnt = power_spectrum(delta, box, n_bins)
    n = np.fft.fftfreq(mesh, d=1.0 / mesh).round()
    nabs = np.sqrt(n[:, None, None] ** 2 + n[None, :, None] ** 2 + n[None, None, :] ** 2)
    b = np.floor(nabs + 0.5).astype(np.int64)
    t = np.zeros(n_bins + 1)
    with np.errstate(invalid="ignore", divide="ignore"):
        t[1:] = np.where(cnt > 0, np.asarray(g_pk, dtype=np.float64) * box ** 3
                         / (mesh ** 6 * cnt), 0.0)
    tk = np.where(b <= n_bins, t[np.minimum(b, n_bins)], 0.0)
    dk = np.fft.fftn(delta)
    return 2.0 * mesh ** 3 * np.real(np.fft.ifftn(tk * dk))
