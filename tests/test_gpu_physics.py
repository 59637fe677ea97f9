"""Physics pins run on the GPU path itself (the oracle has the same pins).

  * Plane-wave growth: white noise made of one Fourier mode gives one plane
    wave of displacement; in the linear regime (A k D(1) = 0.01, no shell
    crossing) its amplitude must grow like the linear growth factor D(a), to
    0.5 % on a 64^3 lattice and 64^3 mesh (the residual is the force deficit of
    the two CIC windows at the fundamental mode plus the KDK time step).
  * Two-body force: the PM force of a point mass on a probe against the
    Ewald-summed periodic force, for separations from 4 cells to a quarter box,
    directions more than 15 degrees from a mesh axis (along the axis lines the
    truncated spectral kernel rings; see the oracle test).
  * Overflow of the fixed-point momenta is detected (forced from the host with
    a huge step scale) and the context recovers.
"""
import numpy as np
import pytest
import torch

from ewald import ewald_force
from gpu_util import CO, context, dev, host
from oracle import cosmology as C
from oracle import pm as opm
from paper_2211_09958_amd import _lib, api
from synthetic import normal, white_noise

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("a_stop,n_steps", [(1.0, 10), (0.5, 5)])
def test_plane_wave_grows_like_linear_theory(a_stop, n_steps):
    np_ = ng = 64
    box = 64.0
    j0 = np.arange(np_)
    mode = np.cos(2 * np.pi * j0 / np_)[:, None, None] * np.ones((1, np_, np_))
    # measure the amplitude per unit noise at a_0, then size the wave so that
    # A k D(1) = 0.01 (D(1) = 1)
    q = opm.lattice(np_, box)
    k = 2 * np.pi / box
    basis = np.sin(k * q[:, 0])
    proj = lambda d: float(np.dot(d[:, 0], basis) / np.dot(basis, basis))
    a_grid = np.array([1.0 / 64, a_stop])
    D = C.growth_D(a_grid, CO.omega_m)
    cfg = api.make_config(np_, ng, box, n_steps, a_stop=a_stop)
    pm = api.PMContext(cfg, CO)
    d0, _ = pm.initial_conditions(dev(mode))
    per_unit = abs(proj(host(d0))) / D[0]
    c = 0.01 / (k * per_unit)
    noise = dev(c * mode)
    d0, _ = pm.initial_conditions(noise)
    disp, mom, dens = pm.forward(noise)
    d0, dN = host(d0), host(disp)
    ratio = proj(dN) / proj(d0)
    err = ratio / (D[1] / D[0]) - 1
    transverse = np.abs(dN[:, 1:]).max() / abs(proj(dN))
    print(f"a = {a_stop}: growth ratio {ratio:.5f}, linear {D[1] / D[0]:.5f}, error {err:.2e}, "
          f"transverse {transverse:.1e}")
    assert abs(err) < 5e-3
    assert transverse < 1e-4


def test_two_body_force_against_ewald():
    """511 particles stacked at one point form the mass; particle 0 is the
    probe (zero self-force).  Mass per particle box^3 / Np^3 on a cell-1 mesh."""
    np_, ng, box = 8, 128, 128.0
    P = np_ ** 3
    pm = context(np_, ng, box, 1)
    q = opm.lattice(np_, box)
    src = np.array([40.3, 61.7, 50.2])
    mass = (P - 1) * box ** 3 / P
    dirs = normal((200, 3), 15)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dirs = dirs[np.max(np.abs(dirs), axis=1) < np.cos(np.radians(15.0))][:64]
    base = src[None, :] - q
    base -= box * np.round(base / box)
    for r, tol_vec in ((4.0, 0.03), (8.0, 0.005), (16.0, 0.005), (32.0, 0.005)):
        f = np.zeros((len(dirs), 3))
        for i, u in enumerate(dirs):
            s = base.copy()
            s[0] = src + r * u - q[0]
            f[i] = host(pm.force(dev(s), 1.0))[0]
        ref = ewald_force(r * dirs, mass, box)
        rr = np.sum(f * dirs, axis=1) / np.sum(ref * dirs, axis=1)
        vec = np.linalg.norm(f - ref, axis=1).mean() / np.linalg.norm(ref, axis=1).mean()
        print(f"r = {r}: radial ratio {rr.mean():.4f} (anisotropy {rr.std():.4f}), vector {vec:.4f}")
        assert abs(rr.mean() - 1) < 0.01, (r, rr.mean())
        assert vec < tol_vec, (r, vec)


def test_momentum_overflow_is_reported_and_context_recovers():
    np_, ng, box, n = 8, 16, 32.0, 4
    pm = api.PMContext(api.make_config(np_, ng, box, n), CO)
    noise = dev(white_noise(np_, 2))
    g = dev(normal((np_ ** 3, 3), 3))
    pm.forward(noise)
    ref = pm.adjoint(g_disp=g)[0].clone()
    assert not pm.stats()["momentum_overflow"]
    scales = np.ones((3, n))
    scales[0, 0] = 1e12          # first kick far outside the int32 momentum range
    pm.set_step_scales(scales)
    pm.forward(noise)
    assert pm.stats()["momentum_overflow"]
    with pytest.raises(api.PMError) as e:
        pm.adjoint(g_disp=g)
    assert e.value.code == _lib.PM_ENUMERIC
    pm.set_step_scales(np.ones((3, n)))
    pm.forward(noise)
    assert not pm.stats()["momentum_overflow"]
    assert torch.equal(pm.adjoint(g_disp=g)[0], ref)
