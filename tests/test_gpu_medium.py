"""GPU checks at the 256^3-particle / 512^3-mesh / 256 Mpc/h geometry.

  * The whole 63-step run with the MSE loss against a second seed: reverse-time
    reconstruction of the initial state bit for bit, finite gradients.
  * Gradients against finite differences of the GPU's own loss (central
    differences along a noise direction, along Omega_m and along sigma_8) on the
    first two steps of the same geometry.
  * The first two steps against the FP64 oracle's stored results
    (tests/golden/medium_truncated_2steps.json, written by
    tests/golden/make_oracle_fixtures.py): loss, Omega_m and sigma_8 gradients,
    the noise gradient at sampled lattice sites and by shells, final
    displacements at sampled particles and the final P(k).
"""
import json
import os
from dataclasses import replace

import numpy as np
import pytest

from gpu_util import CO, dev, host, periodic_cells, rel_l2
from paper_2211_09958_amd import api
from synthetic import MEDIUM, normal, white_noise

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "medium_truncated_2steps.json")


def _truncated(n_steps):
    return api.make_config(MEDIUM.ptcl_grid, MEDIUM.mesh, MEDIUM.box, n_steps,
                           a_start=MEDIUM.a_start, a_stop=MEDIUM.a_start + n_steps / 64.0)


def test_medium_reconstruction_is_exact():
    pm = api.PMContext(api.config_from_workload(MEDIUM), CO)
    target = pm.forward(dev(white_noise(MEDIUM.ptcl_grid, 1)))[2].clone()
    disp, mom, dens = pm.forward(dev(white_noise(MEDIUM.ptcl_grid, 0)))
    L, g = pm.loss_mse(dens, target)
    g_noise, (g_om, g_s8), _ = pm.adjoint(g)
    st = pm.stats()
    print(f"loss {L:.4e}; dL/dOmega_m {g_om:.4e}, dL/dsigma8 {g_s8:.4e}; reconstruction "
          f"{st['ic_rms_cells']} / {st['ic_max_cells']} cells")
    assert st["ic_max_cells"] == 0.0 and st["ic_mom_rel_rms"] == 0.0
    assert np.isfinite(host(g_noise)).all() and np.isfinite([g_om, g_s8]).all()


def test_medium_gradients_match_finite_differences():
    """Central differences of the GPU loss L(omega, Omega_m, sigma_8) (the first
    two steps of the geometry, loss against seed 1's final density) along each
    of the three inputs against the adjoint's directional derivative.

    Two steps: the loss is piecewise smooth (CIC weights have kinks at node
    planes), and after four steps the derivative already jumps at the 1e-3 level
    between inputs that differ by rounding (the oracle's own gradient moves by
    4e-4 under a 1e-6 relative noise perturbation on a smaller box of the same
    cell size); there the difference quotient settles 1.5e-3 away from the
    adjoint over steps from 1e-4 to 6e-6 |omega|.  After two steps the oracle's
    gradient moves by 7e-6 under the same perturbation.

    The noise direction is v = g/|g| + r/|r| (r seeded Gaussian), normalised,
    so that the derivative along it is of the order of |g| (along a purely
    random direction of 16.8M dimensions it is ~1/4096 of |g|).  The loss is far
    from linear along g over steps of 1e-3 |omega| (a 40 % error there; the
    mesh-scale density is stiff), so the steps are 5e-5 and 2.5e-5 |omega| with
    Richardson extrapolation (4 D(h/2) - D(h)) / 3, which cancels the h^2 term
    of the central difference; likewise 1e-3 and 5e-4 relative for Omega_m and
    sigma_8.  The Omega_m quotient is judged against the sum of the |terms| of
    dL/dOmega_m, which cancel about 11x here.  The loss averages 512^3 cells, so the FP32 rounding of the density
    moves it by ~1e-10, far below these differences."""
    cfg = _truncated(2)
    pm = api.PMContext(cfg, CO)
    npg = MEDIUM.ptcl_grid
    target = pm.forward(dev(white_noise(npg, 1)))[2].clone()
    w = white_noise(npg, 0)

    def loss(noise, cosmo):
        pm.set_cosmology(cosmo)
        return pm.loss_mse(pm.forward(dev(noise))[2], target, want_grad=False)[0]

    pm.set_cosmology(CO)
    dens = pm.forward(dev(w))[2]
    _, g = pm.loss_mse(dens, target)
    g_noise, (g_om, g_s8), _ = pm.adjoint(g)
    sg = pm.step_gradients()
    gn = host(g_noise)
    r = normal((npg,) * 3, 5)
    v = gn / np.linalg.norm(gn) + r / np.linalg.norm(r)
    v /= np.linalg.norm(v)
    gv = float(np.dot(gn.reshape(-1), v.reshape(-1)))
    def richardson(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    fd = richardson(lambda t: loss(w + t * v, CO), 5e-5 * np.linalg.norm(w))
    e_noise = abs(fd / gv - 1)
    fd_om = richardson(lambda t: loss(w, replace(CO, omega_m=CO.omega_m + t)), 1e-3 * CO.omega_m)
    fd_s8 = richardson(lambda t: loss(w, replace(CO, sigma8=CO.sigma8 + t)), 1e-3 * CO.sigma8)
    pm.set_cosmology(CO)
    # dL/dOmega_m sums terms that cancel (about 11x here): the difference quotient
    # inherits the FP32 rounding of every Omega_m-dependent coefficient and table
    # relative to each term, so it is judged against the sum of the |terms|
    # (as against the oracle): per-step terms from the step-scale gradients and
    # the host tables' Omega_m derivatives, plus the initial-condition rest
    t = api.host_tables(cfg, CO)
    steps = [sg[0] / t["kick_a"] * t["d_kick_a"], sg[1] / t["drift"] * t["d_drift"],
             sg[2] / t["kick_b"] * t["d_kick_b"]]
    rest = g_om - sum(float(np.sum(x)) for x in steps)
    om_scale = sum(float(np.sum(np.abs(x))) for x in steps) + abs(rest)
    e_om_scaled = abs(fd_om - g_om) / om_scale
    e_om, e_s8 = abs(fd_om / g_om - 1), abs(fd_s8 / g_s8 - 1)
    print(f"noise direction: adjoint {gv:.6e} fd {fd:.6e} ({e_noise:.1e}); Omega_m: "
          f"{g_om:.6e} vs {fd_om:.6e} ({e_om:.1e} plain, {e_om_scaled:.1e} of the term scale "
          f"{om_scale:.3e}); sigma8: {g_s8:.6e} vs {fd_s8:.6e} ({e_s8:.1e})")
    assert e_noise < 1e-3 and e_om_scaled < 1e-3 and e_s8 < 1e-3


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("run tests/golden/make_oracle_fixtures.py medium first")
    with open(GOLDEN) as f:
        return json.load(f)


def _shell_power(field, n_shells):
    """Same shell sums as the fixture script: Sum |DFT|^2 / N^3 over round(|n|)."""
    import torch
    n = field.shape[0]
    fk = torch.fft.rfftn(torch.as_tensor(field, dtype=torch.float64))
    f = torch.fft.fftfreq(n, 1.0 / n, dtype=torch.float64)
    fz = torch.arange(n // 2 + 1, dtype=torch.float64)
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
    b = torch.floor(torch.sqrt(n2) + 0.5).long()
    w = torch.where((fz == 0) | (fz == n // 2), 1.0, 2.0).expand_as(n2)
    p = fk.abs() ** 2 * w / n ** 3
    out = torch.bincount(b.reshape(-1), weights=p.reshape(-1), minlength=n_shells + 1)
    return out[1:n_shells + 1].numpy()


def test_medium_first_steps_match_oracle(golden):
    c = golden["config"]
    pm = api.PMContext(_truncated(c["n_steps"]), CO)
    npg = c["ptcl_grid"]
    target = pm.forward(dev(white_noise(npg, c["target_seed"])))[2].clone()
    disp, mom, dens = pm.forward(dev(white_noise(npg, c["seed"])))
    L, g = pm.loss_mse(dens, target)
    k, pk, nm = pm.power_spectrum(dens, c["mesh"] // 4)
    g_noise, (g_om, g_s8), _ = pm.adjoint(g)
    sg = pm.step_gradients()
    gn = host(g_noise)
    gi = np.array(golden["g_noise_index"])
    e_sample = rel_l2(gn.reshape(-1)[gi], golden["g_noise_sample"])
    e_norm = abs(np.linalg.norm(gn) / golden["g_noise_norm"] - 1)
    shells = _shell_power(gn, npg // 2)
    e_shell = np.max(np.abs(shells / np.array(golden["g_noise_shell_power"]) - 1))
    e_om = abs(g_om / golden["g_omega_m"] - 1)
    e_s8 = abs(g_s8 / golden["g_sigma8"] - 1)
    pi = np.array(golden["disp_index"])
    d = periodic_cells(host(disp)[pi], golden["disp_sample"], c["box"], c["mesh"])
    e_pk = np.max(np.abs(pk / np.array(golden["pk"]) - 1))
    print(f"loss {L:.6e}/{golden['loss']:.6e}; noise grad samples {e_sample:.1e}, norm "
          f"{e_norm:.1e}, shells {e_shell:.1e}; Omega_m {e_om:.1e}; sigma8 {e_s8:.1e}; "
          f"positions rms {np.sqrt(np.mean(d * d)):.1e} cells; P(k) {e_pk:.1e}")
    np.testing.assert_array_equal(nm, golden["pk_modes"])
    assert abs(L / golden["loss"] - 1) < 1e-4
    assert e_sample < 1e-3 and e_norm < 1e-4 and e_shell < 1e-3
    assert e_om < 1e-3 and e_s8 < 1e-3
    assert np.sqrt(np.mean(d * d)) < 1e-4
    assert e_pk < 1e-4
