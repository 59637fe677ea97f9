"""GPU parity of the 2LPT initial conditions and their adjoint (PM_F_2LPT).

Against the FP64 oracle: the initial state itself (Zel'dovich plus second
order) on several particle/mesh geometries, the 10-step forward run, the
gradients w.r.t. noise, Omega_m and sigma_8, and the exact reverse-time
reconstruction.  At the full 512^3-particle / 1024^3-mesh size: crossed plane
waves of noise, whose 2LPT displacement has a closed form at every particle.
"""
import gc
import math

import numpy as np
import pytest
import torch

from gpu_util import CO, context, dev, host, periodic_cells, rel_l2, setup_for
from oracle import cosmology as C
from oracle import lpt as olpt
from oracle import mesh as M
from oracle import pm as opm
from paper_2211_09958_amd import api
from synthetic import LARGE, SMALL, Workload, normal, white_noise

pytestmark = pytest.mark.gpu

TINY = Workload("tiny", ptcl_grid=8, mesh=16, box=32.0, n_steps=4)


def ctx2(w, **kw):
    return context(w.ptcl_grid, w.mesh, w.box, w.n_steps, lpt_order=2, **kw)


def oracle_ics(w, noise):
    st = setup_for(w, 2)
    s1 = opm.zeldovich_displacement(noise, w.box, opm.ic_radial(w.ptcl_grid, w.box, CO))
    s2 = olpt.second_order_displacement(np.asarray(noise, dtype=np.float64), w.box, CO)
    return s1, s2, opm.initial_state(s1, st, s2)


@pytest.mark.parametrize("np_,ng,box", [(8, 8, 16.0), (8, 16, 32.0), (16, 16, 32.0), (32, 64, 64.0),
                                        (64, 128, 128.0)])
def test_lpt2_initial_state_matches_oracle(np_, ng, box):
    """The state is stored in fixed point: positions in units of box / 2^32 and
    momenta in units of (box / Ng) 2^-22, each rounded to nearest, so the bound
    is half a unit (one unit for a difference of two states) plus FP32 rounding."""
    w = Workload("ic", ptcl_grid=np_, mesh=ng, box=box, n_steps=10)
    noise = white_noise(np_, 21)
    s1, s2, (d_ref, p_ref) = oracle_ics(w, noise)
    co = C.kdk_coefficients(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    disp, mom = ctx2(w).initial_conditions(dev(noise))
    disp1, mom1 = context(np_, ng, box, 10).initial_conditions(dev(noise))
    disp, mom, disp1, mom1 = host(disp), host(mom), host(disp1), host(mom1)
    qx, qp = box / 2.0 ** 32, box / ng * 2.0 ** -22
    fx, fp = 2e-6 * np.abs(d_ref).max(), 2e-6 * np.abs(p_ref).max()
    e_d, e_p = np.abs(disp - d_ref).max(), np.abs(mom - p_ref).max()
    # the second-order part alone: 2LPT minus Zel'dovich state of the same noise
    e_2d = np.abs(disp - disp1 - co.D20 * s2).max()
    e_2p = np.abs(mom - mom1 - co.G20 * s2).max()
    print(f"{np_}/{ng}: state {e_d:.2e} ({0.5 * qx + fx:.2e}) {e_p:.2e} ({0.5 * qp + fp:.2e}); "
          f"second order {e_2d:.2e} {e_2p:.2e} of {np.abs(co.D20 * s2).max():.2e} "
          f"{np.abs(co.G20 * s2).max():.2e}")
    assert e_d <= 0.5 * qx + fx and e_p <= 0.5 * qp + fp
    assert e_2d <= qx + fx and e_2p <= qp + fp
    assert rel_l2(disp - disp1, co.D20 * s2) < 1e-3


@pytest.fixture(scope="module")
def small_lpt2_runs():
    noise = white_noise(SMALL.ptcl_grid, 0)
    run = opm.forward(noise, setup_for(SMALL, 2))
    disp, mom, dens = ctx2(SMALL).forward(dev(noise))
    return run, host(disp), host(mom), host(dens)


def test_lpt2_small_positions_within_1e3_cells(small_lpt2_runs):
    run, disp, mom, dens = small_lpt2_runs
    d = periodic_cells(disp, run.disp[-1], SMALL.box, SMALL.mesh)
    rms = float(np.sqrt(np.mean(d * d)))
    print(f"position RMS {rms:.3e} cells, max {d.max():.3e}")
    assert rms < 1e-3
    assert rel_l2(mom, run.mom) < 1e-3


def test_lpt2_small_power_spectrum_within_1e4(small_lpt2_runs):
    run, disp, mom, dens = small_lpt2_runs
    k, P, _ = ctx2(SMALL).power_spectrum(dev(dens), SMALL.mesh // 2)
    kr, Pr, _ = M.power_spectrum(run.dens, SMALL.box, SMALL.mesh // 2)
    sel = kr < 0.5 * np.pi * SMALL.mesh / SMALL.box
    err = np.abs(P[sel] / Pr[sel] - 1)
    print("P(k) relative errors", err.max())
    assert err.max() < 1e-4


def _omega_m_scale(w, ref):
    """Sum of |terms| of dL/dOmega_m in the oracle's decomposition."""
    d = C.kdk_coefficient_derivatives(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    step = (np.dot(ref.kick_a, d.kick_a) + np.dot(ref.kick_b, d.kick_b)
            + np.dot(ref.drift, d.drift))
    growth = ref.D0 * d.D0 + ref.G0 * d.G0 + ref.D20 * d.D20 + ref.G20 * d.G20
    terms = [np.abs(ref.kick_a * d.kick_a).sum(), np.abs(ref.kick_b * d.kick_b).sum(),
             np.abs(ref.drift * d.drift).sum(), abs(ref.D0 * d.D0), abs(ref.G0 * d.G0),
             abs(ref.D20 * d.D20), abs(ref.G20 * d.G20)]
    return float(sum(terms) + abs(ref.omega_m - step - growth))


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_lpt2_gradients_match_oracle(w):
    st = setup_for(w, 2)
    noise = white_noise(w.ptcl_grid, 3)
    target = opm.forward(white_noise(w.ptcl_grid, 4), st).dens
    run = opm.forward(noise, st)
    _, gd_ref = opm.mse_loss(run.dens, target)
    P = w.ptcl_grid ** 3
    gdisp, gmom = normal((P, 3), 9) * 1e-3, normal((P, 3), 10) * 1e-3
    ref = opm.adjoint(run, noise, g_dens=gd_ref, g_disp=gdisp, g_mom=gmom)
    pm = ctx2(w)
    disp, mom, dens = pm.forward(dev(noise))
    _, gd = pm.loss_mse(dens, dev(target))
    g_noise, (g_om, g_s8), _ = pm.adjoint(gd, dev(gdisp), dev(gmom))
    e_noise = rel_l2(host(g_noise), ref.noise)
    e_om = abs(g_om - ref.omega_m) / _omega_m_scale(w, ref)
    e_s8 = abs(g_s8 / ref.sigma8 - 1)
    print(f"{w.name}: noise {e_noise:.2e} Om {e_om:.2e} (plain rel "
          f"{abs(g_om / ref.omega_m - 1):.2e}) s8 {e_s8:.2e}")
    assert e_noise < 1e-3 and e_om < 1e-3 and e_s8 < 1e-3


def test_lpt2_gradient_differs_from_zeldovich():
    """The second-order terms change the gradient (the pins above would also
    pass if both sides dropped them, so check that they matter here)."""
    w = SMALL
    noise = white_noise(w.ptcl_grid, 3)
    g = []
    for pm in (context(w.ptcl_grid, w.mesh, w.box, w.n_steps), ctx2(w)):
        pm.forward(dev(noise))
        g.append(host(pm.adjoint(g_disp=dev(np.ones((w.ptcl_grid ** 3, 3))))[0]))
    assert rel_l2(g[1], g[0]) > 1e-3


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_lpt2_reverse_time_reconstruction(w):
    pm = ctx2(w)
    pm.forward(dev(white_noise(w.ptcl_grid, 1)))
    pm.adjoint(g_disp=dev(np.zeros((w.ptcl_grid ** 3, 3))))
    st = pm.stats()
    assert st["ic_max_cells"] == 0.0 and st["ic_mom_rel_rms"] == 0.0


def test_initial_conditions_call_keeps_the_stored_run():
    w = TINY
    pm = ctx2(w)
    noise = dev(white_noise(w.ptcl_grid, 2))
    gdisp = dev(normal((w.ptcl_grid ** 3, 3), 3))
    pm.forward(noise)
    a = pm.adjoint(g_disp=gdisp)[0].clone()
    pm.forward(noise)
    d0, _ = pm.initial_conditions(dev(white_noise(w.ptcl_grid, 9)))
    b = pm.adjoint(g_disp=gdisp)[0]
    assert torch.equal(a, b)
    assert pm.stats()["ic_max_cells"] == 0.0


def test_lpt2_full_size_crossed_waves_closed_form():
    """512^3 particles, 1024^3 mesh: noise = eps [cos(al x) + cos(be y)] gives
    delta_lin = A cos(al x) + B cos(be y) with A = eps sqrt(P(k_al)/V_c), and
    s1 = -(A/al sin(al x), B/be sin(be y), 0),
    s2 = A B / (al^2 + be^2) (al sin(al x) cos(be y), be cos(al x) sin(be y), 0)."""
    w = LARGE
    n, L = w.ptcl_grid, w.box
    m_a, m_b, eps = 3, 5, 0.05
    cfg = api.config_from_workload(w)
    cfg.flags |= api._lib.PM_F_2LPT
    pm = api.PMContext(cfg, CO)
    try:
        j = torch.arange(n, device="cuda", dtype=torch.float64)
        ca = torch.cos(2 * math.pi * m_a * j / n)
        cb = torch.cos(2 * math.pi * m_b * j / n)
        noise = (eps * (ca[:, None, None] + cb[None, :, None])).expand(n, n, n)
        disp, mom = pm.initial_conditions(noise.float().contiguous())
        del noise
        t = api.host_tables(cfg, CO)
        g2 = api.lpt2_growth(cfg, CO)
        vc = (L / n) ** 3
        A = eps * math.sqrt(t["pk"][m_a * m_a] / vc)
        B = eps * math.sqrt(t["pk"][m_b * m_b] / vc)
        al, be = 2 * math.pi * m_a / L, 2 * math.pi * m_b / L
        sa, sb = torch.sin(2 * math.pi * m_a * j / n), torch.sin(2 * math.pi * m_b * j / n)
        c = A * B / (al * al + be * be)
        for out, g1, g2c in ((disp, t["D0"], g2["D2"]), (mom, t["G0"], g2["G2"])):
            v = out.view(n, n, n, 3).double()
            # axis 0 depends on j0 only through (sa, ca), on j1 through cb
            want0 = (g1 * (-A / al) * sa[:, None, None]
                     + g2c * c * al * sa[:, None, None] * cb[None, :, None])
            want1 = (g1 * (-B / be) * sb[None, :, None]
                     + g2c * c * be * ca[:, None, None] * sb[None, :, None])
            second = abs(g2c) * c * max(al, be)
            e0 = (v[..., 0] - want0).abs().max().item()
            e1 = (v[..., 1] - want1).abs().max().item()
            e2 = v[..., 2].abs().max().item()
            print(f"max errors {e0:.3e} {e1:.3e} {e2:.3e} vs second-order amplitude {second:.3e}")
            assert max(e0, e1, e2) < 1e-3 * second
            del v, want0, want1
    finally:
        del pm
        gc.collect()
        torch.cuda.empty_cache()
