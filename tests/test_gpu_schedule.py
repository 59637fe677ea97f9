"""GPU parity of the per-step KDK scales (pm_set_step_scales) and their
gradients (pm_step_gradients) against the FP64 oracle, exact reverse-time
reconstruction with scaled steps, and a short schedule training through the
adjoint."""
from dataclasses import replace

import numpy as np
import pytest
import torch

from gpu_util import CO, context, dev, host, periodic_cells, rel_l2, setup_for
from oracle import cosmology as C
from oracle import pm as opm
from paper_2211_09958_amd import _lib, api
from synthetic import SMALL, Workload, normal, white_noise

pytestmark = pytest.mark.gpu

TINY = Workload("tiny", ptcl_grid=8, mesh=16, box=32.0, n_steps=4)


def fresh(w):
    return api.PMContext(api.config_from_workload(w), CO)


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_step_scale_gradients_match_oracle(w):
    scales = 1.0 + 0.05 * normal((3, w.n_steps), 70)
    st = replace(setup_for(w), step_scales=scales)
    noise = white_noise(w.ptcl_grid, 3)
    target = opm.forward(white_noise(w.ptcl_grid, 4), st).dens
    run = opm.forward(noise, st)
    _, gd_ref = opm.mse_loss(run.dens, target)
    P = w.ptcl_grid ** 3
    gdisp = normal((P, 3), 9) * 1e-3
    ref = opm.adjoint(run, noise, g_dens=gd_ref, g_disp=gdisp)
    pm = fresh(w)
    pm.set_step_scales(scales)
    disp, _, dens = pm.forward(dev(noise))
    d = periodic_cells(host(disp), run.disp[-1], w.box, w.mesh)
    _, gd = pm.loss_mse(dens, dev(target))
    g_noise, (g_om, g_s8), _ = pm.adjoint(gd, dev(gdisp))
    g_steps = pm.step_gradients()
    e_steps = rel_l2(g_steps, ref.step_scales)
    e_noise = rel_l2(host(g_noise), ref.noise)
    e_s8 = abs(g_s8 / ref.sigma8 - 1)
    print(f"{w.name}: position rms {np.sqrt(np.mean(d * d)):.2e} cells; step scales {e_steps:.2e} "
          f"noise {e_noise:.2e} s8 {e_s8:.2e} Om {abs(g_om / ref.omega_m - 1):.2e}")
    assert np.sqrt(np.mean(d * d)) < 1e-3
    assert e_steps < 1e-3 and e_noise < 1e-3 and e_s8 < 1e-3
    # each of the three rows separately (kick_a, drift, kick_b)
    for r in range(3):
        assert rel_l2(g_steps[r], ref.step_scales[r]) < 1e-3


def test_unit_step_scales_reproduce_plain_bitwise():
    pm, plain = fresh(TINY), context(TINY.ptcl_grid, TINY.mesh, TINY.box, TINY.n_steps)
    n = dev(white_noise(8, 5))
    pm.set_step_scales(np.ones((3, TINY.n_steps)))
    for x, y in zip(pm.forward(n), plain.forward(n)):
        assert torch.equal(x, y)


def test_scaled_steps_reconstruct_exactly():
    pm = fresh(SMALL)
    pm.set_step_scales(1.0 + 0.2 * normal((3, SMALL.n_steps), 71))
    pm.forward(dev(white_noise(SMALL.ptcl_grid, 1)))
    pm.adjoint(g_disp=dev(np.zeros((SMALL.ptcl_grid ** 3, 3))))
    st = pm.stats()
    assert st["ic_max_cells"] == 0.0 and st["ic_mom_rel_rms"] == 0.0


def test_step_gradients_need_an_adjoint():
    pm = fresh(TINY)
    pm.forward(dev(white_noise(8, 2)))
    with pytest.raises(_lib.PMError):
        pm.step_gradients()
    pm.adjoint(g_disp=dev(np.ones((512, 3))))
    assert pm.step_gradients().shape == (3, TINY.n_steps)
    with pytest.raises(_lib.PMError):
        pm.set_step_scales(np.full((3, TINY.n_steps), np.nan))


def test_schedule_training_reduces_loss():
    """Per-step scales alone, trained through the adjoint against a finer-mesh
    run: the training loss falls."""
    from paper_2211_09958_amd import train_filter as tf
    a = tf.parse(["--ptcl", "32", "--fine-factor", "2", "--box", "64", "--steps", "8",
                  "--train-seeds", "4", "--heldout", "0", "--batch", "4", "--train", "schedule",
                  "--lr-schedule", "0.02"])
    tr = tf.Trainer(a, CO)
    first = sum(tr.step([0, 1, 2, 3]))
    for _ in range(24):
        last = sum(tr.step([0, 1, 2, 3]))
    print(f"schedule training loss {first:.4e} -> {last:.4e}")
    assert last < 0.9 * first
    assert not torch.equal(tr.scales, torch.ones_like(tr.scales))


def test_autograd_function_with_step_scales():
    w = TINY
    pm = fresh(w)
    scales_np = 1.0 + 0.05 * normal((3, w.n_steps), 72)
    noise = dev(white_noise(8, 2)).requires_grad_(True)
    om = torch.tensor(CO.omega_m, dtype=torch.float64, requires_grad=True)
    s8 = torch.tensor(CO.sigma8, dtype=torch.float64, requires_grad=True)
    scales = torch.tensor(scales_np, dtype=torch.float64, requires_grad=True)
    disp, mom, dens = api.simulate(pm, noise, om, s8, None, scales)
    (dens.double() ** 2).mean().backward()
    st = replace(setup_for(w), step_scales=scales_np)
    run = opm.forward(white_noise(8, 2), st)
    ref = opm.adjoint(run, white_noise(8, 2), g_dens=2 * run.dens / run.dens.size)
    assert scales.grad.shape == (3, w.n_steps)
    assert rel_l2(scales.grad.numpy(), ref.step_scales) < 1e-3
    assert rel_l2(host(noise.grad), ref.noise) < 1e-3


def test_all_options_together_match_oracle():
    """2LPT ICs, learned filter, step scales and checkpoints in one run: every
    gradient against the oracle, and the checkpointed adjoint against the pure one."""
    from oracle import mlp as omlp
    from synthetic import mlp_init
    w = SMALL
    theta = 0.3 * mlp_init(1, zero_last=False)
    scales = 1.0 + 0.05 * normal((3, w.n_steps), 73)
    st = replace(setup_for(w, 2), step_scales=scales)
    noise = white_noise(w.ptcl_grid, 3)
    target = opm.forward(white_noise(w.ptcl_grid, 4), st).dens
    run = opm.forward(noise, st, theta)
    _, gd_ref = opm.mse_loss(run.dens, target)
    ref = opm.adjoint(run, noise, g_dens=gd_ref)
    out = []
    for ck in (0, 3):
        cfg = api.make_config(w.ptcl_grid, w.mesh, w.box, w.n_steps, checkpoint_every=ck,
                              filter=True, lpt_order=2)
        pm = api.PMContext(cfg, CO)
        pm.set_filter(dev(theta))
        pm.set_step_scales(scales)
        disp, _, dens = pm.forward(dev(noise))
        _, gd = pm.loss_mse(dens, dev(target))
        g_noise, (g_om, g_s8), g_w = pm.adjoint(gd, want_filter=True)
        out.append((host(g_noise), g_om, g_s8, host(g_w), pm.step_gradients(), pm.stats()))
    for g_noise, g_om, g_s8, g_w, g_steps, stats in out:
        d = periodic_cells(host(disp), run.disp[-1], w.box, w.mesh)
        assert np.sqrt(np.mean(d * d)) < 1e-3
        assert rel_l2(g_noise, ref.noise) < 1e-3
        assert rel_l2(g_w, ref.theta) < 1e-3
        assert rel_l2(g_steps, ref.step_scales) < 1e-3
        assert abs(g_s8 / ref.sigma8 - 1) < 1e-3
        assert stats["ic_max_cells"] == 0.0
    assert out[1][5]["n_checkpoints"] == 3 and max(out[1][5]["ckpt_max_cells"]) == 0.0
    assert rel_l2(out[1][0], out[0][0]) < 1e-4
    assert rel_l2(out[1][4], out[0][4]) < 1e-4


def test_step_scales_persist_across_set_cosmology():
    scales = 1.0 + 0.1 * normal((3, TINY.n_steps), 74)
    new = replace(CO, omega_m=0.27)
    a = fresh(TINY)
    a.set_step_scales(scales)
    a.set_cosmology(new)
    b = api.PMContext(api.config_from_workload(TINY), new)
    b.set_step_scales(scales)
    n = dev(white_noise(8, 6))
    for x, y in zip(a.forward(n), b.forward(n)):
        assert torch.equal(x, y)
