"""End-to-end GPU parity: forward run, reverse-time adjoint, gradients, filter."""
import numpy as np
import pytest
import torch

from gpu_util import (CO, context, ctx_for, dev, gradient_envelope, host, oracle_gradients,
                      periodic_cells, rel_l2, setup_for)
from oracle import mesh as M
from oracle import mlp as omlp
from oracle import pm as opm
from paper_2211_09958_amd import _lib, api
from synthetic import SMALL, Workload, mlp_init, normal, white_noise

pytestmark = pytest.mark.gpu

TINY = Workload("tiny", ptcl_grid=8, mesh=16, box=32.0, n_steps=4)


@pytest.fixture(scope="module")
def small_runs():
    noise = white_noise(SMALL.ptcl_grid, 0)
    run = opm.forward(noise, setup_for(SMALL))
    pm = ctx_for(SMALL)
    disp, mom, dens = pm.forward(dev(noise))
    return noise, run, host(disp), host(mom), host(dens)


def test_small_positions_within_1e3_cells(small_runs):
    noise, run, disp, mom, dens = small_runs
    d = periodic_cells(disp, run.disp[-1], SMALL.box, SMALL.mesh)
    rms = float(np.sqrt(np.mean(d * d)))
    print(f"position RMS {rms:.3e} cells, max {d.max():.3e}")
    assert rms < 1e-3


def test_small_power_spectrum_within_1e4(small_runs):
    noise, run, disp, mom, dens = small_runs
    k, P, N = ctx_for(SMALL).power_spectrum(dev(dens), SMALL.mesh // 2)
    kr, Pr, Nr = M.power_spectrum(run.dens, SMALL.box, SMALL.mesh // 2)
    k_nyq = np.pi * SMALL.mesh / SMALL.box
    sel = kr < 0.5 * k_nyq
    err = np.abs(P[sel] / Pr[sel] - 1)
    print("P(k) relative errors", err.max())
    assert err.max() < 1e-4


def test_small_momentum_and_density(small_runs):
    noise, run, disp, mom, dens = small_runs
    assert rel_l2(mom, run.mom) < 1e-3
    assert np.max(np.abs(dens - run.dens)) < 5e-2 * np.abs(run.dens).max()


def test_forward_bitwise_repeatable():
    pm = ctx_for(TINY)
    n = dev(white_noise(8, 5))
    a = pm.forward(n)
    b = pm.forward(n)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def omega_m_scale(w, ref):
    """Sum of |terms| of dL/dOmega_m in the oracle's decomposition."""
    from oracle import cosmology as C
    d = C.kdk_coefficient_derivatives(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    terms = [np.abs(ref.kick_a * d.kick_a).sum(), np.abs(ref.kick_b * d.kick_b).sum(),
             np.abs(ref.drift * d.drift).sum(), abs(ref.D0 * d.D0), abs(ref.G0 * d.G0)]
    ic = ref.omega_m - (np.dot(ref.kick_a, d.kick_a) + np.dot(ref.kick_b, d.kick_b)
                        + np.dot(ref.drift, d.drift) + ref.D0 * d.D0 + ref.G0 * d.G0)
    return float(sum(terms) + abs(ic))


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_gradients_match_oracle(w):
    noise, target, gdisp, gmom, ref, run = oracle_gradients(w, 3, 4)
    pm = ctx_for(w)
    disp, mom, dens = pm.forward(dev(noise))
    L, gd = pm.loss_mse(dens, dev(target))
    g_noise, (g_om, g_s8), _ = pm.adjoint(gd, dev(gdisp), dev(gmom))
    e_noise = rel_l2(host(g_noise), ref.noise)
    # dL/dOmega_m is a sum of terms that largely cancel; FP32 rounding scales
    # with the sum of their magnitudes, so the error is measured against it
    e_om = abs(g_om - ref.omega_m) / omega_m_scale(w, ref)
    e_s8 = abs(g_s8 / ref.sigma8 - 1)
    e_om_plain = abs(g_om / ref.omega_m - 1)
    print(f"{w.name}: noise {e_noise:.2e} Om {e_om:.2e} (plain rel {e_om_plain:.2e}) "
          f"s8 {e_s8:.2e}")
    assert e_noise < 1e-3 and e_om < 1e-3 and e_s8 < 1e-3
    if w is SMALL:
        # the 32^3 / 64^3 workload against plain relative bars: 1e-3, or three
        # times the oracle's own envelope where the trajectory's CIC kinks make
        # the exact gradient move more than that under FP32-sized perturbations
        env, dpos = gradient_envelope(w, 3, 4, ref, run)
        print(f"oracle envelope {env} (positions moved {dpos:.1e} cells)")
        assert e_noise < max(1e-3, 3 * env["noise"])
        assert e_om_plain < max(1e-3, 3 * env["omega_m"])
        assert e_s8 < max(1e-3, 3 * env["sigma8"])


@pytest.mark.parametrize("w", [TINY, SMALL])
def test_reverse_time_reconstruction(w):
    pm = ctx_for(w)
    pm.forward(dev(white_noise(w.ptcl_grid, 1)))
    pm.adjoint(g_disp=dev(np.zeros((w.ptcl_grid ** 3, 3))))
    st = pm.stats()
    print(w.name, st["ic_rms_cells"], st["ic_max_cells"], st["ic_mom_rel_rms"])
    assert st["ic_rms_cells"] < 1e-4
    # fixed-point kick/drift + bitwise-reproducible force: the reverse pass
    # recovers the initial state bit for bit
    assert st["ic_max_cells"] == 0.0 and st["ic_mom_rel_rms"] == 0.0


def test_checkpointed_adjoint_matches_pure():
    w = SMALL
    noise, target, gdisp, gmom, ref, run = oracle_gradients(w, 5, 6)
    out = []
    for ck in (0, 3):
        pm = context(w.ptcl_grid, w.mesh, w.box, w.n_steps, checkpoint_every=ck)
        disp, mom, dens = pm.forward(dev(noise))
        _, gd = pm.loss_mse(dens, dev(target))
        out.append(pm.adjoint(gd, dev(gdisp), dev(gmom)))
        if ck:
            st = pm.stats()
            assert st["n_checkpoints"] == 3
            assert max(st["ckpt_max_cells"]) == 0.0
    assert rel_l2(host(out[1][0]), host(out[0][0])) < 1e-4
    assert abs(out[1][1][0] / out[0][1][0] - 1) < 1e-4
    # and both against the oracle's stored-trajectory adjoint, to the oracle's
    # own envelope under FP32-sized input perturbations (gradient_envelope)
    env, dpos = gradient_envelope(w, 5, 6, ref, run)
    bar = {k: max(1e-3, 3 * v) for k, v in env.items()}
    for g_noise, (g_om, g_s8), _ in out:
        e = {"noise": rel_l2(host(g_noise), ref.noise), "omega_m": abs(g_om / ref.omega_m - 1),
             "sigma8": abs(g_s8 / ref.sigma8 - 1)}
        print(f"errors {e}; oracle envelope {env} (positions moved {dpos:.1e} cells)")
        for k in e:
            assert e[k] < bar[k], (k, e[k], bar[k])


def test_autograd_function():
    w = TINY
    pm = ctx_for(w)
    noise = dev(white_noise(8, 2)).requires_grad_(True)
    om = torch.tensor(CO.omega_m, dtype=torch.float64, requires_grad=True)
    s8 = torch.tensor(CO.sigma8, dtype=torch.float64, requires_grad=True)
    disp, mom, dens = api.simulate(pm, noise, om, s8)
    loss = (dens.double() ** 2).mean()
    loss.backward()
    run = opm.forward(white_noise(8, 2), setup_for(w))
    ref = opm.adjoint(run, white_noise(8, 2), g_dens=2 * run.dens / run.dens.size)
    assert rel_l2(host(noise.grad), ref.noise) < 1e-3
    assert abs(float(om.grad) / ref.omega_m - 1) < 1e-3


def test_autograd_rejects_a_stale_graph():
    """The context keeps one forward run: backward of a graph whose run was
    replaced by a later simulate() on the same context must raise, not return the
    later run's gradients."""
    pm = ctx_for(TINY)
    om = torch.tensor(CO.omega_m, dtype=torch.float64, requires_grad=True)
    s8 = torch.tensor(CO.sigma8, dtype=torch.float64, requires_grad=True)
    n1 = dev(white_noise(8, 2)).requires_grad_(True)
    n2 = dev(white_noise(8, 3)).requires_grad_(True)
    d1 = api.simulate(pm, n1, om, s8)[2]
    d2 = api.simulate(pm, n2, om, s8)[2]
    with pytest.raises(RuntimeError, match="another forward"):
        (d1.double() ** 2).mean().backward()
    (d2.double() ** 2).mean().backward()        # the latest graph still works
    assert torch.isfinite(n2.grad).all()


# ---------------------------------------------------------------- filter

def test_filter_table_matches_oracle():
    pm = context(8, 32, 32.0, 2, filter=True)
    theta = mlp_init(1, zero_last=False)
    pm.set_filter(dev(theta))
    for a in (0.1, 0.7):
        got = host(pm.filter_table(a))
        ref, _ = omlp.filter_table(theta, 32, 32.0, a)
        assert np.max(np.abs(got - ref)) < 2e-5 * np.abs(ref).max()


def test_zero_last_layer_reproduces_plain_pm_bitwise():
    plain = ctx_for(TINY)
    filt = context(TINY.ptcl_grid, TINY.mesh, TINY.box, TINY.n_steps, filter=True)
    filt.set_filter(dev(mlp_init(0)))
    n = dev(white_noise(8, 7))
    a, b = plain.forward(n), filt.forward(n)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_filter_gradients_match_oracle():
    w = TINY
    theta = 0.5 * mlp_init(0, zero_last=False)
    noise, target, gdisp, gmom, ref, _ = oracle_gradients(w, 3, 4, theta)
    pm = context(w.ptcl_grid, w.mesh, w.box, w.n_steps, filter=True)
    pm.set_filter(dev(theta))
    disp, mom, dens = pm.forward(dev(noise))
    _, gd = pm.loss_mse(dens, dev(target))
    g_noise, (g_om, g_s8), g_w = pm.adjoint(gd, dev(gdisp), dev(gmom), want_filter=True)
    e_w = rel_l2(host(g_w), ref.theta)
    e_n = rel_l2(host(g_noise), ref.noise)
    print(f"filter grads: W {e_w:.2e} noise {e_n:.2e}")
    assert e_w < 1e-3 and e_n < 1e-3


def test_adam_matches_torch():
    pm = ctx_for(TINY)
    p0 = normal(100, 1).astype(np.float32)
    p = dev(p0)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    ref = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float64))
    opt = torch.optim.Adam([ref], lr=1e-2)
    for t in range(1, 6):
        g = normal(100, 10 + t).astype(np.float32)
        pm.adam(p, dev(g), m, v, t, lr=1e-2)
        ref.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(host(p), ref.detach().numpy(), rtol=1e-5, atol=1e-6)


def test_adam_on_batch_mean_matches_torch():
    pm = ctx_for(TINY)
    p0 = normal(300, 2).astype(np.float32)
    p = dev(p0)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    ref = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float64))
    opt = torch.optim.Adam([ref], lr=3e-3)
    for t in range(1, 5):
        g = normal((4, 300), 20 + t).astype(np.float32)
        pm.adam(p, dev(g), m, v, t, lr=3e-3)
        ref.grad = torch.tensor(g.astype(np.float64).mean(axis=0))
        opt.step()
    np.testing.assert_allclose(host(p), ref.detach().numpy(), rtol=1e-5, atol=1e-6)


def test_training_objective_gradient_matches_oracle():
    """Filter gradient of the training objective (P(k) ratio + weighted position
    loss against a finer-mesh run) through pm_loss_pk, pm_loss_disp and the
    reverse-time adjoint, against the oracle over a stored trajectory."""
    np_, ng, box, steps, nb, wd = 16, 16, 16.0, 6, 8, 1e-2
    theta = 0.5 * mlp_init(2, zero_last=False)
    noise = white_noise(np_, 11)
    fine = opm.forward(noise, opm.Setup(np_, 4 * ng, box, steps, CO))
    disp_t = fine.disp[-1].astype(np.float32)
    pk_t = M.power_spectrum(M.density(fine.q + fine.disp[-1], ng, box, np_ ** 3), box, nb)[1]
    st = opm.Setup(np_, ng, box, steps, CO)
    run = opm.forward(noise, st, theta)
    Lp_ref, gd = opm.pk_loss(run.dens, pk_t, box, nb)
    Ld_ref, gx = opm.disp_loss(run.disp[-1], disp_t, box, ng, wd)
    ref = opm.adjoint(run, noise, g_dens=gd, g_disp=gx)

    pm = context(np_, ng, box, steps, filter=True)
    pm.set_filter(dev(theta))
    disp, mom, dens = pm.forward(dev(noise))
    Lp, g_dens = pm.loss_pk(dens, pk_t, nb)
    Ld, g_disp = pm.loss_disp(disp, dev(disp_t), weight=wd)
    _, _, g_w = pm.adjoint(g_dens=g_dens, g_disp=g_disp, want_filter=True)
    e_w = rel_l2(host(g_w), ref.theta)
    print(f"losses {Lp:.4e}/{Lp_ref:.4e} {Ld:.4e}/{Ld_ref:.4e}; filter grad {e_w:.2e}")
    assert abs(Lp / Lp_ref - 1) < 1e-3 and abs(Ld / Ld_ref - 1) < 1e-3
    assert e_w < 1e-3


def test_filter_training_reduces_loss():
    from paper_2211_09958_amd import train_filter
    rep = train_filter.main(["--ptcl", "16", "--box", "16", "--steps", "8", "--train-seeds", "4",
                             "--heldout", "2", "--batch", "2", "--epochs", "24", "--lr", "1e-2",
                             "--n-bins", "8", "--log-every", "8"])
    h = rep["history"]
    assert rep["adam_steps"] == 48
    total = [e["loss_pk"] + e["loss_disp"] for e in h]
    assert total[-1] < 0.75 * total[0] and total[-1] < total[len(total) // 2]


@pytest.mark.parametrize("weights,fine_mesh,factor", [("filter_128p_128m_to_512m.npy", 512, 0.6),
                                                    ("filter_128p_128m_to_256m.npy", 256, 0.3)])
def test_trained_filter_beats_plain_on_heldout_seeds(weights, fine_mesh, factor):
    """The committed filters (trained by train_filter on seeds 0..55 at 128^3
    particles, 128^3 vs 512^3 or 256^3 meshes, box 128, 31 steps) against plain PM
    on two held-out seeds: P(k) of the final density against the finer-mesh run of
    the same seed, both on the 128^3 mesh, max over shells k <= k_Nyq/2."""
    import os
    here = os.path.dirname(os.path.abspath(api.__file__))
    theta = np.load(os.path.join(here, "weights", weights))
    fine = context(128, fine_mesh, 128.0, 31)
    coarse = context(128, 128, 128.0, 31, filter=True)
    errs = {"plain": [], "learned": []}
    for seed in (56, 63):
        n = dev(white_noise(128, seed))
        ref = coarse.power_spectrum(coarse.density(fine.forward(n, want_density=False)[0]), 32)[1]
        for name, w in (("plain", mlp_init(0)), ("learned", theta)):
            coarse.set_filter(dev(w))
            pk = coarse.power_spectrum(coarse.forward(n)[2], 32)[1]
            errs[name].append(np.max(np.abs(pk / ref - 1)))
    print({k: np.round(v, 4) for k, v in errs.items()})
    assert np.mean(errs["learned"]) < factor * np.mean(errs["plain"])


@pytest.mark.parametrize("lpt", [1, 2])
def test_field_level_reconstruction_recovers_the_noise(lpt):
    """Adam on the white noise through the reverse-time adjoint: fitting the final
    density of a held-back seed (32^3 particles, 64^3 mesh, 32 Mpc/h particle
    spacing, 10 steps; Zel'dovich or 2LPT initial conditions) drives the loss down
    by orders of magnitude and recovers the noise (cross-correlation with the
    truth near 1 in every shell)."""
    from paper_2211_09958_amd import reconstruct
    rep = reconstruct.main(["--ptcl", "32", "--mesh", "64", "--box", "1024", "--steps", "10",
                            "--iters", "200", "--lr", "0.03", "--log-every", "50",
                            "--lpt-order", str(lpt)])
    assert rep["loss_last"] < 0.05 * rep["loss_first"]
    r = np.array(rep["noise_cross_correlation"])
    print(np.round(r, 4))
    assert r[: 3 * len(r) // 4].min() > 0.95, r


def test_field_level_reconstruction_in_a_nonlinear_box():
    """The same fit where the final field is nonlinear (64^3 particles, 128^3
    mesh, box 128 Mpc/h: 2 Mpc/h spacing, 15 steps to a = 1).  Adam's step must
    be small there (lr 0.02 stalls, 0.05 diverges); with lr 0.01 and 300 steps
    the loss drops below half and the recovered noise correlates with the truth
    at r > 0.75 on average over the four largest-scale shells, each above 0.65.
    The 300 nonlinear steps amplify rounding: two builds whose noise gradients
    differ by 3e-7 (relative L2) gave r = 0.78, 0.88, 0.86, 0.78 and 0.72, 0.86,
    0.88, 0.84 (mean 0.82 both), the first shell holding the fewest modes."""
    from paper_2211_09958_amd import reconstruct
    rep = reconstruct.main(["--ptcl", "64", "--mesh", "128", "--box", "128", "--steps", "15",
                            "--iters", "300", "--lr", "0.01", "--log-every", "100"])
    r = np.array(rep["noise_cross_correlation"])
    print(f"loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}; r(k) {np.round(r[:8], 3)}")
    assert rep["loss_last"] < 0.5 * rep["loss_first"]
    assert r[:4].mean() > 0.75 and r[:4].min() > 0.65, r[:4]


# ------------------------------------------------------- failure handling, resume

def test_nonfinite_cotangent_reports_enumeric_and_context_recovers():
    """A NaN cotangent makes the adjoint's FP64 sums non-finite: PM_ENUMERIC, and
    the context stays usable (positions never depend on cotangents)."""
    w = TINY
    pm = api.PMContext(api.config_from_workload(w), CO)
    noise = dev(white_noise(8, 2))
    gd = dev(normal((512, 3), 3))
    pm.forward(noise)
    ref = pm.adjoint(g_disp=gd)[0].clone()
    pm.forward(noise)
    bad = torch.full((512, 3), float("nan"), device="cuda")
    with pytest.raises(api.PMError) as e:
        pm.adjoint(g_mom=bad)
    assert e.value.code == _lib.PM_ENUMERIC
    pm.forward(noise)
    assert torch.equal(pm.adjoint(g_disp=gd)[0], ref)
    assert pm.stats()["ic_max_cells"] == 0.0


def test_filter_training_resumes_from_its_state(tmp_path):
    """Two epochs in one go against one epoch, stop, resume for the second: the
    same weights (up to the order of the FP64 filter-gradient atomics)."""
    from paper_2211_09958_amd import train_filter as tf
    base = ["--ptcl", "16", "--fine-factor", "2", "--box", "32", "--steps", "4",
            "--train-seeds", "4", "--heldout", "0", "--batch", "2", "--n-bins", "8",
            "--lr", "1e-2", "--log-every", "100"]
    tf.main(base + ["--epochs", "2", "--out", str(tmp_path / "a.npy")])
    st = str(tmp_path / "state.npz")
    tf.main(base + ["--epochs", "1", "--state", st])
    r = tf.main(base + ["--epochs", "2", "--state", st, "--out", str(tmp_path / "b.npy")])
    a, b = np.load(tmp_path / "a.npy"), np.load(tmp_path / "b.npy")
    assert r["adam_steps"] == 4 and len(r["history"]) == 2
    assert not np.array_equal(a, mlp_init(0, zero_last=True))
    assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(a))


def test_adjoint_repeatable_and_checkpoint_invariant():
    """Run twice, compare bits: catches LDS races and order-dependent atomics.

    The state and the noise gradient are bitwise repeatable, and so is the
    noise gradient of a checkpointed adjoint, since the reverse pass rebuilds
    every checkpointed state exactly.  The parameter sums are FP64 block sums
    over tiles whose particle order follows the binning atomics, so they repeat
    to rounding only; the filter gradient is folded with FP32 atomics."""
    w = SMALL
    theta = dev(0.3 * mlp_init(1, zero_last=False))
    noise = dev(white_noise(w.ptcl_grid, 3))
    g_dens = dev(normal((w.mesh,) * 3, 11) * 1e-3)
    g_disp = dev(normal((w.ptcl_grid ** 3, 3), 12) * 1e-3)
    runs = []
    for ck in (0, 0, 3, 3):
        cfg = api.make_config(w.ptcl_grid, w.mesh, w.box, w.n_steps, checkpoint_every=ck,
                              filter=True)
        pm = api.PMContext(cfg, CO)
        pm.set_filter(theta)
        out = pm.forward(noise)
        g_noise, g_cosmo, g_w = pm.adjoint(g_dens, g_disp, want_filter=True)
        runs.append((out, g_noise.clone(), np.array(g_cosmo), host(g_w), pm.step_gradients(),
                     pm.stats()))
    ref = runs[0]
    for out, g_noise, g_cosmo, g_w, g_steps, st in runs[1:]:
        for x, y in zip(out, ref[0]):
            assert torch.equal(x, y)
        assert torch.equal(g_noise, ref[1])
        assert np.allclose(g_cosmo, ref[2], rtol=1e-12, atol=0)
        assert np.allclose(g_steps, ref[4], rtol=1e-12, atol=1e-12 * np.abs(ref[4]).max())
        assert rel_l2(g_w, ref[3]) < 1e-5
        assert st["ic_max_cells"] == 0.0
    assert max(runs[2][5]["ckpt_max_cells"]) == 0.0
