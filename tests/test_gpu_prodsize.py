"""GPU parity against the FP64 oracle at the mesh sizes of the production runs.

The transforms change shape with the mesh (fft_plan.h, fft.hip): up to 128
points a column holds 8 values per lane; 256 and 1024 hold 16 values over 16
and 64 lanes; 512 and 1024 switch the strided passes to 8-column tiles with a
register cap.  The filter cotangent pairs the modes n0 and -n0 across lanes
once a column spans several lanes, and the network backward loops over several
chunks of the |n|^2 table per block once the table exceeds 256 chunks of 64
entries (a 256^3 mesh has 49153 entries).  These tests run every one of those
code paths against the oracle, with few particles so that the oracle's meshes
stay cheap:
  * the force and its transpose (force VJP) at 128^3, 256^3 and 512^3 meshes,
    plain and with the learned filter, on clustered and smooth particle sets;
  * a whole forward run and reverse-time adjoint with the learned filter on a
    256^3 mesh: gradients with respect to the noise, Omega_m, sigma_8 and the
    4417 filter weights;
  * the same on a 512^3 mesh against the oracle's stored result
    (tests/golden/filter_32p_512m_2steps.json, written by
    tests/golden/make_oracle_fixtures.py, since the FP64 run takes minutes).
Few particles on a large mesh are heavy (16^3 particles on 256^3 cells weigh
4096 cells each), and their trajectories amplify rounding differences within a
few large steps: run to a = 1/4 in three steps, the oracle's own gradients move
by 1-2 % under a 1e-6 relative perturbation of the noise.  The whole runs
therefore take two steps of 1/64 from a = 1/64, where that sensitivity is below
1e-4 and per-element parity is well defined.

Force bar: FP32 rounding of the four 3-D transforms grows with the number of
butterfly stages, log2(Ng^3); 1e-5 at a 64^3 mesh, scaled by log2(Ng) / 6.
"""
import json
import os

import numpy as np
import pytest

from gpu_util import CO, context, dev, host, periodic_cells, rel_l2, setup_for
from oracle import mesh as M
from oracle import pm as opm
from paper_2211_09958_amd import api
from synthetic import Workload, mlp_init, normal, uniform, white_noise

pytestmark = pytest.mark.gpu

THETA = 0.5 * mlp_init(0, zero_last=False)


@pytest.fixture(autouse=True)
def _workers(monkeypatch):
    monkeypatch.setattr(M, "WORKERS", 16)


def _displacements(np_, box, seed, kind):
    """Lattice displacements: 'smooth' Gaussian of 2 cells, or 'clustered' (half
    the particles pulled into four blobs a few cells wide, so some tiles hold
    thousands of particles and others none)."""
    cell = 1.0   # box = mesh in these tests
    s = normal((np_ ** 3, 3), seed) * 2.0 * cell
    if kind == "clustered":
        q = opm.lattice(np_, box)
        centres = uniform((4, 3), seed + 1, 0.0, box)
        pick = np.arange(np_ ** 3) % 2 == 0
        which = np.arange(np_ ** 3) % 8 // 2
        target = centres[which] + normal((np_ ** 3, 3), seed + 2) * 3.0 * cell
        d = target - q
        d -= box * np.round(d / box)
        s = np.where(pick[:, None], d, s)
    return s


CASES = [(32, 128, "clustered"), (64, 256, "smooth"), (16, 256, "clustered"),
         (16, 512, "smooth")]


@pytest.mark.parametrize("np_,ng,kind", CASES)
@pytest.mark.parametrize("filtered", [False, True])
def test_force_and_vjp_match_oracle(np_, ng, kind, filtered):
    box, a = float(ng), 0.6
    pm = context(np_, ng, box, 1, filter=filtered)
    if filtered:
        pm.set_filter(dev(THETA))
    s = _displacements(np_, box, 40 + ng, kind).astype(np.float32)
    v = normal((np_ ** 3, 3), 50 + ng).astype(np.float32)
    print(f"case np={np_} ng={ng} {kind} filter={filtered}", flush=True)
    F = host(pm.force(dev(s), a))
    xi = host(pm.force_vjp(dev(s), a, dev(v)))
    st = opm.Setup(np_, ng, box, 1, CO)
    filt = opm.filter_at(THETA, st, a)[0] if filtered else None
    x = opm.lattice(np_, box) + s.astype(np.float64)
    xi_ref, _, F_ref = opm.pm_force_vjp(x, v.astype(np.float64), st, filt)
    eF, ex = rel_l2(F, F_ref), rel_l2(xi, xi_ref)
    print(f"  force rel L2 {eF:.2e}, VJP rel L2 {ex:.2e}")
    assert eF < 1e-5 * np.log2(ng) / 6
    assert ex < 1e-4


def test_filter_whole_run_gradients_at_256_mesh():
    """Forward + reverse-time adjoint with the learned filter on a 256^3 mesh
    (16^3 particles, box 256, 2 steps a = 1/64 -> 3/64): the filter gradient
    takes the multi-lane +-n0 pairing and the multi-chunk network backward."""
    w = Workload("filter-16p-256m-2s", ptcl_grid=16, mesh=256, box=256.0, n_steps=2,
                 a_stop=3.0 / 64)
    st = setup_for(w)
    noise = white_noise(w.ptcl_grid, 21)
    target = opm.forward(white_noise(w.ptcl_grid, 22), st, THETA).dens
    run = opm.forward(noise, st, THETA)
    _, gd = opm.mse_loss(run.dens, target)
    P = w.ptcl_grid ** 3
    gdisp = normal((P, 3), 23) * 1e-3
    ref = opm.adjoint(run, noise, g_dens=gd, g_disp=gdisp)

    pm = api.PMContext(api.make_config(w.ptcl_grid, w.mesh, w.box, w.n_steps,
                                       a_stop=w.a_stop, filter=True), CO)
    pm.set_filter(dev(THETA))
    disp, mom, dens = pm.forward(dev(noise))
    _, g = pm.loss_mse(dens, dev(target))
    g_noise, (g_om, g_s8), g_w = pm.adjoint(g, dev(gdisp), want_filter=True)
    e_w = rel_l2(host(g_w), ref.theta)
    e_n = rel_l2(host(g_noise), ref.noise)
    e_om, e_s8 = abs(g_om / ref.omega_m - 1), abs(g_s8 / ref.sigma8 - 1)
    print(f"filter {e_w:.2e} noise {e_n:.2e} Omega_m {e_om:.2e} sigma8 {e_s8:.2e}")
    assert e_w < 1e-3 and e_n < 1e-3 and e_om < 1e-3 and e_s8 < 1e-3
    # every block of the table sum is used: all 4417 entries carry gradient
    assert np.count_nonzero(host(g_w)) == np.count_nonzero(ref.theta)


def test_filter_whole_run_gradients_at_512_mesh():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "filter_32p_512m_2steps.json")
    if not os.path.exists(path):
        pytest.skip("run tests/golden/make_oracle_fixtures.py filter first")
    with open(path) as f:
        ref = json.load(f)
    c = ref["config"]
    np_, ng = c["ptcl_grid"], c["mesh"]
    pm = api.PMContext(api.make_config(np_, ng, c["box"], c["n_steps"], a_start=c["a_start"],
                                       a_stop=c["a_stop"], filter=True), CO)
    pm.set_filter(dev(THETA))
    target = pm.forward(dev(white_noise(np_, c["target_seed"])))[2].clone()
    disp, mom, dens = pm.forward(dev(white_noise(np_, c["seed"])))
    L, g = pm.loss_mse(dens, target)
    gdisp = normal((np_ ** 3, 3), 33) * 1e-3
    g_noise, (g_om, g_s8), g_w = pm.adjoint(g, dev(gdisp), want_filter=True)
    e_w = rel_l2(host(g_w), ref["g_theta"])
    gn = host(g_noise).reshape(-1)
    e_n = rel_l2(gn[np.array(ref["g_noise_index"])], ref["g_noise_sample"])
    e_norm = abs(np.linalg.norm(gn) / ref["g_noise_norm"] - 1)
    e_om, e_s8 = abs(g_om / ref["g_omega_m"] - 1), abs(g_s8 / ref["g_sigma8"] - 1)
    d = periodic_cells(host(disp)[np.array(ref["disp_index"])], np.array(ref["disp_sample"]),
                       c["box"], ng)
    e_x = float(np.sqrt(np.mean(d * d)))
    print(f"loss {L:.6e}/{ref['loss']:.6e}; filter {e_w:.2e} noise {e_n:.2e} Omega_m {e_om:.2e} "
          f"sigma8 {e_s8:.2e} positions {e_x:.2e} cells RMS")
    assert e_x < 1e-4
    assert abs(L / ref["loss"] - 1) < 1e-4
    assert e_w < 1e-3 and e_n < 1e-3 and e_norm < 1e-3 and e_om < 1e-3 and e_s8 < 1e-3
