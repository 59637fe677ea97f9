"""Write the stored oracle results of tests/golden/ (calls only oracle/ and synthetic/).

Some parity cases run at sizes where the FP64 oracle takes minutes, too long to
repeat inside every GPU test run.  This script runs the oracle once on the host
and stores what the GPU tests compare against:

  medium_truncated_2steps.json
      The 256^3-particle / 512^3-mesh / 256 Mpc/h geometry with the integration
      cut to its first two steps (a = 1/64 -> 3/64, the same step of 1/64), run
      seed 0 against the final density of seed 1 (MSE loss).  Early enough
      that the exact gradient is smooth in the inputs (on a 64^3/128^3 box of
      the same cell size the oracle's own gradient moves by 7e-6 under a 1e-6
      relative perturbation of the noise after two steps, 4e-4 after four), so
      per-element parity holds.  Stored: the loss, the gradients
      with respect to Omega_m and sigma_8 (and the terms of the Omega_m sum),
      the norm and shell spectrum of the noise gradient, the noise gradient and
      final displacement at seeded sample indices, and the final P(k).
  filter_32p_512m_2steps.json
      32^3 particles, 512^3 mesh, box 512, two steps a = 1/64 -> 3/64, learned
      filter with weights 0.5 * mlp_init(0, zero_last=False): the 4417 filter
      gradients, the Omega_m and sigma_8 gradients, the noise gradient (norm and
      4096 sampled sites) and 2048 sampled final displacements (MSE loss against
      seed 32 plus a seeded displacement cotangent).  Few heavy particles make trajectories sensitive to rounding:
      with 16^3 particles (32^3 cells each) the oracle's own filter gradient moves
      by 12 % under a 1e-6 relative perturbation of the noise even in these two
      early steps; with 32^3 particles (16^3 cells each, as 16^3 particles on the
      256^3 mesh, where that sensitivity is 1e-5) the run is well conditioned.

Run:  python tests/golden/make_oracle_fixtures.py [medium|filter|all]
Takes about 15 minutes (medium) and 3 minutes (filter) on 8 cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cosmology as C  # noqa: E402
from oracle import mesh as M  # noqa: E402
from oracle import pm as opm  # noqa: E402
from synthetic import Cosmology, mlp_init, normal, white_noise  # noqa: E402

CO = Cosmology()
MEDIUM_FILE = os.path.join(HERE, "medium_truncated_2steps.json")
FILTER_FILE = os.path.join(HERE, "filter_32p_512m_2steps.json")


def shell_power(field, n_shells):
    """Sum over |n| shells (round(|n|) = 1..n_shells) of |DFT(field)|^2 / N^3,
    full spectrum (the half spectrum weighted 2 off the n_z = 0, N/2 planes)."""
    n = field.shape[0]
    fk = M.rfftn(field)
    f = np.fft.fftfreq(n, 1.0 / n)
    fz = np.arange(n // 2 + 1, dtype=np.float64)
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
    b = np.floor(np.sqrt(n2) + 0.5).astype(np.int64)
    w = np.where((fz == 0) | (fz == n // 2), 1.0, 2.0)[None, None, :] * np.ones_like(n2)
    p = np.abs(fk) ** 2 * w / n ** 3
    out = np.bincount(b.ravel(), weights=p.ravel(), minlength=n_shells + 1)
    return out[1:n_shells + 1]


def sample_indices(n, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=count, replace=False))


def medium():
    np_, ng, box, steps = 256, 512, 256.0, 2
    a0 = 1.0 / 64
    st = opm.Setup(np_, ng, box, steps, CO, a0, a0 + steps / 64.0)
    t0 = time.time()
    target = opm.forward(white_noise(np_, 1), st).dens
    print(f"target run {time.time() - t0:.0f} s", flush=True)
    noise = white_noise(np_, 0)
    run = opm.forward(noise, st)
    print(f"run {time.time() - t0:.0f} s", flush=True)
    loss, gd = opm.mse_loss(run.dens, target)
    del target
    ref = opm.adjoint(run, noise, g_dens=gd)
    print(f"adjoint {time.time() - t0:.0f} s", flush=True)
    d = C.kdk_coefficient_derivatives(CO.omega_m, st.a_start, st.a_stop, steps)
    terms = {"kick_a": float(np.dot(ref.kick_a, d.kick_a)),
             "kick_b": float(np.dot(ref.kick_b, d.kick_b)),
             "drift": float(np.dot(ref.drift, d.drift)),
             "D0": float(ref.D0 * d.D0), "G0": float(ref.G0 * d.G0)}
    terms["power_spectrum"] = ref.omega_m - sum(terms.values())
    P = np_ ** 3
    gi = sample_indices(P, 4096, 7)
    pi = sample_indices(P, 2048, 8)
    _, pk, cnt = M.power_spectrum(run.dens, box, ng // 4)
    out = {
        "config": {"ptcl_grid": np_, "mesh": ng, "box": box, "n_steps": steps,
                   "a_start": st.a_start, "a_stop": st.a_stop, "seed": 0, "target_seed": 1,
                   "cosmology": CO.__dict__},
        "loss": loss,
        "g_omega_m": ref.omega_m, "g_sigma8": ref.sigma8, "g_omega_m_terms": terms,
        "g_noise_norm": float(np.linalg.norm(ref.noise)),
        "g_noise_shell_power": shell_power(ref.noise, np_ // 2).tolist(),
        "g_noise_index": gi.tolist(),
        "g_noise_sample": ref.noise.reshape(-1)[gi].tolist(),
        "disp_index": pi.tolist(),
        "disp_sample": run.disp[-1][pi].tolist(),
        "pk": pk.tolist(), "pk_modes": cnt.tolist(),
    }
    with open(MEDIUM_FILE, "w") as f:
        json.dump(out, f)
    print(f"wrote {MEDIUM_FILE}", flush=True)


def filter_case():
    np_, ng, box, steps = 32, 512, 512.0, 2
    a0 = 1.0 / 64
    st = opm.Setup(np_, ng, box, steps, CO, a0, a0 + steps / 64.0)
    theta = 0.5 * mlp_init(0, zero_last=False)
    t0 = time.time()
    target = opm.forward(white_noise(np_, 32), st, theta).dens
    noise = white_noise(np_, 31)
    run = opm.forward(noise, st, theta)
    loss, gd = opm.mse_loss(run.dens, target)
    del target
    gdisp = normal((np_ ** 3, 3), 33) * 1e-3
    ref = opm.adjoint(run, noise, g_dens=gd, g_disp=gdisp)
    print(f"filter case {time.time() - t0:.0f} s", flush=True)
    gi = sample_indices(np_ ** 3, 4096, 9)
    pi = sample_indices(np_ ** 3, 2048, 10)
    out = {
        "config": {"ptcl_grid": np_, "mesh": ng, "box": box, "n_steps": steps,
                   "a_start": st.a_start, "a_stop": st.a_stop, "seed": 31, "target_seed": 32,
                   "theta": "0.5 * mlp_init(0, zero_last=False)",
                   "g_disp": "1e-3 * normal((32**3, 3), 33)", "cosmology": CO.__dict__},
        "loss": loss,
        "g_omega_m": ref.omega_m, "g_sigma8": ref.sigma8,
        "g_theta": ref.theta.tolist(),
        "g_noise_norm": float(np.linalg.norm(ref.noise)),
        "g_noise_index": gi.tolist(),
        "g_noise_sample": ref.noise.reshape(-1)[gi].tolist(),
        "disp_index": pi.tolist(),
        "disp_sample": run.disp[-1][pi].tolist(),
    }
    with open(FILTER_FILE, "w") as f:
        json.dump(out, f)
    print(f"wrote {FILTER_FILE}", flush=True)


if __name__ == "__main__":
    M.WORKERS = os.cpu_count() or 1
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("filter", "all"):
        filter_case()
    if what in ("medium", "all"):
        medium()
