"""Train the learned PM force filter f(|k|, a) through the reverse-time adjoint.

The paper motivates learned corrections of the PM force (a differentiable
simulator lets a model be optimised through it).  Here a 2-64-64-1 SiLU network
f = 1 + g(|k|/k_Nyq, a) multiplies the Poisson kernel of a coarse run
(Np^3 particles on an Np^3 mesh) and is trained so that the coarse run reproduces
a run of the same seeded initial conditions on a finer mesh: the power spectrum
of the final density (both runs' particles assigned to the coarse mesh) and the
final particle positions.

Every arithmetic step runs in libpmx through the C ABI: fine and coarse forward
runs, the two losses and their cotangents (pm_loss_pk, pm_loss_disp), the
reverse-time adjoint with the filter gradient, and Adam on the batch mean.

The temporal half (``--train schedule`` or ``both``): per-step multipliers of
the kick and drift factors (pm_set_step_scales), trained with Adam on the
gradients the same adjoint returns (pm_step_gradients), alone or jointly with
the filter.

    python -m paper_2211_09958_amd.train_filter --out weights.npy --report report.json

Defaults: 128^3 particles, coarse 128^3 and fine 512^3 meshes, box 128 Mpc/h, 31
steps, seeds 0..55 for training in batches of 8, seeds 56..63 held out.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import api
from ._lib import N_FILTER_PARAMS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
from synthetic import Cosmology, mlp_init, white_noise  # noqa: E402  (seeded inputs only)


def parse(argv=None):
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    p.add_argument("--ptcl", type=int, default=128)
    p.add_argument("--fine-factor", type=int, default=4, help="fine mesh = factor x coarse mesh")
    p.add_argument("--box", type=float, default=128.0)
    p.add_argument("--steps", type=int, default=31)
    p.add_argument("--train-seeds", type=int, default=56, help="seeds 0..N-1 train")
    p.add_argument("--first-seed", type=int, default=0,
                   help="offset of the seed range (training seeds start here)")
    p.add_argument("--heldout", type=int, default=8, help="the next seeds are held out")
    p.add_argument("--batch", type=int, default=8)
    p.add_argument("--epochs", type=int, default=200)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--w-disp", type=float, default=1e-2, help="weight of the position loss")
    p.add_argument("--n-bins", type=int, default=0,
                   help="P(k) shells in the loss (0: Ng/4, the shells up to k_Nyq/2)")
    p.add_argument("--init-seed", type=int, default=0)
    p.add_argument("--init", default="", help="start from these weights (.npy) instead")
    p.add_argument("--train", choices=("filter", "schedule", "both"), default="filter",
                   help="what to learn: the force filter, the per-step KDK scales, or both")
    p.add_argument("--lr-schedule", type=float, default=1e-3, help="Adam rate of the step scales")
    p.add_argument("--lpt-order", type=int, choices=(1, 2), default=1,
                   help="initial conditions of every run: 1 Zel'dovich, 2 with the 2LPT term")
    p.add_argument("--out-schedule", default="", help="write the step scales (.npy, [3, steps])")
    p.add_argument("--out", default="", help="write the trained weights (.npy, float32)")
    p.add_argument("--report", default="", help="write losses and held-out errors (.json)")
    p.add_argument("--log-every", type=int, default=1)
    p.add_argument("--state", default="",
                   help="training state (.npz: weights, step scales, Adam moments, step count, "
                        "epoch, shuffling RNG) written after every epoch and resumed from when "
                        "it exists")
    return p.parse_args(argv)


def save_state(path, tr, epoch, rng, history):
    """Weights, step scales, their Adam moments and step count, the next epoch, the
    shuffling RNG state and the loss history, written atomically."""
    cpu = lambda t: t.detach().cpu().numpy()
    tmp = path + ".tmp.npz"
    np.savez(tmp, theta=cpu(tr.theta), m=cpu(tr.m), v=cpu(tr.v), scales=cpu(tr.scales),
             sm=cpu(tr.sm), sv=cpu(tr.sv), t=tr.t, epoch=epoch,
             rng=json.dumps(rng.bit_generator.state), history=json.dumps(history))
    os.replace(tmp, path)


def load_state(path, tr, rng):
    """Restore what save_state wrote; returns (next epoch, history)."""
    with np.load(path) as z:
        for name in ("theta", "m", "v", "scales", "sm", "sv"):
            getattr(tr, name).copy_(torch.as_tensor(z[name]))
        tr.t = int(z["t"])
        rng.bit_generator.state = json.loads(str(z["rng"]))
        return int(z["epoch"]), json.loads(str(z["history"]))


class Trainer:
    def __init__(self, a, cosmo=None):
        self.a = a
        self.cosmo = cosmo or Cosmology()
        self.dev = torch.device("cuda", torch.cuda.current_device())
        ng = a.ptcl
        # the 2 % criterion is judged on k <= k_Nyq/2, i.e. shells |n| <= Ng/4
        self.n_bins = a.n_bins or ng // 4
        lpt = getattr(a, "lpt_order", 1)
        self.coarse = api.PMContext(api.make_config(a.ptcl, ng, a.box, a.steps, filter=True,
                                                    lpt_order=lpt), self.cosmo, device=self.dev)
        first = getattr(a, "first_seed", 0)
        self.seeds = list(range(first, first + a.train_seeds + a.heldout))
        self.noise, self.disp_f, self.pk_f = {}, {}, {}
        fine = api.PMContext(api.make_config(a.ptcl, a.fine_factor * ng, a.box, a.steps,
                                             lpt_order=lpt), self.cosmo, device=self.dev)
        for s in self.seeds:
            self.noise[s] = torch.as_tensor(white_noise(a.ptcl, s), dtype=torch.float32,
                                            device=self.dev)
            disp, _, _ = fine.forward(self.noise[s], want_density=False)
            self.disp_f[s] = disp
            self.pk_f[s] = self.coarse.power_spectrum(self.coarse.density(disp), self.n_bins)[1]
        fine.close()
        del fine
        torch.cuda.empty_cache()
        w0 = np.load(a.init) if a.init else mlp_init(a.init_seed, zero_last=True)
        self.theta = torch.as_tensor(np.asarray(w0, dtype=np.float32), device=self.dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grads = torch.empty((a.batch, N_FILTER_PARAMS), dtype=torch.float32, device=self.dev)
        self.train_filter = a.train in ("filter", "both")
        self.train_schedule = a.train in ("schedule", "both")
        ns = 3 * a.steps
        self.scales = torch.ones(ns, dtype=torch.float32, device=self.dev)
        self.sm = torch.zeros_like(self.scales)
        self.sv = torch.zeros_like(self.scales)
        self.sgrads = torch.empty((a.batch, ns), dtype=torch.float32, device=self.dev)
        self.t = 0

    def step(self, batch):
        """One Adam step on the mean gradient (filter weights and/or step scales)
        of the runs in `batch`."""
        c = self.coarse
        c.set_filter(self.theta)
        c.set_step_scales(self.scales.cpu().numpy())
        lp = ld = 0.0
        for i, s in enumerate(batch):
            disp, _, dens = c.forward(self.noise[s])
            Lp, g_dens = c.loss_pk(dens, self.pk_f[s], self.n_bins)
            Ld, g_disp = c.loss_disp(disp, self.disp_f[s], weight=self.a.w_disp)
            c.adjoint(g_dens=g_dens, g_disp=g_disp,
                      g_filter_out=self.grads[i] if self.train_filter else None)
            if self.train_schedule:
                self.sgrads[i].copy_(torch.as_tensor(c.step_gradients().reshape(-1),
                                                     dtype=torch.float32))
            lp += Lp
            ld += Ld
        self.t += 1
        if self.train_filter:
            c.adam(self.theta, self.grads[:len(batch)], self.m, self.v, self.t, lr=self.a.lr)
        if self.train_schedule:
            c.adam(self.scales, self.sgrads[:len(batch)], self.sm, self.sv, self.t,
                   lr=self.a.lr_schedule)
        return lp / len(batch), ld / len(batch)

    def evaluate(self, theta, seeds, scales=None):
        """P(k) error against the fine run on the common coarse mesh, per held-out
        seed: max over shells with k <= k_Nyq/2 of |P/P_fine - 1|; and the RMS
        position error in coarse cells."""
        c = self.coarse
        c.set_filter(theta)
        c.set_step_scales(np.ones(3 * self.a.steps) if scales is None
                          else scales.cpu().numpy())
        half = self.a.ptcl // 4   # shell b ~ |n|; k_Nyq/2 is |n| = Ng/4
        errs, rms, ratios = [], [], []
        for s in seeds:
            disp, _, dens = c.forward(self.noise[s])
            pk = c.power_spectrum(dens, self.n_bins)[1]
            r = pk / self.pk_f[s]
            ratios.append(r)
            errs.append(float(np.max(np.abs(r[:half] - 1.0))))
            L, _ = c.loss_disp(disp, self.disp_f[s], want_grad=False)
            rms.append(float(np.sqrt(L)))
        return {"pk_maxerr_half_nyq_mean": float(np.mean(errs)), "pk_maxerr_per_seed": errs,
                "pos_rms_cells_mean": float(np.mean(rms)),
                "pk_ratio_mean": np.mean(ratios, axis=0).tolist()}


def main(argv=None):
    a = parse(argv)
    t0 = time.perf_counter()
    tr = Trainer(a)
    print(f"targets: {len(tr.seeds)} fine runs ({a.ptcl}^3 on {a.fine_factor * a.ptcl}^3) in "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    train = tr.seeds[:a.train_seeds]
    held = tr.seeds[a.train_seeds:]
    plain = torch.as_tensor(mlp_init(a.init_seed, zero_last=True), dtype=torch.float32,
                            device=tr.dev)
    history = []
    rng = np.random.Generator(np.random.PCG64(12345))
    start = 0
    if a.state and os.path.exists(a.state):
        start, history = load_state(a.state, tr, rng)
        print(f"resumed from {a.state} at epoch {start} (Adam step {tr.t})", flush=True)
    t1 = time.perf_counter()
    for ep in range(start, a.epochs):
        order = rng.permutation(train)
        lps, lds = [], []
        for b0 in range(0, len(order), a.batch):
            lp, ld = tr.step([int(s) for s in order[b0:b0 + a.batch]])
            lps.append(lp)
            lds.append(ld)
        history.append({"epoch": ep, "loss_pk": float(np.mean(lps)), "loss_disp": float(np.mean(lds))})
        if a.state:
            save_state(a.state, tr, ep + 1, rng, history)
        if ep % a.log_every == 0 or ep == a.epochs - 1:
            print(f"epoch {ep:4d}  loss_pk {np.mean(lps):.4e}  loss_disp {np.mean(lds):.4e}  "
                  f"{time.perf_counter() - t1:.1f} s", flush=True)
    train_s = time.perf_counter() - t1
    report = {"config": vars(a), "train_seconds": train_s, "adam_steps": tr.t, "history": history}
    if held:
        report["heldout_plain"] = tr.evaluate(plain, held)
        report["heldout_learned"] = tr.evaluate(tr.theta, held, tr.scales)
        print(f"held-out max |P/P_fine - 1| (k <= k_Nyq/2): plain "
              f"{report['heldout_plain']['pk_maxerr_half_nyq_mean']:.4f}, learned "
              f"{report['heldout_learned']['pk_maxerr_half_nyq_mean']:.4f}; position rms cells: "
              f"plain {report['heldout_plain']['pos_rms_cells_mean']:.4f}, learned "
              f"{report['heldout_learned']['pos_rms_cells_mean']:.4f}", flush=True)
    if a.out:
        np.save(a.out, tr.theta.cpu().numpy().astype(np.float32))
    if a.out_schedule:
        np.save(a.out_schedule, tr.scales.cpu().numpy().reshape(3, a.steps).astype(np.float64))
    if tr.train_schedule:
        report["step_scales"] = tr.scales.cpu().numpy().reshape(3, a.steps).tolist()
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main()
