"""Benchmark: forward + reverse-time adjoint particle-steps/s on one MI355X.

One step = one whole pass of the hot path over one batch: Zel'dovich ICs from
seeded white noise, 63 KDK steps of the PM force (CIC scatter, 3-D real FFT,
Poisson gradient, 3 inverse FFTs, CIC gather, kick/drift), the MSE loss against
a second seeded run, and the reverse-time adjoint back to dL/dnoise,
dL/dOmega_m and dL/dsigma_8.  Throughput = particles * time steps * K / time
of K such passes, with all inputs resident in HBM.

Prints one JSON line (see the keys below).  `--gpus N` with N > 1 exits: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adjoint particle-steps/s at 512³/1024³; learned vs plain speed at 2% P(k)"
PEAK_HBM_GBS = 8000.0
CPU_STEPS = 10          # oracle sample: about 10-20 s on a 16-core host
# trained against the 2x-finer mesh, the resolution of the plain run it is compared with
WEIGHTS = os.path.join(ROOT, "paper_2211_09958_amd", "weights", "filter_128p_128m_to_256m.npy")
# per-step KDK scales trained at 63 steps (alone, and jointly with a filter)
SCHEDULE = os.path.join(ROOT, "paper_2211_09958_amd", "weights",
                        "schedule_128p_128m_63s_to_256m.npy")
JOINT = (os.path.join(ROOT, "paper_2211_09958_amd", "weights", "joint_filter_128p_128m_63s_to_256m.npy"),
         os.path.join(ROOT, "paper_2211_09958_amd", "weights", "joint_schedule_128p_128m_63s_to_256m.npy"))
FAMILY_KERNELS = {
    "fft_strided": ["k_fft_strided", "k_fft_y_split", "k_fft_y_merge"], "fft_x": ["k_fft_x_r2c", "k_fft_x_c2r"],
    "grad_z": ["k_grad_z"], "grad_adj_z": ["k_grad_adj_z"],
    "scatter": ["k_scatter_tile<16, false>"], "scatter_vec": ["k_scatter_tile<16, true>"],
    "gather": ["k_gather_tile<16, 0>"], "unkick_vjp": ["k_gather_tile<16, 2>"],
    "wgrad": ["k_gather_tile<16, 3>"],
    "bin": ["k_bin_count", "k_scan_local", "k_scan_bsum", "k_scan_add", "k_permute"],
}


def parse():
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="pm-512p-1024m-63s")
    p.add_argument("--checkpoint-every", type=int, default=16)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-pure-variant", action="store_true")
    p.add_argument("--no-medium", action="store_true",
                   help="skip the 256^3-particle / 512^3-mesh run reported beside the headline")
    p.add_argument("--no-learned", action="store_true",
                   help="skip the learned-filter 512^3-mesh vs plain 1024^3-mesh comparison")
    p.add_argument("--weights", default=WEIGHTS, help="trained filter weights (.npy)")
    p.add_argument("--no-lpt2", action="store_true",
                   help="skip the run from second-order (2LPT) initial conditions")
    p.add_argument("--cpu-only", action="store_true", help="only the oracle CPU baseline")
    p.add_argument("--calib-copy-gib", type=float, default=0.0,
                   help="also run one device copy of this many GiB (HBM counter calibration)")
    return p.parse_args()


def progress(msg):
    """One line per finished piece of work, on stderr (stdout carries the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline():
    """The FP64 oracle, as it stands, on a bounded sample of the workload: 64^3
    particles on a 128^3 mesh in a 64 Mpc/h box (the headline's cell size and
    particle spacing), CPU_STEPS KDK steps, forward + MSE loss + stored-trajectory adjoint."""
    import numpy as np
    from oracle import mesh as M
    from oracle import pm as opm
    from synthetic import Cosmology, white_noise
    cores = len(os.sched_getaffinity(0))
    M.WORKERS = cores
    st = opm.Setup(64, 128, 64.0, CPU_STEPS, Cosmology())
    target = opm.forward(white_noise(64, 1), st).dens
    t0 = time.perf_counter()
    run = opm.forward(white_noise(64, 0), st)
    _, gd = opm.mse_loss(run.dens, target)
    opm.adjoint(run, white_noise(64, 0), g_dens=gd)
    dt = time.perf_counter() - t0
    return {"value": 64 ** 3 * CPU_STEPS / dt, "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": "64^3 particles, 128^3 mesh, box 64 Mpc/h (same cell size and particle "
                      f"spacing as 512^3/1024^3), {CPU_STEPS} KDK steps, fwd + MSE loss + adjoint, FP64; "
                      f"scipy.fft with {cores} workers, CIC single-threaded numpy; {dt:.1f} s"}


def traffic_for(family, alg_bytes_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary: the family's
    measured/algorithmic byte ratio (FETCH_SIZE + WRITE_SIZE, calibrated) times its
    algorithmic bytes per launch here.  None when the summary is absent or was taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_2211_09958_amd.rocprof_summary import sources_sha256
    with open(path) as f:
        data = json.load(f)
    entry = data.get("families", {}).get(family)
    if not entry or entry.get("sources_sha256") != sources_sha256(family):
        return None
    return entry["measured_over_algorithmic"] * alg_bytes_per_launch


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.cpu_only:
        print(json.dumps({"cpu_baseline": cpu_baseline()}))
        return

    import numpy as np
    import torch

    from paper_2211_09958_amd import api
    from synthetic import WORKLOADS, Cosmology, white_noise

    w = WORKLOADS[args.workload]
    co = Cosmology()
    P = w.ptcl_grid ** 3

    def make(ck):
        return api.PMContext(api.config_from_workload(w, checkpoint_every=ck, timing=True), co,
                             device="cuda:0")

    pm = make(args.checkpoint_every)
    noise = torch.as_tensor(white_noise(w.ptcl_grid, 0), dtype=torch.float32, device="cuda:0")
    _, _, target = pm.forward(torch.as_tensor(white_noise(w.ptcl_grid, 1), dtype=torch.float32,
                                              device="cuda:0"))
    target = target.clone()

    last = {}

    def step(ctx):
        disp, mom, dens = ctx.forward(noise)
        _, g = ctx.loss_mse(dens, target)
        g_noise, g_cosmo, _ = ctx.adjoint(g_dens=g)
        last["disp"] = disp
        return g_cosmo

    for i in range(args.warmup):
        step(pm)
        progress(f"warm-up run {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    pm.reset_stats()
    if args.calib_copy_gib > 0:
        # a device copy of known size, for calibrating HBM byte counters under a profiler
        n = int(args.calib_copy_gib * 2 ** 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # one-element uint8 fills mark the timed region for kernel-trace summaries
    marker = torch.empty(1, dtype=torch.uint8, device="cuda:0")
    marker.fill_(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        g_cosmo = step(pm)   # returns host values: the stream has synchronised
        progress(f"timed run {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    marker.fill_(2)
    torch.cuda.synchronize()
    st = pm.stats()
    value = P * w.n_steps * args.steps / dt

    fams = st["kernels"]
    dom = max(fams, key=lambda k: fams[k]["ms"])
    f = fams[dom]
    achieved = f["bytes"] / (f["ms"] * 1e-3) / 1e9 if f["ms"] > 0 else 0.0
    per_launch = f["bytes"] / max(f["launches"], 1)
    traffic = traffic_for(dom, per_launch)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                "kernel": dom, "kernel_symbols": FAMILY_KERNELS.get(dom, []),
                "avg_launch_ms": f["ms"] / max(f["launches"], 1),
                "algorithmic_bytes_per_launch": per_launch}
    total_ms = sum(v["ms"] for v in fams.values())
    breakdown = {}
    for k, v in fams.items():
        if v["ms"] <= 0:
            continue
        gbps = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        e = {"ms_per_step": v["ms"] / args.steps, "share": v["ms"] / total_ms,
             "GBps": gbps, "frac_alg": gbps / PEAK_HBM_GBS}
        # counter bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE) where the committed
        # summary was taken on the current kernel sources
        launches = max(v["launches"], 1)
        t = traffic_for(k, v["bytes"] / launches) if v["bytes"] > 0 else None
        if t is not None:
            e["frac_counter"] = t * launches / (v["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS
        breakdown[k] = e
    # the initial conditions and their adjoint (and the reconstruction checks)
    # are the "other" family: throughput of the time steps alone
    other_s = fams.get("other", {}).get("ms", 0.0) * 1e-3
    value_steps_only = P * w.n_steps * args.steps / (dt - other_s) if dt > other_s else None

    out = {"metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded white-noise LCDM ICs)",
           "config": {"workload": w.name if not args.checkpoint_every else
                      f"{w.name}-ckpt{args.checkpoint_every}",
                      "ptcl_grid": w.ptcl_grid, "mesh": w.mesh, "box": w.box,
                      "n_steps": w.n_steps, "checkpoint_every": args.checkpoint_every,
                      "loss": "MSE of final CIC density vs seed-1 run"},
           "roofline": roofline,
           "reconstruction": {"ic_rms_cells": st["ic_rms_cells"], "ic_max_cells": st["ic_max_cells"],
                              "ckpt_rms_cells": st["ckpt_rms_cells"]},
           "value_excluding_ics": value_steps_only,
           "grad_cosmo": list(g_cosmo), "kernel_breakdown": breakdown}

    if not args.no_pure_variant and args.checkpoint_every:
        del pm
        torch.cuda.empty_cache()
        pure = make(0)
        step(pure)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(pure)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        sp = pure.stats()
        out["pure_reverse"] = {"value": P * w.n_steps / dtp, "ms_per_step": dtp * 1e3,
                               "ic_rms_cells": sp["ic_rms_cells"],
                               "ic_max_cells": sp["ic_max_cells"]}
        progress("pure reverse-time variant done")
    if not args.no_medium and w.name == "pm-512p-1024m-63s":
        pm = pure = None
        torch.cuda.empty_cache()
        out["medium"] = medium_leg(args, co)
        progress("256^3/512^3 leg done")
    if not args.no_lpt2:
        pm = pure = None
        torch.cuda.empty_cache()
        out["lpt2"] = lpt2_leg(args, w, co, noise, target, fams, make)
        progress("2LPT leg done")
    if not args.no_learned and os.path.exists(args.weights) and w.name == "pm-512p-1024m-63s":
        pm = pure = None   # release the 1024^3 workspaces
        torch.cuda.empty_cache()
        out["learned_vs_plain"] = learned_vs_plain(args, co, noise, last["disp"], value)
        progress("learned-filter leg done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        progress("CPU baseline done")
    print(json.dumps(out))


def medium_leg(args, co):
    """The same forward + MSE loss + adjoint run at 256^3 particles / 512^3 mesh /
    box 256 / 63 steps (pure reverse time), seeds 0 (run) and 1 (target):
    1 warm-up, then `steps` timed runs."""
    import torch

    from paper_2211_09958_amd import api
    from synthetic import MEDIUM, white_noise
    w = MEDIUM
    pm = api.PMContext(api.config_from_workload(w), co, device="cuda:0")
    dev = lambda seed: torch.as_tensor(white_noise(w.ptcl_grid, seed), dtype=torch.float32,
                                       device="cuda:0")
    noise = dev(0)
    target = pm.forward(dev(1))[2].clone()

    def run():
        disp, mom, dens = pm.forward(noise)
        _, g = pm.loss_mse(dens, target)
        return pm.adjoint(g_dens=g)[1]

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g_cosmo = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = pm.stats()
    return {"workload": w.name, "value": w.ptcl_grid ** 3 * w.n_steps / dt,
            "unit": "particle-steps/s", "ms_per_run": dt * 1e3, "ic_max_cells": st["ic_max_cells"],
            "grad_cosmo": list(g_cosmo)}


def lpt2_leg(args, w, co, noise, target, plain_fams, make):
    """The same forward + adjoint run from 2LPT initial conditions: whole-run
    rate, the extra initial-condition time (the "other" kernel family holds the
    ICs, their adjoint and the reconstruction checks) and the time of the
    initial conditions alone, Zel'dovich vs 2LPT (HIP events, 5 calls each)."""
    import torch

    from paper_2211_09958_amd import api
    P = w.ptcl_grid ** 3
    cfg = api.config_from_workload(w, checkpoint_every=args.checkpoint_every, timing=True)
    cfg.flags |= api._lib.PM_F_2LPT
    pm = api.PMContext(cfg, co, device="cuda:0")

    def run():
        disp, mom, dens = pm.forward(noise)
        _, g = pm.loss_mse(dens, target)
        return pm.adjoint(g_dens=g)[1]

    run()
    torch.cuda.synchronize()
    pm.reset_stats()
    t0 = time.perf_counter()
    g_cosmo = run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = pm.stats()
    other = st["kernels"].get("other", {}).get("ms", 0.0)
    plain_other = plain_fams.get("other", {}).get("ms", 0.0) / args.steps
    ic_ms = {}
    for name, ctx in (("zeldovich", make(args.checkpoint_every)), ("2lpt", pm)):
        ctx.initial_conditions(noise)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            ctx.initial_conditions(noise)
        e1.record()
        torch.cuda.synchronize()
        ic_ms[name] = e0.elapsed_time(e1) / 5
        del ctx
    return {"value": P * w.n_steps / dt, "unit": "particle-steps/s", "ms_per_run": dt * 1e3,
            "other_family_ms_per_run": other, "plain_other_family_ms_per_run": plain_other,
            "initial_conditions_ms": ic_ms, "ic_max_cells": st["ic_max_cells"],
            "ic_mom_rel_rms": st["ic_mom_rel_rms"], "grad_cosmo": list(g_cosmo)}


def learned_vs_plain(args, co, noise, disp_plain, plain_value):
    """The learned-filter run on a 512^3 mesh (512^3 particles, box 512, 63 steps,
    forward + MSE loss + adjoint including the filter gradient) timed like the
    headline, and its P(k) against the plain 1024^3-mesh run of the same seed, both
    measured on the 512^3 mesh; the plain 512^3-mesh run is shown beside it."""
    import numpy as np
    import torch

    from paper_2211_09958_amd import api
    from synthetic import FILTER_PROD, white_noise

    w = FILTER_PROD
    P = w.ptcl_grid ** 3
    theta = torch.as_tensor(np.load(args.weights).astype(np.float32), device="cuda:0")
    lp = api.PMContext(api.config_from_workload(w, filter=True, timing=True), co,
                       device="cuda:0")
    lp.set_filter(theta)
    _, _, target = lp.forward(torch.as_tensor(white_noise(w.ptcl_grid, 1), dtype=torch.float32,
                                              device="cuda:0"))
    target = target.clone()

    def step():
        disp, mom, dens = lp.forward(noise)
        _, g = lp.loss_mse(dens, target)
        lp.adjoint(g_dens=g, want_filter=True)
        return dens

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lp.reset_stats()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dens = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = P * w.n_steps * args.steps / dt
    fams = lp.stats()["kernels"]
    breakdown = {k: round(v["ms"] / args.steps, 1) for k, v in
                 sorted(fams.items(), key=lambda kv: -kv[1]["ms"]) if v["ms"] > 0}
    half = w.mesh // 4                     # shells with k <= k_Nyq / 2
    pk_ref = lp.power_spectrum(lp.density(disp_plain), w.mesh // 2)[1]
    pk_learned = lp.power_spectrum(dens, w.mesh // 2)[1]
    plain = api.PMContext(api.config_from_workload(w), co, device="cuda:0")
    pk_plain = plain.power_spectrum(plain.forward(noise)[2], w.mesh // 2)[1]
    err = lambda pk: float(np.max(np.abs(pk[:half] / pk_ref[:half] - 1.0)))
    worst = lambda pk: int(np.argmax(np.abs(pk[:half] / pk_ref[:half] - 1.0))) + 1
    e_l, e_p = err(pk_learned), err(pk_plain)
    # the temporal half: learned per-step scales, alone and with their jointly
    # trained filter (accuracy only: the scales leave the cost of a run unchanged)
    temporal = {}
    if os.path.exists(SCHEDULE):
        plain.set_step_scales(np.load(SCHEDULE))
        pk = plain.power_spectrum(plain.forward(noise)[2], w.mesh // 2)[1]
        temporal["schedule_only_512"] = {"pk_maxerr_to_half_nyq": err(pk), "worst_shell": worst(pk),
                                         "scales": os.path.relpath(SCHEDULE, ROOT)}
    if all(os.path.exists(f) for f in JOINT):
        lp.set_filter(torch.as_tensor(np.load(JOINT[0]).astype(np.float32), device="cuda:0"))
        lp.set_step_scales(np.load(JOINT[1]))
        pk = lp.power_spectrum(lp.forward(noise)[2], w.mesh // 2)[1]
        temporal["filter_and_schedule_512"] = {"pk_maxerr_to_half_nyq": err(pk),
                                               "worst_shell": worst(pk),
                                               "weights": [os.path.relpath(f, ROOT) for f in JOINT]}
    return {"workload": f"{w.name} learned f(|k|,a)", "value": value, "unit": "particle-steps/s",
            "ms_per_step": dt / args.steps * 1e3, "speedup_vs_plain_1024": value / plain_value,
            "pk_maxerr_to_half_nyq": {"learned_512": e_l, "plain_512": e_p},
            "worst_shell": {"learned_512": worst(pk_learned), "plain_512": worst(pk_plain)},
            "pk_ratio_learned_shells_1_16": [round(float(x), 4) for x in
                                             (pk_learned[:16] / pk_ref[:16])],
            "reference": "plain 512^3 particles on the 1024^3 mesh, same seed; all P(k) on the "
                         "512^3 mesh",
            "within_2pct": e_l <= 0.02, "weights": os.path.relpath(args.weights, ROOT),
            "temporal": temporal, "kernel_ms_per_run": breakdown}


if __name__ == "__main__":
    main()
