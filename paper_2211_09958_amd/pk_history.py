"""Time history of the coarse-to-fine power-spectrum ratio (plain and learned force).

For the filter-training geometry (Np^3 particles, box L, N steps linear in a from
1/64 to 1), runs the same seeded initial conditions on a coarse mesh and on finer
meshes, stopped after n steps for several n (each stop is a run of n steps with
a_stop = a_n, i.e. exactly the first n steps of the full schedule), assigns both
final particle sets to the coarse mesh and reports the mean over seeds of
P_coarse/P_fine in the lowest shells: where and when the coarse run's excess or
deficit of power appears.  With --weights the coarse run also uses a learned
filter (and --scales learned step scales, which only apply at the full N).

    python -m paper_2211_09958_amd.pk_history --ptcl 128 --box 128 --steps 31 \
        --fine 512 256 --seeds 56 57 58 59 --stops 4 8 16 24 31 --report hist.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

from . import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
from synthetic import Cosmology, white_noise  # noqa: E402  (seeded inputs only)


def parse(argv=None):
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    p.add_argument("--ptcl", type=int, default=128)
    p.add_argument("--box", type=float, default=128.0)
    p.add_argument("--steps", type=int, default=31)
    p.add_argument("--coarse", type=int, default=0, help="coarse mesh (0: Np)")
    p.add_argument("--fine", type=int, nargs="+", default=[512, 256])
    p.add_argument("--seeds", type=int, nargs="+", default=[56, 57, 58, 59, 60, 61, 62, 63])
    p.add_argument("--stops", type=int, nargs="+", default=[2, 4, 8, 12, 16, 20, 24, 28, 31])
    p.add_argument("--shells", type=int, default=8)
    p.add_argument("--weights", default="", help="learned filter for the coarse run (.npy)")
    p.add_argument("--report", default="")
    return p.parse_args(argv)


def main(argv=None):
    a = parse(argv)
    dev = torch.device("cuda", torch.cuda.current_device())
    co = Cosmology()
    ng = a.coarse or a.ptcl
    a0 = 1.0 / 64
    da = (1.0 - a0) / a.steps
    theta = None
    if a.weights:
        theta = torch.as_tensor(np.load(a.weights), dtype=torch.float32, device=dev)
    rows = []
    for n in a.stops:
        a_n = a0 + n * da
        mk = lambda mesh, filt=False: api.PMContext(
            api.make_config(a.ptcl, mesh, a.box, n, a_stop=a_n, filter=filt), co, device=dev)
        coarse = mk(ng, theta is not None)
        if theta is not None:
            coarse.set_filter(theta)
        fines = {m: mk(m) for m in a.fine}
        ratios = {m: [] for m in a.fine}
        for s in a.seeds:
            w = torch.as_tensor(white_noise(a.ptcl, s), dtype=torch.float32, device=dev)
            pc = coarse.power_spectrum(coarse.forward(w)[2], a.shells)[1]
            for m, f in fines.items():
                disp = f.forward(w, want_density=False)[0]
                pf = coarse.power_spectrum(coarse.density(disp), a.shells)[1]
                ratios[m].append(pc / pf)
        row = {"steps": n, "a": a_n}
        for m in a.fine:
            row[f"ratio_vs_{m}"] = np.mean(ratios[m], axis=0).round(4).tolist()
        rows.append(row)
        print(f"n = {n:3d}  a = {a_n:.3f}  " + "  ".join(
            f"vs {m}: " + " ".join(f"{x:.3f}" for x in row[f'ratio_vs_{m}'][:4])
            for m in a.fine), flush=True)
        for c in [coarse, *fines.values()]:
            c.close()
    rep = {"ptcl": a.ptcl, "box": a.box, "coarse_mesh": ng, "fine_meshes": a.fine,
           "schedule_steps": a.steps, "seeds": a.seeds, "weights": a.weights or None,
           "shells": "round(|n|) = 1.., P on the coarse mesh", "history": rows}
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


if __name__ == "__main__":
    main()
