"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import functools

import numpy as np
import torch

from oracle import pm as opm
from paper_2211_09958_amd import api
from synthetic import Cosmology, Workload

CO = Cosmology()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


@functools.lru_cache(maxsize=None)
def context(ptcl_grid, mesh, box, n_steps, checkpoint_every=0, filter=False, lpt_order=1):
    cfg = api.make_config(ptcl_grid, mesh, box, n_steps, checkpoint_every=checkpoint_every,
                          filter=filter, lpt_order=lpt_order)
    return api.PMContext(cfg, CO)


def ctx_for(w: Workload, **kw):
    return context(w.ptcl_grid, w.mesh, w.box, w.n_steps, **kw)


def setup_for(w: Workload, lpt_order=1):
    return opm.Setup(w.ptcl_grid, w.mesh, w.box, w.n_steps, CO, w.a_start, w.a_stop, lpt_order)


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def periodic_cells(a, b, box, mesh):
    """Per-particle minimum-image distance between displacement sets, in cells."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    d -= box * np.round(d / box)
    return np.sqrt(np.sum(d * d, axis=1)) * mesh / box
