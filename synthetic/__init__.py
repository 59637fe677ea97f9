"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds workload *definitions* (sizes, seeds, cosmological parameters)
and the white-noise generator only.  It contains none of the particle-mesh
arithmetic: both the FP64 oracle and the HIP path receive the same noise array
as an input, so neither side re-implements the random draw.

The white noise is the Gaussian random field from which the initial conditions
are synthesised (pmwd paper, Summary: forward modelling from initial conditions;
workload statement: "seeded Gaussian white noise").  It is drawn in FP64 with
NumPy's PCG64 stream, C order with the last axis fastest, then handed to each
side in the precision that side computes in.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Cosmology:
    """Flat LambdaCDM parameters (no radiation)."""
    omega_m: float = 0.3
    omega_b: float = 0.05
    h: float = 0.7
    sigma8: float = 0.8
    n_s: float = 0.96
    T_cmb: float = 2.7255


@dataclass(frozen=True)
class Workload:
    """One simulation geometry.

    ptcl_grid  particles per side (Np); the particle lattice has Np**3 points
    mesh       mesh cells per side (Ng)
    box        comoving box side L in Mpc/h
    n_steps    number of kick-drift-kick steps, linear in scale factor a
    a_start, a_stop   integration range in a
    checkpoint_every  0 for the pure reverse-time adjoint
    """
    name: str
    ptcl_grid: int
    mesh: int
    box: float
    n_steps: int
    a_start: float = 1.0 / 64
    a_stop: float = 1.0
    checkpoint_every: int = 0
    cosmo: Cosmology = field(default_factory=Cosmology)

    @property
    def n_particles(self) -> int:
        return self.ptcl_grid ** 3

    @property
    def cell(self) -> float:
        return self.box / self.mesh

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five geometries of the evaluation (sizes only).
SMALL = Workload("pm-32p-64m-10s", ptcl_grid=32, mesh=64, box=64.0, n_steps=10)
MEDIUM = Workload("pm-256p-512m-63s", ptcl_grid=256, mesh=512, box=256.0, n_steps=63)
LARGE = Workload("pm-512p-1024m-63s", ptcl_grid=512, mesh=1024, box=512.0, n_steps=63)
LARGE_CKPT = LARGE.with_(name="pm-512p-1024m-63s-ckpt16", checkpoint_every=16)
FILTER_COARSE = Workload("pm-128p-128m-31s", ptcl_grid=128, mesh=128, box=128.0, n_steps=31)
FILTER_FINE = Workload("pm-128p-512m-31s", ptcl_grid=128, mesh=512, box=128.0, n_steps=31)
FILTER_PROD = Workload("pm-512p-512m-63s", ptcl_grid=512, mesh=512, box=512.0, n_steps=63)

WORKLOADS = {w.name: w for w in
             (SMALL, MEDIUM, LARGE, LARGE_CKPT, FILTER_COARSE, FILTER_FINE, FILTER_PROD)}


def white_noise(ptcl_grid: int, seed: int) -> np.ndarray:
    """Unit-variance Gaussian white noise on the Np**3 lattice, FP64, C order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((ptcl_grid, ptcl_grid, ptcl_grid))


def uniform(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Seeded uniform draws (FP64) used for positions and cotangents in tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape)


def normal(shape, seed: int) -> np.ndarray:
    """Seeded standard-normal draws (FP64) used for cotangents and directions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape)


MLP_HIDDEN = 64
MLP_N_PARAMS = MLP_HIDDEN * 2 + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1


def mlp_init(seed: int = 0, zero_last: bool = True) -> np.ndarray:
    """Seeded initial weights of the 2-64-64-1 filter network, FP64, packed
    W1[64,2], b1[64], W2[64,64], b2[64], W3[1,64], b3[1] (output index first).

    Hidden layers draw uniform(+-1/sqrt(fan_in)); the last layer is zero by
    default so that the filter starts out as the plain force (f = 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_out, fan_in in ((MLP_HIDDEN, 2), (MLP_HIDDEN, MLP_HIDDEN), (1, MLP_HIDDEN)):
        bound = 1.0 / np.sqrt(fan_in)
        w = rng.uniform(-bound, bound, (fan_out, fan_in))
        b = rng.uniform(-bound, bound, fan_out)
        if fan_out == 1 and zero_last:
            w, b = np.zeros_like(w), np.zeros_like(b)
        parts += [w.reshape(-1), b]
    return np.concatenate(parts)
