"""FP64 CPU oracle for the particle-mesh force step and its reverse-time adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, tables or constants with the HIP
library; the only common input is the seeded noise from ``synthetic``.

Method (pmwd paper, Summary and Statement of Need): a cosmological
particle-mesh (PM) N-body simulation whose gradients come from the adjoint
method, evolving the dual equations backward in time with the forward states
recovered by reverse time integration, discretize-then-optimize so that the
gradient follows the same discrete trajectory as the forward run.  The paper
prints no equations; every formula here is standard published physics written
out plainly and pinned by the tests under ``tests/`` (closed forms, brute-force
DFTs, invariants, finite differences).  Where the paper is silent, each module's
docstring states the reading it takes.

Modules
  cosmology  background E(a), linear growth D, G, Eisenstein-Hu no-wiggle
             transfer function, sigma_8 normalisation, KDK coefficients
  mesh       cloud-in-cell scatter/gather/gradient, spectral Poisson force,
             power spectrum and its transpose
  mlp        the 2-64-64-1 SiLU force filter, forward and backward
  lpt        second-order (2LPT) initial-condition term, its transpose and
             Omega_m tangent
  pm         initial conditions, KDK time stepping, discrete adjoint over a
             stored trajectory, gradients w.r.t. noise, Omega_m, sigma_8 and
             filter weights; the filter-training losses
"""
