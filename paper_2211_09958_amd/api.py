"""Python binding of libpmx: argument marshalling over the C ABI only.

PyTorch provides device memory (the workspace and all inputs/outputs are torch
tensors, so torch's caching allocator is the only allocator) and the stream
(the current torch stream).  Every step of the simulation runs in the HIP
kernels behind the C ABI.
"""
from __future__ import annotations

import ctypes
import math
from ctypes import byref, c_double, c_int, c_void_p

import torch

from . import _lib
from ._lib import Config, Cosmology, N_FILTER_PARAMS, PMError, Stats, check


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _cosmo_struct(c) -> Cosmology:
    return Cosmology(float(c.omega_m), float(c.omega_b), float(c.h), float(c.sigma8),
                     float(c.n_s), float(getattr(c, "T_cmb", 2.7255)))


def make_config(ptcl_grid, mesh, box, n_steps, a_start=1.0 / 64, a_stop=1.0,
                checkpoint_every=0, filter=False, timing=False, lpt_order=1) -> Config:
    """pm_config; lpt_order 2 selects 2LPT initial conditions (PM_F_2LPT)."""
    if lpt_order not in (1, 2):
        raise ValueError("lpt_order must be 1 or 2")
    flags = (_lib.PM_F_TIMING if timing else 0) | (_lib.PM_F_2LPT if lpt_order == 2 else 0)
    return Config(int(ptcl_grid), int(mesh), float(box), float(a_start), float(a_stop),
                  int(n_steps), int(checkpoint_every), int(bool(filter)), flags)


def config_from_workload(w, filter=False, checkpoint_every=None, timing=False) -> Config:
    return make_config(w.ptcl_grid, w.mesh, w.box, w.n_steps, w.a_start, w.a_stop,
                       w.checkpoint_every if checkpoint_every is None else checkpoint_every,
                       filter, timing)


def workspace_bytes(cfg: Config) -> int:
    lib = _lib.load()
    st = c_int(0)
    n = lib.pm_workspace_bytes(byref(cfg), byref(st))
    check(st.value)
    return int(n)


def host_tables(cfg: Config, cosmo):
    """FP64 host tables of the library (no GPU): coefficients, their Omega_m
    derivatives, growth (D, dD/da, G at a_n) and P_lin on the particle grid."""
    import numpy as np
    N = cfg.n_steps
    co = np.zeros(3 * N + 2)
    dco = np.zeros(3 * N + 2)
    gr = np.zeros(3 * (N + 1))
    pk = np.zeros(3 * (cfg.ptcl_grid // 2) ** 2 + 1)
    cs = _cosmo_struct(cosmo)
    p = lambda a: a.ctypes.data_as(c_void_p)
    check(_lib.load().pm_host_tables(byref(cfg), byref(cs), p(co), p(dco), p(gr), p(pk)))
    return {"kick_a": co[:N], "drift": co[N:2 * N], "kick_b": co[2 * N:3 * N],
            "D0": co[3 * N], "G0": co[3 * N + 1],
            "d_kick_a": dco[:N], "d_drift": dco[N:2 * N], "d_kick_b": dco[2 * N:3 * N],
            "d_D0": dco[3 * N], "d_G0": dco[3 * N + 1],
            "D": gr[:N + 1], "dD": gr[N + 1:2 * N + 2], "G": gr[2 * N + 2:], "pk": pk}


def state_units(cfg: Config):
    """Fixed-point units of the particle state (no GPU): position unit, momentum
    unit and momentum range (the largest representable |p|)."""
    import numpy as np
    out = np.zeros(3)
    check(_lib.load().pm_state_units(byref(cfg), out.ctypes.data_as(c_void_p)))
    return {"position_unit": out[0], "momentum_unit": out[1], "momentum_range": out[2]}


def lpt2_growth(cfg: Config, cosmo):
    """Second-order growth at a_start (no GPU): D2, G2 and their Omega_m derivatives."""
    import numpy as np
    out = np.zeros(4)
    cs = _cosmo_struct(cosmo)
    check(_lib.load().pm_lpt2_growth(byref(cfg), byref(cs), out.ctypes.data_as(c_void_p)))
    return {"D2": out[0], "G2": out[1], "d_D2": out[2], "d_G2": out[3]}


def power_spectrum_noalloc(dens, box, n_bins=None, stream=None):
    """pm_power_spectrum_noalloc: P(k) of an [Ng]^3 float32 overdensity on the
    current device without a context (no device allocation by the library;
    Ng <= PM_NOALLOC_MAX_MESH).  Returns (k, P, modes) as host arrays."""
    import numpy as np
    if dens.dtype != torch.float32 or not dens.is_contiguous() or dens.dim() != 3:
        raise ValueError("dens must be a contiguous [Ng]^3 float32 tensor")
    ng = dens.shape[0]
    n_bins = ng // 2 if n_bins is None else n_bins
    k, pk, nm = np.zeros(n_bins), np.zeros(n_bins), np.zeros(n_bins)
    s = torch.cuda.current_stream(dens.device) if stream is None else stream
    p = lambda a: a.ctypes.data_as(c_void_p)
    with torch.cuda.device(dens.device):
        check(_lib.load().pm_power_spectrum_noalloc(_ptr(dens), ng, float(box), n_bins, p(k),
                                                    p(pk), p(nm), c_void_p(s.cuda_stream)))
    return k, pk, nm


class PMContext:
    """One simulation geometry on one GPU (a pm_ctx plus its torch workspace)."""

    def __init__(self, cfg: Config, cosmo, device="cuda"):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libpmx needs a ROCm GPU (torch.cuda is unavailable)")
        self.cfg = cfg
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.np = cfg.ptcl_grid
        self.ng = cfg.mesh
        self.P = self.np ** 3
        self._cosmo = _cosmo_struct(cosmo)
        self.cosmo = cosmo
        nbytes = workspace_bytes(cfg)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        self.ctx = c_void_p()
        # number of pm_forward calls on this context: the adjoint differentiates
        # the most recent one, so an autograd graph remembers which run it owns
        self.forward_count = 0
        check(self.lib.pm_init(byref(cfg), byref(self._cosmo), _ptr(self.workspace), nbytes,
                               c_void_p(self.stream.cuda_stream), byref(self.ctx)))

    # -- helpers -------------------------------------------------------
    def _check(self, rc):
        check(rc, self.ctx)

    def _vec(self):
        return torch.empty((self.P, 3), dtype=torch.float32, device=self.device)

    def _mesh(self):
        return torch.empty((self.ng,) * 3, dtype=torch.float32, device=self.device)

    def _in(self, t, shape):
        if t is None:
            return None
        if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("inputs must be contiguous float32 tensors on the context's device")
        if t.numel() != math.prod(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t

    def close(self):
        if self.ctx:
            self.lib.pm_destroy(self.ctx)
            self.ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls -----------------------------------------------------------
    def set_cosmology(self, cosmo):
        self._cosmo = _cosmo_struct(cosmo)
        self.cosmo = cosmo
        self._check(self.lib.pm_set_cosmology(self.ctx, byref(self._cosmo)))

    def set_filter(self, weights):
        w = self._in(weights, (N_FILTER_PARAMS,))
        self._check(self.lib.pm_set_filter(self.ctx, _ptr(w)))

    def forward(self, noise, want_density=True):
        noise = self._in(noise, (self.np,) * 3)
        disp, mom = self._vec(), self._vec()
        dens = self._mesh() if want_density else None
        self.forward_count += 1
        self._check(self.lib.pm_forward(self.ctx, _ptr(noise), _ptr(disp), _ptr(mom), _ptr(dens)))
        return disp, mom, dens

    def set_step_scales(self, scales):
        """Per-step multipliers [3, n_steps] of kick_a, drift, kick_b (host array)."""
        import numpy as np
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64).reshape(-1))
        if sc.size != 3 * self.cfg.n_steps:
            raise ValueError(f"need {3 * self.cfg.n_steps} scales")
        self._check(self.lib.pm_set_step_scales(self.ctx, sc.ctypes.data_as(c_void_p)))

    def step_gradients(self):
        """dL/d(step scales) [3, n_steps] of the last adjoint."""
        import numpy as np
        out = np.zeros(3 * self.cfg.n_steps)
        self._check(self.lib.pm_step_gradients(self.ctx, out.ctypes.data_as(c_void_p)))
        return out.reshape(3, self.cfg.n_steps)

    def initial_conditions(self, noise):
        """(x_0 - q, p_0) [P, 3] exactly as pm_forward starts (Zel'dovich or 2LPT)."""
        noise = self._in(noise, (self.np,) * 3)
        disp, mom = self._vec(), self._vec()
        self._check(self.lib.pm_initial_conditions(self.ctx, _ptr(noise), _ptr(disp), _ptr(mom)))
        return disp, mom

    def adjoint(self, g_dens=None, g_disp=None, g_mom=None, want_filter=False, g_filter_out=None):
        """Reverse-time adjoint; g_filter_out (a [4417] tensor) receives the filter
        gradient in place when given."""
        g_dens = self._in(g_dens, (self.ng,) * 3)
        g_disp = self._in(g_disp, (self.P, 3))
        g_mom = self._in(g_mom, (self.P, 3))
        g_noise = torch.empty((self.np,) * 3, dtype=torch.float32, device=self.device)
        g_cosmo = (c_double * 2)()
        if g_filter_out is not None:
            g_filter = self._in(g_filter_out, (N_FILTER_PARAMS,))
        else:
            g_filter = (torch.empty(N_FILTER_PARAMS, dtype=torch.float32, device=self.device)
                        if want_filter else None)
        self._check(self.lib.pm_adjoint(self.ctx, _ptr(g_dens), _ptr(g_disp), _ptr(g_mom),
                                        _ptr(g_noise), g_cosmo, _ptr(g_filter)))
        return g_noise, (g_cosmo[0], g_cosmo[1]), g_filter

    def loss_mse(self, dens, target, want_grad=True):
        dens = self._in(dens, (self.ng,) * 3)
        target = self._in(target, (self.ng,) * 3)
        g = self._mesh() if want_grad else None
        loss = c_double(0.0)
        self._check(self.lib.pm_loss_mse(self.ctx, _ptr(dens), _ptr(target), _ptr(g), byref(loss)))
        return loss.value, g

    def loss_pk(self, dens, pk_target, n_bins=None, weight=1.0, want_grad=True):
        """Filter-training P(k) loss (pm_loss_pk); pk_target is a host array."""
        import numpy as np
        dens = self._in(dens, (self.ng,) * 3)
        n_bins = self.ng // 2 if n_bins is None else n_bins
        pt = np.ascontiguousarray(np.asarray(pk_target, dtype=np.float64)[:n_bins])
        if pt.shape != (n_bins,):
            raise ValueError(f"pk_target needs {n_bins} values")
        g = self._mesh() if want_grad else None
        loss = c_double(0.0)
        self._check(self.lib.pm_loss_pk(self.ctx, _ptr(dens), n_bins, pt.ctypes.data_as(c_void_p),
                                        float(weight), byref(loss), _ptr(g)))
        return loss.value, g

    def loss_disp(self, disp, disp_target, weight=1.0, want_grad=True):
        """Filter-training position loss (pm_loss_disp)."""
        disp = self._in(disp, (self.P, 3))
        disp_target = self._in(disp_target, (self.P, 3))
        g = self._vec() if want_grad else None
        loss = c_double(0.0)
        self._check(self.lib.pm_loss_disp(self.ctx, _ptr(disp), _ptr(disp_target), float(weight),
                                          byref(loss), _ptr(g)))
        return loss.value, g

    def power_spectrum(self, dens, n_bins=None):
        import numpy as np
        dens = self._in(dens, (self.ng,) * 3)
        n_bins = self.ng // 2 if n_bins is None else n_bins
        k, pk, nm = np.zeros(n_bins), np.zeros(n_bins), np.zeros(n_bins)
        p = lambda a: a.ctypes.data_as(c_void_p)
        self._check(self.lib.pm_power_spectrum(self.ctx, _ptr(dens), n_bins, p(k), p(pk), p(nm)))
        return k, pk, nm

    def density(self, disp):
        disp = self._in(disp, (self.P, 3))
        out = self._mesh()
        self._check(self.lib.pm_density(self.ctx, _ptr(disp), _ptr(out)))
        return out

    def force(self, disp, a):
        disp = self._in(disp, (self.P, 3))
        out = self._vec()
        self._check(self.lib.pm_force(self.ctx, _ptr(disp), float(a), _ptr(out)))
        return out

    def force_vjp(self, disp, a, v):
        disp = self._in(disp, (self.P, 3))
        v = self._in(v, (self.P, 3))
        out = self._vec()
        self._check(self.lib.pm_force_vjp(self.ctx, _ptr(disp), float(a), _ptr(v), _ptr(out)))
        return out

    def fft_r2c(self, real):
        real = self._in(real, (self.ng,) * 3)
        spec = torch.empty((self.ng, self.ng, self.ng // 2 + 1), dtype=torch.complex64,
                           device=self.device)
        self._check(self.lib.pm_fft_r2c(self.ctx, _ptr(real), _ptr(spec)))
        return spec

    def fft_c2r(self, spec):
        if spec.dtype != torch.complex64 or not spec.is_contiguous() or spec.device != self.device:
            raise ValueError("spec must be contiguous complex64 on the context's device")
        out = self._mesh()
        self._check(self.lib.pm_fft_c2r(self.ctx, _ptr(spec), _ptr(out)))
        return out

    def filter_table(self, a):
        out = torch.empty(3 * (self.ng // 2) ** 2 + 1, dtype=torch.float32, device=self.device)
        self._check(self.lib.pm_filter_table(self.ctx, float(a), _ptr(out)))
        return out

    def adam(self, param, grad, m, v, t, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        """One Adam step on param; grad is [n] or a batch [B][n] whose mean is used."""
        n = param.numel()
        for x in (param, m, v):
            self._in(x, (n,))
        nb = grad.numel() // n
        if grad.numel() != nb * n or nb < 1:
            raise ValueError("grad must hold a whole number of parameter vectors")
        self._in(grad, tuple(grad.shape))
        self._check(self.lib.pm_adam(self.ctx, _ptr(param), _ptr(grad), nb, _ptr(m), _ptr(v),
                                     n, lr, betas[0], betas[1], eps, int(t)))

    def reset_stats(self):
        self._check(self.lib.pm_stats_reset(self.ctx))

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.pm_stats_get(self.ctx, byref(s)))
        n = s.n_checkpoints
        kernels = {name: {"ms": s.kernel_ms[i], "launches": int(s.kernel_launches[i]),
                          "bytes": s.kernel_bytes[i]}
                   for i, name in enumerate(_lib.KERNEL_FAMILIES)}
        return {"forward_ms": s.forward_ms, "adjoint_ms": s.adjoint_ms, "kernels": kernels,
                "n_checkpoints": n, "ckpt_rms_cells": list(s.ckpt_rms_cells[:n]),
                "ckpt_max_cells": list(s.ckpt_max_cells[:n]),
                "ic_rms_cells": s.ic_rms_cells, "ic_max_cells": s.ic_max_cells,
                "ic_mom_rel_rms": s.ic_mom_rel_rms, "workspace_bytes": s.workspace_bytes,
                "momentum_overflow": bool(s.momentum_overflow)}


class Simulate(torch.autograd.Function):
    """(noise, omega_m, sigma8, filter weights, step scales) -> (disp, mom, dens).

    forward calls pm_forward; backward calls pm_adjoint (the reverse-time
    adjoint), returning dL/dnoise, dL/dOmega_m, dL/dsigma_8, dL/dweights and
    dL/d(step scales).  The context keeps one forward run, so backward raises if
    the context ran another forward after this graph was built.  omega_m and sigma8 are 0-d tensors (their values update
    the context's cosmology when they change); weights may be None for the plain
    force; step_scales ([3, n_steps] multipliers of kick_a, drift, kick_b) may be
    None for plain KDK.
    """

    @staticmethod
    def forward(fctx, pm: PMContext, noise, omega_m, sigma8, weights, step_scales):
        from dataclasses import replace
        om, s8 = float(omega_m), float(sigma8)
        if om != pm.cosmo.omega_m or s8 != pm.cosmo.sigma8:
            pm.set_cosmology(replace(pm.cosmo, omega_m=om, sigma8=s8))
        if weights is not None:
            pm.set_filter(weights.detach().contiguous())
        if step_scales is not None:
            pm.set_step_scales(step_scales.detach().double().cpu().numpy())
        disp, mom, dens = pm.forward(noise.detach().contiguous())
        fctx.pm = pm
        fctx.run = pm.forward_count
        fctx.has_w = weights is not None
        fctx.scales = None if step_scales is None else (step_scales.shape, step_scales.dtype,
                                                        step_scales.device)
        fctx.dev = noise.device
        return disp, mom, dens

    @staticmethod
    def backward(fctx, g_disp, g_mom, g_dens):
        pm = fctx.pm
        if pm.forward_count != fctx.run:
            raise RuntimeError("the PMContext ran another forward after this graph was built; "
                               "pm_adjoint only differentiates the most recent run (use one "
                               "context per graph, or call backward before the next simulate)")
        c = lambda t: None if t is None else t.contiguous()
        g_noise, (g_om, g_s8), g_w = pm.adjoint(c(g_dens), c(g_disp), c(g_mom), want_filter=fctx.has_w)
        dev = fctx.dev
        g_sc = None
        if fctx.scales is not None:
            shape, dtype, sdev = fctx.scales
            g_sc = torch.as_tensor(pm.step_gradients(), dtype=dtype, device=sdev).reshape(shape)
        return (None, g_noise, torch.tensor(g_om, device=dev), torch.tensor(g_s8, device=dev), g_w,
                g_sc)


def simulate(pm: PMContext, noise, omega_m, sigma8, weights=None, step_scales=None):
    return Simulate.apply(pm, noise, omega_m, sigma8, weights, step_scales)
