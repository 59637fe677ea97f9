"""ctypes loader and signatures of libpmx (the C ABI in include/pm.h).

Loading fails loudly when the shared library is missing: there is no CPU
fallback on the product path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmx.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EHIP, PM_ESTATE, PM_ENUMERIC = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "PM_OK", -1: "PM_EINVAL", -2: "PM_ENOMEM", -3: "PM_EHIP",
                -4: "PM_ESTATE", -5: "PM_ENUMERIC"}
PM_MAX_CHECKPOINTS = 64
N_FILTER_PARAMS = 4417
PM_F_TIMING = 1
PM_F_2LPT = 2
PM_NOALLOC_MAX_MESH = 128
KERNEL_FAMILIES = ("bin", "scatter", "scatter_vec", "fft_x", "fft_strided", "grad_z",
                   "grad_adj_z", "gather", "unkick_vjp", "wgrad", "mlp", "other")

# exported entry points, in the order include/pm.h declares them
EXPORTS = ("pm_workspace_bytes", "pm_host_tables", "pm_state_units", "pm_init",
           "pm_set_cosmology", "pm_set_filter", "pm_forward", "pm_adjoint", "pm_loss_mse", "pm_loss_pk",
           "pm_loss_disp", "pm_power_spectrum", "pm_power_spectrum_noalloc",
           "pm_density", "pm_force", "pm_force_vjp", "pm_fft_r2c", "pm_fft_c2r",
           "pm_lpt2_growth", "pm_initial_conditions", "pm_set_step_scales",
           "pm_step_gradients",
           "pm_filter_table", "pm_adam", "pm_stats_get", "pm_stats_reset", "pm_destroy",
           "pm_last_error")


class Cosmology(ctypes.Structure):
    _fields_ = [("omega_m", c_double), ("omega_b", c_double), ("h", c_double),
                ("sigma8", c_double), ("n_s", c_double), ("T_cmb", c_double)]


class Config(ctypes.Structure):
    _fields_ = [("ptcl_grid", c_int32), ("mesh", c_int32), ("box", c_double),
                ("a_start", c_double), ("a_stop", c_double), ("n_steps", c_int32),
                ("checkpoint_every", c_int32), ("filter", c_int32), ("flags", c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("forward_ms", c_double), ("adjoint_ms", c_double),
                ("n_checkpoints", c_int32),
                ("ckpt_rms_cells", c_double * PM_MAX_CHECKPOINTS),
                ("ckpt_max_cells", c_double * PM_MAX_CHECKPOINTS),
                ("ic_rms_cells", c_double), ("ic_max_cells", c_double),
                ("ic_mom_rel_rms", c_double), ("workspace_bytes", c_size_t),
                ("kernel_ms", c_double * len(KERNEL_FAMILIES)),
                ("kernel_launches", ctypes.c_int64 * len(KERNEL_FAMILIES)),
                ("kernel_bytes", c_double * len(KERNEL_FAMILIES)),
                ("momentum_overflow", c_int32)]


class PMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpmx.so once; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"libpmx.so not found at {path}; run paper_2211_09958_amd.build.build()")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "pm_workspace_bytes": (c_size_t, [POINTER(Config), POINTER(c_int)]),
        "pm_host_tables": (c_int, [POINTER(Config), POINTER(Cosmology), P, P, P, P]),
        "pm_state_units": (c_int, [POINTER(Config), P]),
        "pm_init": (c_int, [POINTER(Config), POINTER(Cosmology), P, c_size_t, P, POINTER(P)]),
        "pm_set_cosmology": (c_int, [P, POINTER(Cosmology)]),
        "pm_set_filter": (c_int, [P, P]),
        "pm_forward": (c_int, [P, P, P, P, P]),
        "pm_adjoint": (c_int, [P, P, P, P, P, P, P]),
        "pm_loss_mse": (c_int, [P, P, P, P, P]),
        "pm_loss_pk": (c_int, [P, P, c_int32, P, c_double, P, P]),
        "pm_loss_disp": (c_int, [P, P, P, c_double, P, P]),
        "pm_power_spectrum": (c_int, [P, P, c_int32, P, P, P]),
        "pm_power_spectrum_noalloc": (c_int, [P, c_int32, c_double, c_int32, P, P, P, P]),
        "pm_density": (c_int, [P, P, P]),
        "pm_force": (c_int, [P, P, c_double, P]),
        "pm_force_vjp": (c_int, [P, P, c_double, P, P]),
        "pm_fft_r2c": (c_int, [P, P, P]),
        "pm_fft_c2r": (c_int, [P, P, P]),
        "pm_lpt2_growth": (c_int, [POINTER(Config), POINTER(Cosmology), P]),
        "pm_initial_conditions": (c_int, [P, P, P, P]),
        "pm_set_step_scales": (c_int, [P, P]),
        "pm_step_gradients": (c_int, [P, P]),
        "pm_filter_table": (c_int, [P, c_double, P]),
        "pm_adam": (c_int, [P, P, P, c_int32, P, P, c_int32, c_double, c_double, c_double, c_double,
                            c_int32]),
        "pm_stats_get": (c_int, [P, POINTER(Stats)]),
        "pm_stats_reset": (c_int, [P]),
        "pm_destroy": (None, [P]),
        "pm_last_error": (c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(rc: int, ctx=None) -> None:
    if rc != PM_OK:
        msg = load().pm_last_error(ctx)
        raise PMError(rc, msg.decode() if msg else "")
