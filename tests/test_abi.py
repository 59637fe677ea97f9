"""The C ABI without a GPU: symbols, host-side validation, host tables (pinned
against the oracle's independent hypergeometric/quad implementation)."""
import ctypes
import subprocess

import numpy as np
import pytest

from oracle import cosmology as C
from oracle import pm as opm
from paper_2211_09958_amd import _lib, api
from synthetic import LARGE, MEDIUM, SMALL, WORKLOADS, Cosmology

CO = Cosmology()


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _lib.EXPORTS:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    header = open(_lib.HERE + "/../include/pm.h").read()
    import re
    declared = set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", header))
    assert declared == set(_lib.EXPORTS)
    assert declared <= exported


@pytest.mark.parametrize("field,value", [("ptcl_grid", 48), ("mesh", 12), ("mesh", 2048),
                                         ("box", -1.0), ("n_steps", 0), ("a_start", 0.0),
                                         ("filter", 2), ("flags", 4), ("checkpoint_every", -1)])
def test_invalid_config_rejected_on_host(field, value):
    cfg = api.config_from_workload(SMALL)
    setattr(cfg, field, value)
    st = ctypes.c_int(0)
    n = _lib.load().pm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(st))
    assert n == 0 and st.value == _lib.PM_EINVAL
    assert _lib.load().pm_last_error(None)


def test_mesh_must_be_multiple_of_particles():
    cfg = api.make_config(64, 32, 64.0, 10)
    with pytest.raises(_lib.PMError):
        api.workspace_bytes(cfg)


def test_pm_init_validates_before_touching_the_gpu():
    lib = _lib.load()
    cfg = api.config_from_workload(SMALL)
    cs = api._cosmo_struct(CO)
    out = ctypes.c_void_p()
    assert lib.pm_init(ctypes.byref(cfg), ctypes.byref(cs), None, 0, None, ctypes.byref(out)) == _lib.PM_EINVAL
    bad = api._cosmo_struct(CO)
    bad.omega_m = -0.1
    assert lib.pm_init(ctypes.byref(cfg), ctypes.byref(bad), ctypes.c_void_p(256), 10 ** 12, None,
                       ctypes.byref(out)) == _lib.PM_EINVAL
    # unaligned workspace
    assert lib.pm_init(ctypes.byref(cfg), ctypes.byref(cs), ctypes.c_void_p(4), 10 ** 12, None,
                       ctypes.byref(out)) == _lib.PM_EINVAL
    # too small
    assert lib.pm_init(ctypes.byref(cfg), ctypes.byref(cs), ctypes.c_void_p(256), 16, None,
                       ctypes.byref(out)) == _lib.PM_ENOMEM
    assert lib.pm_adjoint(None, None, None, None, None, None, None) == _lib.PM_EINVAL


def test_noalloc_power_spectrum_validates_before_touching_the_gpu():
    lib = _lib.load()
    k = (ctypes.c_double * 8)()
    fake = ctypes.c_void_p(256)   # never dereferenced: every case fails validation
    for mesh, box, nb, dens in ((12, 12.0, 4, fake), (256, 256.0, 8, fake), (64, -1.0, 8, fake),
                                (64, 64.0, 0, fake), (64, 64.0, 65, fake), (64, 64.0, 8, None)):
        rc = lib.pm_power_spectrum_noalloc(dens, mesh, box, nb, k, k, k, None)
        assert rc == _lib.PM_EINVAL, (mesh, box, nb)
        assert lib.pm_last_error(None)


def test_workspace_scales_with_mesh_not_steps():
    a = api.workspace_bytes(api.config_from_workload(MEDIUM))
    b = api.workspace_bytes(api.config_from_workload(MEDIUM.with_(n_steps=630)))
    assert 0 <= b - a < 1 << 20   # reverse-time adjoint: only scalar slots grow with steps
    big = api.workspace_bytes(api.config_from_workload(LARGE))
    assert big < 60e9


def test_state_units_cover_the_momentum_bound():
    """Momenta are int32 multiples of cell * 2^-22, coarsened by powers of two
    for small cells until the range covers |p| <= 100 Mpc/h per unit time."""
    u = api.state_units(api.config_from_workload(LARGE))          # cell 0.5
    assert u["position_unit"] == 512.0 / 2 ** 32
    assert u["momentum_unit"] == 0.5 * 2.0 ** -22 and u["momentum_range"] == 256.0
    for w in WORKLOADS.values():
        r = api.state_units(api.config_from_workload(w))
        assert r["momentum_range"] >= 100.0
        assert r["momentum_unit"] == w.cell * 2.0 ** -22 or r["momentum_range"] < 200.0
    tiny = api.state_units(api.make_config(64, 1024, 64.0, 10))    # cell 1/16: range 32 by default
    assert 100.0 <= tiny["momentum_range"] < 200.0
    ratio = tiny["momentum_unit"] / (64.0 / 1024 * 2.0 ** -22)
    assert ratio == 4.0
    cfg = api.config_from_workload(SMALL)
    cfg.mesh = 12
    with pytest.raises(_lib.PMError):
        api.state_units(cfg)


@pytest.mark.parametrize("w", [SMALL, MEDIUM])
def test_host_tables_match_oracle(w):
    cfg = api.config_from_workload(w)
    t = api.host_tables(cfg, CO)
    co = C.kdk_coefficients(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    np.testing.assert_allclose(t["kick_a"], co.kick_a, rtol=1e-11)
    np.testing.assert_allclose(t["drift"], co.drift, rtol=1e-11)
    np.testing.assert_allclose(t["kick_b"], co.kick_b, rtol=1e-11)
    assert abs(t["D0"] / co.D0 - 1) < 1e-12 and abs(t["G0"] / co.G0 - 1) < 1e-11
    np.testing.assert_allclose(t["D"], C.growth_D(co.a, CO.omega_m), rtol=1e-12)
    np.testing.assert_allclose(t["G"], C.growth_G(co.a, CO.omega_m), rtol=1e-11)
    d = C.kdk_coefficient_derivatives(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    for key, ref in (("d_kick_a", d.kick_a), ("d_drift", d.drift), ("d_kick_b", d.kick_b)):
        np.testing.assert_allclose(t[key], ref, rtol=1e-6, atol=1e-8 * np.abs(ref).max())
    assert abs(t["d_D0"] / d.D0 - 1) < 1e-6
    nsq = np.arange(t["pk"].size)
    ref = C.linear_pk(2 * np.pi / w.box * np.sqrt(nsq), CO)
    np.testing.assert_allclose(t["pk"][1:], ref[1:], rtol=1e-9)
    assert t["pk"][0] == 0.0


@pytest.mark.parametrize("w", [SMALL, MEDIUM])
def test_lpt2_growth_matches_oracle(w):
    cfg = api.config_from_workload(w)
    g = api.lpt2_growth(cfg, CO)
    co = C.kdk_coefficients(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    d = C.kdk_coefficient_derivatives(CO.omega_m, w.a_start, w.a_stop, w.n_steps)
    assert abs(g["D2"] / co.D20 - 1) < 1e-11 and abs(g["G2"] / co.G20 - 1) < 1e-10
    assert abs(g["d_D2"] / d.D20 - 1) < 1e-6 and abs(g["d_G2"] / d.G20 - 1) < 1e-6
    assert g["D2"] < 0 and g["G2"] < 0


def test_lpt_order_sets_the_flag():
    assert api.make_config(32, 64, 64.0, 10, lpt_order=2).flags == _lib.PM_F_2LPT
    assert api.make_config(32, 64, 64.0, 10).flags == 0
    with pytest.raises(ValueError):
        api.make_config(32, 64, 64.0, 10, lpt_order=3)


def test_new_calls_validate_on_the_host():
    lib = _lib.load()
    cfg = api.config_from_workload(SMALL)
    cs = api._cosmo_struct(CO)
    out = np.zeros(4)
    assert lib.pm_lpt2_growth(ctypes.byref(cfg), ctypes.byref(cs), None) == _lib.PM_EINVAL
    assert lib.pm_lpt2_growth(None, ctypes.byref(cs), out.ctypes.data_as(ctypes.c_void_p)) == _lib.PM_EINVAL
    bad = api._cosmo_struct(CO)
    bad.omega_m = 2.0
    assert lib.pm_lpt2_growth(ctypes.byref(cfg), ctypes.byref(bad),
                              out.ctypes.data_as(ctypes.c_void_p)) == _lib.PM_EINVAL
    scales = np.ones(3 * SMALL.n_steps)
    assert lib.pm_set_step_scales(None, scales.ctypes.data_as(ctypes.c_void_p)) == _lib.PM_EINVAL
    assert lib.pm_step_gradients(None, scales.ctypes.data_as(ctypes.c_void_p)) == _lib.PM_EINVAL
    assert lib.pm_initial_conditions(None, None, None, None) == _lib.PM_EINVAL


def test_einstein_de_sitter_host_tables():
    """Omega_m = 1 (no Lambda): D = a, G = a^3 E dD/da = a^(3/2), D2 = -(3/7) a^2,
    G2 = -(6/7) a^(5/2), and kick/drift factors in closed form."""
    from dataclasses import replace
    co = replace(CO, omega_m=1.0)
    cfg = api.make_config(32, 64, 64.0, 8, a_start=0.1, a_stop=0.9)
    t = api.host_tables(cfg, co)
    a = 0.1 + 0.1 * np.arange(9)
    np.testing.assert_allclose(t["D"], a, rtol=1e-12)
    np.testing.assert_allclose(t["G"], a ** 1.5, rtol=1e-11)
    ah = 0.5 * (a[:-1] + a[1:])
    np.testing.assert_allclose(t["kick_a"], (ah ** 1.5 - a[:-1] ** 1.5) / a[:-1], rtol=1e-11)
    np.testing.assert_allclose(t["drift"], (a[1:] - a[:-1]) / ah ** 1.5, rtol=1e-11)
    np.testing.assert_allclose(t["kick_b"], (a[1:] ** 1.5 - ah ** 1.5) / a[1:], rtol=1e-11)
    g2 = api.lpt2_growth(cfg, co)
    assert abs(g2["D2"] / (-3 / 7 * 0.01) - 1) < 1e-12
    assert abs(g2["G2"] / (-6 / 7 * 0.1 ** 2.5) - 1) < 1e-11
    ref = C.kdk_coefficients(1.0, 0.1, 0.9, 8)
    np.testing.assert_allclose(t["kick_a"], ref.kick_a, rtol=1e-11)
    assert abs(ref.D20 / g2["D2"] - 1) < 1e-12


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built library every call path raises."""
    monkeypatch.setattr(_lib, "_LIB", None)
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "libpmx.so"))


def test_context_without_a_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the path taken when no GPU is present")
    with pytest.raises(RuntimeError):
        api.PMContext(api.config_from_workload(SMALL), CO)
