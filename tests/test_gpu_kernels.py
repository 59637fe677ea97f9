"""GPU parity of the building blocks against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from gpu_util import CO, context, dev, host, rel_l2
from oracle import mesh as M
from oracle import pm as opm
from synthetic import normal, uniform

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ng", [8, 16, 32, 64, 128, 256, 512])
def test_fft_r2c_matches_oracle(ng, monkeypatch):
    monkeypatch.setattr(M, "WORKERS", 16)
    pm = context(8, ng, float(ng), 1)
    x = normal((ng,) * 3, 100 + ng).astype(np.float32)
    got = pm.fft_r2c(dev(x)).cpu().numpy().astype(np.complex128)
    ref = M.rfftn(x.astype(np.float64))
    err = np.sqrt(np.mean(np.abs(got - ref) ** 2) / np.mean(np.abs(ref) ** 2))
    assert err < 2e-6, err
    back = host(pm.fft_c2r(torch.as_tensor(got.astype(np.complex64), device="cuda"))) / ng ** 3
    assert rel_l2(back, x) < 2e-6


def test_fft_hermitian_planes_and_nyquist():
    ng = 32
    pm = context(8, ng, 32.0, 1)
    c = (np.arange(ng) + 0.5)
    X = np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1)
    x = np.cos(2 * np.pi * (X @ np.array([16, 0, 16])) / ng)     # Nyquist along 0 and 2
    got = pm.fft_r2c(dev(x)).cpu().numpy()
    ref = M.rfftn(x.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(got - ref)) < 1e-3 * np.max(np.abs(ref))


def _lattice_disp(np_, box, seed, sigma):
    return normal((np_ ** 3, 3), seed) * sigma


@pytest.mark.parametrize("np_,ng,sigma", [(32, 64, 3.0), (16, 64, 10.0), (8, 16, 5.0), (32, 32, 0.7)])
def test_density_matches_oracle(np_, ng, sigma):
    box = float(ng)
    pm = context(np_, ng, box, 1)
    s = _lattice_disp(np_, box, 7, sigma).astype(np.float32)
    got = host(pm.density(dev(s)))
    q = opm.lattice(np_, box)
    ref = M.density(q + s.astype(np.float64), ng, box, np_ ** 3)
    mass = (ng / np_) ** 3
    assert np.max(np.abs(got - ref)) < 2e-6 * mass
    assert abs((got + 1).sum() / ng ** 3 - 1) < 1e-6


def test_density_edge_cases():
    np_, ng, box = 16, 32, 32.0
    pm = context(np_, ng, box, 1)
    q = opm.lattice(np_, box)
    cases = {
        # every particle in one cell (all CIC footprints overlap)
        "one_cell": np.array([5.3, 17.2, 30.9]) - q,
        # exactly on cell faces (t = 1/2) and exactly on mesh nodes (t = 0)
        "faces": np.round(uniform(q.shape, 3, 0, box)) - q,
        "nodes": np.round(uniform(q.shape, 5, 0, box)) + 0.5 - q,
        # just below the box edge and at negative coordinates (wrap)
        "edge": np.full(q.shape, box - 1e-4) - q + np.where(np.arange(q.shape[0])[:, None] % 2, -box, 0.0),
        # far outside the box in both directions
        "wrap": q * 0 + normal(q.shape, 4) * 3 * box,
    }
    for name, s in cases.items():
        s32 = s.astype(np.float32)
        got = host(pm.density(dev(s32)))
        ref = M.density(q + s32.astype(np.float64), ng, box, np_ ** 3)
        assert np.max(np.abs(got - ref)) < 1e-5 * (ng / np_) ** 3 * max(1, np.abs(ref).max()), name


def test_density_bitwise_repeatable():
    pm = context(32, 64, 64.0, 1)
    s = dev(_lattice_disp(32, 64.0, 9, 4.0))
    a, b = pm.density(s), pm.density(s)
    assert torch.equal(a, b)


@pytest.mark.parametrize("np_,ng,sigma", [(32, 64, 1.0), (16, 32, 3.0), (8, 16, 2.0)])
def test_force_matches_oracle(np_, ng, sigma):
    box = float(ng)
    pm = context(np_, ng, box, 1)
    s = _lattice_disp(np_, box, 11, sigma).astype(np.float32)
    got = host(pm.force(dev(s), 0.5))
    st = opm.Setup(np_, ng, box, 1, CO)
    ref, _, _ = opm.pm_force(opm.lattice(np_, box) + s.astype(np.float64), st)
    assert rel_l2(got, ref) < 1e-5


def test_force_sums_to_zero_on_gpu():
    pm = context(32, 64, 64.0, 1)
    s = _lattice_disp(32, 64.0, 12, 2.0)
    F = host(pm.force(dev(s), 0.5))
    assert np.max(np.abs(F.sum(axis=0))) < 1e-4 * np.abs(F).sum() / 3


@pytest.mark.parametrize("np_,ng,sigma", [(16, 32, 2.0), (8, 16, 1.5)])
def test_force_vjp_matches_oracle(np_, ng, sigma):
    box = float(ng)
    pm = context(np_, ng, box, 1)
    s = _lattice_disp(np_, box, 13, sigma).astype(np.float32)
    v = normal((np_ ** 3, 3), 14).astype(np.float32)
    got = host(pm.force_vjp(dev(s), 0.5, dev(v)))
    st = opm.Setup(np_, ng, box, 1, CO)
    ref, _, _ = opm.pm_force_vjp(opm.lattice(np_, box) + s.astype(np.float64),
                                 v.astype(np.float64), st)
    assert rel_l2(got, ref) < 1e-4


def test_power_spectrum_matches_oracle():
    ng, box = 64, 128.0
    pm = context(32, ng, box, 1)
    d = normal((ng,) * 3, 15).astype(np.float32)
    k, P, N = pm.power_spectrum(dev(d), ng // 2)
    kr, Pr, Nr = M.power_spectrum(d.astype(np.float64), box, ng // 2)
    np.testing.assert_array_equal(N, Nr)
    np.testing.assert_allclose(P, Pr, rtol=1e-5)
    np.testing.assert_allclose(k, kr, rtol=1e-12)


def test_loss_mse():
    pm = context(32, 64, 64.0, 1)
    a, b = normal((64,) * 3, 16).astype(np.float32), normal((64,) * 3, 17).astype(np.float32)
    L, g = pm.loss_mse(dev(a), dev(b))
    ref = np.mean((a.astype(np.float64) - b) ** 2)
    assert abs(L / ref - 1) < 1e-6
    np.testing.assert_allclose(host(g), 2 * (a.astype(np.float64) - b) / a.size, rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("n_bins", [32, 56, 64])
def test_loss_pk_matches_oracle(n_bins):
    """P(k) training loss and its mesh cotangent; 56 and 64 include empty corner
    shells (round(|n|) > 55 holds no mode of a 64^3 mesh)."""
    pm = context(32, 64, 64.0, 1)
    # a clustered field: CIC density of displaced lattice particles
    q = (np.indices((32,) * 3).reshape(3, -1).T + 0.5) * 2.0
    d = M.density(q + normal((32 ** 3, 3), 60) * 2.5, 64, 64.0, 32 ** 3)
    t = M.density(q + normal((32 ** 3, 3), 61) * 2.0, 64, 64.0, 32 ** 3)
    pt = M.power_spectrum(t, 64.0, n_bins)[1]
    pt = np.where(np.isfinite(pt), pt, 0.0)
    L_ref, g_ref = opm.pk_loss(d, pt, 64.0, n_bins, weight=0.3)
    L, g = pm.loss_pk(dev(d), pt, n_bins, weight=0.3)
    assert abs(L / L_ref - 1) < 1e-5
    assert rel_l2(host(g), g_ref) < 1e-5


def test_loss_pk_skips_zero_targets_and_rejects_empty():
    pm = context(8, 16, 16.0, 1)
    d = normal((16,) * 3, 62)
    pt = M.power_spectrum(normal((16,) * 3, 63), 16.0, 8)[1]
    pt[[0, 3]] = 0.0                      # shells without a target are left out
    L_ref, g_ref = opm.pk_loss(d, pt, 16.0, 8)
    L, g = pm.loss_pk(dev(d), pt, 8)
    assert abs(L / L_ref - 1) < 1e-5
    assert rel_l2(host(g), g_ref) < 1e-5
    with pytest.raises(Exception, match="PM_EINVAL"):
        pm.loss_pk(dev(d), np.zeros(8), 8)


def test_loss_disp_matches_oracle_with_wrap():
    pm = context(16, 32, 32.0, 1)
    P = 16 ** 3
    s = uniform((P, 3), 64, -3.0, 3.0)
    shifts = np.round(uniform((P, 3), 65, -1.0, 1.0)) * 32.0
    t = s + normal((P, 3), 66) * 0.5 + shifts
    t[:10, 0] = s[:10, 0] + 15.9             # separations near half a box
    t[10:20, 1] = s[10:20, 1] - 16.1
    s32, t32 = s.astype(np.float32), t.astype(np.float32)
    L_ref, g_ref = opm.disp_loss(s32, t32, 32.0, 32, weight=0.01)
    L, g = pm.loss_disp(dev(s32), dev(t32), weight=0.01)
    assert abs(L / L_ref - 1) < 1e-5
    assert rel_l2(host(g), g_ref) < 1e-5
