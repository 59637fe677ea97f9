"""GPU checks at the full sizes of the 512^3-particle / 1024^3-mesh workload.

The FP64 oracle cannot run these sizes in seconds, so the checks use results that
hold at any size:
  * 1024^3 real FFTs against the closed-form spectrum of a sum of plane waves;
  * the CIC density of an evolved 512^3-particle state on the 1024^3 mesh at
    sampled cells (random ones and the densest) against a brute-force FP64 sum over
    the particles that touch them;
  * the 63-step forward run and reverse-time adjoint in the launch configuration
    the benchmark times: exact reconstruction of the initial state and of every
    checkpoint, mass conservation, checkpointed vs pure adjoint.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import CO, context, dev, host, rel_l2
from paper_2211_09958_amd import api
from synthetic import LARGE, uniform, white_noise

pytestmark = pytest.mark.gpu

N = 1024
MODES = [((3, -5, 7), 1.0, 0.3), ((-100, 200, 300), 0.5, 1.1), ((17, 0, 1), 0.25, -2.0),
         ((511, -511, 511), 0.125, 0.7)]


def plane_waves(n, modes):
    """Sum of A cos(2 pi n.i / N + phi) on the GPU, phases reduced mod N in int64."""
    i = torch.arange(n, device="cuda", dtype=torch.int64)
    x = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    for (n0, n1, n2), A, phi in modes:
        for a in range(0, n, 128):   # 128 planes at a time
            idx = (n0 * i[a:a + 128, None, None] + n1 * i[None, :, None]
                   + n2 * i[None, None, :]) % n
            x[a:a + 128] += (A * torch.cos(2 * math.pi * idx.double() / n + phi)).float()
    return x


def mode_index(m, n):
    return (m[0] % n, m[1] % n, m[2])


def test_fft_1024_r2c_plane_waves():
    pm = context(8, N, float(N), 1)
    spec = pm.fft_r2c(plane_waves(N, MODES))
    peak = 0.5 * N ** 3
    for m, A, phi in MODES:
        got = complex(spec[mode_index(m, N)].item())
        want = A * peak * complex(math.cos(phi), math.sin(phi))
        assert abs(got - want) < 1e-6 * A * peak, (m, got, want)
        spec[mode_index(m, N)] = 0
    rest = spec.abs().max().item()
    assert rest < 1e-7 * peak, rest


def test_fft_1024_c2r_plane_waves():
    pm = context(8, N, float(N), 1)
    spec = torch.zeros((N, N, N // 2 + 1), dtype=torch.complex64, device="cuda")
    for m, A, phi in MODES:
        spec[mode_index(m, N)] = A * 0.5 * N ** 3 * complex(math.cos(phi), math.sin(phi))
    back = pm.fft_c2r(spec) / N ** 3
    err = (back - plane_waves(N, MODES)).abs().max().item()
    assert err < 2e-6, err


@pytest.fixture(scope="module")
def large_forward():
    pm = api.PMContext(api.config_from_workload(LARGE.with_(checkpoint_every=16)), CO)
    disp, mom, dens = pm.forward(dev(white_noise(LARGE.ptcl_grid, 0)))
    torch.cuda.synchronize()
    return pm, disp, mom, dens


def cic_sampled(disp, cells, np_, ng, box):
    """FP64 CIC density at the given cells from all particles that touch them."""
    P = np_ ** 3
    cell = box / ng
    j = np.arange(P, dtype=np.int64)
    q = np.stack([j // (np_ * np_), (j // np_) % np_, j % np_], axis=1) * (box / np_)
    x = np.mod(q + disp.astype(np.float64), box)
    u = x / cell - 0.5
    base = np.floor(u).astype(np.int64)
    t = u - base
    base %= ng
    key = (base[:, 0] * ng + base[:, 1]) * ng + base[:, 2]
    need = {}
    for ci, c in enumerate(cells):
        for a in (0, 1):
            for b in (0, 1):
                for d in (0, 1):
                    k = (((c[0] - a) % ng) * ng + (c[1] - b) % ng) * ng + (c[2] - d) % ng
                    need.setdefault(k, []).append((ci, a, b, d))
    table = np.zeros(ng ** 3, dtype=bool)
    table[np.fromiter(need, dtype=np.int64)] = True
    sel = np.flatnonzero(table[key])
    rho = np.zeros(len(cells))
    m = (ng / np_) ** 3
    for p in sel:
        for ci, a, b, d in need[int(key[p])]:
            w = ((t[p, 0] if a else 1 - t[p, 0]) * (t[p, 1] if b else 1 - t[p, 1])
                 * (t[p, 2] if d else 1 - t[p, 2]))
            rho[ci] += m * w
    return rho - 1.0


def test_density_full_size_sampled_cells(large_forward):
    pm, disp, _, dens = large_forward
    d2 = pm.density(disp)
    flat = d2.reshape(-1)
    top = torch.topk(flat, 8).indices.cpu().numpy()
    rnd = (uniform(32, 70) * N ** 3).astype(np.int64)
    idx = np.concatenate([top, rnd])
    cells = [(i // (N * N), (i // N) % N, i % N) for i in idx]
    ref = cic_sampled(host(disp), cells, LARGE.ptcl_grid, N, LARGE.box)
    got = flat[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    assert ref[:8].min() > 20           # halo cells at a = 1
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5)
    # the density returned by the run itself is that of its internal state
    assert rel_l2(host(dens.reshape(-1)[torch.as_tensor(idx, device="cuda")]), ref) < 1e-5


def test_full_size_forward_adjoint_properties(large_forward):
    pm, disp, mom, dens = large_forward
    assert abs(dens.double().mean().item()) < 1e-6          # mass conservation
    tgt = api.PMContext(api.config_from_workload(LARGE), CO)
    _, _, target = tgt.forward(dev(white_noise(LARGE.ptcl_grid, 1)))
    _, gd = pm.loss_mse(dens, target)
    g_ck, cosmo_ck, _ = pm.adjoint(g_dens=gd)
    st = pm.stats()
    assert st["n_checkpoints"] == 3
    assert max(st["ckpt_max_cells"]) == 0.0
    assert st["ic_max_cells"] == 0.0 and st["ic_mom_rel_rms"] == 0.0
    # pure reverse-time adjoint on the same run (a context without checkpoints)
    tgt.forward(dev(white_noise(LARGE.ptcl_grid, 0)))
    g_pure, cosmo_pure, _ = tgt.adjoint(g_dens=gd)
    st2 = tgt.stats()
    assert st2["ic_max_cells"] == 0.0
    assert torch.isfinite(g_ck).all() and torch.isfinite(g_pure).all()
    assert rel_l2(host(g_ck), host(g_pure)) < 1e-5
    assert abs(cosmo_ck[0] / cosmo_pure[0] - 1) < 1e-5 and abs(cosmo_ck[1] / cosmo_pure[1] - 1) < 1e-5
