"""pm_power_spectrum_noalloc (for callers that cannot allocate device memory)
against pm_power_spectrum of a context on the same field: two calls in a row,
the second on a smaller mesh, then the first size again (the scratch array keeps
the previous call's contents)."""
import numpy as np
import pytest

from gpu_util import context, dev
from oracle import pm as opm
from paper_2211_09958_amd import _lib, api
from synthetic import normal

pytestmark = pytest.mark.gpu


def _field(ng, box, seed):
    """A clustered overdensity: CIC density of displaced lattice particles."""
    pm = context(32, ng, box, 1)
    s = normal((32 ** 3, 3), seed) * (box / 32) * 0.7
    return pm, pm.density(dev(s))


@pytest.mark.parametrize("order", [(128, 64, 128)])
def test_noalloc_power_spectrum_matches_context_call(order):
    boxes = {128: 128.0, 64: 96.0}
    for i, ng in enumerate(order):
        box = boxes[ng]
        pm, dens = _field(ng, box, 70 + i)
        nb = ng // 2 if i != 1 else ng // 3
        k_ref, p_ref, n_ref = pm.power_spectrum(dens, nb)
        k, p, n = api.power_spectrum_noalloc(dens, box, nb)
        print(f"call {i}: mesh {ng}, {nb} shells, max rel P diff "
              f"{np.nanmax(np.abs(p / p_ref - 1)):.2e}")
        np.testing.assert_array_equal(n, n_ref)
        np.testing.assert_allclose(p, p_ref, rtol=1e-12)
        np.testing.assert_allclose(k, k_ref, rtol=1e-12)


def test_noalloc_rejects_meshes_above_its_limit():
    pm, dens = _field(128, 128.0, 79)
    big = dev(np.zeros((256,) * 3))
    with pytest.raises(_lib.PMError) as e:
        api.power_spectrum_noalloc(big, 256.0, 64)
    assert e.value.code == _lib.PM_EINVAL
    with pytest.raises(_lib.PMError):
        api.power_spectrum_noalloc(dens, -1.0, 8)
    with pytest.raises(_lib.PMError):
        api.power_spectrum_noalloc(dens, 128.0, 129)
