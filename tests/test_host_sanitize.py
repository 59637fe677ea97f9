"""The host C++ cosmology tables under AddressSanitizer and UBSan (CPU only).

g++ builds host_cosmo.cpp with a small driver (no HIP code is involved); the run
must be clean under the sanitizers and print the same tables the library
returns through pm_host_tables / pm_lpt2_growth."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2211_09958_amd import api
from synthetic import Cosmology

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2211_09958_amd", "csrc")


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "host_cosmo_driver")
    flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd = [gxx, *flags, f"-I{CSRC}", os.path.join(HERE, "host_cosmo_driver.cpp"),
           os.path.join(CSRC, "host_cosmo.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    return res.stdout


def test_host_tables_clean_under_sanitizers(driver_output):
    lines = driver_output.splitlines()
    co = Cosmology()
    k = 0
    for steps in (1, 10, 63):
        assert lines[k] == f"steps {steps}"
        rows = np.array([[float(v) for v in lines[k + 1 + n].split()] for n in range(steps)])
        ic = np.array([float(v) for v in lines[k + 1 + steps].split()[1:]])
        k += steps + 2
        cfg = api.make_config(32, 64, 64.0, steps)
        t = api.host_tables(cfg, co)
        g2 = api.lpt2_growth(cfg, co)
        np.testing.assert_allclose(rows[:, 0], t["kick_a"], rtol=1e-12)
        np.testing.assert_allclose(rows[:, 1], t["drift"], rtol=1e-12)
        np.testing.assert_allclose(rows[:, 2], t["kick_b"], rtol=1e-12)
        np.testing.assert_allclose(rows[:, 3], t["d_kick_a"], rtol=1e-9)
        np.testing.assert_allclose(ic[[0, 1, 4, 5]], [t["D0"], t["G0"], t["d_D0"], t["d_G0"]], rtol=1e-12)
        np.testing.assert_allclose(ic[[2, 3, 6, 7]], [g2["D2"], g2["G2"], g2["d_D2"], g2["d_G2"]], rtol=1e-12)
    assert lines[k].startswith("pk ")
    pk = np.array([float(v) for v in lines[k + 1:]])
    ref = api.host_tables(api.make_config(32, 64, 64.0, 1), co)["pk"]
    np.testing.assert_allclose(pk, ref, rtol=1e-12)
