"""Host-side check of the mesh row order (csrc/layout.h): a bijection of the n^2
rows with an exact inverse, plain order for n < 16, and 16 x 16 blocks beyond."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2211_09958_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "layout.h"
int main() {
    for (int n = 8; n <= 1024; n *= 2) {
        std::vector<int> seen((size_t)n * n, 0);
        for (int i0 = 0; i0 < n; ++i0)
            for (int i1 = 0; i1 < n; ++i1) {
                const long r = pmx::mesh_row(i0, i1, n);
                if (r < 0 || r >= (long)n * n || seen[r]++) { printf("collision\n"); return 1; }
                int a, b;
                pmx::mesh_row_inv(r, n, a, b);
                if (a != i0 || b != i1) { printf("inverse\n"); return 1; }
                if (n < 16 && r != (long)i0 * n + i1) { printf("plain\n"); return 1; }
                // rows of one 16 x 16 block are contiguous
                if (n >= 16 && r / 256 != (long)(i0 / 16) * (n / 16) + i1 / 16) { printf("block\n"); return 1; }
            }
    }
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_mesh_row_order_is_a_blocked_bijection(tmp_path):
    src = tmp_path / "layout_check.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "layout_check"
    subprocess.run(["hipcc", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60)
    assert out.stdout.strip() == "ok"
