"""The learned radial force filter f(|k|, a) = 1 + g(|k|/k_Nyq, a), FP64.

Test infrastructure (see ``oracle/__init__.py``).

Passage followed: pmwd paper, Statement of Need, on deep-learning components
running with the simulation and the ongoing spatiotemporal optimisation of the
PM gravity solver.  The paper gives no architecture; the reading used here is
a 2 -> 64 -> 64 -> 1 perceptron with SiLU activations whose output g is added
to 1, so a zero last layer reproduces the plain PM force exactly.

Parameters are one flat vector of 4417 values packed as
  W1 [64, 2], b1 [64], W2 [64, 64], b2 [64], W3 [1, 64], b3 [1]
(row-major, output index first, the layout of torch.nn.Linear.weight).
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
N_PARAMS = HIDDEN * 2 + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1   # 4417


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    o = 0
    parts = []
    for shape in ((HIDDEN, 2), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (1, HIDDEN), (1,)):
        n = int(np.prod(shape))
        parts.append(theta[o:o + n].reshape(shape))
        o += n
    return parts


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def features(mesh, box, a):
    """Inputs (|k| / k_Nyq, a) for every integer |n|^2 in [0, 3 (mesh/2)^2]."""
    nsq = np.arange(3 * (mesh // 2) ** 2 + 1, dtype=np.float64)
    kabs = 2.0 * np.pi / box * np.sqrt(nsq)
    k_nyq = np.pi * mesh / box
    return np.stack([kabs / k_nyq, np.full_like(kabs, a)], axis=1)


def forward(theta, x):
    """g(x) for inputs x [n, 2]; returns (g [n], cache for backward)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = x @ W1.T + b1
    h1 = _silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = _silu(z2)
    g = (h2 @ W3.T + b3)[:, 0]
    return g, (x, z1, h1, z2, h2)


def backward(theta, cache, g_bar):
    """Vector-Jacobian product: dL/dtheta given dL/dg [n]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    x, z1, h1, z2, h2 = cache
    gb = g_bar[:, None]
    dW3 = gb.T @ h2
    db3 = gb.sum(axis=0)
    dh2 = gb @ W3
    dz2 = dh2 * _silu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * _silu_grad(z1)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def filter_table(theta, mesh, box, a):
    """f(|n|^2, a) = 1 + g for every integer |n|^2, plus the backward cache."""
    g, cache = forward(theta, features(mesh, box, a))
    return 1.0 + g, cache

