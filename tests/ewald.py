"""Ewald-summed periodic force of a point mass: the reference that the PM
two-body force is pinned against (a test helper, not collected by pytest).

Periodic gravity of a point mass in a box with a neutralising uniform
background (lap(phi) = mass (sum of image deltas) - mass / box^3, F = -grad phi),
summed by the Ewald method (Hernquist, Bouchet & Suto 1991): a real-space sum
over images with the erfc screen plus a reciprocal-space sum.
"""
import numpy as np


def ewald_force(d, mass, box, alpha=None, nreal=2, nfour=8):
    """Periodic force of a point mass with a neutralising background (lap(phi) =
    mass (sum of deltas) - mass / box^3, F = -grad(phi)) at separations d [m, 3], by
    Ewald summation (Hernquist, Bouchet & Suto 1991): a real-space erfc sum over
    images plus a reciprocal-space sum."""
    from scipy.special import erfc
    alpha = 2.0 / box if alpha is None else alpha
    out = np.zeros_like(d)
    rng = range(-nreal, nreal + 1)
    for n0 in rng:
        for n1 in rng:
            for n2 in rng:
                s = d - box * np.array([n0, n1, n2])
                r = np.linalg.norm(s, axis=1, keepdims=True)
                g = erfc(alpha * r) + 2 * alpha * r / np.sqrt(np.pi) * np.exp(-(alpha * r) ** 2)
                out -= mass / (4 * np.pi) * s / r ** 3 * g
    h = np.arange(-nfour, nfour + 1)
    hv = np.stack(np.meshgrid(h, h, h, indexing="ij"), axis=-1).reshape(-1, 3)
    hv = hv[np.any(hv != 0, axis=1)]
    k = 2 * np.pi / box * hv
    k2 = np.sum(k * k, axis=1)
    coef = np.exp(-k2 / (4 * alpha ** 2)) / k2
    out -= mass / box ** 3 * (np.sin(d @ k.T) * coef) @ k
    return out
