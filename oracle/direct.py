"""Oracle direct summation for isolated particle sets (FP64, O(N^2)).

TEST INFRASTRUCTURE ONLY.  Used to pin the PM force (Sec. 2.4: PM forces are
the discretised derivative of the potential; Table 1 contrasts them with
direct summation).  With Lap Phi = S delta and particle masses equal to the
volume per particle V/N0 (in units of the mean density), the isolated
potential and force of a set of point masses are

    Phi(x) = -(S/4 pi) (V/N0) sum_j 1/|x - x_j|
    g(x_i) = -(S/4 pi) (V/N0) sum_{j != i} (x_i - x_j)/|x_i - x_j|^3.
"""
from __future__ import annotations

import numpy as np


def potential(points: np.ndarray, src: np.ndarray, s: float, mass: float) -> np.ndarray:
    """Isolated potential of point masses `src` evaluated at `points`."""
    out = np.zeros(points.shape[0])
    for j in range(src.shape[0]):
        d = np.sqrt(((points - src[j]) ** 2).sum(axis=1))
        out -= s * mass / (4.0 * np.pi) / d
    return out


def forces(x: np.ndarray, s: float, mass: float) -> np.ndarray:
    """Pairwise direct-sum acceleration g = -grad Phi on each particle."""
    n = x.shape[0]
    g = np.zeros((n, 3))
    for i in range(n):
        d = x[i] - x                        # (n, 3)
        r2 = (d * d).sum(axis=1)
        r2[i] = np.inf
        g[i] = -(s * mass / (4.0 * np.pi)) * (d / r2[:, None] ** 1.5).sum(axis=0)
    return g
