"""Oracle of the paper's alternating-direction explicit (ADE) integrator of the
gravity diffusion equation (FP64, plain loops).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

What the paper fixes (Sec. 2.1 Eq. 4, Sec. 2.3): the potential obeys a
diffusion equation, 3 calH dPhi/dtau - c^2 Lap Phi = -c^2 S delta, advanced on
the mesh by an ADE method: the new value of a cell is written from its old
value and its neighbours, and two consecutive steps run in alternate
directions, which makes the scheme unconditionally stable.  The potential
advances in two half sub-steps per time step (Table 2).

Readings (the paper names the method, not its stencil):
* Eq. 4 divided by 3 calH is dPhi/dtau = D (Lap Phi - S delta) with
  D = c^2 / (3 calH).  One ADE step of length dt is a Saul'yev sweep: the
  cells of the active box are visited in one lexicographic order (forward:
  z, then y, then x index increasing; backward: all decreasing) and each is
  replaced in place by the solution of
      (1 + 3 lam) Phi_c' = (1 - 3 lam) Phi_c + lam (S6 - f_c),
  lam = D dt / h^2, f = S h^2 delta (the mesh source of Eq. 3), S6 the sum
  of the six neighbours' current values: a neighbour visited earlier in the
  sweep already holds its new value, one not yet visited its old one.  On
  the periodic mesh the wrap-around neighbours follow the same rule; on a
  frozen-exterior box the cells outside keep their values.  In the 7-point
  Laplacian the centre term is split equally between the old and the new
  value, the visited neighbours are taken at the new time and the others at
  the old.
* Each half sub-step of a time step is one sweep, the first forward and the
  second backward (the two consecutive steps in alternate directions), with
  lam = 1 / (kappa h^2) for the kappa of the implicit reading of the same
  half sub-step (kappa = 3 calH / (c^2 dtau / 2), calH at the sub-step end).

Pinned by tests/test_oracle_ade.py: the steady state of the discrete
Poisson problem is a fixed point; each sweep equals the solution of its
lower-triangular linear system (built from the visiting order, solved
densely) on small meshes; a forward-backward pair has spectral radius <= 1
for any lam (the stability the paper states); and alternating sweeps
converge to the exact solution of the semi-discrete equation
(matrix exponential) as dt -> 0.
"""
from __future__ import annotations

import numpy as np


def sweep(phi: np.ndarray, f: np.ndarray, lam: float, lo, hi, periodic: bool,
          forward: bool = True) -> np.ndarray:
    """One Saul'yev sweep over the inclusive index box [lo, hi] (axis order
    x, y, z) of the (N, N, N) array phi indexed [k, j, i]; returns the new
    array (phi is not modified).  periodic: the box is the whole mesh and
    neighbour indices wrap."""
    n = phi.shape[0]
    u = [float(v) for v in phi.ravel()]
    src = [float(v) for v in f.ravel()]
    c_old = 1.0 - 3.0 * lam
    inv = 1.0 / (1.0 + 3.0 * lam)
    ks = range(lo[2], hi[2] + 1)
    js = range(lo[1], hi[1] + 1)
    is_ = range(lo[0], hi[0] + 1)
    if not forward:
        ks, js, is_ = reversed(ks), reversed(js), reversed(is_)
    js, is_ = list(js), list(is_)

    def idx(i, j, k):
        if periodic:
            i, j, k = i % n, j % n, k % n
        return (k * n + j) * n + i

    for k in ks:
        for j in js:
            for i in is_:
                c = idx(i, j, k)
                s6 = (u[idx(i - 1, j, k)] + u[idx(i + 1, j, k)] + u[idx(i, j - 1, k)]
                      + u[idx(i, j + 1, k)] + u[idx(i, j, k - 1)] + u[idx(i, j, k + 1)])
                u[c] = (c_old * u[c] + lam * (s6 - src[c])) * inv
    return np.array(u).reshape(phi.shape)


def half_step_sweeps(phi: np.ndarray, f: np.ndarray, kappa1_h2: float, kappa2_h2: float,
                     lo, hi, periodic: bool):
    """The two half sub-steps of a time step as ADE sweeps: forward with
    lam = 1 / kappa1_h2 to t + dt/2, backward with lam = 1 / kappa2_h2 to
    t + dt (the same source f).  Returns (phi_half, phi_end); the second is
    computed by the caller after the kick in a full step, here for the
    field alone."""
    ph = sweep(phi, f, 1.0 / kappa1_h2, lo, hi, periodic, True)
    pe = sweep(ph, f, 1.0 / kappa2_h2, lo, hi, periodic, False)
    return ph, pe
