"""Host-side check of the rounding bound behind the estimating correction pass,
CPU only.

After a defect correction phi += e, where e solved A e = r_old for the stored
residual r_old (FP32 in mixed precision) of the implicit step's operator
A = Lap_h - kappa h^2 (Sec. 2.1 Eq. 4, 7-point Laplacian in grid units), the
library estimates the new residual as r_old - A e instead of recomputing
rhs - A phi in FP64, and stops when the estimate plus a bound is below the
threshold.  The bound is

    u_T / (1 - u_T) |r_old| + g16 (2 |rhs| + |r_old| + (12 + kappa h^2)(4 |phi| + 3 |e|)),

u_T the unit roundoff of the stored residual's type, g16 = 16 u / (1 - 16 u)
with u that of FP64, norms over the solved cells.  Here both residuals are
evaluated in FP64 with numpy in the library's order of operations on random
and adversarial periodic fields (a potential far larger than the source, a
correction that leaves almost nothing, FP32 and FP64 storage), and the
distance between them must stay within the bound.
"""
import numpy as np
import pytest


def _apply(phi, kappa):
    nb = (np.roll(phi, 1, 0) + np.roll(phi, -1, 0) + np.roll(phi, 1, 1) + np.roll(phi, -1, 1)
          + np.roll(phi, 1, 2) + np.roll(phi, -1, 2))
    return nb - 6.0 * phi - kappa * phi


def _bound(no, nb, nphi, ne, kappa, ut):
    u = 0.5 * np.finfo(np.float64).eps
    g16 = 16.0 * u / (1.0 - 16.0 * u)
    return ut / (1.0 - ut) * no + g16 * (2.0 * nb + no + (12.0 + kappa) * (4.0 * nphi + 3.0 * ne))


def _solve_periodic(r, kappa):
    # exact inverse of the 7-point operator by FFT (kappa > 0)
    n = r.shape[0]
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    lam = sum(np.meshgrid(*(2.0 - 2.0 * np.cos(k),) * 3, indexing="ij"))
    return np.real(np.fft.ifftn(np.fft.fftn(r) / (-lam - kappa)))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("case", ["random", "large_phi", "nearly_solved"])
def test_estimate_within_bound(dtype, case):
    rng = np.random.Generator(np.random.PCG64(4703 + len(case)))
    n, kappa = 16, 0.113
    rhs = rng.normal(size=(n, n, n))
    phi_old = rng.normal(size=(n, n, n)) * (1e4 if case == "large_phi" else 1.0)
    r_old = rhs - _apply(phi_old, kappa)                      # the FP64 residual pass
    r_stored = r_old.astype(dtype)                            # what the cycles solve for
    if case == "nearly_solved":
        e = _solve_periodic(r_stored.astype(np.float64), kappa)
    else:
        e = _solve_periodic(r_stored.astype(np.float64), kappa) + 1e-3 * rng.normal(size=(n, n, n))
    e = e.astype(dtype).astype(np.float64)                    # the stored correction
    phi_new = phi_old + e
    true = rhs - _apply(phi_new, kappa)                       # what the FP64 pass would give
    est = r_stored.astype(np.float64) - _apply(e, kappa)      # the estimating pass
    ut = 0.5 * float(np.finfo(dtype).eps)
    b = _bound(np.linalg.norm(r_stored), np.linalg.norm(rhs), np.linalg.norm(phi_new),
               np.linalg.norm(e), kappa, ut)
    dist = np.linalg.norm(true - est)
    assert dist <= b
    # the bound is not vacuous: well below the residual left by a correction
    # that is not nearly exact
    if case == "random":
        assert b < 1e-3 * np.linalg.norm(true)


def test_acceptance_implies_fp64_check():
    # an estimate accepted with its bound (est + bound <= threshold) means the
    # FP64 residual is below the threshold too, for a threshold just above the
    # accepted value
    rng = np.random.Generator(np.random.PCG64(17))
    n, kappa = 16, 0.05
    rhs = rng.normal(size=(n, n, n))
    phi_old = rng.normal(size=(n, n, n))
    r32 = (rhs - _apply(phi_old, kappa)).astype(np.float32).astype(np.float64)
    e = _solve_periodic(r32, kappa).astype(np.float32).astype(np.float64)
    phi_new = phi_old + e
    true = np.linalg.norm(rhs - _apply(phi_new, kappa))
    est = np.linalg.norm(r32 - _apply(e, kappa))
    b = _bound(np.linalg.norm(r32), np.linalg.norm(rhs), np.linalg.norm(phi_new),
               np.linalg.norm(e), kappa, 0.5 * float(np.finfo(np.float32).eps))
    thresh = (est + b) * (1.0 + 1e-9)
    assert true <= thresh


@pytest.mark.parametrize("exterior", [1.0, 1e3, 1e5])
def test_estimate_within_bound_on_a_frozen_exterior_box(exterior):
    # a Dirichlet box inside the mesh: the correction is zero outside it, the
    # residuals and the norms are taken over its cells, and the frozen
    # exterior potential (here up to 1e5 times the interior one) enters the
    # FP64 residual evaluations at the box's faces
    rng = np.random.Generator(np.random.PCG64(5))
    n, kappa, lo, hi = 16, 0.113, 2, 13
    sl = (slice(lo, hi + 1),) * 3
    inner = (hi - lo + 1,) * 3
    rhs = rng.normal(size=(n, n, n))
    phi_old = rng.normal(size=(n, n, n)) * exterior
    phi_old[sl] = rng.normal(size=inner)
    r_old = np.zeros_like(rhs)
    r_old[sl] = (rhs - _apply(phi_old, kappa))[sl]
    r32 = r_old.astype(np.float32).astype(np.float64)
    e = np.zeros_like(rhs)
    e[sl] = (1e-2 * rng.normal(size=inner)).astype(np.float32)
    phi_new = phi_old + e
    true = (rhs - _apply(phi_new, kappa))[sl]
    est = (r32 - _apply(e, kappa))[sl]
    b = _bound(np.linalg.norm(r32[sl]), np.linalg.norm(rhs[sl]), np.linalg.norm(phi_new[sl]),
               np.linalg.norm(e[sl]), kappa, 0.5 * float(np.finfo(np.float32).eps))
    assert np.linalg.norm(true - est) <= b
