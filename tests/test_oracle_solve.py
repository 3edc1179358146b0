"""Pins for the oracle's exact mesh solves (CPU only): explicit stencil
residuals, a single Fourier mode in closed form, a dense direct solve on a
tiny box, and O(h^2) convergence to analytic isolated potentials."""
import math

import numpy as np
import pytest

from oracle import pm


def test_periodic_solve_residual_and_gauge():
    rng = np.random.Generator(np.random.PCG64(1))
    ng = 24
    f = rng.normal(size=(ng, ng, ng))
    f -= f.mean()
    phi = pm.solve_periodic(f, 0.0)
    assert abs(phi.mean()) < 1e-14
    r = f - pm.laplacian_periodic(phi)
    assert np.abs(r).max() < 1e-12 * np.abs(f).max() * 10


@pytest.mark.parametrize("kh2", [0.05, 0.4])
def test_periodic_screened_residual(kh2):
    rng = np.random.Generator(np.random.PCG64(2))
    ng = 16
    f = rng.normal(size=(ng, ng, ng))
    phi = pm.solve_periodic(f, kh2)
    r = f - (pm.laplacian_periodic(phi) - kh2 * phi)
    assert np.abs(r).max() < 1e-12


@pytest.mark.parametrize("n,kh2", [(1, 0.0), (3, 0.0), (2, 0.3)])
def test_single_fourier_mode_closed_form(n, kh2):
    ng, box = 32, 100.0
    h = box / ng
    s = 1.5 * 0.3 / 0.5
    xs = np.arange(ng) * h
    delta = np.cos(2 * np.pi * n * xs / box)[None, None, :] * np.ones((ng, ng, 1))
    phi = pm.solve_periodic(s * h * h * delta, kh2)
    ref = -s * h * h * delta / (2.0 - 2.0 * np.cos(2 * np.pi * n / ng) + kh2)
    assert np.abs(phi - ref).max() < 1e-12 * np.abs(ref).max()


def test_box_solve_residual_with_frozen_ring():
    rng = np.random.Generator(np.random.PCG64(3))
    ng = 20
    phi0 = rng.normal(size=(ng, ng, ng))
    rhs = rng.normal(size=(ng, ng, ng))
    lo, hi = np.array([2, 3, 4]), np.array([15, 14, 12])
    for kh2 in (0.0, 0.2):
        phi = pm.solve_box(phi0, rhs, lo, hi, kh2)
        r = pm.residual_box(phi, rhs, lo, hi, kh2)
        assert np.abs(r).max() < 1e-11
        mask = np.ones_like(phi, dtype=bool)
        mask[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = False
        assert np.array_equal(phi[mask], phi0[mask])


def test_box_solve_against_dense_matrix():
    # tiny box: assemble the 7-point operator as a dense matrix and solve
    rng = np.random.Generator(np.random.PCG64(4))
    ng = 7
    phi0 = rng.normal(size=(ng, ng, ng))
    rhs = rng.normal(size=(ng, ng, ng))
    lo, hi = np.array([1, 2, 1]), np.array([4, 4, 3])
    kh2 = 0.15
    cells = [(i, j, k) for k in range(lo[2], hi[2] + 1) for j in range(lo[1], hi[1] + 1)
             for i in range(lo[0], hi[0] + 1)]
    index = {c: n for n, c in enumerate(cells)}
    a = np.zeros((len(cells), len(cells)))
    b = np.zeros(len(cells))
    for n, (i, j, k) in enumerate(cells):
        a[n, n] = -6.0 - kh2
        b[n] = rhs[k, j, i]
        for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            nb = (i + di, j + dj, k + dk)
            if nb in index:
                a[n, index[nb]] += 1.0
            else:
                b[n] -= phi0[nb[2], nb[1], nb[0]]
    sol = np.linalg.solve(a, b)
    phi = pm.solve_box(phi0, rhs, lo, hi, kh2)
    for n, (i, j, k) in enumerate(cells):
        assert phi[k, j, i] == pytest.approx(sol[n], abs=1e-12)


def _isolated_error(ng, source_fn, exact_fn, box=1.0, probe=0.3):
    """Solve Lap Phi = S rho on a Dirichlet box with exact ring data and
    return |Phi - Phi_exact| at cells in a shell at distance ~probe."""
    h = box / ng
    s = 1.0
    c = np.arange(ng) * h - 0.5 * box
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    rhs = s * h * h * source_fn(r, h)
    phi0 = exact_fn(np.where(r > 0, r, h))
    lo, hi = np.array([1, 1, 1]), np.array([ng - 2] * 3)
    phi = pm.solve_box(phi0, rhs, lo, hi, 0.0)
    shell = np.abs(r - probe) < 0.5 * h + 1e-12
    shell &= (r > 0)
    return np.sqrt(np.mean((phi[shell] - exact_fn(r[shell])) ** 2)) / np.sqrt(np.mean(exact_fn(r[shell]) ** 2))


def test_point_mass_converges_second_order():
    # a unit point mass on a node: rho = delta_cell / h^3 -> Phi = -S m / (4 pi r)
    def src(r, h):
        out = np.zeros_like(r)
        out[r == 0] = 1.0 / h**3
        return out

    exact = lambda r: -1.0 / (4 * np.pi * r)  # noqa: E731
    e1 = _isolated_error(32, src, exact)
    e2 = _isolated_error(64, src, exact)
    assert e1 < 0.02
    assert e1 / e2 == pytest.approx(4.0, rel=0.25)


def test_smooth_sphere_converges_second_order():
    # rho = rho0 (1 - r^2/R^2)^2 inside R (Gauss's law, integrated by hand):
    # Phi = S rho0 (r^2/6 - r^4/(10 R^2) + r^6/(42 R^4) - R^2/6) inside,
    # -8 S rho0 R^3 / (105 r) outside
    big_r, rho0 = 0.2, 1.0

    def src(r, h):
        return np.where(r < big_r, rho0 * (1 - r * r / big_r**2) ** 2, 0.0)

    def exact(r):
        inside = rho0 * (r * r / 6 - r**4 / (10 * big_r**2) + r**6 / (42 * big_r**4) - big_r**2 / 6)
        outside = -8 * rho0 * big_r**3 / (105 * r)
        return np.where(r < big_r, inside, outside)

    e1 = _isolated_error(32, src, exact, probe=0.1)
    e2 = _isolated_error(64, src, exact, probe=0.1)
    assert e1 < 0.02
    assert e1 / e2 == pytest.approx(4.0, rel=0.2)


def test_uniform_sphere_exterior():
    # literal uniform sphere: Phi = -S rho0 R^3 / (3 r) outside; the staircase
    # surface makes convergence irregular, so only a bound is asserted
    big_r = 0.2

    def src(r, h):
        return np.where(r < big_r, 1.0, 0.0)

    def exact(r):
        return np.where(r < big_r, (r * r - 3 * big_r**2) / 6, -big_r**3 / (3 * r))

    assert _isolated_error(64, src, exact, probe=0.35) < 0.03
