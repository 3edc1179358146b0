"""Pins of the ADE oracle (oracle/ade.py) against facts fixed by mathematics
rather than by its own formula: the steady state of the discrete Poisson
problem, the lower-triangular linear system a sweep solves, the unconditional
stability the paper states for alternating directions (Sec. 2.3), and
convergence to the exact solution of the semi-discrete diffusion equation
(Sec. 2.1 Eq. 4)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ade, pm

NB = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def _box_cells(lo, hi):
    return [(i, j, k) for k in range(lo[2], hi[2] + 1) for j in range(lo[1], hi[1] + 1)
            for i in range(lo[0], hi[0] + 1)]


def _at(a, c):
    return a[c[2], c[1], c[0]]


@pytest.mark.parametrize("lam", [0.1, 8.8, 1e4])
@pytest.mark.parametrize("forward", [True, False])
def test_steady_state_is_fixed_point_periodic(lam, forward):
    # phi solving Lap_h phi = f exactly is left unchanged by any sweep
    n = 8
    rng = np.random.default_rng(3)
    phi = rng.normal(size=(n, n, n))
    f = pm.laplacian_periodic(phi)
    out = ade.sweep(phi, f, lam, (0, 0, 0), (n - 1,) * 3, True, forward)
    assert np.max(np.abs(out - phi)) <= 1e-12 * np.max(np.abs(phi)) * max(1.0, lam)


@pytest.mark.parametrize("forward", [True, False])
def test_steady_state_is_fixed_point_box(forward):
    n, lo, hi = 10, (2, 1, 3), (7, 8, 6)
    rng = np.random.default_rng(4)
    phi = rng.normal(size=(n, n, n))
    # f = Lap_h phi on the box (exterior values included) = -(0 - Lap_h phi)
    f = np.zeros_like(phi)
    f[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = -pm.residual_box(
        phi, np.zeros_like(phi), lo, hi, 0.0)
    out = ade.sweep(phi, f, 5.0, lo, hi, False, forward)
    assert np.max(np.abs(out - phi)) <= 1e-12 * 20
    inside = np.zeros(phi.shape, dtype=bool)
    inside[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = True
    assert np.array_equal(out[~inside], phi[~inside])


def _triangular_solve(phi, f, lam, lo, hi, periodic, forward):
    """The sweep as one linear system: unknowns are the new box values; a
    neighbour that comes earlier in the visiting order enters with its new
    value (matrix), a later one or one outside the box with its old value."""
    n = phi.shape[0]
    cells = _box_cells(lo, hi)
    order = {c: q for q, c in enumerate(cells if forward else cells[::-1])}
    col = {c: q for q, c in enumerate(cells)}
    m = len(cells)
    M = np.zeros((m, m))
    rhs = np.zeros(m)
    for c in cells:
        q = col[c]
        M[q, q] = 1.0 + 3.0 * lam
        rhs[q] = (1.0 - 3.0 * lam) * _at(phi, c) - lam * _at(f, c)
        for d in NB:
            nb = tuple(c[a] + d[a] for a in range(3))
            if periodic:
                nb = tuple(v % n for v in nb)
            if nb in order and order[nb] < order[c]:
                M[q, col[nb]] -= lam
            else:
                rhs[q] += lam * _at(phi, nb)
    sol = np.linalg.solve(M, rhs)
    out = phi.copy()
    for c in cells:
        out[c[2], c[1], c[0]] = sol[col[c]]
    return out


@pytest.mark.parametrize("forward", [True, False])
@pytest.mark.parametrize("case", ["periodic", "box"])
def test_sweep_solves_its_triangular_system(forward, case):
    rng = np.random.default_rng(5)
    if case == "periodic":
        n, lo, hi, per = 4, (0, 0, 0), (3, 3, 3), True
    else:
        n, lo, hi, per = 7, (1, 2, 1), (5, 4, 3), False
    phi = rng.normal(size=(n, n, n))
    f = rng.normal(size=(n, n, n))
    for lam in (0.3, 8.8, 300.0):
        got = ade.sweep(phi, f, lam, lo, hi, per, forward)
        ref = _triangular_solve(phi, f, lam, lo, hi, per, forward)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", ["periodic", "box"])
def test_alternating_pair_is_stable_for_any_step(case):
    # homogeneous problem (f = 0, zero exterior): the amplification matrix of
    # a forward + backward pair has spectral radius <= 1 however large lam is
    if case == "periodic":
        n, lo, hi, per = 4, (0, 0, 0), (3, 3, 3), True
    else:
        n, lo, hi, per = 6, (1, 1, 1), (4, 4, 3), False
    cells = _box_cells(lo, hi)
    f = np.zeros((n, n, n))
    for lam in (0.5, 8.8, 1e3, 1e6):
        G = np.zeros((len(cells), len(cells)))
        for q, c in enumerate(cells):
            e = np.zeros((n, n, n))
            e[c[2], c[1], c[0]] = 1.0
            u = ade.sweep(e, f, lam, lo, hi, per, True)
            u = ade.sweep(u, f, lam, lo, hi, per, False)
            G[:, q] = [_at(u, d) for d in cells]
        rho = np.max(np.abs(np.linalg.eigvals(G)))
        assert rho <= 1.0 + 1e-10
        if not per:
            assert rho < 1.0


def test_converges_to_exact_semidiscrete_solution():
    # du/ds = Lap_h u - f on a frozen-exterior box (s = D t / h^2): exact
    # u(S) = u* + expm(S L) (u0 - u*); alternating sweeps of lam = S / (2 m)
    # converge at second order in lam
    n, lo, hi = 6, (1, 1, 1), (4, 4, 4)
    rng = np.random.default_rng(1)
    phi0 = rng.normal(size=(n, n, n))
    f = rng.normal(size=(n, n, n))
    cells = _box_cells(lo, hi)
    col = {c: q for q, c in enumerate(cells)}
    m = len(cells)
    L = np.zeros((m, m))
    g = np.zeros(m)
    for c in cells:
        q = col[c]
        L[q, q] = -6.0
        for d in NB:
            nb = tuple(c[a] + d[a] for a in range(3))
            if nb in col:
                L[q, col[nb]] += 1.0
            else:
                g[q] += _at(phi0, nb)
        g[q] -= _at(f, c)
    u0 = np.array([_at(phi0, c) for c in cells])
    ustar = -np.linalg.solve(L, g)
    S = 1.0
    exact = ustar + sla.expm(S * L) @ (u0 - ustar)
    errs = []
    for pairs in (4, 8, 16, 32):
        lam = S / (2 * pairs)
        u = phi0
        for _ in range(pairs):
            u = ade.sweep(u, f, lam, lo, hi, False, True)
            u = ade.sweep(u, f, lam, lo, hi, False, False)
        v = np.array([_at(u, c) for c in cells])
        errs.append(np.linalg.norm(v - exact) / np.linalg.norm(exact - u0))
    ratios = [errs[q] / errs[q + 1] for q in range(len(errs) - 1)]
    assert all(r > 3.5 for r in ratios), ratios
    assert errs[-1] < 1e-4
