"""Pins for the oracle's fixed-point CIC deposit and interpolation (CPU only):
brute force with Python integers, exact mass invariant, node particles,
exact periodic shifts, edge positions."""
import math

import numpy as np
import pytest

from oracle import pm
from synth import clustered_particles, edge_particles, uniform_particles

B = 14


def brute_counts(x, ng, box, frac_bits, periodic):
    """Per-particle loop with Python ints; the coordinate is the FP64 product
    x * (ng 2^B / L) floored, as the deposit defines it."""
    s = float(ng * (1 << frac_bits)) / box
    one = 1 << frac_bits
    out = {}
    for row in x:
        cells, ws = [], []
        for d in range(3):
            u = math.floor(float(row[d]) * s)
            if periodic:
                u %= ng << frac_bits
            cells.append(u >> frac_bits)
            q = u & (one - 1)
            ws.append((one - q, q))
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    i, j, k = cells[0] + dx, cells[1] + dy, cells[2] + dz
                    if periodic:
                        i, j, k = i % ng, j % ng, k % ng
                    key = (k * ng + j) * ng + i
                    out[key] = out.get(key, 0) + ws[0][dx] * ws[1][dy] * ws[2][dz]
    c = np.zeros(ng**3, dtype=np.uint64)
    for key, v in out.items():
        c[key] = v
    return c.reshape(ng, ng, ng)


@pytest.mark.parametrize("maker", ["uniform", "clustered", "edge"])
def test_deposit_matches_brute_force(maker):
    ng, box = 16, 100.0
    if maker == "uniform":
        x, _, _ = uniform_particles(300, box, 11)
    elif maker == "clustered":
        x, _, _ = clustered_particles(300, box, 12, ng=ng)
    else:
        x, _, _ = edge_particles(ng, box)
    got = pm.deposit(x, ng, box, B, True)
    ref = brute_counts(x, ng, box, B, True)
    assert np.array_equal(got, ref)


def test_mass_invariant_exact():
    ng, box = 32, 2000.0
    x, _, _ = clustered_particles(20000, box, 3, ng=ng, width_cells=0.7)
    c = pm.deposit(x, ng, box, B, True)
    assert int(c.sum(dtype=np.uint64)) == x.shape[0] * (1 << (3 * B))


def test_node_particle_single_cell():
    ng, box = 16, 16.0       # h = 1: nodes are integers
    x = np.array([[3.0, 7.0, 11.0]])
    c = pm.deposit(x, ng, box, B, True)
    assert c[11, 7, 3] == 1 << (3 * B)
    assert np.count_nonzero(c) == 1


def test_integer_cell_shift_permutes_counts():
    # With h = 1 and dyadic positions the shifted coordinates are exact, so a
    # shift by whole cells must permute C exactly.
    ng = 16
    rng = np.random.Generator(np.random.PCG64(5))
    x = np.floor(rng.uniform(0, ng, size=(500, 3)) * 1024.0) / 1024.0
    c0 = pm.deposit(x, ng, float(ng), B, True)
    shift = np.array([3.0, 5.0, 1.0])
    x1 = np.mod(x + shift, ng)
    c1 = pm.deposit(x1, ng, float(ng), B, True)
    assert np.array_equal(c1, np.roll(c0, (1, 5, 3), axis=(0, 1, 2)))


def test_periodic_wrap_of_last_coordinate():
    # x just below L rounds to U = N 2^B; the periodic deposit wraps it to 0.
    ng, box = 8, 1000.0
    below = np.nextafter(box, 0.0)
    x = np.array([[below, 0.0, 0.0]])
    c = pm.deposit(x, ng, box, B, True)
    ref = brute_counts(x, ng, box, B, True)
    assert np.array_equal(c, ref)
    assert int(c.sum()) == 1 << (3 * B)


def test_interpolation_is_deposit_transpose():
    # sum_p w_pc g_c over particles equals sum_c C_c g_c / 2^(3B)
    ng, box = 16, 50.0
    x, _, _ = uniform_particles(400, box, 9)
    rng = np.random.Generator(np.random.PCG64(10))
    g = rng.normal(size=(3, ng, ng, ng))
    gp = pm.interpolate(x, g, ng, box, B, True)
    c = pm.deposit(x, ng, box, B, True).astype(np.float64) / 2.0 ** (3 * B)
    for comp in range(3):
        assert gp[:, comp].sum() == pytest.approx((c * g[comp]).sum(), rel=1e-12)


def test_interpolation_of_linear_field_is_exact_in_bulk():
    # CIC reproduces a linear function between nodes (up to the 2^-B quantum)
    ng, box = 16, 16.0
    x, _, _ = uniform_particles(200, box, 4)
    x = np.clip(x, 1.0, 14.0)
    ii = np.arange(ng, dtype=np.float64)
    z, y, xx = np.meshgrid(ii, ii, ii, indexing="ij")
    g = np.stack([2.0 * xx + 0.5 * y, -y + 3.0 * z, z.copy()])
    gp = pm.interpolate(x, g, ng, box, B, True)
    xq = np.floor(x * (1 << B)) / (1 << B)
    ref = np.stack([2 * xq[:, 0] + 0.5 * xq[:, 1], -xq[:, 1] + 3 * xq[:, 2], xq[:, 2]], axis=1)
    assert np.allclose(gp, ref, rtol=0, atol=1e-12)
