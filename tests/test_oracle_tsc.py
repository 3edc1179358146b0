"""Pins of the oracle's fixed-point TSC assignment (oracle/pm.py,
tsc_weights / deposit / interpolate with assignment="tsc") against facts that
hold for the TSC kernel itself: the weights at a node (1/8, 3/4, 1/8) and
midway between nodes (1/2, 1/2, 0), closeness to the continuous kernel for
any offset, the first moment (centre of mass kept to one unit), exact mass,
exact interpolation of constant and linear fields, and zero self-force."""
import numpy as np
import pytest

from oracle import pm

B = 14
ONE = 1 << B


def _w(d_units):
    u = np.array([[1000 * ONE + d] for d in d_units], dtype=np.int64)   # node 1000 + offset
    node, w = pm.tsc_weights(u, B)
    return node[:, 0], np.stack([w[0][:, 0], w[1][:, 0], w[2][:, 0]], axis=1)


def test_weights_at_a_node_and_midway():
    node, w = _w([0])
    assert node[0] == 1000
    assert list(w[0]) == [ONE // 8, 3 * ONE // 4, ONE // 8]
    # U = node 2^B - 2^(B-1): exactly midway between nodes 999 and 1000
    node, w = _w([-ONE // 2])
    assert node[0] == 1000 and list(w[0]) == [ONE // 2, ONE // 2, 0]


def test_weights_close_to_the_continuous_kernel_and_sum_exactly():
    rng = np.random.default_rng(4)
    d = rng.integers(-ONE // 2, ONE // 2, size=5000)
    node, w = _w(d)
    assert np.all(node == 1000)
    assert np.all(w.sum(axis=1) == ONE) and np.all(w >= 0)
    t = d / ONE
    cont = np.stack([0.5 * (0.5 - t) ** 2, 0.75 - t * t, 0.5 * (0.5 + t) ** 2], axis=1)
    err = np.abs(w / ONE - cont)
    assert err[:, [0, 2]].max() <= 0.5 / ONE + 1e-15
    assert err[:, 1].max() <= 1.0 / ONE + 1e-15
    # first moment: the weighted node offset is the particle offset to one unit
    assert np.abs((w[:, 2] - w[:, 0]) - d).max() <= 1


def test_node_assignment_across_a_cell():
    # U from one node to the next: the nearest node switches at the midpoint
    u = np.arange(999 * ONE, 1001 * ONE + 1, 997, dtype=np.int64)[:, None]
    node, _ = pm.tsc_weights(u, B)
    assert np.array_equal(node[:, 0], (u[:, 0] + ONE // 2) >> B)


def test_deposit_conserves_mass_and_interpolates_fields_exactly():
    ng, box, n = 16, 40.0, 3000
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, box, size=(n, 3))
    c = pm.deposit(x, ng, box, B, True, "tsc")
    assert int(c.sum(dtype=np.uint64)) == n << (3 * B)
    # constant field: exact (weights sum to 2^3B)
    g = np.ones((3, ng, ng, ng)) * np.array([1.5, -2.0, 0.25])[:, None, None, None]
    gi = pm.interpolate(x, g, ng, box, B, True, "tsc")
    assert np.array_equal(gi, np.broadcast_to([1.5, -2.0, 0.25], gi.shape))
    # linear field along x on a non-periodic mesh: the position to 2^-B cells
    h = box / ng
    xs = rng.uniform(3 * h, box - 3 * h, size=(n, 3))
    lin = np.zeros((3, ng, ng, ng))
    lin[0] = np.arange(ng)[None, None, :] * 1.0          # value = node index along x
    gl = pm.interpolate(xs, lin, ng, box, B, False, "tsc")
    u = pm.fixed_point_coords(xs, ng, box, B, False)
    assert np.abs(gl[:, 0] - u[:, 0] / ONE).max() <= 1.0 / ONE + 1e-12


def test_zero_self_force_on_a_node():
    ng, box = 16, 16.0
    x = np.array([[8.0, 8.0, 8.0]])                      # exactly on node (8, 8, 8)
    c = pm.deposit(x, ng, box, B, True, "tsc")
    f = pm.source(c, 1, B, 1.0, box / ng, True)
    phi = pm.solve_periodic(f, 0.0)
    g = pm.interpolate(x, pm.force_mesh(phi, box / ng), ng, box, B, True, "tsc")
    assert np.abs(g).max() <= 1e-12 * np.abs(pm.force_mesh(phi, box / ng)).max()


def test_tsc_step_runs_and_keeps_mass():
    # the oracle's whole step with TSC assignment on a small periodic run
    from synth import zeldovich_ics
    ng, box, a0 = 16, 100.0, 0.05
    x, p, ids = zeldovich_ics(ng, box, a0, 3, "powerlaw-2")
    cfg = pm.Config(ng=ng, box=box, c_grav=-1.0, n_initial=ng**3, assignment="tsc")
    st = pm.init_state(x, p, ids, cfg, a0)
    diag = {}
    st2 = pm.step(st, cfg, 0.01, diag)
    assert int(diag["counts"].sum(dtype=np.uint64)) == ng**3 << (3 * B)
    assert np.isfinite(st2.p).all()
    with pytest.raises(ValueError):
        pm.deposit(x, ng, box, B, True, "ngp")
