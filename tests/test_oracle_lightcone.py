"""Pins for the oracle's lightcone crossing (CPU only): closed forms for
radial and static motion, the on-sphere invariant of every recorded point,
and the clamps at the step's ends."""
import numpy as np
import pytest

from oracle import pm

XO = np.array([50.0, 50.0, 50.0])


def test_radial_outward_closed_form():
    # |d| - u |w| = r + u L  =>  u = (|d| - r) / (|w| + L)
    x1 = np.array([[XO[0] + 80.0, XO[1], XO[2]], [XO[0], XO[1] - 77.0, XO[2]]])
    w = np.array([[1.0, 0.0, 0.0], [0.0, -2.5, 0.0]])
    disp, light, r1 = 0.5, 16.0, 75.0
    u, a, xc, pc = pm.lightcone_crossing(x1, w / disp, XO, r1, light, disp, 0.975, 0.005)
    ref = (np.array([80.0, 77.0]) - r1) / (np.array([1.0, 2.5]) + light)
    assert np.allclose(u, ref, rtol=1e-13, atol=0)
    assert np.allclose(a, 0.975 - ref * 0.005, rtol=1e-15)
    assert np.array_equal(pc, w / disp)


def test_radial_inward_and_static_closed_forms():
    # inward: |d| + u |w| = r + u L  =>  u = (|d| - r) / (L - |w|); static: (|d| - r) / L
    x1 = np.array([[XO[0], XO[1], XO[2] + 76.0], [XO[0] - 78.0, XO[1], XO[2]]])
    p1 = np.array([[0.0, 0.0, -3.0], [0.0, 0.0, 0.0]])
    disp, light, r1 = 1.0, 12.0, 75.0
    u, _, xc, _ = pm.lightcone_crossing(x1, p1, XO, r1, light, disp, 1.0, 0.01)
    assert u[0] == pytest.approx(1.0 / (12.0 - 3.0), rel=1e-13)
    assert u[1] == pytest.approx(3.0 / 12.0, rel=1e-13)
    assert np.allclose(xc[1], x1[1])


def test_recorded_points_lie_on_the_lightcone():
    rng = np.random.Generator(np.random.PCG64(5))
    n, r1, light, disp = 2000, 70.0, 15.0, 0.7
    direc = rng.normal(size=(n, 3))
    direc /= np.linalg.norm(direc, axis=1)[:, None]
    x1 = XO + direc * (r1 + rng.uniform(1e-6, 14.0, size=n))[:, None]
    p1 = rng.normal(size=(n, 3)) * 5.0
    u, a, xc, _ = pm.lightcone_crossing(x1, p1, XO, r1, light, disp, 0.9, 0.01)
    inside = u < 1.0
    assert inside.sum() > n // 2
    dist = np.linalg.norm(xc - XO, axis=1)
    assert np.allclose(dist[inside], r1 + u[inside] * light, rtol=1e-12)
    assert np.all((u >= 0.0) & (u <= 1.0))
    # outside at the step's start (f(1) > 0): the record is the start
    far = ~inside
    y = x1[far] - XO - p1[far] * disp
    assert np.all(np.sum(y * y, axis=1) >= (r1 + light) ** 2 * (1 - 1e-12))


def test_no_light_travel_records_the_removal_instant():
    x1 = XO + np.array([[90.0, 0.0, 0.0]])
    u, a, xc, _ = pm.lightcone_crossing(x1, np.ones((1, 3)), XO, 75.0, 0.0, 0.0, 0.6, 0.0)
    assert u[0] == 0.0 and a[0] == 0.6 and np.array_equal(xc, x1)


def test_fixed_domain_crossing_step_of_radial_motion():
    # Fixed domain (nothing removed): a particle moving radially at constant
    # comoving speed v, d(tau) = d0 + v (tau - tau0), meets the shrinking
    # lightcone r(tau) = c (tau(1) - tau) at tau* = (c tau(1) - d0 + v tau0) / (c + v).
    # In Einstein-de Sitter (H0 = 1) tau = 2 sqrt(a), so r(a) = 2 c (1 - sqrt(a)).
    # lightcone_crossed must flag each particle in exactly the step that
    # contains tau*, and in no other.
    c = 2997.92458
    a_edges = np.linspace(0.5, 1.0, 41)
    tau = 2.0 * np.sqrt(a_edges)
    tau0, tau1 = tau[0], 2.0
    rng = np.random.Generator(np.random.PCG64(11))
    n = 400
    direc = rng.normal(size=(n, 3))
    direc /= np.linalg.norm(direc, axis=1)[:, None]
    v = rng.uniform(-0.3, 0.3, size=n) * c          # inward and outward
    r0 = c * (tau1 - tau0)
    # inward movers must not reach the observer before a = 1
    lower = np.maximum(0.02 * r0, -v * (tau1 - tau0) + 1.0)
    d0 = lower + rng.uniform(0.0, 1.0, size=n) * (0.98 * r0 - lower)
    t_star = (c * tau1 - d0 + v * tau0) / (c + v)
    expect = np.searchsorted(tau, t_star, side="left") - 1   # tau_j < tau* <= tau_{j+1}
    assert np.all((expect >= 0) & (expect < len(tau) - 1))
    # keep clear of step edges by far more than rounding
    gap = np.min(np.abs(t_star[:, None] - tau[None, :]), axis=1)
    keep = gap > 1e-9
    hits = np.zeros(n, dtype=np.int64)
    first = np.full(n, -1)
    for j in range(len(tau) - 1):
        xs = XO + direc * (d0 + v * (tau[j] - tau0))[:, None]
        xe = XO + direc * (d0 + v * (tau[j + 1] - tau0))[:, None]
        rs = 2.0 * c * (1.0 - np.sqrt(a_edges[j]))
        re = 2.0 * c * (1.0 - np.sqrt(a_edges[j + 1]))
        got = pm.lightcone_crossed(xs, xe, XO, rs, re)
        hits += got
        first = np.where(got & (first < 0), j, first)
    assert np.count_nonzero(keep) > 0.99 * n
    assert np.all(hits[keep] == 1)
    assert np.array_equal(first[keep], expect[keep])
