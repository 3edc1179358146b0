"""Physics pins for the oracle's full step (CPU only): Zel'dovich plane wave
(second-order convergence in h and in dtau), linear growth D(a), momentum
conservation, exact free drift, zero self-force, and direct summation."""
import math

import numpy as np
import pytest

from oracle import cosmology as oc
from oracle import direct, pm
from synth import clustered_particles, lattice_positions

OM, OL = 0.3, 0.7


def _plane_wave(ng, nsteps, a0, a1, amp_final, box=100.0, kvec=(1, 0, 0), c_grav=0.0):
    """Evolve a single Zel'dovich plane wave with the oracle; return the
    signed relative error of the displacement and momentum amplitudes."""
    kv = 2 * np.pi * np.asarray(kvec, dtype=np.float64) / box
    k = np.linalg.norm(kv)
    amp = amp_final / oc.growth_d(a1, OM, OL)
    q = lattice_positions(ng, box)
    s = np.sin(q @ kv)
    khat = kv / k

    def zel(a):
        d = oc.growth_d(a, OM, OL)
        f = oc.growth_f(a, OM, OL)
        psi = -(amp / k) * s[:, None] * khat[None, :]
        return np.mod(q + d * psi, box), a * (a * oc.hubble_e(a, OM, OL)) * f * d * psi

    x0, p0 = zel(a0)
    cfg = pm.Config(ng=ng, box=box, n_initial=ng**3, c_grav=c_grav)
    st = pm.init_state(x0, p0, np.arange(ng**3), cfg, a0)
    da = (a1 - a0) / nsteps
    for _ in range(nsteps):
        st = pm.step(st, cfg, da)
    xe, pe = zel(a1)
    order = np.argsort(st.ids)
    x, p = st.x[order], st.p[order]
    dx = x - q
    dx = (dx + box / 2) % box - box / 2
    disp = dx @ khat
    mom = p @ khat
    ss = (s * s).sum()
    ax = (disp * s).sum() / ss
    axe = (((xe - q + box / 2) % box - box / 2) @ khat * s).sum() / ss
    ap = (mom * s).sum() / ss
    ape = ((pe @ khat) * s).sum() / ss
    return ax / axe - 1.0, ap / ape - 1.0


def test_zeldovich_plane_wave_second_order_in_h():
    # spatial error ~ C h^2 + (same time error): successive differences shrink 4x
    e = [_plane_wave(n, 10, 0.1, 0.5, 0.05) for n in (16, 32, 64)]
    for comp in (0, 1):
        d1 = e[0][comp] - e[1][comp]
        d2 = e[1][comp] - e[2][comp]
        assert d1 / d2 == pytest.approx(4.0, rel=0.2)
    assert abs(e[2][0]) < 0.01 and abs(e[2][1]) < 0.01


def test_zeldovich_plane_wave_second_order_in_dtau():
    e = [_plane_wave(16, n, 0.1, 0.5, 0.05) for n in (10, 20, 40)]
    for comp in (0, 1):
        d1 = e[0][comp] - e[1][comp]
        d2 = e[1][comp] - e[2][comp]
        assert d1 / d2 == pytest.approx(4.0, rel=0.35)


def test_zeldovich_large_amplitude_before_shell_crossing():
    # D A = 0.5 at the end (shell crossing at D A = 1): still tracked closely
    ex, ep = _plane_wave(32, 20, 0.1, 0.5, 0.5)
    assert abs(ex) < 0.02 and abs(ep) < 0.03


def _growth_ratio_error(ng, nsteps, a0, a1, kvec, box=100.0, delta0=1e-4):
    """Evolve a small single mode (delta ~ delta0 at a0) with steps uniform
    in ln a and return (measured growth) / (D(a1)/D(a0)) - 1."""
    kv = 2 * np.pi * np.asarray(kvec, dtype=np.float64) / box
    k = np.linalg.norm(kv)
    khat = kv / k
    q = lattice_positions(ng, box)
    s = np.sin(q @ kv)
    amp = delta0 / k
    psi = -amp * s[:, None] * khat[None, :]
    x0 = np.mod(q + psi, box)
    p0 = a0 * a0 * oc.hubble_e(a0, OM, OL) * oc.growth_f(a0, OM, OL) * psi
    cfg = pm.Config(ng=ng, box=box, n_initial=ng**3)
    st = pm.init_state(x0, p0, np.arange(ng**3), cfg, a0)
    edges = np.geomspace(a0, a1, nsteps + 1)
    for i in range(nsteps):
        st.a = edges[i]
        st = pm.step(st, cfg, edges[i + 1] - edges[i])
    x = st.x[np.argsort(st.ids)]
    dx = (x - q + box / 2) % box - box / 2
    grown = ((dx @ khat) * s).sum() / (s * s).sum() / (-amp)
    return grown / (oc.growth_d(a1, OM, OL) / oc.growth_d(a0, OM, OL)) - 1.0


def test_linear_growth_of_small_mode():
    # delta ~ 1e-4 at a = 0.02 grows by D(1)/D(0.02) (about 39x) to within the
    # O((kh)^2) force error of a 32^3 mesh
    assert abs(_growth_ratio_error(32, 20, 0.02, 1.0, (1, 0, 0))) < 0.04
    assert abs(_growth_ratio_error(32, 20, 0.02, 1.0, (1, 1, 0))) < 0.06


def test_diffusion_gravity_tracks_poisson_on_large_scales():
    # with the gravity speed -> infinity the screened solve tends to Poisson;
    # with the paper's c_eff the large-scale growth stays within a few per cent
    ex0, _ = _plane_wave(16, 10, 0.1, 0.5, 0.05, box=1000.0)
    ex_fast, _ = _plane_wave(16, 10, 0.1, 0.5, 0.05, box=1000.0, c_grav=1e9)
    assert ex_fast == pytest.approx(ex0, abs=1e-9)
    ex_eff, _ = _plane_wave(16, 10, 0.1, 0.5, 0.05, box=1000.0, c_grav=-1.0)
    assert abs(ex_eff - ex0) < 0.2


def test_momentum_conservation_periodic_poisson():
    ng, box = 32, 100.0
    x, _, _ = clustered_particles(3000, box, 21, ng=ng, width_cells=1.0)
    h = box / ng
    c = pm.deposit(x, ng, box, 14, True)
    f = pm.source(c, x.shape[0], 14, 1.0, h, True)
    phi = pm.solve_periodic(f, 0.0)
    g = pm.interpolate(x, pm.force_mesh(phi, h), ng, box, 14, True)
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * np.abs(g).sum()


def test_node_particle_has_zero_self_force():
    ng, box = 16, 16.0
    x = np.array([[5.0, 9.0, 2.0]])
    c = pm.deposit(x, ng, box, 14, True)
    f = pm.source(c, ng**3, 14, 1.0, 1.0, True)
    phi = pm.solve_periodic(f, 0.0)
    g = pm.interpolate(x, pm.force_mesh(phi, 1.0), ng, box, 14, True)
    assert np.abs(g).max() < 1e-14 * np.abs(phi).max()


@pytest.mark.parametrize("c_grav", [0.0, -1.0])
def test_free_drift_of_uniform_lattice(c_grav):
    # one particle per cell moving rigidly: CIC density is exactly uniform,
    # so g = 0 and x_N = x_0 + p sum_n (dtau_n/2)(1/a_n + 1/a_{n+1})
    ng, box = 8, 64.0
    x0 = lattice_positions(ng, box)
    p0 = np.tile([0.3, -1.7, 2.2], (ng**3, 1))
    cfg = pm.Config(ng=ng, box=box, n_initial=ng**3, c_grav=c_grav)
    st = pm.init_state(x0, p0, np.arange(ng**3), cfg, 0.1)
    a, da, travel = 0.1, 0.05, 0.0
    for _ in range(6):
        dt = oc.dtau(a, a + da, OM, OL)
        travel += 0.5 * dt * (1.0 / a + 1.0 / (a + da))
        st = pm.step(st, cfg, da)
        a += da
    assert np.array_equal(st.p, p0)
    assert np.abs(st.phi).max() == 0.0
    ref = np.mod(x0 + p0 * travel, box)
    d = (st.x - ref + box / 2) % box - box / 2
    assert np.abs(d).max() < 1e-12 * box


def test_pm_forces_match_direct_summation_isolated():
    # isolated set of particles: Dirichlet box with exact ring potential;
    # PM forces match direct summation for well-separated particles
    ng, box, npart, b = 64, 1.0, 120, 14
    rng = np.random.Generator(np.random.PCG64(7))
    x = rng.uniform(0.2, 0.8, size=(npart, 3))
    h = box / ng
    s, mass = 1.0, box**3 / npart
    c = pm.deposit(x, ng, box, b, False)
    nbar = npart / ng**3
    rhs = s * h * h * c.astype(np.float64) / (nbar * 2.0 ** (3 * b))
    grid = np.arange(ng) * h
    zz, yy, xx = np.meshgrid(grid, grid, grid, indexing="ij")
    ring = np.ones((ng, ng, ng), dtype=bool)
    ring[1:-1, 1:-1, 1:-1] = False
    pts = np.stack([xx[ring], yy[ring], zz[ring]], axis=1)
    phi0 = np.zeros((ng, ng, ng))
    phi0[ring] = direct.potential(pts, x, s, mass)
    phi = pm.solve_box(phi0, rhs, [1, 1, 1], [ng - 2] * 3, 0.0)
    g_pm = pm.interpolate(x, pm.force_mesh(phi, h), ng, box, b, False)
    g_dir = direct.forces(x, s, mass)
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    isolated = d.min(axis=1) > 4 * h
    assert isolated.sum() > 40
    err = np.linalg.norm(g_pm - g_dir, axis=1) / np.linalg.norm(g_dir, axis=1)
    assert np.median(err[isolated]) < 0.03
    assert np.sqrt(np.mean(err[isolated] ** 2)) < 0.08
