"""GPU parity of the lightcone output (removed particles recorded where they
cross the lightcone).  One step from an identical state, plain FP64 with
static gravity, a = 0.970 -> 0.975, where the lightcone (about 76 Mpc/h at
the step's end) cuts the corners of a 100 Mpc/h box: the records against the
oracle's own step and its bisection for the crossing; the u = 0 records of
sdpm_shrink(a); and a full output buffer (SDPM_EFULL, the run goes on)."""
import numpy as np
import pytest

from oracle import cosmology as oc
from oracle import pm
from synth import uniform_particles

from helpers import lib_config, log, make_sim, oracle_config

pytestmark = pytest.mark.gpu

NG, BOX, N = 32, 100.0, 20000


def _setup(capacity, seed=31):
    import torch
    import paper_1709_04703_amd as P
    x, p, ids = uniform_particles(N, BOX, seed)
    cfg = lib_config(NG, BOX, precision=P.SDPM_PLAIN_FP64, c_grav=0.0, shrink=1, tol=1e-10,
                     n_initial=N)
    sim = make_sim(cfg, N)
    sim.bind(x, p, ids)
    sim.set_lightcone(capacity)
    a = 0.970
    sim.init_potential(a)
    ost = pm.init_state(x, p, ids, oracle_config(cfg), a)
    sim.phi.copy_(torch.as_tensor(ost.phi))
    return sim, cfg, ost, a


def test_step_records_match_oracle():
    sim, cfg, ost, a = _setup(N)
    da = 0.005
    assert ost.n_active == N
    st = sim.step(a, da)
    ost = pm.step(ost, oracle_config(cfg), da, {})
    k = ost.n_active
    log(f"lightcone step: removed {st['n_removed']} (oracle {N - k})")
    assert st["n_removed"] == N - k > 100
    gid, ga, gx, gp = sim.lightcone_records()
    assert np.array_equal(gid, ost.ids[k:N])
    sc = oc.step_scalars(a, da, cfg.omega_m, cfg.omega_l, BOX, NG, 0.0, cfg.c_light)
    xo = np.asarray(cfg.x_obs)
    u, a_ref, x_ref, p_ref = pm.lightcone_crossing(
        ost.x[k:N], ost.p[k:N], xo, sc["r_lc_end"], cfg.c_light * sc["dtau"],
        sc["dtau"] / (a + da), a + da, da)
    log(f"  crossing u in [{u.min():.3f}, {u.max():.3f}]; max |da| {np.abs(ga - a_ref).max():.2e}, "
        f"max |dx| {np.abs(gx - x_ref).max():.2e}")
    assert 0.0 < u.min() and u.max() < 1.0          # every crossing falls inside the step
    assert np.abs(ga - a_ref).max() <= 1e-9
    assert np.abs(gx - x_ref).max() <= 1e-8 * BOX
    assert np.abs(gp - p_ref).max() <= 1e-9 * np.abs(p_ref).max()
    sim.close()


def test_shrink_records_at_the_removal_instant():
    sim, cfg, ost, a = _setup(N, seed=32)
    x, p, ids = sim.particles()
    a2 = 0.99
    r = oc.lightcone_radius(a2, cfg.omega_m, cfg.omega_l, cfg.c_light)
    out = pm.outside_lightcone(x, np.asarray(cfg.x_obs), r)
    nr = sim.shrink(a2)
    assert nr == int(out.sum()) > 0
    gid, ga, gx, gp = sim.lightcone_records()
    assert np.array_equal(gid, ids[out])
    assert np.all(ga == a2)
    assert np.array_equal(gx, x[out]) and np.array_equal(gp, p[out])
    sim.close()


def test_full_output_returns_efull_and_continues():
    import paper_1709_04703_amd as P
    sim, cfg, ost, a = _setup(10, seed=33)
    st = sim.step(a, 0.005, raise_on_error=False)
    assert st["rc"] == P.SDPM_EFULL and st["n_removed"] > 10
    assert sim.lightcone_count() == 10
    gid, _, _, _ = sim.lightcone_records()
    _, _, ids_all = sim.particles(all_particles=True)
    n_act = st["n_active"]
    assert np.array_equal(gid, ids_all[n_act:n_act + 10])
    st2 = sim.step(a + 0.005, 0.005, raise_on_error=False)
    assert st2["rc"] in (P.SDPM_OK, P.SDPM_EFULL)
    assert st2["n_active"] <= n_act and sim.lightcone_count() == 10
    sim.close()
