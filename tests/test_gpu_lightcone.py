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


def _setup(capacity, seed=31, shrink=1):
    import torch
    import paper_1709_04703_amd as P
    x, p, ids = uniform_particles(N, BOX, seed)
    cfg = lib_config(NG, BOX, precision=P.SDPM_PLAIN_FP64, c_grav=0.0, shrink=shrink, tol=1e-10,
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


def test_fixed_domain_records_crossings_without_removal():
    # shrink = 0: two steps record the particles that cross the lightcone
    # (outside at a step's end, inside at its start), none is removed and
    # none is recorded twice
    sim, cfg, ost, a = _setup(N, seed=34, shrink=0)
    ocfg = oracle_config(cfg)
    xo = np.asarray(cfg.x_obs)
    r_start = oc.lightcone_radius(a, cfg.omega_m, cfg.omega_l, cfg.c_light)
    # (the second step starts with the first step's crossers outside)
    seen = 0
    for da in (0.005, 0.005):
        x0 = ost.x.copy()
        st = sim.step(a, da)
        ost = pm.step(ost, ocfg, da, {})
        assert st["n_removed"] == 0 and sim.n_active == N and ost.n_active == N
        sc = oc.step_scalars(a, da, cfg.omega_m, cfg.omega_l, BOX, NG, 0.0, cfg.c_light)
        crossed = pm.lightcone_crossed(x0, ost.x, xo, r_start, sc["r_lc_end"])
        gid, ga, gx, gp = sim.lightcone_records()
        gid, ga, gx, gp = gid[seen:], ga[seen:], gx[seen:], gp[seen:]
        order = np.argsort(gid)
        ref_ids = np.sort(ost.ids[crossed])
        log(f"fixed-domain step a={a:.3f}: recorded {len(gid)}, oracle {len(ref_ids)}")
        assert len(ref_ids) > 50
        assert np.array_equal(gid[order], ref_ids)
        sel = np.argsort(ost.ids[crossed])
        u, a_ref, x_ref, p_ref = pm.lightcone_crossing(
            ost.x[crossed][sel], ost.p[crossed][sel], xo, sc["r_lc_end"],
            cfg.c_light * sc["dtau"], sc["dtau"] / (a + da), a + da, da)
        assert np.abs(ga[order] - a_ref).max() <= 1e-9
        assert np.abs(gx[order] - x_ref).max() <= 1e-8 * BOX
        assert np.abs(gp[order] - p_ref).max() <= 1e-9 * np.abs(p_ref).max()
        seen += len(gid)
        a, r_start = a + da, sc["r_lc_end"]
    all_ids = sim.lightcone_records()[0]
    assert len(np.unique(all_ids)) == len(all_ids) == sim.lightcone_count()
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


def test_shrinking_and_fixed_domain_lightcones_agree():
    # the paper's check (Sec. 3.2): a run that shrinks the domain and one on
    # the fixed periodic domain record the same particles on the lightcone
    # at nearly the same places (64^3, 2000 Mpc/h, z = 49 -> 0 in 32 steps,
    # diffusion gravity, FP64).  The runs part once the shrinking run freezes
    # the exterior and empties the box corners outside the sphere, which acts
    # on the largest scales; the spectra are compared on wavelengths up to a
    # quarter of the box.  There a position change dx_j moves each term
    # exp(-i k.x_j) of the density transform by at most |k| |dx_j|, so to
    # first order the relative change of P(k) is at most 2 |k| times the
    # typical position change: the bound is 2 k_max rms(dx).
    import paper_1709_04703_amd as P
    from synth import zeldovich_ics
    ng, box, nsteps = 64, 2000.0, 32
    a0 = 1.0 / 50.0
    x, p, ids = zeldovich_ics(ng, box, a0, 4703)
    rec = {}
    for shrink in (1, 0):
        cfg = lib_config(ng, box, c_grav=-1.0, shrink=shrink, precision=P.SDPM_PLAIN_FP64,
                         n_initial=ng**3, tol=1e-10)
        sim = make_sim(cfg, ng**3)
        sim.bind(x, p, ids)
        sim.set_lightcone(ng**3)
        sim.init_potential(a0)
        edges = np.linspace(a0, 1.0, nsteps + 1)
        for q in range(nsteps):
            sim.step(edges[q], edges[q + 1] - edges[q])
        gid, ga, gx, _ = sim.lightcone_records()
        o = np.argsort(gid)
        rec[shrink] = (gid[o], ga[o], gx[o])
        sim.close()
    assert np.array_equal(rec[1][0], rec[0][0]) and len(rec[1][0]) == ng**3
    d = np.abs(rec[1][2] - rec[0][2])
    d = np.minimum(d, box - d) / (box / ng)
    pk_s = P.power_spectrum(_dev_wrapped(rec[1][2], box), box, ng, shot=False, jing=False)
    pk_f = P.power_spectrum(_dev_wrapped(rec[0][2], box), box, ng, shot=False, jing=False)
    kf = 2.0 * np.pi / box
    sel = (pk_f["modes"] >= 20) & (pk_f["k"] >= 4.0 * kf)
    dp = np.abs(pk_s["p_raw"][sel] / pk_f["p_raw"][sel] - 1.0).max()
    rms_dx = float(np.sqrt(np.mean(np.sum((d * (box / ng)) ** 2, axis=1))))
    bound = 2.0 * pk_f["k"][sel].max() * rms_dx
    log(f"shrink vs fixed: max position difference {d.max():.2e} cells (rms {rms_dx:.2e} Mpc/h), "
        f"max |da| {np.abs(rec[1][1] - rec[0][1]).max():.2e}, P(k) max rel diff {dp:.2e} "
        f"(bound {bound:.2e}) at k >= 4 k_f")
    assert d.max() < 0.05
    assert dp < bound


def _dev_wrapped(x, box):
    import torch
    xw = np.mod(x, box)
    xw[xw >= box] = 0.0
    return torch.as_tensor(np.ascontiguousarray(xw.T)).cuda()
