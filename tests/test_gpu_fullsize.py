"""Parity at the benchmark's full size and launch configuration: 512^3
particles on a 512^3 mesh, 2000 Mpc/h, synthetic LCDM Zel'dovich ICs at z = 49
(seed 512), the paper's reduced gravity speed, FP32 V-cycles in FP64 defect
correction to 1e-8, Morton re-sort every 10 steps.  The oracle cannot redo a
whole step at this size in seconds, so it checks what it can compute one by
one and properties that hold at any size, on one full sdpm_step (the first of
the run, which also sorts):

 * sort: the particle order is exactly the stable sort by the key (Morton
   code of the 16^3-cell block, then the cell row inside it; a stable sort
   has one result);
 * drift + deposit: positions after the first drift equal x + p c evaluated
   in FP64 (no fused multiply-add), so the total mass (sum of counts =
   n 2^(3B)) and the counts of whole z-planes (both periodic edges and the
   middle) are bit-exact against the oracle's deposit of the particles that
   reach those planes; a separate test checks the whole counts array
   bit for bit at step 25 of the run, where the particles have moved off
   their sorted rows;
 * both solves: the potentials against the oracle's exact FFT solves of the
   oracle's own source of those counts, within cond(A) * tol;
 * kick + second drift: sampled momenta within FP32 rounding plus a 1e-5
   relative force error, and positions bit-exact given the GPU's momenta;
 * force: sampled interpolated forces at the end of the step, 1e-5 relative
   RMS against central differences of the exact potential;
 * removal: the removed set and the stable order of the survivors, exact, for
   a sphere that cuts the box, and the Dirichlet index box it implies."""
import numpy as np
import pytest

from oracle import cosmology as ocosmo
from oracle import pm
from synth import zeldovich_ics

from helpers import cond_periodic, lib_config, log, make_sim, rel_rms

pytestmark = pytest.mark.gpu

NG, BOX, Z_INIT, SEED, SCHEDULE, B = 512, 2000.0, 49.0, 512, 200, 14


def morton_key(x, ng, box, shift):
    """Sort key: the Morton code of the cell's block (cells >> shift; bit b
    of the block's x, y, z index goes to bit 3b, 3b+1, 3b+2, from a table of
    the bit spreading of 0..1023), then the z and y index of the cell's row
    inside the block."""
    table = np.array([sum(((v >> b) & 1) << (3 * b) for b in range(10)) for v in range(1024)],
                     dtype=np.int64)
    key = np.zeros(x.shape[0], dtype=np.int64)
    inner = (1 << shift) - 1
    rows = np.zeros(x.shape[0], dtype=np.int64)
    for d in range(3):
        c = np.clip(np.floor(x[:, d] * (ng / box)), 0, ng - 1).astype(np.int64)
        key |= table[c >> shift] << d
        if d == 1:
            rows |= c & inner
        elif d == 2:
            rows |= (c & inner) << shift
    return (key << (2 * shift)) | rows


def exact_counts(x, periodic):
    """The oracle's CIC deposit (its fixed-point coordinates and corner
    weights) summed exactly at full size: np.add.at over 10^9 corner
    contributions takes minutes, so each uint64 weight (< 2^42) is split
    into two 21-bit halves accumulated by np.bincount in float64, where
    every partial sum is an integer below 2^53 and hence exact in any order."""
    u = pm.fixed_point_coords(x, NG, BOX, B, periodic)
    lo_sum = np.zeros(NG**3)
    hi_sum = np.zeros(NG**3)
    mask = np.uint64((1 << 21) - 1)
    for flat, wt in pm._corners(u, NG, B, periodic):
        lo_sum += np.bincount(flat, weights=(wt & mask).astype(np.float64), minlength=NG**3)
        hi_sum += np.bincount(flat, weights=(wt >> np.uint64(21)).astype(np.float64),
                              minlength=NG**3)
        del flat, wt
    assert max(lo_sum.max(), hi_sum.max()) < 2.0**53
    return ((hi_sum.astype(np.uint64) << np.uint64(21)) + lo_sum.astype(np.uint64)).reshape(
        NG, NG, NG)


def wrap(x, box):
    x = np.where(x < 0.0, x + box, x)
    return np.where(x >= box, x - box, x)


@pytest.fixture(scope="module")
def big():
    import paper_1709_04703_amd as P
    a0 = 1.0 / (1.0 + Z_INIT)
    log(f"full size: ICs {NG}^3, seed {SEED}")
    x, p, ids = zeldovich_ics(NG, BOX, a0, SEED)
    n = x.shape[0]
    cfg = lib_config(NG, BOX, c_grav=-1.0, shrink=1, precision=P.SDPM_MIXED, n_initial=n,
                     sort_every=10)
    sim = make_sim(cfg, n)
    sim.bind(x, p, ids)
    del x, p, ids
    sim.init_potential(a0)
    yield dict(sim=sim, cfg=cfg, n=n, a0=a0, edges=np.linspace(a0, 1.0, SCHEDULE + 1))
    sim.close()


def test_fullsize_step(big):
    sim, cfg, n = big["sim"], big["cfg"], big["n"]
    a, da = big["edges"][0], big["edges"][1] - big["edges"][0]
    h = BOX / NG
    x0, p0, ids0 = sim.particles()
    phi0 = sim.phi_numpy().copy()
    log("full size: one step (sorts first)")
    st = sim.step(a, da)
    assert st["n_active"] == n and st["periodic"] == 1
    assert max(st["res"]) <= cfg.tol
    x1, p1, ids1 = sim.particles()

    # sort: exactly the stable sort by the block Morton + row key (ids are the initial
    # indices): a permutation with non-decreasing keys, ties in index order
    assert np.array_equal(ids0, np.arange(n, dtype=np.uint32))
    order = ids1.astype(np.int64)
    seen = np.zeros(n, dtype=bool)
    seen[order] = True
    assert seen.all()
    key = morton_key(x0, NG, BOX, cfg.sort_shift)[order]
    dk = np.diff(key)
    assert np.all(dk >= 0)
    assert np.all(np.diff(order)[dk == 0] > 0)
    del seen, key, dk
    x0, p0 = x0[order], p0[order]
    del order

    # first drift and the deposit: exact
    c1 = 0.5 * st["dtau"] / a
    xh = wrap(x0 + p0 * c1, BOX)
    counts = sim.counts_numpy().reshape(NG, NG, NG)
    lo = int((counts & np.uint64(0xFFFFFFFF)).sum(dtype=np.uint64))
    hi = int((counts >> np.uint64(32)).sum(dtype=np.uint64))
    assert (hi << 32) + lo == n << (3 * B)
    kz = pm.fixed_point_coords(xh[:, 2:3], NG, BOX, B, True)[:, 0] >> B
    for k in (0, 1, 255, 256, NG - 1):
        sel = (kz == k) | (kz == (k - 1) % NG)
        ref = pm.deposit(xh[sel], NG, BOX, B, True)[k]
        assert np.array_equal(counts[k], ref), f"plane {k}"
    del kz
    log("  sort, drift and deposit planes exact")

    # both solves against the oracle's exact solves of its own source
    sc = ocosmo.step_scalars(a, da, cfg.omega_m, cfg.omega_l, BOX, NG, cfg.c_grav, cfg.c_light)
    k1, k2 = st["kappa_h2"]
    assert k1 == pytest.approx(sc["kappa1_h2"], rel=1e-12)
    assert k2 == pytest.approx(sc["kappa2_h2"], rel=1e-12)
    f = pm.source(counts, n, B, sc["s_half"], h, True)
    del counts
    phi_half = pm.solve_periodic(f - k1 * phi0, k1)
    del phi0
    rhs2 = sim.rhs.cpu().numpy()
    phi_half_gpu = (f - rhs2) / k2
    err1 = rel_rms(phi_half_gpu, phi_half)
    phi1 = pm.solve_periodic(f - k2 * phi_half, k2)
    err2 = rel_rms(sim.phi_numpy(), phi1)
    log(f"  potential errors: half step {err1:.2e}, full step {err2:.2e}")
    assert err1 <= cond_periodic(NG, k1) * cfg.tol
    assert err2 <= 2.0 * cond_periodic(NG, k2) * cfg.tol
    del f, rhs2, phi_half_gpu

    # kick with the exact force at the drifted positions, second drift exact
    rng = np.random.Generator(np.random.PCG64(5))
    idx = np.sort(rng.choice(n, size=1 << 17, replace=False))
    g = pm.interpolate(xh[idx], pm.force_mesh(phi_half, h), NG, BOX, B, True)
    kick = st["a_half"] * st["dtau"]
    p_ref = p0[idx] + g * kick
    dp = np.sqrt(np.mean((p1[idx] - p_ref) ** 2))
    bound = 2.0**-24 * np.sqrt(np.mean(p_ref**2)) + 1e-5 * kick * np.sqrt(np.mean(g**2))
    log(f"  momentum rms error {dp:.3e} (bound {bound:.3e})")
    assert dp <= bound
    c2 = 0.5 * st["dtau"] / (a + da)
    assert np.array_equal(x1[idx], wrap(xh[idx] + p1[idx] * c2, BOX))
    del phi_half, xh

    # force at the end of the step
    g_gpu = sim.interp_force()[:, idx].cpu().numpy().T
    g_ref = pm.interpolate(x1[idx], pm.force_mesh(phi1, h), NG, BOX, B, True)
    ferr = rel_rms(g_gpu, g_ref)
    log(f"  force rel rms {ferr:.2e}")
    assert ferr <= 1e-5


@pytest.mark.timeout(600)
def test_fullsize_deposit_whole_array_at_step_25():
    """The whole 512^3 counts array of the deposit in step 25 (five steps
    after the last sort, particles moved off their sorted rows, some deposit
    workgroups with outliers) equals the oracle's deposit of the drifted
    positions, bit for bit."""
    import paper_1709_04703_amd as P
    a0 = 1.0 / (1.0 + Z_INIT)
    x, p, ids = zeldovich_ics(NG, BOX, a0, SEED)
    n = x.shape[0]
    cfg = lib_config(NG, BOX, c_grav=-1.0, shrink=1, precision=P.SDPM_MIXED, n_initial=n,
                     sort_every=10, warm_start=P.SDPM_WS_PREV | P.SDPM_WS_EXTRAP)
    sim = make_sim(cfg, n)
    sim.bind(x, p, ids)
    del x, p, ids
    sim.init_potential(a0)
    edges = np.linspace(a0, 1.0, SCHEDULE + 1)
    log("full size: 25 steps, then the whole counts array of step 25")
    for s_ in range(25):
        sim.step(edges[s_], edges[s_ + 1] - edges[s_])
    x0, p0, _ = sim.particles()
    a, da = edges[25], edges[26] - edges[25]
    st = sim.step(a, da)
    assert st["periodic"] == 1
    xh = wrap(x0 + p0 * (0.5 * st["dtau"] / a), BOX)
    del x0, p0
    got = sim.counts_numpy().reshape(NG, NG, NG)
    sim.close()
    ref = exact_counts(xh, True)
    del xh
    bad = int(np.count_nonzero(got != ref))
    log(f"  cells differing: {bad}")
    assert bad == 0


def test_fullsize_removal(big):
    sim, cfg = big["sim"], big["cfg"]
    x, _, ids = sim.particles()
    n = x.shape[0]
    r = 600.0
    out = pm.outside_lightcone(x, np.asarray(cfg.x_obs), r)
    log(f"full size: removal at r = {r}, {int(out.sum())} of {n} outside")
    nr = sim.shrink_radius(r)
    assert nr == int(out.sum())
    xa, _, ida = sim.particles(all_particles=True)
    keep = ~out
    assert np.array_equal(ida[: n - nr], ids[keep])
    assert np.array_equal(ida[n - nr: n], ids[out])
    assert np.array_equal(xa[: n - nr], x[keep])
    st = sim.state()
    dirichlet, lo, hi = pm.box_for_radius(r, np.asarray(cfg.x_obs), BOX / NG, NG, cfg.margin,
                                          cfg.box_align)
    assert dirichlet and st["periodic"] == 0
    assert list(st["lo"]) == list(lo) and list(st["hi"]) == list(hi)


def test_fullsize_extrapolated_start_step():
    """The headline solve configuration at full size: mixed precision with the
    extrapolated start, two steps; the second applies the start (each solve
    begins from the potential plus the previous step's scaled change, the
    finer cycles per correction and the short hierarchy as in the bench), and
    both of its potentials are the exact solves of the oracle's own source of
    the library's (exact) counts within cond(A) tol."""
    import paper_1709_04703_amd as P
    a0 = 1.0 / (1.0 + Z_INIT)
    x, p, ids = zeldovich_ics(NG, BOX, a0, SEED)
    n = x.shape[0]
    cfg = lib_config(NG, BOX, c_grav=-1.0, shrink=1, precision=P.SDPM_MIXED, n_initial=n,
                     sort_every=10, warm_start=P.SDPM_WS_EXTRAP)
    sim = make_sim(cfg, n)
    sim.bind(x, p, ids)
    del x, p, ids
    sim.init_potential(a0)
    edges = np.linspace(a0, 1.0, SCHEDULE + 1)
    h = BOX / NG
    sim.step(edges[0], edges[1] - edges[0])
    phi0 = sim.phi_numpy().copy()
    a, da = edges[1], edges[2] - edges[1]
    log("full size: second step with the extrapolated start")
    st = sim.step(a, da)
    assert max(st["res"]) <= cfg.tol
    log(f"  V-cycles {st['vcycles']}, outer iterations {st['outer_iters']}, "
        f"start residual {st['res0']}")
    sc = ocosmo.step_scalars(a, da, cfg.omega_m, cfg.omega_l, BOX, NG, cfg.c_grav, cfg.c_light)
    k1, k2 = st["kappa_h2"]
    f = pm.source(sim.counts_numpy().reshape(NG, NG, NG), n, B, sc["s_half"], h, True)
    phi_half = pm.solve_periodic(f - k1 * phi0, k1)
    del phi0
    phi_half_gpu = (f - sim.rhs.cpu().numpy()) / k2
    err1 = rel_rms(phi_half_gpu, phi_half)
    del phi_half_gpu
    phi1 = pm.solve_periodic(f - k2 * phi_half, k2)
    err2 = rel_rms(sim.phi_numpy(), phi1)
    log(f"  potential errors: half step {err1:.2e}, full step {err2:.2e}")
    assert err1 <= cond_periodic(NG, k1) * cfg.tol
    assert err2 <= 2.0 * cond_periodic(NG, k2) * cfg.tol
    sim.close()


def test_fullsize_frozen_exterior_step():
    """The shrinking phase at full size, as the bench times it: the 512^3 run
    to step 160 of the 200-step schedule (z = 0.24: a 383^3-cell
    frozen-exterior box, 17 % of the particles active), then one step whose
    two potentials, on the box, are the oracle's exact Dirichlet solves (DST)
    of the source of the library's exact counts with the frozen exterior,
    within cond(A) tol; the exterior is left as it was; its deposit is exact
    (total mass and whole planes); and its lightcone records are the removed
    particles, in removal order, on the sphere."""
    import paper_1709_04703_amd as P
    a0 = 1.0 / (1.0 + Z_INIT)
    x, p, ids = zeldovich_ics(NG, BOX, a0, SEED)
    n = x.shape[0]
    cfg = lib_config(NG, BOX, c_grav=-1.0, shrink=1, precision=P.SDPM_MIXED, n_initial=n,
                     sort_every=10)
    sim = make_sim(cfg, n)
    sim.bind(x, p, ids)
    del x, p, ids
    sim.init_potential(a0)
    edges = np.linspace(a0, 1.0, SCHEDULE + 1)
    log("full size: 160 steps into the shrinking phase")
    for s in range(160):
        sim.step(edges[s], edges[s + 1] - edges[s])
    st0 = sim.state()
    lo, hi = np.array(st0["lo"]), np.array(st0["hi"])
    log(f"  box {st0['lo']} .. {st0['hi']}, active {sim.n_active} of {n}")
    assert st0["periodic"] == 0
    phi0 = sim.phi_numpy().copy()
    a, da = edges[160], edges[161] - edges[160]
    h = BOX / NG
    x0, p0, _ = sim.particles()
    sim.set_lightcone(4_000_000)
    n_before = sim.n_active
    st = sim.step(a, da)
    assert max(st["res"]) <= cfg.tol
    # the deposit of the drifted positions (no wrap on the box): the total
    # mass and whole z-planes exact (late in the run the deposit takes its
    # larger LDS tile)
    xh = x0 + p0 * (0.5 * st["dtau"] / a)
    del x0, p0
    counts = sim.counts_numpy().reshape(NG, NG, NG)
    tot = int((counts & np.uint64(0xFFFFFFFF)).sum(dtype=np.uint64)) + \
        (int((counts >> np.uint64(32)).sum(dtype=np.uint64)) << 32)
    assert tot == n_before << (3 * B)
    kz = pm.fixed_point_coords(xh[:, 2:3], NG, BOX, B, False)[:, 0] >> B
    for kp in (int(lo[2]), 200, 256, int(hi[2])):
        sel = (kz == kp) | (kz == kp - 1)
        assert np.array_equal(counts[kp], pm.deposit(xh[sel], NG, BOX, B, False)[kp]), kp
    del counts, kz, xh
    # lightcone output: one record per removed particle, in removal order,
    # each (crossing strictly inside the step) on the sphere r_lc + u c dtau
    rid, ra, rx, _ = sim.lightcone_records()
    _, _, ids_all = sim.particles(all_particles=True)
    k = sim.n_active
    assert st["n_removed"] == n_before - k > 0
    assert np.array_equal(rid.astype(np.uint32), ids_all[k:n_before])
    u = (a + da - ra) / da
    inner = (u > 0.0) & (u < 1.0)
    dist = np.linalg.norm(rx[inner] - np.asarray(cfg.x_obs), axis=1)
    r_u = st["r_lc"] + u[inner] * cfg.c_light * st["dtau"]
    log(f"  {len(rid)} lightcone records, {int(inner.sum())} inside the step, "
        f"max |distance - r| = {np.abs(dist - r_u).max():.2e} Mpc/h")
    assert inner.sum() > 0.9 * len(rid)
    assert np.abs(dist - r_u).max() <= 1e-9 * r_u.max()
    del rid, ra, rx, ids_all
    sc = ocosmo.step_scalars(a, da, cfg.omega_m, cfg.omega_l, BOX, NG, cfg.c_grav, cfg.c_light)
    k1, k2 = st["kappa_h2"]
    sl = (slice(lo[2], hi[2] + 1), slice(lo[1], hi[1] + 1), slice(lo[0], hi[0] + 1))
    f = pm.source(sim.counts_numpy().reshape(NG, NG, NG), n, B, sc["s_half"], h, False)
    phi_half = pm.solve_box(phi0, f - k1 * phi0, lo, hi, k1)
    rhs2 = sim.rhs.cpu().numpy()
    err1 = rel_rms(((f - rhs2) / k2)[sl], phi_half[sl])
    del rhs2
    phi1 = pm.solve_box(phi_half, f - k2 * phi_half, lo, hi, k2)
    phi = sim.phi_numpy()
    err2 = rel_rms(phi[sl], phi1[sl])
    log(f"  potential errors on the box: half step {err1:.2e}, full step {err2:.2e}")
    nmax = int(max(hi - lo + 1))
    cond = lambda kap: (12.0 + kap) / (3 * (2 - 2 * np.cos(np.pi / (nmax + 1))) + kap)
    assert err1 <= cond(k1) * cfg.tol
    assert err2 <= 2.0 * cond(k2) * cfg.tol
    outside = np.ones(phi.shape, dtype=bool)
    outside[sl] = False
    assert np.array_equal(phi[outside], phi0[outside])
    sim.close()
