"""Oracle particle-mesh step on the shrinking domain (FP64 NumPy/SciPy).

TEST INFRASTRUCTURE ONLY: imported by tests, smoke() and the cpu_baseline leg
of bench.py, never by the product path.  Plain, slow and written to be read
against the paper.

Conventions
-----------
* Mesh values live at x_i = i h, h = L / N_g; a grid array G has shape
  (N_g, N_g, N_g) indexed G[k, j, i] (z, y, x), so the flat index of cell
  (i, j, k) is (k N_g + j) N_g + i.  Particle arrays are (n, 3) with columns
  (x, y, z).
* The discrete operator is the 7-point Laplacian in grid units,
  (Lap_h Phi)_c = sum of the 6 neighbours - 6 Phi_c, and the mesh equation is
  (Lap_h - kappa h^2) Phi = rhs with rhs carrying the h^2 factor.
* Sign: the paper prints dp/dtau = a grad Phi (Eq. 2) together with
  Lap Phi = +S delta (Eq. 3).  Gravity is attractive, so the force used is
  g = -grad Phi and dp/dtau = a g.

Readings of the paper where it is silent or garbled (each also listed in the
design notes):
* Gravity (Sec. 2.1 Eq. 4) is advanced by one backward-Euler step per half
  sub-step (the paper names implicit solvers as the intended route, Sec. 3.1.1;
  Config.solver = "ade" takes the paper's own ADE sweeps instead, oracle/ade.py):
  3 calH (Phi+ - Phi-)/(dtau/2) - c^2 Lap Phi+ = -c^2 S delta, i.e.
  (Lap - kappa) Phi+ = S delta - kappa Phi-,  kappa = 3 calH / (c^2 dtau/2).
  kappa = 0 is Poisson (Eq. 3).  Both half sub-steps (Table 2) reuse the
  mid-step density.
* The CIC weights are fixed point with B fractional bits so that the deposit
  is exact and order independent: U = floor(x s), s = N_g 2^B / L,
  cell = U >> B, q = U mod 2^B, axis weights (2^B - q, q).
* Active cells (Sec. 2.4): an index box per axis, floor((x_o -+ r)/h) -+ m,
  rounded outward so the planes next to it are multiples of `align`, and
  never growing.  While that box does not fit strictly inside the mesh the
  whole mesh is active and periodic (Sec. 3: periodic until the lightcone
  reaches the box borders); afterwards it is Dirichlet with the exterior
  values frozen at their last solved value and positions no longer wrap.
* Removal (Table 2 last row, Sec. 2.4): a particle is removed when
  ((dx^2 + dy^2) + dz^2) > r_lc^2 in FP64 (tie kept).  Removed particles are
  kept in memory after the active ones (stable partition).
* Mean density n_bar = N_initial / N_g^3; the FP64 mean of the source is
  subtracted only while the mesh is periodic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as sfft

from . import ade
from . import cosmology as cosmo


# --------------------------------------------------------------------------
# configuration and state
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Config:
    ng: int
    box: float
    omega_m: float = 0.3
    omega_l: float = 0.7
    c_light: float = cosmo.C_LIGHT
    c_grav: float = 0.0          # 0: static Poisson; <0: 0.019 h c (Eq. 12)
    x_obs: tuple = None          # default: box centre
    shrink: bool = False
    margin: int = 2
    align: int = 1               # planes next to the box at multiples of this
    frac_bits: int = 14
    n_initial: int = 0
    solver: str = "implicit"     # "implicit": backward Euler; "ade": the paper's ADE sweeps
    assignment: str = "cic"      # "cic" or "tsc" (Sec. 2.4 names both schemes)

    def observer(self) -> np.ndarray:
        if self.x_obs is None:
            return np.full(3, 0.5 * self.box)
        return np.asarray(self.x_obs, dtype=np.float64)


@dataclasses.dataclass
class State:
    x: np.ndarray        # (n, 3) float64 positions; active first
    p: np.ndarray        # (n, 3) float64 momenta p = a dx/dtau
    ids: np.ndarray      # (n,) uint32
    n_active: int
    phi: np.ndarray      # (N, N, N) float64
    a: float
    periodic: bool = True
    lo: np.ndarray = None   # (3,) int, inclusive, axis order (x, y, z)
    hi: np.ndarray = None

    def copy(self) -> "State":
        return State(self.x.copy(), self.p.copy(), self.ids.copy(), self.n_active,
                     self.phi.copy(), self.a, self.periodic,
                     None if self.lo is None else self.lo.copy(),
                     None if self.hi is None else self.hi.copy())


# --------------------------------------------------------------------------
# CIC deposit (Sec. 2.4: CIC; fixed-point weights)
# --------------------------------------------------------------------------
def fixed_point_scale(ng: int, box: float, frac_bits: int) -> float:
    """s = N_g 2^B / L, one FP64 division."""
    return float(ng * (1 << frac_bits)) / box


def fixed_point_coords(x: np.ndarray, ng: int, box: float, frac_bits: int,
                       periodic: bool) -> np.ndarray:
    """U = floor(x s) as int64 (one FP64 multiply and a floor); periodic
    meshes wrap U modulo N_g 2^B."""
    s = fixed_point_scale(ng, box, frac_bits)
    u = np.floor(x * s).astype(np.int64)
    if periodic:
        u = np.mod(u, np.int64(ng) << frac_bits)
    return u


def _corners(u: np.ndarray, ng: int, frac_bits: int, periodic: bool):
    """Yield (flat cell index, uint64 weight product) for the 8 CIC corners."""
    one = np.uint64(1 << frac_bits)
    cell = u >> frac_bits
    q = (u & ((1 << frac_bits) - 1)).astype(np.uint64)
    w = [one - q, q]                       # weight of the lower / upper cell
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                ii = cell[:, 0] + dx
                jj = cell[:, 1] + dy
                kk = cell[:, 2] + dz
                if periodic:
                    ii %= ng
                    jj %= ng
                    kk %= ng
                if ii.size and (ii.max() >= ng or jj.max() >= ng or kk.max() >= ng
                                or ii.min() < 0 or jj.min() < 0 or kk.min() < 0):
                    raise ValueError("CIC corner outside the mesh")
                wt = w[dx][:, 0] * w[dy][:, 1] * w[dz][:, 2]
                yield (kk * ng + jj) * ng + ii, wt


def tsc_weights(u: np.ndarray, frac_bits: int):
    """TSC in fixed point (Sec. 2.4 names TSC beside CIC; the integer form is
    a reading): the nearest node i = (U + 2^(B-1)) >> B of the coordinate U,
    the offset D = U - i 2^B in [-2^(B-1), 2^(B-1)), and the three weights of
    nodes i - 1, i, i + 1 in units of 2^-B: the continuous TSC weights
    (1/2 - d)^2 / 2 and (1/2 + d)^2 / 2 (d = D / 2^B) rounded to the nearest
    unit, and the middle one 2^B minus both, so that they sum to 2^B exactly.
    Returns (node, [w_minus, w_mid, w_plus]) as int64 arrays."""
    one = np.int64(1) << frac_bits
    half = one >> 1
    node = (u + half) >> frac_bits
    d = u - (node << frac_bits)
    wm = ((half - d) ** 2 + one) >> (frac_bits + 1)
    wp = ((half + d) ** 2 + one) >> (frac_bits + 1)
    return node, [wm, one - wm - wp, wp]


def _tsc_corners(u: np.ndarray, ng: int, frac_bits: int, periodic: bool):
    """Yield (flat cell index, uint64 weight product) for the 27 TSC nodes."""
    node, w = tsc_weights(u, frac_bits)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ii = node[:, 0] + dx
                jj = node[:, 1] + dy
                kk = node[:, 2] + dz
                if periodic:
                    ii %= ng
                    jj %= ng
                    kk %= ng
                if ii.size and (ii.max() >= ng or jj.max() >= ng or kk.max() >= ng
                                or ii.min() < 0 or jj.min() < 0 or kk.min() < 0):
                    raise ValueError("TSC node outside the mesh")
                wt = (w[dx + 1][:, 0].astype(np.uint64) * w[dy + 1][:, 1].astype(np.uint64)
                      * w[dz + 1][:, 2].astype(np.uint64))
                yield (kk * ng + jj) * ng + ii, wt


def _assignment_corners(assignment: str):
    if assignment == "cic":
        return _corners
    if assignment == "tsc":
        return _tsc_corners
    raise ValueError(f"unknown assignment {assignment!r}")


def deposit(x: np.ndarray, ng: int, box: float, frac_bits: int,
            periodic: bool, assignment: str = "cic") -> np.ndarray:
    """Exact mass counts C (uint64, shape (N,N,N)) of the CIC (default) or
    TSC assignment; each particle adds weight products summing to 2^(3B)."""
    u = fixed_point_coords(x, ng, box, frac_bits, periodic)
    c = np.zeros(ng**3, dtype=np.uint64)
    for flat, wt in _assignment_corners(assignment)(u, ng, frac_bits, periodic):
        np.add.at(c, flat, wt)
    return c.reshape(ng, ng, ng)


def source(counts: np.ndarray, n_initial: int, frac_bits: int, s_half: float,
           h: float, periodic: bool) -> np.ndarray:
    """f = S h^2 delta, delta = C / (n_bar 2^(3B)) - 1  (Eq. 3 source);
    the mean is subtracted on a periodic mesh."""
    ng = counts.shape[0]
    nbar = n_initial / float(ng**3)
    delta = counts.astype(np.float64) / (nbar * 2.0**(3 * frac_bits)) - 1.0
    f = s_half * h * h * delta
    if periodic:
        f = f - f.mean()
    return f


# --------------------------------------------------------------------------
# exact mesh solves of (Lap_h - kappa h^2) Phi = rhs
# --------------------------------------------------------------------------
def laplacian_periodic(phi: np.ndarray) -> np.ndarray:
    """7-point Laplacian in grid units on a periodic mesh (by index shifts)."""
    out = -6.0 * phi
    for ax in range(3):
        out = out + np.roll(phi, 1, axis=ax) + np.roll(phi, -1, axis=ax)
    return out


def solve_periodic(rhs: np.ndarray, kappa_h2: float) -> np.ndarray:
    """Exact periodic solve by FFT: the operator's symbol is
    -sum_d (2 - 2 cos(2 pi k_d / N)) - kappa h^2.  With kappa = 0 the k = 0
    mode is set to zero (zero-mean gauge)."""
    ng = rhs.shape[0]
    k = np.arange(ng)
    lam1 = 2.0 - 2.0 * np.cos(2.0 * np.pi * k / ng)
    sym = -(lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]) - kappa_h2
    rk = sfft.fftn(rhs, workers=-1)
    if kappa_h2 == 0.0:
        sym[0, 0, 0] = 1.0
        rk[0, 0, 0] = 0.0
    return np.real(sfft.ifftn(rk / sym, workers=-1))


def solve_box(phi: np.ndarray, rhs: np.ndarray, lo, hi, kappa_h2: float) -> np.ndarray:
    """Exact Dirichlet solve on the active index box [lo, hi] (inclusive,
    axis order x, y, z).  Values outside the box are frozen: the ring next to
    the box is moved to the right-hand side, then the interior problem is
    solved with DST-I, whose basis diagonalises the Dirichlet second
    difference with eigenvalues -(2 - 2 cos(pi m / (n + 1)))."""
    lo = [int(v) for v in lo]
    hi = [int(v) for v in hi]
    sl = (slice(lo[2], hi[2] + 1), slice(lo[1], hi[1] + 1), slice(lo[0], hi[0] + 1))
    b = rhs[sl].copy()
    # ring contributions (array axis 0 = z, 1 = y, 2 = x)
    for arr_ax, dim in ((2, 0), (1, 1), (0, 2)):
        l, h = lo[dim], hi[dim]
        idx_lo = [sl[0], sl[1], sl[2]]
        idx_lo[arr_ax] = slice(l - 1, l)
        idx_hi = [sl[0], sl[1], sl[2]]
        idx_hi[arr_ax] = slice(h + 1, h + 2)
        first = [slice(None)] * 3
        first[arr_ax] = slice(0, 1)
        last = [slice(None)] * 3
        last[arr_ax] = slice(-1, None)
        b[tuple(first)] -= phi[tuple(idx_lo)]
        b[tuple(last)] -= phi[tuple(idx_hi)]
    nz, ny, nx = b.shape
    def lam(n):
        m = np.arange(1, n + 1)
        return 2.0 - 2.0 * np.cos(np.pi * m / (n + 1))
    sym = -(lam(nz)[:, None, None] + lam(ny)[None, :, None] + lam(nx)[None, None, :]) - kappa_h2
    bk = sfft.dstn(b, type=1, norm="ortho", workers=-1)
    sol = sfft.idstn(bk / sym, type=1, norm="ortho", workers=-1)
    out = phi.copy()
    out[sl] = sol
    return out


def residual_box(phi: np.ndarray, rhs: np.ndarray, lo, hi, kappa_h2: float) -> np.ndarray:
    """rhs - (Lap_h - kappa h^2) phi on the box, by explicit neighbour reads
    (used to check the DST solve)."""
    lo = [int(v) for v in lo]
    hi = [int(v) for v in hi]
    k0, k1 = lo[2], hi[2] + 1
    j0, j1 = lo[1], hi[1] + 1
    i0, i1 = lo[0], hi[0] + 1
    c = phi[k0:k1, j0:j1, i0:i1]
    nb = (phi[k0:k1, j0:j1, i0 - 1:i1 - 1] + phi[k0:k1, j0:j1, i0 + 1:i1 + 1]
          + phi[k0:k1, j0 - 1:j1 - 1, i0:i1] + phi[k0:k1, j0 + 1:j1 + 1, i0:i1]
          + phi[k0 - 1:k1 - 1, j0:j1, i0:i1] + phi[k0 + 1:k1 + 1, j0:j1, i0:i1])
    return rhs[k0:k1, j0:j1, i0:i1] - (nb - 6.0 * c - kappa_h2 * c)


# --------------------------------------------------------------------------
# force and interpolation
# --------------------------------------------------------------------------
def force_mesh(phi: np.ndarray, h: float) -> np.ndarray:
    """g = -grad Phi by 2-point central differences; returns (3, N, N, N)
    with components (x, y, z).  Uses periodic index shifts; in Dirichlet
    mode only cells inside the active box are ever read by the
    interpolation, and their neighbours exist in the full mesh."""
    g = np.empty((3,) + phi.shape)
    for comp, arr_ax in ((0, 2), (1, 1), (2, 0)):
        g[comp] = -(np.roll(phi, -1, axis=arr_ax) - np.roll(phi, 1, axis=arr_ax)) / (2.0 * h)
    return g


def interpolate(x: np.ndarray, g: np.ndarray, ng: int, box: float, frac_bits: int,
                periodic: bool, assignment: str = "cic") -> np.ndarray:
    """Interpolation with the deposit's own fixed-point weights (same
    scheme both ways, the footnote of Sec. 2.4); returns (n, 3)."""
    u = fixed_point_coords(x, ng, box, frac_bits, periodic)
    out = np.zeros((x.shape[0], 3))
    norm = 2.0 ** (-3 * frac_bits)
    gf = g.reshape(3, -1)
    for flat, wt in _assignment_corners(assignment)(u, ng, frac_bits, periodic):
        wf = wt.astype(np.float64) * norm
        for comp in range(3):
            out[:, comp] += wf * gf[comp][flat]
    return out


# --------------------------------------------------------------------------
# domain: lightcone removal and active box
# --------------------------------------------------------------------------
def outside_lightcone(x: np.ndarray, x_obs: np.ndarray, r_lc: float) -> np.ndarray:
    """True where ((dx^2 + dy^2) + dz^2) > r_lc^2 (FP64, no fused multiply-add)."""
    dx = x[:, 0] - x_obs[0]
    dy = x[:, 1] - x_obs[1]
    dz = x[:, 2] - x_obs[2]
    d2 = (dx * dx + dy * dy) + dz * dz
    return d2 > r_lc * r_lc


def lightcone_crossed(x_start: np.ndarray, x_end: np.ndarray, x_obs: np.ndarray, r_start: float,
                      r_end: float) -> np.ndarray:
    """Fixed domain (nothing removed): the particles that cross the lightcone
    during a step, outside at its end and not outside at its start, each by
    the removal predicate with that instant's radius."""
    return outside_lightcone(x_end, x_obs, r_end) & ~outside_lightcone(x_start, x_obs, r_start)


def lightcone_crossing(x1: np.ndarray, p1: np.ndarray, x_obs: np.ndarray, r1: float,
                       light: float, disp: float, a1: float, da: float):
    """Where removed particles crossed the lightcone during their last step
    (the lightcone output; the reading stated in the C header): the particle
    is traced back from its end-of-step position x1 along w = p1 disp
    (disp = dtau / a1), x(u) = x1 - u w, while the radius grows back as
    r(u) = r1 + u light (light = c dtau), u in [0, 1] the fraction of the step
    before its end.  u is the root of f(u) = |x(u) - x_obs|^2 - r(u)^2, found
    by bisection (f(0) > 0 for a removed particle); u = 1 when f(1) > 0 (the
    particle was already outside at the step's start), u = 0 when light = 0.
    Returns (u, a = a1 - u da, x(u), p1)."""
    d = x1 - x_obs
    w = p1 * disp

    def f(u):
        y = d - u[:, None] * w
        return np.sum(y * y, axis=1) - (r1 + u * light) ** 2

    n = x1.shape[0]
    if light <= 0.0:
        u = np.zeros(n)
    else:
        lo, hi = np.zeros(n), np.ones(n)
        outside_at_start = f(hi) > 0.0
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            pos = f(mid) > 0.0
            lo = np.where(pos, mid, lo)
            hi = np.where(pos, hi, mid)
        u = np.where(outside_at_start, 1.0, 0.5 * (lo + hi))
        u = np.where(np.sum(d * d, axis=1) - r1 * r1 > 0.0, u, 0.0)
    return u, a1 - u * da, x1 - u[:, None] * w, p1.copy()


def box_for_radius(r_lc: float, x_obs: np.ndarray, h: float, ng: int, margin: int,
                   align: int = 1):
    """Index box covering the sphere of radius r_lc about x_obs plus `margin`
    cells, rounded outward so that the planes just outside it (lo - 1 and
    hi + 1) are multiples of `align`.  Returns (dirichlet, lo, hi); dirichlet
    is False (whole periodic mesh) unless the box lies inside [1, N_g - 2] on
    every axis."""
    lo = np.array([math.floor((x_obs[d] - r_lc) / h) - margin for d in range(3)], dtype=np.int64)
    hi = np.array([math.floor((x_obs[d] + r_lc) / h) + margin for d in range(3)], dtype=np.int64)
    lo = ((lo - 1) // align) * align + 1
    hi = -((-(hi + 1)) // align) * align - 1
    if np.all(lo >= 1) and np.all(hi <= ng - 2):
        return True, lo, hi
    return False, np.zeros(3, dtype=np.int64), np.full(3, ng - 1, dtype=np.int64)


def shrink(state: State, cfg: Config, a: float) -> np.ndarray:
    """Lightcone at a: remove particles outside it (stable partition, kept
    first) and update the active box / boundary mode.  Returns removed ids
    in their array order."""
    r = cosmo.lightcone_radius(a, cfg.omega_m, cfg.omega_l, cfg.c_light)
    return shrink_radius(state, cfg, r)


def shrink_radius(state: State, cfg: Config, r: float) -> np.ndarray:
    x_obs = cfg.observer()
    n = state.n_active
    removed = np.zeros(0, dtype=np.uint32)
    if cfg.shrink:
        out = outside_lightcone(state.x[:n], x_obs, r)
        if out.any():
            keep = np.nonzero(~out)[0]
            gone = np.nonzero(out)[0]
            order = np.concatenate([keep, gone, np.arange(n, state.x.shape[0])])
            state.x = state.x[order]
            state.p = state.p[order]
            state.ids = state.ids[order]
            removed = state.ids[keep.size:n].copy()
            state.n_active = keep.size
        h = cfg.box / cfg.ng
        # TSC reaches one node further than CIC: one more cell of margin
        margin = cfg.margin + (1 if cfg.assignment == "tsc" else 0)
        dirichlet, lo, hi = box_for_radius(r, x_obs, h, cfg.ng, margin, cfg.align)
        if dirichlet:
            if not state.periodic:
                lo = np.maximum(lo, state.lo)
                hi = np.minimum(hi, state.hi)
            state.periodic = False
            state.lo, state.hi = lo, hi
    return removed


# --------------------------------------------------------------------------
# the step (Table 2, right column)
# --------------------------------------------------------------------------
def _wrap(x: np.ndarray, box: float) -> np.ndarray:
    x = np.where(x < 0.0, x + box, x)
    return np.where(x >= box, x - box, x)


def _check_domain(x: np.ndarray, state: State, cfg: Config) -> None:
    if state.periodic or x.shape[0] == 0:
        return
    u = fixed_point_coords(x, cfg.ng, cfg.box, cfg.frac_bits, False)
    if cfg.assignment == "tsc":
        node, _ = tsc_weights(u, cfg.frac_bits)
        first, last = node - 1, node + 1
    else:
        first = u >> cfg.frac_bits
        last = first + 1
    if np.any(first < state.lo) or np.any(last > state.hi):
        raise ValueError("particle assignment support leaves the active box")


def solve(phi: np.ndarray, rhs: np.ndarray, state: State, kappa_h2: float) -> np.ndarray:
    if state.periodic:
        return solve_periodic(rhs, kappa_h2)
    return solve_box(phi, rhs, state.lo, state.hi, kappa_h2)


def ade_sweep(phi: np.ndarray, f: np.ndarray, state: State, kappa_h2: float,
              forward: bool) -> np.ndarray:
    """One ADE sweep (oracle/ade.py) of a half sub-step over the active box,
    lam = 1 / (kappa h^2)."""
    n = phi.shape[0]
    if state.periodic:
        return ade.sweep(phi, f, 1.0 / kappa_h2, (0, 0, 0), (n - 1,) * 3, True, forward)
    return ade.sweep(phi, f, 1.0 / kappa_h2, tuple(state.lo), tuple(state.hi), False, forward)


def init_state(x, p, ids, cfg: Config, a: float) -> State:
    """Bind particles at scale factor a, apply the lightcone at a, and set the
    field from linear theory by one static (kappa = 0) solve of the initial
    density (Table 1, initial conditions for the fields)."""
    ng = cfg.ng
    st = State(np.array(x, dtype=np.float64), np.array(p, dtype=np.float64),
               np.array(ids, dtype=np.uint32), len(x), np.zeros((ng, ng, ng)), a,
               True, np.zeros(3, dtype=np.int64), np.full(3, ng - 1, dtype=np.int64))
    if st.periodic:
        st.x[:st.n_active] = _wrap(st.x[:st.n_active], cfg.box)
    shrink(st, cfg, a)
    n = st.n_active
    h = cfg.box / ng
    counts = deposit(st.x[:n], ng, cfg.box, cfg.frac_bits, st.periodic, cfg.assignment)
    f = source(counts, cfg.n_initial, cfg.frac_bits, 1.5 * cfg.omega_m / a, h, st.periodic)
    st.phi = solve(st.phi, f, st, 0.0)
    return st


def step(state: State, cfg: Config, da: float, diag: dict | None = None) -> State:
    """One synchronised leapfrog step a -> a + da (Eqs. 7-9) in the order of
    Table 2: drift 1/2, delta, Phi to t+dt/2, grad Phi, kick, drift 1/2,
    Phi to t+dt, advance time, lightcone and elimination."""
    st = state.copy()
    a = st.a
    sc = cosmo.step_scalars(a, da, cfg.omega_m, cfg.omega_l, cfg.box, cfg.ng,
                            cfg.c_grav, cfg.c_light)
    h = cfg.box / cfg.ng
    n = st.n_active
    x = st.x[:n]
    p = st.p[:n]
    half = 0.5 * sc["dtau"]
    # drift 1/2 with a(t)  (Eq. 7)
    x = x + p * (half / a)
    if st.periodic:
        x = _wrap(x, cfg.box)
    _check_domain(x, st, cfg)
    # density at t + dt/2
    counts = deposit(x, cfg.ng, cfg.box, cfg.frac_bits, st.periodic, cfg.assignment)
    f = source(counts, cfg.n_initial, cfg.frac_bits, sc["s_half"], h, st.periodic)
    # Phi from t to t + dt/2
    k1 = sc["kappa1_h2"]
    if cfg.solver == "ade":
        if not k1 > 0.0:
            raise ValueError("the ADE integrator needs a finite gravity speed")
        phi_half = ade_sweep(st.phi, f, st, k1, True)
    else:
        phi_half = solve(st.phi, f - k1 * st.phi, st, k1)
    # grad Phi, interpolation, kick with a(t + dt/2)  (Eq. 8)
    g = force_mesh(phi_half, h)
    gp = interpolate(x, g, cfg.ng, cfg.box, cfg.frac_bits, st.periodic, cfg.assignment)
    p = p + gp * (sc["a_half"] * sc["dtau"])
    # drift 1/2 with a(t + dt)  (Eq. 9)
    x = x + p * (half / (a + da))
    if st.periodic:
        x = _wrap(x, cfg.box)
    # Phi from t + dt/2 to t + dt (same density); static gravity: unchanged
    k2 = sc["kappa2_h2"]
    if cfg.solver == "ade":
        phi_new = ade_sweep(phi_half, f, st, k2, False)
    elif k2 > 0.0:
        phi_new = solve(phi_half, f - k2 * phi_half, st, k2)
    else:
        phi_new = phi_half
    st.x[:n] = x
    st.p[:n] = p
    st.phi = phi_new
    st.a = a + da
    removed = shrink_radius(st, cfg, sc["r_lc_end"])
    if diag is not None:
        diag.update(sc)
        diag["counts"] = counts
        diag["f"] = f
        diag["phi_half"] = phi_half
        diag["g_particles"] = gp
        diag["removed"] = removed
    return st
