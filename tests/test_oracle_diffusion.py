"""Pins of the time discretisation of the gravity diffusion equation (Sec. 2.1
Eq. 4; two half sub-steps per step, Sec. 2.3 Table 2) in the oracle's step,
CPU only.  None of them re-evaluates the oracle's screening formula: they
start from Eq. 4 itself.

For one Fourier mode of the mesh potential the 7-point Laplacian is
multiplication by -lam_k / h^2, lam_k = sum_d (2 - 2 cos(2 pi n_d / N)), so
Eq. 4 with no source is the scalar equation

    3 calH(tau) dPhi_k/dtau = -c_g^2 lam_k / h^2 Phi_k.

In an Einstein-de Sitter background (Omega_m = 1, H0 = 1) calH = a E(a) =
a^(-1/2) and dtau = da / sqrt(a), so the integral of dtau / calH is the
change of a, and the exact solution over a -> a1 is

    Phi_k(a1) = Phi_k(a0) exp(-c_g^2 lam_k (a1 - a0) / (3 h^2)).

A step that takes the wrong sub-step length (dtau for dtau/2), drops the
factor 3 or scales the rate in any other way converges to a different decay
and fails the convergence checks below; the order of the two Hubble rates
inside one step is fixed by comparing a single large step with a textbook
backward-Euler step of the same equation on the conformal half sub-steps,
solved by a generic root finder.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import pm

NG, BOX, CG = 8, 80.0, 50.0          # h = 10 Mpc/h; gravity speed in (Mpc/h) H0
H = BOX / NG
K = CG * CG / (3.0 * H * H)          # Eq. 4 divided by 3 calH, per unit lam_k


def _mode(nx, ny=0, nz=0):
    i = np.arange(NG)
    return (np.cos(2 * np.pi * nz * i / NG)[:, None, None]
            * np.cos(2 * np.pi * ny * i / NG)[None, :, None]
            * np.cos(2 * np.pi * nx * i / NG)[None, None, :])


def _lam(*n):
    return sum(2.0 - 2.0 * math.cos(2 * math.pi * v / NG) for v in n)


def _empty_state(phi, a):
    # no particles: the periodic source S h^2 (delta - mean delta) is zero
    return pm.State(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, dtype=np.uint32), 0,
                    phi.copy(), a, True, np.zeros(3, dtype=np.int64),
                    np.full(3, NG - 1, dtype=np.int64))


def _cfg(solver="implicit"):
    return pm.Config(ng=NG, box=BOX, omega_m=1.0, omega_l=0.0, c_grav=CG, n_initial=NG**3,
                     solver=solver)


def _run(phi0, a0, a1, nsteps, solver="implicit"):
    st = _empty_state(phi0, a0)
    cfg = _cfg(solver)
    edges = np.linspace(a0, a1, nsteps + 1)
    for s in range(nsteps):
        st = pm.step(st, cfg, edges[s + 1] - edges[s])
    return st.phi


def _amplitude(phi, mode):
    return float(np.sum(phi * mode) / np.sum(mode * mode))


@pytest.mark.parametrize("n,a1", [((1, 0, 0), 0.7), ((2, 1, 0), 0.6), ((1, 1, 3), 0.55)])
def test_implicit_steps_converge_to_eq4_relaxation(n, a1):
    a0 = 0.5
    mode = _mode(*n)
    exact = -K * _lam(*n) * (a1 - a0)          # log of the exact decay
    errs = []
    for nsteps in (16, 32, 64, 128):
        amp = _amplitude(_run(mode, a0, a1, nsteps), mode)
        errs.append(math.log(amp) - exact)
    errs = np.array(errs)
    # first order in the step: each halving halves the error
    ratios = errs[:-1] / errs[1:]
    assert np.all(np.abs(ratios - 2.0) < 0.15), (errs, ratios)
    # the Richardson limit is the exact decay of Eq. 4
    assert abs(2 * errs[-1] - errs[-2]) < 2e-3 * abs(exact), errs


def test_implicit_field_stays_a_single_mode():
    # the periodic operator is diagonal in Fourier space: no other mode appears
    mode = _mode(1, 2, 0)
    phi = _run(mode, 0.3, 0.32, 3)
    amp = _amplitude(phi, mode)
    assert np.max(np.abs(phi - amp * mode)) < 1e-14


def _backward_euler(y, t0, t1, rate):
    """Textbook backward Euler for dy/dtau = -rate(tau) y over [t0, t1]:
    the new value solves y1 = y + (t1 - t0) (-rate(t1) y1), here by a root
    finder rather than by rearranging."""
    g = lambda y1: y1 - y + (t1 - t0) * rate(t1) * y1
    return optimize.brentq(g, -2.0 * abs(y) - 1.0, 2.0 * abs(y) + 1.0, xtol=1e-15, rtol=1e-15)


def test_one_large_step_is_backward_euler_on_half_substeps():
    # a -> a + da in Einstein-de Sitter: tau = 2 sqrt(a), calH(tau) = 2 / tau.
    # The potential advances by one backward-Euler step of Eq. 4 over each
    # conformal half of the step (Table 2: to t + dt/2, then to t + dt), the
    # Hubble rate taken where each sub-step ends (an implicit step evaluates
    # its whole right-hand side at the new time).
    a0, da = 0.3, 0.3
    n = (1, 1, 0)
    lam = _lam(*n)
    mode = _mode(*n)
    rate = lambda tau: CG * CG * lam / (3.0 * (2.0 / tau) * H * H)
    t0, t1 = 2.0 * math.sqrt(a0), 2.0 * math.sqrt(a0 + da)
    tm = 0.5 * (t0 + t1)
    y_half = _backward_euler(1.0, t0, tm, rate)
    y_end = _backward_euler(y_half, tm, t1, rate)
    diag = {}
    st = pm.step(_empty_state(mode, a0), _cfg(), da, diag)
    assert _amplitude(diag["phi_half"], mode) == pytest.approx(y_half, rel=1e-11)
    assert _amplitude(st.phi, mode) == pytest.approx(y_end, rel=1e-11)
    # the two Hubble rates differ by 10 % here, so their order is visible
    swapped = _backward_euler(1.0, t0, tm, lambda tau: rate(t1))
    assert abs(swapped / y_half - 1.0) > 1e-2


def test_ade_steps_converge_to_eq4_relaxation():
    # the paper's integrator (alternating Saul'yev sweeps, one per half
    # sub-step) with its mesh ratio lam = D (dtau/2) / h^2, D = c_g^2 / (3 calH):
    # as the step shrinks the field tends to the same exact decay
    a0, a1 = 0.5, 0.6
    n = (1, 0, 0)
    mode = _mode(*n)
    exact = mode * math.exp(-K * _lam(*n) * (a1 - a0))
    errs = []
    for nsteps in (4, 8, 16):
        phi = _run(mode, a0, a1, nsteps, solver="ade")
        errs.append(float(np.sqrt(np.mean((phi - exact) ** 2)) / np.sqrt(np.mean(exact**2))))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[-1] < 1e-2, errs
    assert errs[1] / errs[2] > 1.7, errs
