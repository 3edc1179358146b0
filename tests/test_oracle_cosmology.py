"""Pins for the oracle's background scalars (closed forms and an independent
ODE integration), CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import cosmology as oc

C = oc.C_LIGHT


@pytest.mark.parametrize("a0,a1", [(0.02, 0.07), (0.5, 0.51), (0.1, 1.0)])
def test_eds_conformal_time_closed_form(a0, a1):
    # Einstein-de Sitter: E = a^(-3/2) => tau = 2 sqrt(a)
    got = oc.dtau(a0, a1, 1.0, 0.0)
    assert got == pytest.approx(2.0 * (math.sqrt(a1) - math.sqrt(a0)), rel=1e-13)


def test_eds_midpoint_and_lightcone():
    a0, a1 = 0.3, 0.35
    sc = oc.step_scalars(a0, a1 - a0, 1.0, 0.0, 100.0, 32, 0.0)
    # tau(a_half) = (tau0 + tau1)/2 => sqrt(a_half) = (sqrt(a0)+sqrt(a1))/2
    assert sc["a_half"] == pytest.approx(((math.sqrt(a0) + math.sqrt(a1)) / 2) ** 2, rel=1e-13)
    assert sc["r_lc_end"] == pytest.approx(2.0 * C * (1.0 - math.sqrt(a1)), rel=1e-12)
    assert oc.lightcone_radius(1.0, 1.0, 0.0) == 0.0
    assert sc["s_half"] == pytest.approx(1.5 / sc["a_half"], rel=1e-15)
    assert sc["kappa1_h2"] == 0.0 and sc["kappa2_h2"] == 0.0


def test_kappa_uses_paper_c_eff():
    # Eq. 12: c_eff = 0.019 h c with h the cell size (Mpc/h)
    box, ng = 2000.0, 128
    sc = oc.step_scalars(0.5, 0.01, 0.3, 0.7, box, ng, -1.0)
    h = box / ng
    cg = 0.019 * h * C
    assert sc["c_g"] == pytest.approx(cg, rel=1e-15)
    ch = 0.5 * oc.hubble_e(0.5, 0.3, 0.7)
    # kappa h^2 = 3 calH h^2 / (c_g^2 dtau/2) with calH at the sub-step end
    assert sc["kappa1_h2"] == pytest.approx(
        3 * oc.conformal_hubble(sc["a_half"], 0.3, 0.7) * h * h / (cg * cg * 0.5 * sc["dtau"]), rel=1e-14)
    assert sc["kappa2_h2"] / sc["kappa1_h2"] == pytest.approx(
        oc.conformal_hubble(0.51, 0.3, 0.7) / oc.conformal_hubble(sc["a_half"], 0.3, 0.7), rel=1e-14)
    assert ch > 0


def test_eds_growth_is_a():
    for a in (0.02, 0.3, 1.0):
        assert oc.growth_d(a, 1.0, 0.0) == pytest.approx(a, rel=1e-10)
        assert oc.growth_f(a, 1.0, 0.0) == pytest.approx(1.0, rel=1e-10)


def test_open_universe_growth_closed_form():
    # Open matter-only universe: D ~ 1 + 3/x + 3 sqrt(1+x)/x^1.5 ln(sqrt(1+x) - sqrt(x)),
    # x = (1/Om - 1) a  (growing mode, Peebles 1980).
    om = 0.3

    def d1(a):
        x = (1.0 / om - 1.0) * a
        return 1.0 + 3.0 / x + 3.0 * math.sqrt(1 + x) / x**1.5 * math.log(math.sqrt(1 + x) - math.sqrt(x))

    for a in (0.1, 0.4, 0.8):
        assert oc.growth_d(a, om, 0.0) == pytest.approx(d1(a) / d1(1.0), rel=1e-7)


def test_lcdm_growth_against_ode():
    om, ol = 0.3, 0.7

    def rhs(x, y):
        e2 = om / x**3 + ol
        dlne = (-3.0 * om / x**4) / (2.0 * e2)
        return [y[1], -(3.0 / x + dlne) * y[1] + 1.5 * om / (x**5 * e2) * y[0]]

    a0 = 1e-5
    sol = integrate.solve_ivp(rhs, (a0, 1.0), [a0, 1.0], method="DOP853", rtol=1e-12,
                              atol=1e-18, dense_output=True)
    d1 = sol.sol(1.0)[0]
    for a in (0.02, 0.25, 0.6):
        d, dd = sol.sol(a)
        assert oc.growth_d(a, om, ol) == pytest.approx(d / d1, rel=1e-7)
        assert oc.growth_f(a, om, ol) == pytest.approx(a * dd / d, rel=1e-7)


def test_lcdm_conformal_time_against_simpson():
    om, ol = 0.3, 0.7
    a = np.linspace(0.05, 1.0, 40001)
    y = 1.0 / (a * a * np.sqrt(om / a**3 + ol))
    ref = integrate.simpson(y, x=a)
    assert oc.dtau(0.05, 1.0, om, ol) == pytest.approx(ref, rel=1e-10)
