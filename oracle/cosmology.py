"""Oracle background cosmology (FP64, SciPy quadrature).  TEST INFRASTRUCTURE.

Units: comoving length in Mpc/h, conformal time tau in units of 1/H0 (H0 = 1),
so the speed of light is c = 2997.92458 (Mpc/h) H0.

Paper passages followed
-----------------------
* Sec. 2.1, Eqs. 1-3: dots are conformal-time derivatives, the Poisson source
  is 3 H0^2 Omega_m / (2a) * delta.
* Sec. 2.1 Eq. 4 and App. A: H = (da/dtau)/a is the conformal Hubble rate,
  here calH(a) = a E(a).
* Sec. 2.4 Eq. 10: the lightcone radius.  As printed (c times elapsed time
  since the *initial* time) it grows; the past lightcone of a z=0 observer
  shrinks to zero at a = 1 (Sec. 1, Fig. 1).  Reading taken: the comoving
  distance light travels between a and today, r_lc(a) = c (tau(1) - tau(a)).
* Sec. 3: "1000 steps uniform in a" in conformal time: for a step a -> a+da
  the conformal interval is the integral of da/(a^2 E).  The mid-step scale
  factor a(t+dt/2) of Eq. 8 is read as the conformal midpoint.
"""
from __future__ import annotations

import math

from scipy import integrate, optimize

C_LIGHT = 2997.92458  # (Mpc/h) * H0


def hubble_e(a: float, om: float, ol: float) -> float:
    """E(a) = H(a)/H0 for matter + Lambda + curvature (ok = 1 - om - ol)."""
    ok = 1.0 - om - ol
    return math.sqrt(om / a**3 + ok / a**2 + ol)


def conformal_hubble(a: float, om: float, ol: float) -> float:
    """calH = (da/dtau)/a = a E(a)  (the paper's H in Eq. 4, App. A)."""
    return a * hubble_e(a, om, ol)


def dtau(a0: float, a1: float, om: float, ol: float) -> float:
    """Conformal time between a0 and a1: integral of da / (a^2 E(a))."""
    val, _ = integrate.quad(lambda a: 1.0 / (a * a * hubble_e(a, om, ol)),
                            a0, a1, epsabs=1e-16 * abs(a1 - a0), epsrel=1e-13, limit=200)
    return val


def a_of_dtau(a0: float, target: float, a_hi: float, om: float, ol: float) -> float:
    """Scale factor reached after conformal time `target` from a0 (bracketed)."""
    if target == 0.0:
        return a0
    return optimize.brentq(lambda a: dtau(a0, a, om, ol) - target, a0, a_hi,
                           xtol=1e-16, rtol=1e-15, maxiter=200)


def step_scalars(a: float, da: float, om: float, ol: float, box: float, ng: int,
                 c_grav: float, c_light: float = C_LIGHT) -> dict:
    """Scalars of one step a -> a + da (Sec. 2.2 Eqs. 7-9, Sec. 2.3 Eq. 4).

    dtau      conformal step
    a_half    conformal midpoint a(tau_n + dtau/2)
    s_half    Poisson source factor 3 Omega_m/(2 a_half)        (Eq. 3)
    kappa1_h2 screening of the first implicit half sub-step:
              3 calH(a_half) h^2 / (c_g^2 dtau/2)
    kappa2_h2 screening of the second half sub-step, calH at a+da
    c_g       gravity speed: 0 => static Poisson; < 0 => paper's
              c_eff = 0.019 h c with h the cell size in Mpc/h (Eq. 12)
    r_lc_end  lightcone radius at a + da
    """
    a1 = a + da
    dt = dtau(a, a1, om, ol)
    a_half = a_of_dtau(a, 0.5 * dt, a1, om, ol)
    h = box / ng
    if c_grav < 0.0:
        cg = 0.019 * h * c_light
    else:
        cg = c_grav
    if cg == 0.0:
        k1 = k2 = 0.0
    else:
        k1 = 3.0 * conformal_hubble(a_half, om, ol) * h * h / (cg * cg * 0.5 * dt)
        k2 = 3.0 * conformal_hubble(a1, om, ol) * h * h / (cg * cg * 0.5 * dt)
    return dict(dtau=dt, a_half=a_half, s_half=1.5 * om / a_half,
                kappa1_h2=k1, kappa2_h2=k2, c_g=cg,
                r_lc_end=lightcone_radius(a1, om, ol, c_light))


def lightcone_radius(a: float, om: float, ol: float, c_light: float = C_LIGHT) -> float:
    """Comoving radius of the z=0 observer's past lightcone at a (Eq. 10 read
    as c (tau(1) - tau(a)); zero at a = 1)."""
    if a >= 1.0:
        return 0.0
    return c_light * dtau(a, 1.0, om, ol)


def growth_d(a: float, om: float, ol: float) -> float:
    """Linear growing mode, normalised to D(1) = 1 (Heath 1977 integral,
    valid for pressureless matter + Lambda + curvature):
    D(a) proportional to E(a) * integral_0^a da' / (a' E(a'))^3."""
    def unnorm(x):
        i, _ = integrate.quad(lambda y: 1.0 / (y * hubble_e(y, om, ol))**3, 0.0, x,
                              epsabs=0.0, epsrel=1e-13, limit=200)
        return hubble_e(x, om, ol) * i
    return unnorm(a) / unnorm(1.0)


def growth_f(a: float, om: float, ol: float) -> float:
    """f = dlnD/dlna from the Heath form:  a E'/E + 1/(a^2 E^3 I(a))."""
    ok = 1.0 - om - ol
    e = hubble_e(a, om, ol)
    i, _ = integrate.quad(lambda y: 1.0 / (y * hubble_e(y, om, ol))**3, 0.0, a,
                          epsabs=0.0, epsrel=1e-13, limit=200)
    dlne = (-3.0 * om / a**3 - 2.0 * ok / a**2) / (2.0 * e * e)
    return dlne + 1.0 / (a * a * e**3 * i)
