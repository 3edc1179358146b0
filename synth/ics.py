"""Synthetic Lambda-CDM-like initial conditions (seeded, FP64).

The paper's initial conditions (Zel'dovich at z = 40 from a COSMICS power
spectrum, Sec. 3) cannot be reproduced: COSMICS and the runs are not
available.  These inputs stand in for them with the same structure:

* white noise from numpy's PCG64 generator on the particle lattice,
* delta_k = FFT(w) sqrt(P(k) / dV), dV = (L / N)^3,
* displacement psi_k = i k delta_k / k^2 (zero and Nyquist modes removed),
* Zel'dovich positions x = q + D(a_i) psi and momenta p = a_i calH f D psi
  (p = a dx/dtau, Sec. 2.1), lattice q = (j + 1/2) L / N,
* P(k) either a power law or the zero-baryon Eisenstein & Hu (1998) shape,
  normalised to sigma_8 at a = 1 with a top-hat window.

The growth factor here is integrated from its linear ODE with SciPy's
solve_ivp; it is input generation only.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as sfft
from scipy import integrate


@dataclasses.dataclass(frozen=True)
class Cosmology:
    omega_m: float = 0.3
    omega_l: float = 0.7
    h: float = 0.7
    n_s: float = 1.0
    sigma8: float = 0.8

    def e(self, a):
        ok = 1.0 - self.omega_m - self.omega_l
        return np.sqrt(self.omega_m / a**3 + ok / a**2 + self.omega_l)

    def growth(self, a: float):
        """(D(a), f(a)) with D(1) = 1, from D'' + (3/a + E'/E) D'
        - 3 Om / (2 a^5 E^2) D = 0 started in the matter era (D = a)."""
        om = self.omega_m
        ok = 1.0 - om - self.omega_l

        def rhs(x, y):
            e2 = om / x**3 + ok / x**2 + self.omega_l
            dlne = (-3.0 * om / x**4 - 2.0 * ok / x**3) / (2.0 * e2)
            return [y[1], -(3.0 / x + dlne) * y[1] + 1.5 * om / (x**5 * e2) * y[0]]

        a0 = 1e-5
        ends = sorted({a, 1.0})
        sol = integrate.solve_ivp(rhs, (a0, max(ends)), [a0, 1.0], method="DOP853",
                                  rtol=1e-12, atol=1e-16, dense_output=True)
        d_a, dd_a = sol.sol(a)
        d_1 = sol.sol(1.0)[0]
        return d_a / d_1, a * dd_a / d_a


def power_eh(k: np.ndarray, cosmo: Cosmology) -> np.ndarray:
    """Unnormalised k^n_s T(k)^2 with the zero-baryon Eisenstein & Hu (1998)
    transfer function; k in h/Mpc, Gamma = Omega_m h, T_cmb = 2.7255 K."""
    theta = 2.7255 / 2.7
    gamma = cosmo.omega_m * cosmo.h
    q = k * theta**2 / gamma
    l0 = np.log(2.0 * math.e + 1.8 * q)
    c0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    t = l0 / (l0 + c0 * q * q)
    return k**cosmo.n_s * t * t


def power_law(k: np.ndarray, index: float = -2.0) -> np.ndarray:
    return k**index


def sigma_r(pk, r: float = 8.0) -> float:
    """sigma(R) of a power spectrum callable with a top-hat window."""
    lk = np.linspace(math.log(1e-5), math.log(1e3), 20001)
    k = np.exp(lk)
    x = k * r
    w = 3.0 * (np.sin(x) - x * np.cos(x)) / x**3
    w = np.where(x < 1e-3, 1.0 - x * x / 10.0, w)
    integrand = k**3 * pk(k) * w * w / (2.0 * math.pi**2)
    return math.sqrt(integrate.simpson(integrand, x=lk))


def lattice_positions(n1d: int, box: float) -> np.ndarray:
    """Lattice q = (j + 1/2) L / n1d, particle index (iz n + iy) n + ix."""
    c = (np.arange(n1d) + 0.5) * (box / n1d)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def zeldovich_ics(n1d: int, box: float, a_init: float, seed: int,
                  spectrum: str = "eh", cosmo: Cosmology = Cosmology()):
    """Return (x, p, ids): float64 (n, 3), float64 (n, 3), uint32 (n,)."""
    if spectrum == "eh":
        base = lambda k: power_eh(k, cosmo)  # noqa: E731
    elif spectrum == "powerlaw-2":
        base = lambda k: power_law(k, -2.0)  # noqa: E731
    else:
        raise ValueError(spectrum)
    amp = (cosmo.sigma8 / sigma_r(base)) ** 2
    d_i, f_i = cosmo.growth(a_init)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((n1d, n1d, n1d))
    kf = 2.0 * math.pi / box
    k1 = np.fft.fftfreq(n1d, d=1.0 / n1d) * kf
    kz1 = np.fft.rfftfreq(n1d, d=1.0 / n1d) * kf
    kx = kz1[None, None, :]
    ky = k1[None, :, None]
    kz = k1[:, None, None]
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    dv = (box / n1d) ** 3
    with np.errstate(divide="ignore", invalid="ignore"):
        pk = np.where(kk > 0, amp * base(np.where(kk > 0, kk, 1.0)), 0.0)
    wk = sfft.rfftn(w, workers=-1)
    dk = wk * np.sqrt(pk / dv)
    nyq = n1d // 2
    dk[0, 0, 0] = 0.0
    dk[nyq, :, :] = 0.0
    dk[:, nyq, :] = 0.0
    dk[:, :, nyq] = 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_k2 = np.where(kk > 0, 1.0 / (kk * kk), 0.0)
    psi = []
    for kc in (kx, ky, kz):
        comp = sfft.irfftn(1j * kc * dk * inv_k2, s=(n1d, n1d, n1d), workers=-1)
        psi.append(comp.ravel())
    psi = np.stack(psi, axis=1) * d_i
    q = lattice_positions(n1d, box)
    x = np.mod(q + psi, box)
    x = np.where(x >= box, x - box, x)
    calh = a_init * float(cosmo.e(a_init))
    p = a_init * calh * f_i * psi
    ids = np.arange(n1d**3, dtype=np.uint32)
    return x, p, ids


def uniform_particles(n: int, box: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0.0, box, size=(n, 3))
    p = rng.normal(0.0, 1.0, size=(n, 3))
    return x, p, np.arange(n, dtype=np.uint32)


def clustered_particles(n: int, box: float, seed: int, n_halo: int = 8,
                        width_cells: float = 1.5, ng: int = 32, lo: float = 0.0,
                        hi: float | None = None):
    """Gaussian blobs of width `width_cells` cells, inside [lo, hi)^3."""
    hi = box if hi is None else hi
    rng = np.random.Generator(np.random.PCG64(seed))
    h = box / ng
    centres = rng.uniform(lo + 4 * width_cells * h, hi - 4 * width_cells * h, size=(n_halo, 3))
    which = rng.integers(0, n_halo, size=n)
    x = centres[which] + rng.normal(0.0, width_cells * h, size=(n, 3))
    x = np.clip(x, lo, np.nextafter(hi, lo))
    p = rng.normal(0.0, 1.0, size=(n, 3))
    return x, p, np.arange(n, dtype=np.uint32)


def edge_particles(ng: int, box: float):
    """Particles at x = 0, just below L, exactly on mesh nodes and at cell
    midpoints (the deposit's edge cases)."""
    h = box / ng
    below = np.nextafter(box, 0.0)
    pts = [
        (0.0, 0.0, 0.0), (below, below, below), (0.0, below, 0.5 * box),
        (3 * h, 5 * h, 7 * h), ((ng - 1) * h, 0.0, h),
        (2.5 * h, 2.5 * h, 2.5 * h), (below, 0.0, 3.25 * h),
        (np.nextafter(h, 0.0), np.nextafter(h, 2 * h), h),
    ]
    x = np.array(pts, dtype=np.float64)
    p = np.zeros_like(x)
    return x, p, np.arange(x.shape[0], dtype=np.uint32)
