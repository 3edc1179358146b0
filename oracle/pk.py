"""Oracle of the power-spectrum estimator (FP64 NumPy): the paper's accuracy
metric for comparing runs (Sec. 3.1, Sec. 3.2: 3D power spectra of the
lightcone in a cubical box of the original size), with the discreteness
corrections of Jing (2005, ApJ 620, 559) that the paper names for its
spectrum tool (Sec. 2.4).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

Definitions (readings; the paper names the method, not its parameters):
* delta on an n^3 mesh from the fixed-point CIC counts of the particles in a
  periodic box of side L (the deposit of pm.py): delta = C / (nbar 2^(3B)) - 1
  with nbar = N / n^3.
* delta_k = sum_x delta(x) exp(-i k.x) / n^3, P_raw(k) = L^3 |delta_k|^2 for
  the integer frequencies f in [-n/2, n/2)^3, k = f 2 pi / L.
* Shell b collects the modes with rint(|f|) = b, b = 1 .. n/2 (k = 0 and the
  corners beyond the Nyquist sphere are left out); a shell reports the mean
  |k| of its modes, the number of modes, the mean P_raw and P.
* Shot noise of a Poisson sample: P_shot = L^3 / N times the aliased CIC
  window sum C1(f) = prod_d (1 - 2/3 sin^2(pi f_d / n)).
* Jing's alias correction: the observed mean P_raw of a shell is modelled as
  P_b S_b + P_shot <C1>_b with S_b the shell mean of
      S(f) = sum over images m in [-2, 2]^3 of W^2(f + n m) (|f + n m| / |f|)^neff_b,
  W^2(g) = prod_d sinc^4(pi g_d / n) (CIC, sinc x = sin x / x): the true
  spectrum taken as a local power law of slope neff_b around the shell.
  neff starts at 0 and is re-estimated 3 times from the corrected spectrum
  (central log-log differences between neighbouring shells, one-sided at the
  ends, clamped to [-4, 4], 0 where a neighbour is not positive).
"""
from __future__ import annotations

import numpy as np

from . import pm

IMAGES = 2          # images per axis on each side in Jing's alias sum
ITERATIONS = 3      # re-estimates of the local slope
NEFF_CLAMP = 4.0


def frequencies(n: int) -> np.ndarray:
    """Signed integer frequencies of an n-point FFT axis, in FFT order."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def shell_of_modes(n: int):
    """(fx, fy, fz, |f|, shell) over the full n^3 spectrum, arrays indexed
    [kz, ky, kx] like np.fft.fftn of a [z, y, x] field; shell 0 marks modes
    that are left out (k = 0 and |f| beyond n/2 after rounding)."""
    f = frequencies(n)
    fz, fy, fx = np.meshgrid(f, f, f, indexing="ij")
    fa = np.sqrt(fx * fx + fy * fy + fz * fz).astype(np.float64)
    shell = np.rint(fa).astype(np.int64)
    shell[shell > n // 2] = 0
    return fx, fy, fz, fa, shell


def cic_alias_sum(fx, fy, fz, n: int) -> np.ndarray:
    """C1(f) = prod_d (1 - 2/3 sin^2(pi f_d / n)), the sum of the CIC window
    squared over all images (the shot-noise alias factor)."""
    out = np.ones(np.shape(fx))
    for g in (fx, fy, fz):
        s = np.sin(np.pi * g / n)
        out = out * (1.0 - (2.0 / 3.0) * s * s)
    return out


def _sinc4(g, n):
    x = np.pi * np.asarray(g, dtype=np.float64) / n
    s = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
    return s ** 4


def alias_window_sum(fx, fy, fz, neff, n: int, images: int = IMAGES) -> np.ndarray:
    """S(f) = sum_{m in [-images, images]^3} W^2(f + n m) (|f + n m| / |f|)^neff
    per mode (neff per mode)."""
    fa2 = (fx * fx + fy * fy + fz * fz).astype(np.float64)
    out = np.zeros(np.shape(fx))
    for mx in range(-images, images + 1):
        gx = fx + n * mx
        wx = _sinc4(gx, n)
        for my in range(-images, images + 1):
            gy = fy + n * my
            wy = _sinc4(gy, n)
            for mz in range(-images, images + 1):
                gz = fz + n * mz
                g2 = (gx * gx + gy * gy + gz * gz).astype(np.float64)
                ratio = np.where(fa2 > 0.0, g2 / np.where(fa2 > 0.0, fa2, 1.0), 1.0)
                out = out + wx * wy * _sinc4(gz, n) * ratio ** (0.5 * neff)
    return out


def slopes(k: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Local log-log slope of p(k) per shell (see module notes)."""
    nb = len(k)
    out = np.zeros(nb)
    for b in range(nb):
        lo, hi = max(b - 1, 0), min(b + 1, nb - 1)
        if hi == lo or p[lo] <= 0.0 or p[hi] <= 0.0 or k[lo] <= 0.0:
            continue
        out[b] = np.clip(np.log(p[hi] / p[lo]) / np.log(k[hi] / k[lo]), -NEFF_CLAMP, NEFF_CLAMP)
    return out


def shells_from_field(delta: np.ndarray, box: float):
    """Shell means of P_raw of a mesh field: returns (k_mean, p_raw, modes,
    c1_mean) over shells 1 .. n/2 and the per-mode arrays for the correction."""
    n = delta.shape[0]
    dk = np.fft.fftn(delta) / n**3
    praw = box**3 * (dk.real**2 + dk.imag**2)
    fx, fy, fz, fa, shell = shell_of_modes(n)
    nb = n // 2
    kf = 2.0 * np.pi / box
    sel = shell > 0
    idx = shell[sel] - 1
    modes = np.bincount(idx, minlength=nb).astype(np.int64)
    safe = np.maximum(modes, 1)
    k_mean = np.bincount(idx, weights=fa[sel], minlength=nb) / safe * kf
    p_raw = np.bincount(idx, weights=praw[sel], minlength=nb) / safe
    c1 = np.bincount(idx, weights=cic_alias_sum(fx, fy, fz, n)[sel], minlength=nb) / safe
    return k_mean, p_raw, modes, c1, (fx[sel], fy[sel], fz[sel], idx)


def jing_correct(k_mean, p_raw, c1, p_shot, mode_data, n: int, iterations: int = ITERATIONS):
    """Jing's alias-corrected shell spectrum (module notes)."""
    fx, fy, fz, idx = mode_data
    nb = len(k_mean)
    modes = np.maximum(np.bincount(idx, minlength=nb), 1)
    signal = p_raw - p_shot * c1
    neff = np.zeros(nb)
    p = None
    for it in range(iterations + 1):
        s = np.bincount(idx, weights=alias_window_sum(fx, fy, fz, neff[idx], n), minlength=nb)
        p = signal / (s / modes)
        if it < iterations:
            neff = slopes(k_mean, p)
    return p


def power_spectrum(x: np.ndarray, box: float, n: int, shot: bool = True, jing: bool = True,
                   frac_bits: int = 14) -> dict:
    """P(k) of particles x (N, 3) in the periodic box [0, L)^3 on an n^3 mesh."""
    npart = x.shape[0]
    counts = pm.deposit(x, n, box, frac_bits, True)
    nbar = npart / n**3
    delta = counts.astype(np.float64) / (nbar * 2.0 ** (3 * frac_bits)) - 1.0
    k_mean, p_raw, modes, c1, mode_data = shells_from_field(delta, box)
    p_shot = box**3 / npart if shot else 0.0
    if jing:
        p = jing_correct(k_mean, p_raw, c1, p_shot, mode_data, n)
    else:
        p = p_raw - p_shot * c1
    return {"k": k_mean, "p": p, "p_raw": p_raw, "modes": modes, "p_shot": p_shot}
