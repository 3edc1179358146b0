"""Pins of the power-spectrum oracle (oracle/pk.py) against facts fixed by
mathematics: the closed-form spectrum of a single Fourier mode, the closed
form of the CIC window's alias sum (brute-force image sums), the shot noise
of a Poisson sample, and the recovery of a known power law from its exactly
aliased spectrum by Jing's correction (which plain deconvolution misses)."""
import numpy as np
import pytest

from oracle import pk
from synth import uniform_particles


def test_single_mode_spectrum_closed_form():
    n, box, amp = 32, 250.0, 0.3
    m = (3, 1, 0)
    ix = np.arange(n)
    z, y, x = np.meshgrid(ix, ix, ix, indexing="ij")
    delta = amp * np.cos(2.0 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n)
    k, p_raw, modes, _, _ = pk.shells_from_field(delta, box)
    b = int(np.rint(np.sqrt(sum(v * v for v in m))))
    # two modes (+m, -m) of |delta_k| = amp / 2 in a shell of `modes` modes
    assert p_raw[b - 1] == pytest.approx(2.0 * box**3 * (amp / 2) ** 2 / modes[b - 1], rel=1e-12)
    others = np.delete(p_raw, b - 1)
    assert np.abs(others).max() <= 1e-25 * box**3
    # shell bookkeeping: every mode of the Nyquist sphere counted once
    fx, fy, fz, fa, shell = pk.shell_of_modes(n)
    assert modes.sum() == np.count_nonzero(shell)
    assert k[0] == pytest.approx(2.0 * np.pi / box * np.mean(fa[shell == 1]), rel=1e-14)
    assert modes[0] == 6 + 12 + 8 * 0   # |f| in [0.5, 1.5): the 6 axis and 12 edge modes


@pytest.mark.parametrize("f", [0, 1, 5, 8, 15, -16])
def test_cic_alias_sum_closed_form(f):
    n = 32
    m = np.arange(-4000, 4001)
    brute = pk._sinc4(f + n * m, n).sum()
    assert brute == pytest.approx(1.0 - (2.0 / 3.0) * np.sin(np.pi * f / n) ** 2, rel=1e-10)
    c1 = pk.cic_alias_sum(np.array([f]), np.array([0]), np.array([f]), n)[0]
    assert c1 == pytest.approx(brute * pk.cic_alias_sum(np.array([f]), np.array([0]),
                                                        np.array([0]), n)[0], rel=1e-10)


def test_alias_window_sum_at_zero_slope_tends_to_closed_form():
    n = 16
    f = np.array([[1, 0, 0], [3, -2, 5], [8, 8, -8], [-7, 1, 2]])
    fx, fy, fz = f[:, 0], f[:, 1], f[:, 2]
    wide = pk.alias_window_sum(fx, fy, fz, np.zeros(len(f)), n, images=12)
    closed = pk.cic_alias_sum(fx, fy, fz, n)
    assert np.abs(wide / closed - 1.0).max() <= 2e-4
    # the estimator's own truncation (images = 2) stays within 1e-2 of it
    narrow = pk.alias_window_sum(fx, fy, fz, np.zeros(len(f)), n)
    assert np.abs(narrow / closed - 1.0).max() <= 1e-2


def test_poisson_sample_has_shot_noise_spectrum():
    n, box, npart = 32, 100.0, 1 << 20
    x, _, _ = uniform_particles(npart, box, 77)
    out = pk.power_spectrum(x, box, n, shot=False, jing=False)
    fx, fy, fz, fa, shell = pk.shell_of_modes(n)
    sel = shell > 0
    idx = shell[sel] - 1
    c1 = np.bincount(idx, weights=pk.cic_alias_sum(fx, fy, fz, n)[sel]) / out["modes"]
    ratio = out["p_raw"] / (box**3 / npart * c1)
    # mean over all modes within the statistical error of ~16000 modes
    assert np.average(ratio, weights=out["modes"]) == pytest.approx(1.0, abs=0.03)
    with_shot = pk.power_spectrum(x, box, n, shot=True, jing=False)
    assert abs(np.average(with_shot["p"], weights=out["modes"])) <= 0.03 * box**3 / npart


@pytest.mark.parametrize("slope", [-2.0, -1.0, 0.5])
def test_jing_recovers_power_law_from_its_aliased_spectrum(slope):
    # observed spectrum of a power law A k^slope: the exact alias sum over
    # 9^3 images plus the Poisson shot noise; the correction recovers A k^slope
    n, box, amp = 32, 500.0, 2.0e3
    kf = 2.0 * np.pi / box
    fx, fy, fz, fa, shell = pk.shell_of_modes(n)
    sel = shell > 0
    fx, fy, fz, idx = fx[sel], fy[sel], fz[sel], shell[sel] - 1
    pobs = np.zeros(len(fx))
    for mx in range(-4, 5):
        for my in range(-4, 5):
            for mz in range(-4, 5):
                gx, gy, gz = fx + n * mx, fy + n * my, fz + n * mz
                g = np.sqrt(gx * gx + gy * gy + gz * gz) * kf
                pobs += (pk._sinc4(gx, n) * pk._sinc4(gy, n) * pk._sinc4(gz, n)
                         * amp * g**slope)
    p_shot = 3.0
    c1m = pk.cic_alias_sum(fx, fy, fz, n)
    pobs += p_shot * c1m
    nb = n // 2
    modes = np.bincount(idx, minlength=nb)
    kmean = np.bincount(idx, weights=np.sqrt(fx * fx + fy * fy + fz * fz.astype(float)),
                        minlength=nb) / modes * kf
    p_raw = np.bincount(idx, weights=pobs, minlength=nb) / modes
    c1 = np.bincount(idx, weights=c1m, minlength=nb) / modes
    p = pk.jing_correct(kmean, p_raw, c1, p_shot, (fx, fy, fz, idx), n)
    truth = np.bincount(idx, weights=amp * (np.sqrt(fx * fx + fy * fy + fz * fz.astype(float))
                                            * kf) ** slope, minlength=nb) / modes
    err = np.abs(p[1:] / truth[1:] - 1.0)
    assert err.max() <= 0.005, err
    # plain window deconvolution (alias terms ignored) misses near Nyquist
    w2 = np.bincount(idx, weights=pk._sinc4(fx, n) * pk._sinc4(fy, n) * pk._sinc4(fz, n),
                     minlength=nb) / modes
    plain = (p_raw - p_shot * c1) / w2
    assert np.abs(plain[-1] / truth[-1] - 1.0) > 0.1
