"""GPU parity of the power-spectrum estimator (sdpm_power_spectrum) against
the oracle (oracle/pk.py) on the same positions: shell wavenumbers, mode
counts (exact), raw shell powers and the shot-noise / Jing-corrected
spectrum, for 16^3 .. 64^3 meshes and every flag combination; at the 512^3
size the raw spectrum of every shell, and the Jing-corrected value of
sampled shells from the oracle run on the shells that value depends on (a
shell's final value depends on its neighbours within 3 shells: one per slope
re-estimate).  Positions outside the box are an error.

Tolerance: the counts are bit-identical (the same fixed-point deposit); the
FFTs and the shell sums differ in rounding order, so shell values agree to
~1e-13 relative of the largest shell (mean wavenumbers to 1e-13, 1e-11 for
the 512^3 shells of up to ~8e5 modes); 1e-10 relative is the gate for the
powers (1e-9 for the corrected spectrum, which divides by window sums
computed with transcendental functions)."""
import numpy as np
import pytest

from oracle import pk
from synth import clustered_particles, uniform_particles

from helpers import log

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x.T)).cuda()


def _positions(n, box, seed):
    xc, _, _ = clustered_particles(n // 2, box, seed, width_cells=2.0, ng=32)
    xu, _, _ = uniform_particles(n - n // 2, box, seed + 1)
    return np.concatenate([xc, xu])


@pytest.mark.parametrize("ng", [16, 32, 64])
@pytest.mark.parametrize("shot,jing", [(False, False), (True, False), (True, True)])
def test_power_spectrum_matches_oracle(ng, shot, jing):
    import paper_1709_04703_amd as P
    box, n = 300.0, 120_000
    x = _positions(n, box, ng)
    log(f"P(k) ng={ng} shot={shot} jing={jing}")
    got = P.power_spectrum(_dev(x), box, ng, shot=shot, jing=jing)
    ref = pk.power_spectrum(x, box, ng, shot=shot, jing=jing)
    assert np.array_equal(got["modes"], ref["modes"])
    assert np.abs(got["k"] / ref["k"] - 1.0).max() <= 1e-13
    scale = np.abs(ref["p_raw"]).max()
    assert np.abs(got["p_raw"] - ref["p_raw"]).max() <= 1e-10 * scale
    pscale = np.abs(ref["p"]).max()
    err = np.abs(got["p"] - ref["p"]).max() / pscale
    log(f"  max rel err p={err:.2e}")
    assert err <= 1e-9


def test_power_spectrum_rejects_positions_outside_the_box():
    import paper_1709_04703_amd as P
    box = 100.0
    x, _, _ = uniform_particles(1000, box, 3)
    # x = L is the periodic image of 0 (the deposit's own rule)
    x[17, 1] = box
    at_l = P.power_spectrum(_dev(x), box, 16)
    x[17, 1] = 0.0
    # (the same counts; shell sums in LDS atomics may differ in the last bit)
    assert np.allclose(P.power_spectrum(_dev(x), box, 16)["p_raw"], at_l["p_raw"], rtol=1e-13,
                       atol=0.0)
    for bad in (-1e-9, box * (1.0 + 1e-12), np.nan):
        x[17, 1] = bad
        with pytest.raises(P.SdpmError, match="EDOMAIN|EOVERFLOW"):
            P.power_spectrum(_dev(x), box, 16)
    x[17, 1] = 1.0
    with pytest.raises(P.SdpmError, match="EINVAL"):
        P.power_spectrum(_dev(x), box, 12)


def test_fullsize_power_spectrum():
    import paper_1709_04703_amd as P
    ng, box, n = 512, 2000.0, 2_000_000
    x = _positions(n, box, 512)
    log("P(k) 512^3, 2M positions")
    got = P.power_spectrum(_dev(x), box, ng, shot=True, jing=True)
    counts = pk.pm.deposit(x, ng, box, 14, True)
    delta = counts.astype(np.float64) / (n / ng**3 * 2.0 ** 42) - 1.0
    del counts
    k, p_raw, modes, c1, (fx, fy, fz, idx) = pk.shells_from_field(delta, box)
    del delta
    assert np.array_equal(got["modes"], modes)
    # shells of up to ~8e5 modes summed in different orders: ~1e-12 relative
    assert np.abs(got["k"] / k - 1.0).max() <= 1e-11
    assert np.abs(got["p_raw"] - p_raw).max() <= 1e-10 * np.abs(p_raw).max()
    shot = box**3 / n
    for b in (4, 40):
        lo, hi = b - 1 - 3, b - 1 + 3          # shell indices (shell b is index b - 1)
        sel = (idx >= lo) & (idx <= hi)
        win = (fx[sel], fy[sel], fz[sel], idx[sel] - lo)
        pw = pk.jing_correct(k[lo:hi + 1], p_raw[lo:hi + 1], c1[lo:hi + 1], shot, win, ng)
        err = abs(got["p"][b - 1] / pw[b - 1 - lo] - 1.0)
        log(f"  shell {b}: p={got['p'][b - 1]:.6e} oracle={pw[b - 1 - lo]:.6e} rel err {err:.1e}")
        assert err <= 1e-9
