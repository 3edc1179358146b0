"""The per-kernel event profiler (sdpm_profile, sdpm_profile_kernels): one
step profiled in full and, from an identical state, with only some kernels
bracketed, which must record exactly those kernels with the same launch
counts; algorithmic bytes per launch match the kernels' unit costs; unknown
names are rejected and leave profiling as it was."""
import numpy as np
import pytest

from synth import zeldovich_ics

from helpers import lib_config, log, make_sim

pytestmark = pytest.mark.gpu


def _sim(ng, box, a0):
    x, p, ids = zeldovich_ics(ng, box, a0, 77)
    cfg = lib_config(ng, box, c_grav=-1.0, shrink=1, n_initial=ng**3)
    sim = make_sim(cfg, ng**3)
    sim.bind(x, p, ids)
    sim.init_potential(a0)
    return sim


def test_full_and_selected_profiles_agree():
    import paper_1709_04703_amd as P
    ng, box, a0, da = 64, 2000.0, 0.02, 0.0049
    sims = [_sim(ng, box, a0), _sim(ng, box, a0)]
    sims[0].profile(True)
    sims[1].profile(True, kernels=["smooth_color", "rhs"])
    st = [s.step(a0, da) for s in sims]
    assert st[0]["vcycles"] == st[1]["vcycles"]
    full, sel = sims[0].profile_read(), sims[1].profile_read()
    used = {k for k, v in full.items() if v["launches"]}
    log(f"kernels launched: {sorted(used)}")
    assert {"drift_deposit", "rhs", "smooth_color", "residual_fp64", "correct"} <= used
    assert {k for k, v in sel.items() if v["launches"]} == {"smooth_color", "rhs"}
    for k in ("smooth_color", "rhs"):
        assert sel[k]["launches"] == full[k]["launches"] > 0
        assert sel[k]["bytes"] == full[k]["bytes"]
        assert sel[k]["ms"] > 0.0
    # unit costs: the rhs pass, fused with the solve's first FP64 residual,
    # moves 28 B per cell (counts, phi and rhs 8 B each, the FP32 residual
    # 4 B), a finest-level half sweep 6 B per cell of the level (4 B read of
    # the other colour, 4 B source and 4 B written per cell of its colour)
    assert full["rhs"]["bytes"] == 28.0 * ng**3 * full["rhs"]["launches"]
    assert full["smooth_color"]["bytes"] == 6.0 * ng**3 * full["smooth_color"]["launches"]
    # an unknown name is rejected and the selection stays as it was
    with pytest.raises(P.SdpmError, match="EINVAL"):
        sims[1].profile(True, kernels=["smooth_color", "no_such_kernel"])
    sims[1].step(a0 + da, da)
    again = sims[1].profile_read()
    assert {k for k, v in again.items() if v["launches"]} == {"smooth_color", "rhs"}
    sims[1].profile(False)
    sims[1].step(a0 + 2 * da, da)
    assert all(v["launches"] == 0 for v in sims[1].profile_read().values())
    for s in sims:
        s.close()
