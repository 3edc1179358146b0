"""CPU-only checks of the C ABI: the library loads, exports every symbol the
header declares, validates configurations, and its host-side logic (step
scalars, lightcone radius, active box) agrees with the oracle's independent
implementation.  No device work is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import cosmology as oc
from oracle import pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1709_04703_amd as pkg
    from paper_1709_04703_amd import build

    if not os.path.exists(build.LIB):
        build.build()
    pkg.library()
    return pkg


def test_exports_every_declared_symbol(P):
    header = open(os.path.join(ROOT, "include", "sdpm.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(sdpm_\w+)\s*\(", header, re.M))
    assert declared == set(P.EXPORTS)
    lib = P.library()
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout(P):
    assert ctypes.sizeof(P.Config) == 152   # ..., solver, cycles_per_outer, assignment (+4 padding)
    assert ctypes.sizeof(P.StepStats) == 8 * 2 + 4 * 4 + 8 * 4 + 8 * 5 + 4 * 7 + 4 * 8 + 4 + 16


@pytest.mark.parametrize("a,da,cg", [(0.02, 0.0049, -1.0), (0.5, 0.01, 0.0), (0.9, 0.1, 3000.0),
                                     (0.0204, 0.049, 0.0)])
def test_step_scalars_match_oracle(P, a, da, cg):
    cfg = P.config_default(128, 2000.0, c_grav=cg)
    got = P.step_scalars(cfg, a, da)
    ref = oc.step_scalars(a, da, 0.3, 0.7, 2000.0, 128, cg)
    for k in ("dtau", "a_half", "s_half", "kappa1_h2", "kappa2_h2", "r_lc_end", "c_g"):
        assert got[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-300), k


def test_lightcone_radius_matches_oracle(P):
    cfg = P.config_default(64, 100.0)
    for a in (0.02, 0.1, 0.7, 0.999, 1.0):
        assert P.lightcone_radius(cfg, a) == pytest.approx(oc.lightcone_radius(a, 0.3, 0.7),
                                                           rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("ng,align", [(64, 1), (64, 8), (128, 16), (512, 32)])
def test_domain_box_matches_oracle(P, ng, align):
    box = 2000.0
    cfg = P.config_default(ng, box, box_align=align)
    rng = np.random.Generator(np.random.PCG64(ng + align))
    for r in list(rng.uniform(0.0, 1.0, 40) * box) + [0.0, box / 2, 0.3 * box]:
        periodic, lo, hi = P.domain_box(cfg, r)
        dirichlet, lo2, hi2 = pm.box_for_radius(r, np.full(3, box / 2), box / ng, ng, 2, align)
        assert periodic == (not dirichlet)
        if dirichlet:
            assert list(lo) == list(lo2) and list(hi) == list(hi2)


def test_config_validation_errors(P):
    with pytest.raises(P.SdpmError, match="power of two"):
        P.workspace_bytes(P.config_default(100, 10.0), 10)
    with pytest.raises(P.SdpmError, match="coarsest"):
        P.workspace_bytes(P.config_default(512, 10.0, mg_levels=3), 10)
    with pytest.raises(P.SdpmError, match="warm_start"):
        P.workspace_bytes(P.config_default(64, 10.0, warm_start=7), 10)
    with pytest.raises(P.SdpmError):
        P.step_scalars(P.config_default(64, 10.0), 0.5, -0.1)


def test_solver_config_validation(P):
    # the ADE integrator needs a finite gravity speed; neither it nor the FFT
    # solve has an iteration to warm-start
    ok = P.config_default(64, 100.0, c_grav=-1.0, solver=P.SDPM_SOLVER_ADE)
    assert P.workspace_bytes(ok, 10) > 0
    for bad in (dict(c_grav=0.0, solver=P.SDPM_SOLVER_ADE),
                dict(c_grav=-1.0, solver=P.SDPM_SOLVER_ADE, warm_start=P.SDPM_WS_EXTRAP),
                dict(c_grav=-1.0, solver=3),
                dict(solver=P.SDPM_SOLVER_FFT, warm_start=P.SDPM_WS_EXTRAP),
                dict(cycles_per_outer=0), dict(cycles_per_outer=5), dict(assignment=2)):
        with pytest.raises(P.SdpmError, match="EINVAL"):
            P.workspace_bytes(P.config_default(64, 100.0, **bad), 10)
    assert P.config_default(64, 100.0).solver == P.SDPM_SOLVER_IMPLICIT
    assert P.config_default(64, 100.0).cycles_per_outer == 4
    assert P.config_default(64, 100.0).assignment == P.SDPM_ASSIGN_CIC
    assert P.workspace_bytes(P.config_default(64, 100.0, assignment=P.SDPM_ASSIGN_TSC), 10) > 0
    for cpo in (1, 4):
        assert P.workspace_bytes(P.config_default(64, 100.0, cycles_per_outer=cpo), 10) > 0
    # the FFT solver's half spectrum and work area come from the workspace
    fft = P.config_default(64, 100.0, solver=P.SDPM_SOLVER_FFT)
    assert (P.workspace_bytes(fft, 10) - P.workspace_bytes(P.config_default(64, 100.0), 10)
            >= 2 * 64 * 64 * 33 * 16)


def test_extrapolated_start_workspace(P):
    # two FP32 change meshes, one per solve kind (the running change is kept
    # in place; no copy of the start)
    prev = P.workspace_bytes(P.config_default(64, 100.0), 10)
    ex = P.workspace_bytes(P.config_default(64, 100.0, warm_start=P.SDPM_WS_EXTRAP), 10)
    assert ex - prev == 2 * 64**3 * 4


def test_power_spectrum_workspace(P):
    # mesh, half spectrum and FFT work area at least
    assert P.pk_workspace_bytes(64) >= 8 * 64**3 + 2 * 64 * 64 * 33 * 16
    for bad in (12, 4, 2048):
        with pytest.raises(P.SdpmError, match="EINVAL"):
            P.pk_workspace_bytes(bad)


def test_workspace_grows_with_capacity_and_precision(P):
    cfg = P.config_default(64, 100.0)
    a = P.workspace_bytes(cfg, 0)
    b = P.workspace_bytes(cfg, 10**6)
    assert b - a >= 10**6 * (24 + 12 + 4)
    plain = P.config_default(64, 100.0, precision=P.SDPM_PLAIN_FP64)
    assert P.workspace_bytes(plain, 0) > a


def test_defaults(P):
    cfg = P.config_default(512, 2000.0)
    assert cfg.mg_levels == 6 and cfg.box_align == 32 and cfg.tol == 1e-8
    assert P.config_default(1024, 4000.0).mg_levels == 7
    assert P.config_default(32, 100.0).mg_levels == 2


def test_rb_sweeps_argument_checks(P):
    # rejected before any launch: sizes outside [64, 2048] or not powers of
    # two, NULL arrays, the fused form writing the array it reads, and a
    # residual output without a positive scale or aliasing another array
    lib = P.library()
    buf, out, t = ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48)
    for n in (32, 96, 4096):
        assert lib.sdpm_rb_sweeps(n, buf, out, buf, 1.0, 0.1, 0, 1, None, 0.0, None, None) == P.SDPM_EINVAL
    assert lib.sdpm_rb_sweeps(64, None, out, buf, 1.0, 0.1, 0, 1, None, 0.0, None, None) == P.SDPM_EINVAL
    assert lib.sdpm_rb_sweeps(64, buf, None, buf, 1.0, 0.1, 1, 1, None, 0.0, None, None) == P.SDPM_EINVAL
    assert lib.sdpm_rb_sweeps(64, buf, buf, buf, 1.0, 0.1, 0, 1, None, 0.0, None, None) == P.SDPM_EINVAL
    # the residual needs scale > 0 and an array of its own
    assert lib.sdpm_rb_sweeps(64, buf, out, buf, 0.0, 0.1, 0, 1, t, 0.1, None, None) == P.SDPM_EINVAL
    assert lib.sdpm_rb_sweeps(64, buf, out, buf, 1.0, 0.1, 0, 1, out, 0.1, None, None) == P.SDPM_EINVAL
    # a box must keep a plane from every face
    for bad in ((0, 1, 1, 10, 10, 10), (1, 1, 1, 63, 10, 10), (5, 5, 5, 4, 10, 10)):
        bx = (ctypes.c_int32 * 6)(*bad)
        assert lib.sdpm_rb_sweeps(64, buf, out, buf, 1.0, 0.1, 0, 1, None, 0.0, bx, None) == P.SDPM_EINVAL
