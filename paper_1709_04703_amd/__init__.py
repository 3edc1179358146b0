"""Shrinking-domain particle-mesh gravity on AMD MI355X (gfx950).

The data-parallel hot path of Llinares (2017), "The shrinking domain
framework I": fixed-point CIC deposit, multigrid solve of the implicit step of
the paper's gravity equation on the shrinking index box, finite-difference
force, CIC interpolation, synchronised leapfrog and lightcone removal, all in
hand-written HIP kernels behind the C ABI of ``include/sdpm.h``.
"""
from ._lib import (  # noqa: F401
    CONV_BACKWARD_DATA, CONV_MASK, CONV_OUT_FP32_CH0, CONV_RELU, NET_PARAMS, conv3d, conv3d_wgrad,
    net_forward, net_forward_noalloc, net_prep, net_scratch_bytes, net_train_step, pk_workspace_bytes, power_spectrum,
    rb_sweeps,
    SDPM_PK_JING, SDPM_PK_SHOT,
    Config, EXPORTS, SDPM_ASSIGN_CIC, SDPM_ASSIGN_TSC, SDPM_EDOMAIN, SDPM_EFULL, SDPM_EINVAL, SDPM_ENOCONV,
    SDPM_EOVERFLOW, SDPM_OK, SDPM_MIXED, SDPM_PLAIN_FP64, SDPM_SOLVER_ADE, SDPM_SOLVER_FFT, SDPM_SOLVER_IMPLICIT, SDPM_WS_EXTRAP, SDPM_WS_LEARNED, SDPM_WS_LEARNED_GATED, SDPM_WS_PREV, SdpmError,
    Simulation, StepStats, config_default, domain_box, library, lightcone_radius,
    step_scalars, workspace_bytes,
)
