"""Test plumbing shared by the GPU parity tests: building library configs and
the matching oracle configs, and small comparison helpers."""
from __future__ import annotations

import sys

import numpy as np

from oracle import pm


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def lib_config(ng, box, **kw):
    import paper_1709_04703_amd as P

    return P.config_default(ng, box, **kw)


def oracle_config(cfg) -> pm.Config:
    """The oracle's own config with the same physical parameters."""
    return pm.Config(ng=cfg.ng, box=cfg.box, omega_m=cfg.omega_m, omega_l=cfg.omega_l,
                     c_light=cfg.c_light, c_grav=cfg.c_grav, x_obs=tuple(cfg.x_obs),
                     shrink=bool(cfg.shrink), margin=cfg.margin, align=cfg.box_align,
                     frac_bits=cfg.frac_bits, n_initial=cfg.n_initial,
                     assignment="tsc" if cfg.assignment == 1 else "cic")


def make_sim(cfg, capacity):
    import paper_1709_04703_amd as P

    return P.Simulation(cfg, capacity)


def rel_rms(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.mean(b * b))
    return float(np.sqrt(np.mean((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.mean(a * a)))


def periodic_delta(a, b, box):
    d = np.asarray(a) - np.asarray(b)
    return (d + box / 2) % box - box / 2


def cond_periodic(ng: int, kappa_h2: float) -> float:
    """Condition number of (Lap_h - kappa h^2) on the periodic zero-mean space:
    bounds the relative error of phi by cond * relative residual."""
    lam_min = 2.0 - 2.0 * np.cos(2 * np.pi / ng) + kappa_h2
    return (12.0 + kappa_h2) / lam_min
