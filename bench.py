"""Benchmark of the shrinking-domain particle-mesh step on one MI355X.

Workload (default): 512^3 particles on a 512^3 mesh, 2000 Mpc/h box, synthetic
Lambda-CDM Zel'dovich initial conditions at z = 49 (seed 512), steps of the
200-step schedule uniform in a to z = 0, shrinking domain with the paper's
reduced gravity speed, multigrid to 1e-8 relative residual.  A step is one
sdpm_step (all of Table 2, lightcone elimination included) on inputs resident
in HBM.  Two solver modes are timed on the same inputs:
  mixed: FP32 V(2,2) cycles (6 levels) inside FP64 defect correction, FP32
         momenta (the headline value);
  plain: FP64 V-cycles, FP64 momenta.
The oracle (FP64 NumPy/SciPy) is timed on a bounded sample as cpu_baseline.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s and V-cycles/s at 512^3 (plain vs learned+mixed, same residual)"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_mode(P, torch, ics, args, precision, profile):
    x, p, ids = ics
    ng, box = args.ng, args.box
    n = x.shape[0]
    cfg = P.config_default(ng, box, c_grav=-1.0, shrink=1, precision=precision, n_initial=n,
                           sort_every=args.sort_every)
    sim = P.Simulation(cfg, n)
    sim.bind(x, p, ids)
    a0 = 1.0 / (1.0 + args.z_init)
    edges = np.linspace(a0, 1.0, args.schedule + 1)
    sim.init_potential(a0)
    step = 0
    for _ in range(args.warmup):
        sim.step(edges[step], edges[step + 1] - edges[step])
        step += 1
    if profile:
        sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates, vcyc, solve_ms, iters, stats = 0, 0, 0.0, [], []
    for _ in range(args.steps):
        n_act = sim.n_active
        st = sim.step(edges[step], edges[step + 1] - edges[step])
        updates += n_act
        vcyc += st["vcycles"]
        solve_ms += st["ms"][2] + st["ms"][4]
        iters.append(st["outer_iters"])
        stats.append(st)
        step += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = sim.profile_read() if profile else None
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return dict(seconds=dt, updates=updates, vcycles=vcyc, solve_ms=solve_ms, iters=iters,
                stats=stats, prof=prof, cfg=cfg)


def cpu_baseline(ics, args):
    """The oracle as it stands: one full-size mesh solve pair + force mesh at
    ng^3, and the particle phases on a sample, scaled to one full step."""
    import scipy.fft  # noqa: F401

    from oracle import cosmology as oc
    from oracle import pm

    x, p, ids = ics
    n = x.shape[0]
    ng, box = args.ng, args.box
    a0 = 1.0 / (1.0 + args.z_init)
    da = (1.0 - a0) / args.schedule
    cfg = pm.Config(ng=ng, box=box, c_grav=-1.0, shrink=True, n_initial=n, align=32)
    sc = oc.step_scalars(a0, da, 0.3, 0.7, box, ng, -1.0)
    h = box / ng
    m = min(n, args.cpu_sample)
    xs, ps = x[:m].copy(), p[:m].copy()
    t0 = time.perf_counter()
    xs = np.mod(xs + ps * (0.5 * sc["dtau"] / a0), box)
    c = pm.deposit(xs, ng, box, 14, True)
    t_dep = time.perf_counter() - t0
    f = pm.source(c, n, 14, sc["s_half"], h, True)
    t1 = time.perf_counter()
    phi = pm.solve_periodic(f, sc["kappa1_h2"])
    g = pm.force_mesh(phi, h)
    phi2 = pm.solve_periodic(f - sc["kappa2_h2"] * phi, sc["kappa2_h2"])
    t_mesh = time.perf_counter() - t1
    t2 = time.perf_counter()
    gp = pm.interpolate(xs, g, ng, box, 14, True)
    ps = ps + gp * (sc["a_half"] * sc["dtau"])
    xs = xs + ps * (0.5 * sc["dtau"] / (a0 + da))
    t_int = time.perf_counter() - t2
    del phi, phi2, g, f, c
    t_step = t_mesh + (t_dep + t_int) * (n / m)
    return {
        "value": n / t_step, "unit": "particle-updates/s", "cores": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"one {ng}^3 step of the same workload: both FP64 FFT solves and the force "
                   f"mesh timed at full size ({t_mesh:.1f} s), deposit + interpolation + "
                   f"leapfrog timed on the first {m} of {n} particles ({t_dep + t_int:.1f} s) "
                   f"and scaled by n; estimated {t_step:.1f} s per step"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ng", type=int, default=512)
    ap.add_argument("--box", type=float, default=2000.0)
    ap.add_argument("--z-init", type=float, default=49.0)
    ap.add_argument("--schedule", type=int, default=200)
    ap.add_argument("--seed", type=int, default=512)
    ap.add_argument("--modes", default="mixed,plain")
    ap.add_argument("--sort-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the design notes for how the step would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1709_04703_amd as P
    from synth import zeldovich_ics

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t = time.perf_counter()
    ics = zeldovich_ics(args.ng, args.box, 1.0 / (1.0 + args.z_init), args.seed)
    log(f"ICs {args.ng}^3 in {time.perf_counter() - t:.1f} s")
    results = {}
    for mode in args.modes.split(","):
        prec = P.SDPM_MIXED if mode == "mixed" else P.SDPM_PLAIN_FP64
        r = run_mode(P, torch, ics, args, prec, profile=(mode == "mixed"))
        log(f"{mode}: {r['steps'] if 'steps' in r else args.steps} steps in {r['seconds']:.3f} s, "
            f"iters {r['iters']}")
        results[mode] = r
    head = results.get("mixed") or next(iter(results.values()))
    value = head["updates"] / head["seconds"]
    modes = {}
    for mode, r in results.items():
        modes[mode] = {
            "particle_updates_per_s": r["updates"] / r["seconds"],
            "vcycles_per_s": r["vcycles"] / (r["solve_ms"] / 1e3) if r["solve_ms"] > 0 else None,
            "ms_per_step": 1e3 * r["seconds"] / args.steps,
            "outer_iters_per_solve": float(np.mean([sum(i) / 2 for i in r["iters"]])),
            "final_residual_max": max(max(s["res"]) for s in r["stats"]),
            "kappa_h2": r["stats"][0]["kappa_h2"][0],
        }
    roofline = None
    if head["prof"]:
        prof = head["prof"]
        dom = max(prof, key=lambda k: prof[k]["ms"])
        d = prof[dom]
        avg_ms = d["ms"] / max(d["launches"], 1)
        achieved = (d["bytes"] / max(d["launches"], 1)) / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "avg_launch_ms": avg_ms, "launches": d["launches"],
                    "kernels": {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                                    "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
                                    if v["ms"] > 0 else None}
                                for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])
                                if v["launches"]}}
    cpu = None
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        cpu = cpu_baseline(ics, args)
        log(f"cpu baseline in {time.perf_counter() - t:.1f} s")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycles in f64 defect correction; f64 positions, f32 momenta",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.ng}^3 particles, {args.ng}^3 mesh, {args.box:g} Mpc/h, "
                         f"z={args.z_init:g}->0 in {args.schedule} steps (steps "
                         f"{args.warmup}..{args.warmup + args.steps - 1} timed), shrinking "
                         "domain, c_eff = 0.019 h c, multigrid 6 levels V(2,2) to 1e-8"),
            "global_batch": int(ics[0].shape[0]),
            "parallelism": "single GPU",
        },
        "vcycles_per_s": modes[next(iter(modes))]["vcycles_per_s"],
        "modes": modes,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
