"""Benchmark of the shrinking-domain particle-mesh step on one MI355X.

Workload (default): 512^3 particles on a 512^3 mesh, 2000 Mpc/h box, synthetic
Lambda-CDM Zel'dovich initial conditions at z = 49 (seed 512), steps of the
200-step schedule uniform in a to z = 0, shrinking domain with the paper's
reduced gravity speed, multigrid to 1e-8 relative residual.  A step is one
sdpm_step (all of Table 2, lightcone elimination included) on inputs resident
in HBM.  These modes are timed on the same inputs, each implicit one to the same
1e-8 relative residual:
  plain:   FP64 V-cycles warm-started from the previous potential, FP64 momenta;
  mixed:   FP32 V(2,2) cycles (6 levels) inside FP64 defect correction, FP32
           momenta, previous-potential warm start;
  extrap:  mixed, each solve started from the potential plus the change the
           same solve made in the previous step (linear extrapolation in time);
  learned: extrap, plus the conv-net warm start, gated: the library keeps the
           net only while the V-cycles it saves outweigh its measured cost
           (the headline value);
  learned_always: extrap, plus the conv-net guess tried before every solve;
  ade:     the paper's own gravity integrator instead of the implicit solve
           (one alternating-direction explicit sweep per half sub-step, FP64
           mesh, FP32 momenta): a different discretisation in time, so it is
           not held to the residual; its potential and momenta after the timed
           steps are compared with those of the implicit modes (ade_vs_implicit);
  fft:     the implicit step solved exactly by FP64 FFT while the mesh is
           periodic (the standard particle-mesh solver), FP32 momenta; compared
           with the implicit modes like ade (fft_vs_implicit);
  tsc:     extrap with TSC instead of CIC assignment (27 nodes per particle
           both ways).
The net is trained once before the timed regions, on the GPU, on solves
recorded (with the extrapolated start) from the periodic phase of 128^3 runs
(2000 Mpc/h, z = 49 -> 0 in 100 steps, seeds 10001-10013: every solve, the
first 2000), and applied both at 512^3 (the learned modes above) and at 256^3
(learned_transfer: seeds 20001-20003, steps 5-24 of the 100-step schedule,
the extrapolated start with and without the learned guess).
The shrinking phase of the same run (steps 160-164 by default: lightcone
removal, the frozen-exterior box and the lightcone output all active) is
timed separately and reported as shrink_phase.
In the timed steps only the launches of the roofline kernel (the finest level's
fused four-sweep post-smoothing passes; the net's layers in the learned modes) carry
HIP event pairs;
--profile-steps further untimed steps (3) have every kernel bracketed for the
per-kernel breakdown (kernel_ms_per_step, roofline.kernels).
The oracle (FP64 NumPy/SciPy) is timed on a bounded sample as cpu_baseline.
With --table4 N the paper's Table 4 comparison runs as well: whole runs
z = 40 -> 0 of N^3 particles in the paper's three boxes, shrinking vs fixed
domain, timed (opt-in: at N = 512 and 1000 steps it takes a few minutes).
Two accuracy experiments of the paper, on synthetic 128^3 inputs (experiments):
  lightcone: the 3D power spectrum of the lightcone recorded by a shrinking run
    and by a run on the fixed periodic domain (same diffusion gravity), in a
    cubical box of the original size (2000 Mpc/h, z = 49 -> 0 in 100 steps);
  solvers: the z = 0 power spectrum of a 500 Mpc/h box (fixed domain) with
    static Poisson gravity (FFT) against the diffusion equation advanced
    implicitly (multigrid) and by the paper's ADE sweeps (also with 4x the
    steps: its small-scale modes relax only when lam k^2 h^2 is small).

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


# HBM bytes per dispatch measured with rocprofv3 (FETCH_SIZE and WRITE_SIZE passes, each
# scaled by what the counter reads for a 1 GiB device-to-device copy), averaged over the
# kernel's dispatches in the default 512^3 mixed workload (profiles/ holds the summary).
# Valid only for the kernel source it was measured on: sweep4_fused is the 512^3 level's
# fused post-smoothing pass, 607228.6 KiB fetched (x 1.99992 for the copy's 524307.8 KiB per
# GiB) and 534612.2 KiB written per dispatch.
MEASURED_TRAFFIC = {"sweep4_fused": 1791000072}

MFMA_KERNELS = ("conv3d_mfma", "conv3d_wgrad_mfma")
BF16_PEAK_TFLOPS = 2500.0
# forward flops per voxel of the warm-start net: the method's channels
# (2 x 27 x (3 x 16 + 3 x 16 x 16 + 16 x 1)) and what the kernels compute with
# every layer padded to 16 x 16 channels (5 x 2 x 27 x 16 x 16)
NET_METHOD_FLOPS_PER_VOXEL = 2 * 27 * (3 * 16 + 3 * 16 * 16 + 16)
NET_KERNEL_FLOPS_PER_VOXEL = 5 * 2 * 27 * 16 * 16


def kernel_roofline(name, d):
    """Achieved rate of one kernel from the library's live HIP-event profile:
    algorithmic bytes (or matrix-core flops) per launch / mean launch time."""
    avg_ms = d["ms"] / max(d["launches"], 1)
    per_launch = d["bytes"] / max(d["launches"], 1)
    if name in MFMA_KERNELS:
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                "avg_launch_ms": avg_ms, "launches": d["launches"]}
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "avg_launch_ms": avg_ms, "launches": d["launches"]}


# The kernel with the largest share of GPU time in the step (the finest
# level's fused four-sweep post-smoothing passes: 10 bytes per cell); its
# launches alone carry HIP events in the timed
# steps, since an event pair around every launch (~300 per step) would slow
# the timed step itself.  The full per-kernel profile comes from further,
# untimed steps, and names its own largest kernel.
ROOFLINE_KERNEL = "sweep4_fused"


def roofline_of(prof, prof_full=None, full_steps=0):
    """Roofline entry of ROOFLINE_KERNEL from the timed steps' events, plus
    every kernel's time per step and rate from the fully profiled steps
    (None when the mode never launched that kernel, as the FFT and ADE
    solvers do not)."""
    if not prof.get(ROOFLINE_KERNEL, {}).get("launches"):
        return None
    out = kernel_roofline(ROOFLINE_KERNEL, prof[ROOFLINE_KERNEL])
    if prof_full:
        out["largest_kernel_in_full_profile"] = max(prof_full, key=lambda k: prof_full[k]["ms"])
        out["full_profile_steps"] = full_steps
        out["kernels"] = {
            k: {"ms_per_step": round(v["ms"] / full_steps, 3),
                "launches_per_step": round(v["launches"] / full_steps, 2),
                ("TFLOP/s" if k in MFMA_KERNELS else "GB/s"):
                    round(v["bytes"] / (v["ms"] * 1e-3) / (1e12 if k in MFMA_KERNELS else 1e9), 1)
                    if v["ms"] > 0 else None}
            for k, v in sorted(prof_full.items(), key=lambda kv: -kv[1]["ms"]) if v["launches"]}
    return out


def train_net(P, torch, args):
    """Record solves from args.train_ng^3 runs (periodic phase of the
    args.train_schedule-step schedule, every solve of it, up to
    args.train_pairs) and train the warm-start net on them; returns
    (weights, info)."""
    from paper_1709_04703_amd.train import Trainer, init_params, record_pairs
    from synth import zeldovich_ics

    t0 = time.perf_counter()
    a0 = 1.0 / (1.0 + args.z_init)
    seeds = [int(s) for s in args.train_seeds.split(",")]
    ics = [zeldovich_ics(args.train_ng, args.box, a0, s) for s in seeds]
    buf, kap, rms_r, rms_phi = record_pairs(ics, args.train_ng, args.box, a0, args.train_schedule,
                                            args.train_pairs, warm_start=P.SDPM_WS_EXTRAP)
    del ics
    t1 = time.perf_counter()
    tr = Trainer(args.train_ng, init_params(0), lr=args.train_lr)
    hist = tr.train(buf, kap, rms_r, rms_phi, args.train_iters,
                    log_every=max(1, args.train_iters // 5))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    err = tr.evaluate(buf, kap, rms_r, rms_phi, range(0, buf.shape[0], max(1, buf.shape[0] // 20)))
    w = tr.weights()
    del buf, tr
    torch.cuda.empty_cache()
    info = {"train_mesh": args.train_ng, "seeds": seeds, "schedule": args.train_schedule,
            "pairs": int(len(kap)), "iterations": args.train_iters,
            "record_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
            "loss": [(i, round(v, 5)) for i, v in hist], "rel_err_dphi": round(err, 4)}
    log(f"net: {info}")
    return w, info


def learned_transfer(P, torch, args, weights):
    """The trained net applied at args.apply_ng^3 (seeds args.apply_seeds, the
    same box and schedule as the training runs): per seed, args.apply_warmup
    untimed then args.apply_steps timed steps with the extrapolated start
    alone, with the gated learned guess added, and with the learned guess
    before every solve; mixed precision, every solve to 1e-8."""
    from synth import zeldovich_ics

    ng = args.apply_ng
    a0 = 1.0 / (1.0 + args.z_init)
    edges = np.linspace(a0, 1.0, args.train_schedule + 1)
    rows = {m: [] for m in ("extrap", "learned", "learned_always")}
    for seed in (int(v) for v in args.apply_seeds.split(",")):
        x, p, ids = zeldovich_ics(ng, args.box, a0, seed)
        n = x.shape[0]
        for mode in rows:
            ws = P.SDPM_WS_EXTRAP | {"extrap": P.SDPM_WS_PREV, "learned": P.SDPM_WS_LEARNED_GATED,
                                     "learned_always": P.SDPM_WS_LEARNED}[mode]
            cfg = P.config_default(ng, args.box, c_grav=-1.0, shrink=1, precision=P.SDPM_MIXED,
                                   n_initial=n, sort_every=args.sort_every,
                                   sort_shift=args.sort_shift, warm_start=ws,
                                   cycles_per_outer=args.cycles_per_outer)
            sim = P.Simulation(cfg, n)
            if mode != "extrap":
                sim.set_warmstart_weights(weights)
            sim.bind(x, p, ids)
            sim.init_potential(a0)
            for s_ in range(args.apply_warmup):
                sim.step(edges[s_], edges[s_ + 1] - edges[s_])
            sim.profile(True, kernels=["conv3d_mfma"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vc, used = 0, 0
            for s_ in range(args.apply_warmup, args.apply_warmup + args.apply_steps):
                st = sim.step(edges[s_], edges[s_ + 1] - edges[s_])
                vc += st["vcycles"]
                used += st["warm_used"]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            prof = sim.profile_read().get("conv3d_mfma", {"launches": 0, "ms": 0.0})
            rows[mode].append({"seed": seed, "ms_per_step": 1e3 * dt / args.apply_steps,
                               "vcycles_per_solve": vc / (2.0 * args.apply_steps),
                               "net_calls": prof["launches"] // 5, "guesses_accepted": used,
                               "net_ms_per_call": (prof["ms"] / max(1, prof["launches"] // 5))})
            sim.close()
            del sim
        del x, p, ids
    torch.cuda.empty_cache()
    mean = {m: {k: float(np.mean([r[k] for r in v])) for k in v[0] if k != "seed"}
            for m, v in rows.items()}
    out = {"mesh": ng, "seeds": args.apply_seeds, "steps": (f"{args.apply_warmup}.."
                                                             f"{args.apply_warmup + args.apply_steps - 1}"
                                                             f" of {args.train_schedule}"),
           "per_seed": rows, "mean": mean,
           "learned_speedup_vs_extrap": mean["extrap"]["ms_per_step"] / mean["learned"]["ms_per_step"],
           "learned_always_speedup_vs_extrap": (mean["extrap"]["ms_per_step"]
                                                / mean["learned_always"]["ms_per_step"]),
           "vcycles_saved_per_solve_always": (mean["extrap"]["vcycles_per_solve"]
                                              - mean["learned_always"]["vcycles_per_solve"])}
    log(f"learned transfer {ng}^3: {json.dumps(out['mean'])}")
    return out


def run_mode(P, torch, ics, args, precision, profile, weights=None, gated=True, extrap=False,
             solver=0, keep=False, assignment=0):
    x, p, ids = ics
    ng, box = args.ng, args.box
    n = x.shape[0]
    cfg = P.config_default(ng, box, c_grav=-1.0, shrink=1, precision=precision, n_initial=n,
                           sort_every=args.sort_every, sort_shift=args.sort_shift,
                           warm_start=(P.SDPM_WS_PREV if weights is None else
                                       P.SDPM_WS_LEARNED_GATED if gated else P.SDPM_WS_LEARNED)
                           | (P.SDPM_WS_EXTRAP if extrap else 0), solver=solver,
                           cycles_per_outer=args.cycles_per_outer, assignment=assignment)
    sim = P.Simulation(cfg, n)
    if weights is not None:
        sim.set_warmstart_weights(weights)
    sim.bind(x, p, ids)
    a0 = 1.0 / (1.0 + args.z_init)
    edges = np.linspace(a0, 1.0, args.schedule + 1)
    sim.init_potential(a0)
    step = 0
    for _ in range(args.warmup):
        sim.step(edges[step], edges[step + 1] - edges[step])
        step += 1
    if profile:
        sim.profile(True, kernels=[ROOFLINE_KERNEL] + (["conv3d_mfma"] if weights is not None else []))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates, vcyc, solve_ms, iters, stats, used = 0, 0, 0.0, [], [], 0
    for _ in range(args.steps):
        n_act = sim.n_active
        st = sim.step(edges[step], edges[step + 1] - edges[step])
        updates += n_act
        vcyc += st["vcycles"]
        solve_ms += st["ms"][2] + st["ms"][4]
        iters.append(st["outer_iters"])
        used += st["warm_used"]
        stats.append(st)
        step += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = sim.profile_read() if profile else None
    prof_full = None
    if profile and args.profile_steps > 0:
        # untimed: every kernel bracketed, for the per-kernel breakdown
        sim.profile(True)
        for _ in range(args.profile_steps):
            sim.step(edges[step], edges[step + 1] - edges[step])
            step += 1
        prof_full = sim.profile_read()
        sim.profile(False)
    kept = None
    if keep:
        # final potential and momenta (ordered by particle id), left on the GPU
        k = sim.n_active
        order = torch.argsort(sim.ids[:k].to(torch.int64) & 0xFFFFFFFF)
        kept = (sim.phi.clone(), sim.p[:, :k][:, order].to(torch.float64))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return dict(seconds=dt, updates=updates, vcycles=vcyc, solve_ms=solve_ms, iters=iters,
                stats=stats, prof=prof, prof_full=prof_full, cfg=cfg, warm_used=used, kept=kept)


def copy_bandwidth(torch, mib=2048, reps=5):
    """Achieved HBM rate of a plain device-to-device copy (read + write bytes
    over time), a practical ceiling for the streaming kernels."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def _run_to_end(P, ics, ng, box, z_init, steps, lightcone=False, **cfg_kw):
    """One 128^3-scale run z_init -> 0; returns (sim, n) with the run done."""
    x, p, ids = ics
    n = x.shape[0]
    cfg = P.config_default(ng, box, n_initial=n, **cfg_kw)
    sim = P.Simulation(cfg, n)
    sim.bind(x, p, ids)
    if lightcone:
        sim.set_lightcone(n)
    a0 = 1.0 / (1.0 + z_init)
    edges = np.linspace(a0, 1.0, steps + 1)
    sim.init_potential(a0)
    for s_ in range(steps):
        sim.step(edges[s_], edges[s_ + 1] - edges[s_])
    return sim, n


def _pk(P, torch, x, box, ng):
    """P(k) of host positions (n, 3), wrapped into the periodic box; the raw
    shell spectrum (p_raw) is the one compared between runs (the particles
    come from a displaced lattice, so Poisson shot-noise subtraction does not
    apply), the Jing-corrected one is reported beside it."""
    xw = np.mod(x, box)
    xw[xw >= box] = 0.0
    return P.power_spectrum(torch.as_tensor(np.ascontiguousarray(xw.T)).cuda(), box, ng,
                            shot=False, jing=True)


def _rel(pa, pb, modes, min_modes=20):
    sel = modes >= min_modes
    return float(np.max(np.abs(pa[sel] / pb[sel] - 1.0)))


def _rel_curve(pa, pb, every=8):
    return [round(float(v), 5) for v in (pa / pb - 1.0)[::every]]


def experiments(P, torch, args):
    """The paper's two accuracy comparisons on synthetic inputs (module notes)."""
    from synth import zeldovich_ics
    t0 = time.perf_counter()
    ng, steps, z0 = args.exp_ng, args.exp_steps, args.z_init
    out = {}
    # lightcone: shrinking vs fixed domain
    box = 2000.0
    ics = zeldovich_ics(ng, box, 1.0 / (1.0 + z0), args.seed + 1)
    recs = {}
    for shrink in (1, 0):
        sim, n = _run_to_end(P, ics, ng, box, z0, steps, lightcone=True, c_grav=-1.0,
                             shrink=shrink, sort_every=args.sort_every)
        gid, _, gx, _ = sim.lightcone_records()
        recs[shrink] = (gid, gx)
        sim.close()
    same = np.array_equal(np.sort(recs[1][0]), np.sort(recs[0][0]))
    dx = None
    if same:
        xa = recs[1][1][np.argsort(recs[1][0])]
        xb = recs[0][1][np.argsort(recs[0][0])]
        d = np.abs(xa - xb)
        d = np.minimum(d, box - d)
        dx = float(d.max() / (box / ng))
    pks = {s_: _pk(P, torch, recs[s_][1], box, ng) for s_ in (1, 0)}
    out["lightcone"] = {
        "box": box, "particles": ng**3, "steps": steps,
        "records": [int(len(recs[1][0])), int(len(recs[0][0]))], "same_particles": bool(same),
        "max_position_diff_cells": dx,
        "pk_raw_max_rel_diff_shrink_vs_fixed": _rel(pks[1]["p_raw"], pks[0]["p_raw"],
                                                    pks[0]["modes"]),
        "pk_raw_rel_diff_shrink_vs_fixed": _rel_curve(pks[1]["p_raw"], pks[0]["p_raw"]),
        "k": [round(float(v), 5) for v in pks[0]["k"][::8]],
        "pk_raw_fixed": [float(v) for v in pks[0]["p_raw"][::8]],
        "pk_jing_fixed": [float(v) for v in pks[0]["p"][::8]],
    }
    # solvers: static Poisson (FFT) vs diffusion (implicit, ADE), fixed domain
    box = 500.0
    ics = zeldovich_ics(ng, box, 1.0 / (1.0 + z0), args.seed + 2)
    final = {}
    for name, kw, nst in (("static_fft", dict(c_grav=0.0, solver=P.SDPM_SOLVER_FFT), steps),
                          ("diffusion_implicit", dict(c_grav=-1.0), steps),
                          ("diffusion_ade", dict(c_grav=-1.0, solver=P.SDPM_SOLVER_ADE), steps),
                          ("diffusion_ade_4x_steps", dict(c_grav=-1.0, solver=P.SDPM_SOLVER_ADE),
                           4 * steps)):
        sim, n = _run_to_end(P, ics, ng, box, z0, nst, shrink=0, sort_every=args.sort_every,
                             precision=P.SDPM_PLAIN_FP64, **kw)
        x, _, _ = sim.particles()
        final[name] = _pk(P, torch, x, box, ng)
        sim.close()
    ref = final["static_fft"]
    out["solvers"] = {
        "box": box, "particles": ng**3, "steps": steps,
        "pk_raw_max_rel_diff_vs_static": {k: _rel(v["p_raw"], ref["p_raw"], ref["modes"])
                                          for k, v in final.items() if k != "static_fft"},
        "k": [round(float(v), 5) for v in ref["k"][::8]],
        "pk_raw_rel_diff_vs_static": {k: _rel_curve(v["p_raw"], ref["p_raw"])
                                      for k, v in final.items() if k != "static_fft"},
        "pk_raw_static": [float(v) for v in ref["p_raw"][::8]],
    }
    out["seconds"] = round(time.perf_counter() - t0, 1)
    log(f"experiments: {json.dumps(out)[:400]}")
    return out


def table4(P, torch, args):
    """The paper's performance comparison (Table 4): whole runs from z = 40 to
    0 in `table4_steps` steps uniform in a, with the shrinking domain and on
    the fixed periodic domain (same diffusion gravity, mixed precision with the
    extrapolated start), in the paper's three boxes; wall time of the steps
    and its ratio, beside the ratio of particle updates."""
    from synth import zeldovich_ics
    ng, steps, z0 = args.table4, args.table4_steps, 40.0
    a0 = 1.0 / (1.0 + z0)
    edges = np.linspace(a0, 1.0, steps + 1)
    rows = []
    for box in (512.0, 2048.0, 8192.0):
        ics = zeldovich_ics(ng, box, a0, args.seed + 3)
        x, p, ids = ics
        n = x.shape[0]
        t, upd = {}, {}
        for shrink in (0, 1):
            cfg = P.config_default(ng, box, c_grav=-1.0, shrink=shrink, precision=P.SDPM_MIXED,
                                   n_initial=n, sort_every=args.sort_every,
                                   sort_shift=args.sort_shift, warm_start=P.SDPM_WS_EXTRAP)
            sim = P.Simulation(cfg, n)
            sim.bind(x, p, ids)
            sim.init_potential(a0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u = 0
            for q in range(steps):
                u += sim.n_active
                sim.step(edges[q], edges[q + 1] - edges[q])
            torch.cuda.synchronize()
            t[shrink], upd[shrink] = time.perf_counter() - t0, u
            sim.close()
            del sim
            torch.cuda.empty_cache()
            log(f"table4 box {box:g}: shrink={shrink} {t[shrink]:.2f} s")
        rows.append({"box": box, "seconds_fixed": round(t[0], 3), "seconds_shrink": round(t[1], 3),
                     "speedup": round(t[0] / t[1], 3),
                     "particle_update_ratio": round(upd[0] / upd[1], 3)})
        del ics, x, p, ids
    return {"particles": ng**3, "steps": steps, "z_init": z0, "rows": rows,
            "paper_speedups_512^3_1000_steps": {"512": 1.08, "2048": 1.44, "8192": 3.02}}


def shrink_phase(P, torch, ics, args):
    """The shrinking phase of the same run: steps 0 .. shrink_from - 1 untimed,
    then shrink_steps steps timed with lightcone removal, the frozen-exterior
    box and the lightcone output on (mixed precision)."""
    x, p, ids = ics
    n = x.shape[0]
    cfg = P.config_default(args.ng, args.box, c_grav=-1.0, shrink=1, precision=P.SDPM_MIXED,
                           n_initial=n, sort_every=args.sort_every, sort_shift=args.sort_shift)
    sim = P.Simulation(cfg, n)
    sim.bind(x, p, ids)
    sim.set_lightcone(n)
    a0 = 1.0 / (1.0 + args.z_init)
    edges = np.linspace(a0, 1.0, args.schedule + 1)
    sim.init_potential(a0)
    for s in range(args.shrink_from):
        sim.step(edges[s], edges[s + 1] - edges[s])
    n0, rec0 = sim.n_active, sim.lightcone_count()
    st0 = sim.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates, removed = 0, 0
    for s in range(args.shrink_from, args.shrink_from + args.shrink_steps):
        n_act = sim.n_active
        st = sim.step(edges[s], edges[s + 1] - edges[s])
        updates += n_act
        removed += st["n_removed"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_end, rec_end = sim.n_active, sim.lightcone_count()
    # untimed, fully profiled steps after the timed ones
    s_end = args.shrink_from + args.shrink_steps
    n_prof = max(0, min(args.profile_steps, args.schedule - s_end))
    prof = {}
    if n_prof:
        sim.profile(True)
        for s in range(s_end, s_end + n_prof):
            sim.step(edges[s], edges[s + 1] - edges[s])
        prof = sim.profile_read()
    out = {
        "steps": f"{args.shrink_from}..{args.shrink_from + args.shrink_steps - 1}",
        "z": [round(1.0 / edges[args.shrink_from] - 1.0, 3),
              round(1.0 / edges[args.shrink_from + args.shrink_steps] - 1.0, 3)],
        "active_fraction": [round(n0 / n, 4), round(n_end / n, 4)],
        "active_box_cells": int(np.prod([h - l + 1 for l, h in zip(st0["lo"], st0["hi"])])),
        "periodic": int(st0["periodic"]),
        "ms_per_step": 1e3 * dt / args.shrink_steps,
        "particle_updates_per_s": updates / dt,
        "removed": removed, "lightcone_records": rec_end - rec0,
        "kernel_ms_per_step": {k: round(v["ms"] / n_prof, 3) for k, v in
                               sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:10]
                               if v["launches"]},
        "kernel_profile_steps": f"{s_end}..{s_end + n_prof - 1}" if n_prof else None,
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    log(f"shrink phase: {out['ms_per_step']:.1f} ms/step, active {out['active_fraction']}")
    return out


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
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")),
                             None)
    except OSError:
        pass
    return {
        "value": n / t_step, "unit": "particle-updates/s", "cores": os.cpu_count(),
        "kind": "oracle", "cpu_model": cpu_model,
        "sample": (f"one {ng}^3 step of the same workload: both FP64 FFT solves and the force "
                   f"mesh timed at full size ({t_mesh:.1f} s), deposit + interpolation + "
                   f"leapfrog timed on the first {m} of {n} particles ({t_dep + t_int:.1f} s) "
                   f"and scaled by n; estimated {t_step:.1f} s per step. The FFTs use every "
                   f"core (scipy.fft workers=-1); the np.add.at deposit and the interpolation "
                   f"run on one"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ng", type=int, default=512)
    ap.add_argument("--box", type=float, default=2000.0)
    ap.add_argument("--z-init", type=float, default=49.0)
    ap.add_argument("--schedule", type=int, default=200)
    ap.add_argument("--seed", type=int, default=512)
    ap.add_argument("--modes", default="plain,mixed,extrap,learned,learned_always,ade,fft,tsc")
    ap.add_argument("--train-ng", type=int, default=128)
    # the periodic phase of a 100-step 128^3 run holds 77 steps (154 solves):
    # 13 runs give the 2000 pairs
    ap.add_argument("--train-seeds", default=",".join(str(10001 + i) for i in range(13)))
    ap.add_argument("--train-schedule", type=int, default=100,
                    help="steps of the training runs' schedule (z_init -> 0)")
    ap.add_argument("--train-pairs", type=int, default=2000)
    ap.add_argument("--train-iters", type=int, default=6000)
    ap.add_argument("--train-lr", type=float, default=1e-3)
    ap.add_argument("--apply-ng", type=int, default=256)
    ap.add_argument("--apply-seeds", default="20001,20002,20003")
    ap.add_argument("--apply-warmup", type=int, default=5)
    ap.add_argument("--apply-steps", type=int, default=20)
    ap.add_argument("--no-learned-transfer", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="untimed steps after the timed ones with every kernel profiled")
    ap.add_argument("--cycles-per-outer", type=int, default=4, choices=(1, 2, 3, 4),
                    help="V-cycles per FP64 defect-correction iteration, at most")
    # re-sort period: the block deposit keeps the particles of a block in a
    # window with a drift margin and routes the rest to global atomics, so
    # a sort (~10 ms at 512^3) pays back only every ~20 steps (measured over
    # steps 5-44: 25.5 / 24.5 / 24.1 / 23.8 ms per step for 5 / 10 / 20 / 40;
    # over steps 100-139: 31.5 / 31.0 / 30.9 ms for 10 / 20 / 40)
    ap.add_argument("--sort-every", type=int, default=20)
    ap.add_argument("--sort-shift", type=int, default=4,
                    help="Morton key of cell blocks of 2^shift cells per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--shrink-from", type=int, default=160)
    ap.add_argument("--shrink-steps", type=int, default=5)
    ap.add_argument("--no-shrink-phase", action="store_true")
    ap.add_argument("--no-experiments", action="store_true")
    ap.add_argument("--table4", type=int, default=0,
                    help="mesh/particles per axis for the Table 4 runs (0: skip)")
    ap.add_argument("--table4-steps", type=int, default=1000)
    ap.add_argument("--exp-ng", type=int, default=128)
    ap.add_argument("--exp-steps", type=int, default=100)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this size (a "
                         "known-size kernel that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the design notes describe how the step would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1709_04703_amd as P
    from synth import zeldovich_ics

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    t = time.perf_counter()
    ics = zeldovich_ics(args.ng, args.box, 1.0 / (1.0 + args.z_init), args.seed)
    log(f"ICs {args.ng}^3 in {time.perf_counter() - t:.1f} s")
    results = {}
    net_info = None
    for mode in args.modes.split(","):
        prec = P.SDPM_PLAIN_FP64 if mode == "plain" else P.SDPM_MIXED
        weights = None
        if mode.startswith("learned"):
            if net_info is None:
                net_weights, net_info = train_net(P, torch, args)
            weights = net_weights
        r = run_mode(P, torch, ics, args, prec, profile=True, weights=weights,
                     gated=(mode != "learned_always"),
                     extrap=mode not in ("plain", "mixed", "ade", "fft"),
                     solver={"ade": P.SDPM_SOLVER_ADE, "fft": P.SDPM_SOLVER_FFT}.get(
                         mode, P.SDPM_SOLVER_IMPLICIT),
                     keep=mode in ("ade", "fft", "extrap", "mixed"),
                     assignment=P.SDPM_ASSIGN_TSC if mode == "tsc" else P.SDPM_ASSIGN_CIC)
        log(f"{mode}: {r['steps'] if 'steps' in r else args.steps} steps in {r['seconds']:.3f} s, "
            f"iters {r['iters']}")
        results[mode] = r
    head_mode = next(m for m in ("learned", "mixed", "extrap", "plain", "learned_always", "ade",
                                 "fft", "tsc") if m in results)
    cmp = {}
    ref_mode = next((m for m in ("extrap", "mixed") if m in results), None)
    for other in ("ade", "fft"):
        if other in results and ref_mode:
            (pa, ma), (pr, mr) = results[other]["kept"], results[ref_mode]["kept"]
            rr = lambda u, v: float(torch.linalg.vector_norm(u - v) / torch.linalg.vector_norm(v))
            cmp[other] = {"reference_mode": ref_mode, "after_step": args.warmup + args.steps,
                          "phi_rel_rms": rr(pa, pr),
                          "p_rel_rms": rr(ma, mr) if ma.shape == mr.shape else None}
            log(f"{other} vs {ref_mode}: {cmp[other]}")
    for r in results.values():
        r["kept"] = None
    torch.cuda.empty_cache()
    head = results[head_mode]
    value = head["updates"] / head["seconds"]
    modes = {}
    for mode, r in results.items():
        modes[mode] = {
            "particle_updates_per_s": r["updates"] / r["seconds"],
            "vcycles_per_s": r["vcycles"] / (r["solve_ms"] / 1e3) if r["solve_ms"] > 0 else None,
            "ms_per_step": 1e3 * r["seconds"] / args.steps,
            "outer_iters_per_solve": float(np.mean([sum(i) / 2 for i in r["iters"]])),
            "vcycles_per_solve": r["vcycles"] / (2.0 * args.steps),
            # wall time of a solve from the step's HIP events (the second with its rhs)
            "ms_per_solve": r["solve_ms"] / (2.0 * args.steps),
            "final_residual_max": (max(max(s["res"]) for s in r["stats"])
                                   if mode not in ("ade", "fft") else None),
            "kappa_h2": r["stats"][0]["kappa_h2"][0],
            "warm_starts_used": r["warm_used"],
            "net_calls": (r["prof"].get("conv3d_mfma", {}).get("launches", 0) // 5
                          if r["prof"] else 0),
            # from the fully profiled steps after the timed ones
            "kernel_ms_per_step": {k: round(v["ms"] / args.profile_steps, 3) for k, v in
                                   sorted(r["prof_full"].items(), key=lambda kv: -kv[1]["ms"])[:10]
                                   if v["launches"]} if r["prof_full"] else None,
        }
    if "plain" in modes:
        for m in modes.values():
            m["speedup_vs_plain"] = m["particle_updates_per_s"] / modes["plain"]["particle_updates_per_s"]
    roofline = (roofline_of(head["prof"], head["prof_full"], args.profile_steps)
                if head["prof"] else None)
    if roofline and args.ng == 512 and roofline["kernel"] in MEASURED_TRAFFIC:
        roofline["traffic"] = MEASURED_TRAFFIC[roofline["kernel"]]
        roofline["traffic_unit"] = "bytes per launch"
    learned_roofline = None
    lmode = next((m for m in ("learned_always", "learned") if m in results), None)
    if lmode and results[lmode]["prof"]:
        lp = results[lmode]["prof"]
        if lp.get("conv3d_mfma", {}).get("launches"):
            learned_roofline = kernel_roofline("conv3d_mfma", lp["conv3d_mfma"])
            # the library charges each layer its padded 16 x 16 channel work; the
            # method's own work is 3 -> 16, 16 -> 16 (three layers), 16 -> 1
            scale = NET_METHOD_FLOPS_PER_VOXEL / NET_KERNEL_FLOPS_PER_VOXEL
            learned_roofline["achieved"] *= scale
            learned_roofline["frac"] *= scale
            learned_roofline["flops_per_voxel"] = NET_METHOD_FLOPS_PER_VOXEL
            learned_roofline["kernel_flops_per_voxel"] = NET_KERNEL_FLOPS_PER_VOXEL
            learned_roofline["mode"] = lmode
    transfer = None
    if net_info is not None and not args.no_learned_transfer:
        transfer = learned_transfer(P, torch, args, net_weights)
    copy_gbs = copy_bandwidth(torch)
    shrink = None
    if not args.no_shrink_phase and args.shrink_from + args.shrink_steps <= args.schedule:
        shrink = shrink_phase(P, torch, ics, args)
    exps = None if args.no_experiments else experiments(P, torch, args)
    t4 = table4(P, torch, args) if args.table4 else None
    cpu = None
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        cpu = cpu_baseline(ics, args)
        log(f"cpu baseline in {time.perf_counter() - t:.1f} s")
    head_net_calls = modes[head_mode]["net_calls"]
    dtype = {"plain": "f64", "mixed": "f32 V-cycles in f64 defect correction",
             "learned": "f32 V-cycles in f64 defect correction",
             "learned_always": "f32 V-cycles in f64 defect correction",
             "extrap": "f32 V-cycles in f64 defect correction",
             "ade": "f64 ADE sweeps", "fft": "f64 FFT solves",
             "tsc": "f32 V-cycles in f64 defect correction"}[head_mode]
    if head_mode.startswith("learned") and head_net_calls > 0:
        dtype += ", bf16 MFMA net"
    warm = {"plain": "previous potential", "mixed": "previous potential",
            "extrap": "previous potential + extrapolated change",
            "tsc": "previous potential + extrapolated change",
            "learned": ("previous potential + extrapolated change + learned guess, gated "
                        f"({head_net_calls} net calls in the timed steps)"),
            "learned_always": ("previous potential + extrapolated change + learned guess "
                               f"before every solve ({head_net_calls} net calls)"),
            "ade": "none (explicit sweeps)", "fft": "none (exact solve)"}[head_mode]
    learned_gain = {}
    if "extrap" in modes:
        for m in ("learned", "learned_always"):
            if m in modes:
                learned_gain[m] = (modes[m]["particle_updates_per_s"]
                                   / modes["extrap"]["particle_updates_per_s"])
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
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"{args.ng}^3 particles, {args.ng}^3 mesh, {args.box:g} Mpc/h, "
                         f"z={args.z_init:g}->0 in {args.schedule} steps (steps "
                         f"{args.warmup}..{args.warmup + args.steps - 1} timed), shrinking "
                         "domain, c_eff = 0.019 h c, multigrid V(2,2) (up to 6 levels, up to 4 "
                         "cycles per FP64 defect correction) to 1e-8, particles re-sorted every "
                         f"{args.sort_every} steps"),
            "global_batch": int(ics[0].shape[0]),
            "parallelism": "single GPU",
            "mode": head_mode,
            "warm_start": warm,
            "net_calls_in_timed_steps": head_net_calls,
        },
        "headline_mode": head_mode,
        # the learned guess's own share: gated / ungated learned over the same
        # mixed-precision solve with the extrapolated start and no net
        "learned_gain_vs_extrap": learned_gain,
        "vcycles_per_s": modes[head_mode]["vcycles_per_s"],
        "modes": modes,
        "roofline": roofline,
        "hbm_copy_GBps": copy_gbs,
        "shrink_phase": shrink,
        "ade_vs_implicit": cmp.get("ade"),
        "fft_vs_implicit": cmp.get("fft"),
        "experiments": exps,
        "table4": t4,
        "roofline_learned": learned_roofline,
        "net": net_info,
        "learned_transfer": transfer,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
