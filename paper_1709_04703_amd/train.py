"""Training driver for the learned warm start of the multigrid solve.

Training pairs come from the method itself: a shrinking-domain run records,
for every implicit gravity sub-step it solves, the residual of the previous
potential r0, the previous potential phi_old and the converged change
dphi = phi - phi_old (sdpm_record).  The net maps (r0 / rms r0, phi_old /
rms phi_old, kappa h^2) to dphi / rms r0.  Training runs on the GPU with the library's
own forward / backward kernels and Adam (sdpm_net_train_step); this module
only selects samples and moves buffers.  Pairs come from the periodic phase
of the runs (the net pads periodically).
"""
from __future__ import annotations

import math

import numpy as np

from . import _lib as L


def record_pairs(ics_list, ng: int, box: float, a0: float, nsteps: int, max_pairs: int,
                 precision: int = L.SDPM_MIXED, c_grav: float = -1.0, device: str = "cuda:0",
                 steps_per_run: int | None = None, warm_start: int = L.SDPM_WS_PREV):
    """Run the given initial conditions (list of (x, p, ids)) on the schedule
    of nsteps steps uniform in a from a0 to 1, each for at most steps_per_run
    steps of its periodic phase, and record up to max_pairs solves (each from
    the start that warm_start gives: the previous potential, or with
    SDPM_WS_EXTRAP its extrapolation).  Returns
    (buf [P, 3, ng^3] float32 device tensor, kappa h^2, rms_r, rms_phi arrays)."""
    import torch

    V = ng ** 3
    buf = torch.zeros((max_pairs, 3, V), dtype=torch.float32, device=device)
    kap, rr, rp = [], [], []
    got = 0
    for x, p, ids in ics_list:
        if got >= max_pairs:
            break
        cfg = L.config_default(ng, box, c_grav=c_grav, shrink=1, precision=precision,
                               n_initial=x.shape[0], warm_start=warm_start)
        sim = L.Simulation(cfg, x.shape[0], device=device)
        sim.bind(x, p, ids)
        sim.init_potential(a0)
        sim.record(buf[got:], max_pairs - got)
        edges = np.linspace(a0, 1.0, nsteps + 1)
        for s in range(min(nsteps, steps_per_run or nsteps)):
            st = sim.step(edges[s], edges[s + 1] - edges[s])
            if not st["periodic"]:
                break
        n, k, r, ph = sim.record_info()
        # keep solves that changed the potential and ran on the periodic mesh
        kap += list(k)
        rr += list(r)
        rp += list(ph)
        got += n
        sim.close()
    return buf[:got], np.array(kap), np.array(rr), np.array(rp)


class Trainer:
    """Adam training of the warm-start net on recorded pairs (all on device)."""

    def __init__(self, ng: int, params: np.ndarray, lr: float = 1e-3, device: str = "cuda:0"):
        import torch

        self.torch = torch
        self.ng = ng
        V = ng ** 3
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device)
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.act0 = torch.zeros((V, 16), dtype=torch.int16, device=device)
        self.act_a = torch.zeros_like(self.act0)
        self.act_b = torch.zeros_like(self.act0)
        self.out = torch.zeros(V, dtype=torch.float32, device=device)
        self.scratch = torch.zeros(L.net_scratch_bytes(ng), dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.lr = lr
        self.step_count = 0

    def _prep(self, pair, kap, rms_r, rms_phi):
        L.net_prep(self.ng, pair[0], pair[1], 1.0 / rms_r, 1.0 / rms_phi, kap, self.act0)

    def train(self, buf, kap, rms_r, rms_phi, iters: int, seed: int = 0, log_every: int = 0,
              cosine: bool = True):
        """Adam steps, one recorded pair each, drawn uniformly at random, the
        step size decaying from lr to 0 along half a cosine (cosine=False:
        constant), so that the weights at the end are not one noisy
        single-pair step away from where the loss is lowest; returns
        [(iteration, loss)] every log_every iterations."""
        rng = np.random.Generator(np.random.PCG64(seed))
        losses = []
        for it in range(iters):
            q = int(rng.integers(0, buf.shape[0]))
            self._prep(buf[q], kap[q], rms_r[q], rms_phi[q])
            self.step_count += 1
            lr = self.lr * 0.5 * (1.0 + math.cos(math.pi * it / iters)) if cosine else self.lr
            L.net_train_step(self.ng, self.params, self.m1, self.m2, self.step_count, lr,
                             self.act0, buf[q, 2], float(1.0 / rms_r[q]), self.scratch, self.loss)
            if log_every and (it % log_every == 0 or it == iters - 1):
                losses.append((it, float(self.loss.item())))
        return losses

    def predict(self, pair, kap, rms_r, rms_phi):
        """Net output (normalised dphi) for one recorded pair, device tensor."""
        self._prep(pair, kap, rms_r, rms_phi)
        L.net_forward(self.ng, self.params, self.act0, self.act_a, self.act_b, self.out)
        return self.out

    def evaluate(self, buf, kap, rms_r, rms_phi, idx):
        """Mean relative error of the predicted change, ||pred - dphi|| / ||dphi||,
        over the pairs idx (also for the trivial guess dphi = 0, which is 1)."""
        errs = []
        for q in idx:
            pred = self.predict(buf[q], kap[q], rms_r[q], rms_phi[q]) * float(rms_r[q])
            tgt = buf[q, 2]
            errs.append(float((pred - tgt).norm() / tgt.norm().clamp_min(1e-30)))
        return float(np.mean(errs))

    def weights(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().copy()


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised parameters in the ABI layout, output layer scaled down
    so the initial guess is close to phi_old."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for l in range(5):
        fan_in = 27 * (3 if l == 0 else 16)
        w = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(27, 16, 16))
        if l == 0:
            w[:, 3:, :] = 0.0
        if l == 4:
            w[:, :, 1:] = 0.0
            w *= 0.1
        out.append(np.concatenate([w.ravel(), np.zeros(16)]))
    return np.concatenate(out).astype(np.float32)
