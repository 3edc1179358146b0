"""GPU checks of the learned warm start: each matrix-core convolution kernel
against the oracle's FP64 convolution on identical BF16 operands, the whole
net forward, training on the method's own recorded solves, and the warm
start inside the solve (accepted only when it lowers the residual; plain
multigrid is the fallback, including for non-finite weights)."""
import numpy as np
import pytest

from oracle import conv as oc
from synth import zeldovich_ics

from helpers import lib_config, log, make_sim, rel_rms

pytestmark = pytest.mark.gpu


def _bf16_tensor(x):
    """float64 array (already BF16-representable) -> int16 device tensor."""
    import torch
    u = np.asarray(x, dtype=np.float32).view(np.uint32) >> 16
    return torch.as_tensor(u.astype(np.uint16).view(np.int16)).cuda()


def _from_bf16(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _random_act(n, seed, positive=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.normal(size=(n, n, n, 16))
    if positive:
        x = np.maximum(x, 0.0)
    return oc.bf16_round(x)


@pytest.mark.parametrize("n", [16, 32, 64])
def test_conv_forward_matches_oracle(n):
    import torch
    import paper_1709_04703_amd as P
    log(f"conv forward n={n}")
    x = _random_act(n, n)
    rng = np.random.Generator(np.random.PCG64(100 + n))
    w = rng.normal(size=(27, 16, 16)) * 0.1
    b = rng.normal(size=16) * 0.1
    wq = oc.bf16_round(w)
    ref = oc.conv(x, wq, b)
    xin = _bf16_tensor(x).reshape(-1, 16)
    wt = torch.as_tensor(w.astype(np.float32)).cuda()
    bt = torch.as_tensor(b.astype(np.float32)).cuda()
    out0 = torch.zeros(n**3, dtype=torch.float32, device="cuda")
    P.conv3d(n, xin, wt, bt, P.CONV_OUT_FP32_CH0, None, out0)
    got0 = out0.cpu().numpy().reshape(n, n, n)
    assert rel_rms(got0, ref[..., 0]) < 1e-5
    outb = torch.zeros_like(xin)
    P.conv3d(n, xin, wt, bt, P.CONV_RELU, None, outb)
    got = _from_bf16(outb).reshape(n, n, n, 16)
    refr = np.maximum(ref, 0.0)
    refq = oc.bf16_round(refr)
    # equal up to one BF16 rounding step where the FP32 sum straddles a
    # rounding boundary (or the ReLU threshold, within FP32 accumulation error)
    diff = np.abs(got - refq)
    tol = np.maximum(np.abs(refq) * 2.0**-7, 1e-5 * np.sqrt(np.mean(ref**2)))
    assert np.all(diff <= 1.01 * tol)
    assert np.mean(diff > 0) < 0.01


@pytest.mark.parametrize("n", [16, 32])
def test_conv_backward_data_matches_oracle(n):
    import torch
    import paper_1709_04703_amd as P
    g = _random_act(n, 7 + n)
    mask = _random_act(n, 9 + n, positive=True)
    rng = np.random.Generator(np.random.PCG64(n))
    w = rng.normal(size=(27, 16, 16)) * 0.1
    ref = oc.conv_dgrad(g, oc.bf16_round(w)) * (mask > 0)
    out = torch.zeros((n**3, 16), dtype=torch.int16, device="cuda")
    P.conv3d(n, _bf16_tensor(g).reshape(-1, 16), torch.as_tensor(w.astype(np.float32)).cuda(), None,
             P.CONV_BACKWARD_DATA | P.CONV_MASK, _bf16_tensor(mask).reshape(-1, 16), out)
    got = _from_bf16(out).reshape(n, n, n, 16)
    refq = oc.bf16_round(ref)
    diff = np.abs(got - refq)
    tol = np.maximum(np.abs(refq) * 2.0**-7, 1e-5 * np.sqrt(np.mean(ref**2)))
    assert np.all(diff <= 1.01 * tol)
    assert rel_rms(got, ref) < 5e-3


@pytest.mark.parametrize("n", [16, 32, 64])
def test_conv_weight_gradient_matches_oracle(n):
    import torch
    import paper_1709_04703_amd as P
    x = _random_act(n, 3 * n)
    g = _random_act(n, 5 * n)
    dw_ref, db_ref, _ = oc.conv_wgrad(x, g)
    dw = torch.zeros((27, 16, 16), dtype=torch.float32, device="cuda")
    db = torch.zeros(16, dtype=torch.float32, device="cuda")
    scratch = torch.zeros(P.net_scratch_bytes(n), dtype=torch.uint8, device="cuda")
    P.conv3d_wgrad(n, _bf16_tensor(x).reshape(-1, 16), _bf16_tensor(g).reshape(-1, 16), dw, db,
                   scratch)
    assert rel_rms(dw.cpu().numpy(), dw_ref) < 1e-5
    assert rel_rms(db.cpu().numpy(), db_ref) < 1e-5
    dw2 = torch.zeros_like(dw)
    P.conv3d_wgrad(n, _bf16_tensor(x).reshape(-1, 16), _bf16_tensor(g).reshape(-1, 16), dw2, db,
                   scratch)
    assert torch.equal(dw, dw2)                     # deterministic reduction


def test_net_forward_matches_oracle():
    import torch
    import paper_1709_04703_amd as P
    from paper_1709_04703_amd.train import init_params
    n = 16
    rng = np.random.Generator(np.random.PCG64(4))
    r = rng.normal(size=(n, n, n))
    phi = rng.normal(size=(n, n, n))
    vec = init_params(3)
    params = oc.unflatten(vec)
    x0 = np.zeros((n, n, n, 16))
    x0[..., 0] = r * 0.5
    x0[..., 1] = phi * 2.0
    x0[..., 2] = 0.3
    _, ref = oc.forward(x0, params, round_bf16=True)
    act0 = torch.zeros((n**3, 16), dtype=torch.int16, device="cuda")
    P.net_prep(n, torch.as_tensor(r.astype(np.float32)).cuda().reshape(-1),
               torch.as_tensor(phi.astype(np.float32)).cuda().reshape(-1), 0.5, 2.0, 0.3, act0)
    assert np.array_equal(_from_bf16(act0).reshape(n, n, n, 16), oc.bf16_round(x0))
    a = torch.zeros_like(act0)
    b = torch.zeros_like(act0)
    out = torch.zeros(n**3, dtype=torch.float32, device="cuda")
    P.net_forward(n, torch.as_tensor(vec).cuda(), act0, a, b, out)
    err = rel_rms(out.cpu().numpy().reshape(n, n, n), ref)
    log(f"  net forward rel rms vs oracle = {err:.2e}")
    # each layer's BF16 outputs may differ from the oracle's by one BF16 step
    # (2^-8 relative) where the two FP32 sums straddle a rounding boundary,
    # in under 1 % of them (the single-layer test): per layer at most
    # sqrt(0.01) 2^-8 = 3.9e-4 relative RMS, over five layers at most 2e-3
    # (measured 7.4e-4)
    assert err < 2e-3


def test_training_reduces_loss_on_one_sample():
    import torch
    from paper_1709_04703_amd.train import Trainer, init_params
    n = 16
    rng = np.random.Generator(np.random.PCG64(8))
    r = torch.as_tensor(rng.normal(size=n**3).astype(np.float32)).cuda()
    phi = torch.as_tensor(rng.normal(size=n**3).astype(np.float32)).cuda()
    # target: a smooth function of r (a local average), learnable by the net
    rr = r.cpu().numpy().reshape(n, n, n)
    tgt = sum(np.roll(rr, s, axis=a) for a in range(3) for s in (-1, 1)) / 6.0
    buf = torch.stack([r, phi, torch.as_tensor(tgt.astype(np.float32).ravel()).cuda()])[None]
    tr = Trainer(n, init_params(1), lr=3e-3)
    hist = tr.train(buf, np.array([0.2]), np.array([1.0]), np.array([1.0]), 300, log_every=50)
    log(f"  loss history {hist}")
    assert hist[-1][1] < 0.2 * hist[0][1]


def test_learned_warm_start_trains_and_falls_back():
    """Train on the method's own solves (64^3, periodic phase) and use the
    net as the initial guess of the same configuration with another seed:
    the solve still reaches tol, the accepted guesses lower the starting
    residual, non-finite weights fall back to plain multigrid, and the gated
    mode runs the net at most as often as the ungated one."""
    import paper_1709_04703_amd as P
    from paper_1709_04703_amd.train import Trainer, init_params, record_pairs
    ng, box, a0, nsteps = 64, 2000.0, 1.0 / 50.0, 40
    ics = [zeldovich_ics(ng, box, a0, s) for s in (11, 12)]
    buf, kap, rms_r, rms_phi = record_pairs(ics, ng, box, a0, nsteps, 60)
    log(f"  recorded {buf.shape[0]} solves")
    assert buf.shape[0] >= 40
    tr = Trainer(ng, init_params(0), lr=4e-4)
    hist = tr.train(buf, kap, rms_r, rms_phi, 1500, log_every=250)
    log(f"  loss history {hist}")
    err = tr.evaluate(buf, kap, rms_r, rms_phi, range(0, buf.shape[0], 7))
    log(f"  relative error of the predicted change on training pairs: {err:.3f}")
    weights = tr.weights()
    x, p, ids = zeldovich_ics(ng, box, a0, 13)
    res = {}
    ws = {"prev": P.SDPM_WS_PREV, "learned": P.SDPM_WS_LEARNED, "nan": P.SDPM_WS_LEARNED,
          "gated": P.SDPM_WS_LEARNED_GATED}
    net_calls = {}
    for mode in ("prev", "learned", "gated", "nan"):
        cfg = lib_config(ng, box, c_grav=-1.0, shrink=1, n_initial=ng**3, warm_start=ws[mode])
        sim = make_sim(cfg, ng**3)
        sim.profile(True)
        if mode in ("learned", "gated"):
            sim.set_warmstart_weights(weights)
        elif mode == "nan":
            bad = weights.copy()
            bad[::7] = np.nan
            sim.set_warmstart_weights(bad)
        sim.bind(x, p, ids)
        sim.init_potential(a0)
        edges = np.linspace(a0, 1.0, nsteps + 1)
        iters, used, g0, r0 = [], 0, [], []
        for s in range(12):
            st = sim.step(edges[s], edges[s + 1] - edges[s])
            assert max(st["res"]) <= cfg.tol
            iters.append(st["vcycles"])
            used += st["warm_used"]
            g0.append(st["res_guess"][0])
            r0.append(st["res0"][0])
        res[mode] = (np.array(iters), used, np.array(g0), np.array(r0), sim.phi_numpy().copy())
        net_calls[mode] = sim.profile_read().get("conv3d_mfma", {}).get("launches", 0) // 5
        log(f"  {mode}: V-cycles {iters} guesses used {used} "
            f"median res0 {np.median(r0):.2e} -> guess {np.median(g0):.2e} "
            f"net calls {net_calls[mode]}")
        sim.close()
    assert res["nan"][1] == 0
    assert np.array_equal(res["nan"][0], res["prev"][0])
    # every accepted guess lowered the residual; the trained net never costs
    # V-cycles (it gains few at this size: 2 of 132 when measured, its 11^3
    # receptive field reaching about half of the weight of the step's Green's
    # function); the converged fields agree
    iters_l, used_l, g_l, r_l, phi_l = res["learned"]
    log(f"  V-cycles over 12 steps: prev {res['prev'][0].sum()}, learned {iters_l.sum()}")
    assert iters_l.sum() <= res["prev"][0].sum()
    assert np.all(g_l <= r_l)
    assert rel_rms(phi_l, res["prev"][4]) < 1e-5
    assert net_calls["prev"] == 0 and net_calls["learned"] >= 12
    assert 1 <= net_calls["gated"] <= net_calls["learned"]
    assert np.all(res["gated"][2] <= res["gated"][3])
    assert rel_rms(res["gated"][4], res["prev"][4]) < 1e-5


def test_train_step_matches_oracle_adam():
    """One training step (forward, MSE loss, backward through every layer,
    Adam at step 5 from nonzero moments, so the update depends on the
    gradient's size, not only its sign) against the oracle's BF16-rounded
    forward / backward and its Adam (Kingma & Ba 2015): the loss, both moment
    updates, the parameter change, and the frozen parameters left at zero."""
    import torch
    import paper_1709_04703_amd as P
    from paper_1709_04703_amd.train import init_params
    n = 16
    rng = np.random.Generator(np.random.PCG64(21))
    r32 = rng.normal(size=(n, n, n)).astype(np.float32)
    phi32 = rng.normal(size=(n, n, n)).astype(np.float32)
    tgt32 = rng.normal(size=(n, n, n)).astype(np.float32)
    s_r, s_phi, kap, ts = np.float32(0.7), np.float32(1.3), np.float32(0.2), np.float32(0.5)
    vec32 = init_params(2)
    mask = oc.frozen_mask()
    assert np.all(vec32[mask] == 0.0)
    # oracle: the prep's FP32 products, rounded to BF16 by forward()
    x0 = np.zeros((n, n, n, 16))
    x0[..., 0] = (r32 * s_r).astype(np.float64)
    x0[..., 1] = (phi32 * s_phi).astype(np.float64)
    x0[..., 2] = float(kap)
    loss_o, g = oc.train_step_grads(x0, oc.unflatten(vec32), tgt32.astype(np.float64), float(ts))
    gr = np.sqrt(np.mean(g[~mask] ** 2))
    m1 = (rng.normal(size=g.size) * gr).astype(np.float32)
    m2 = (rng.uniform(0.5, 1.5, size=g.size) * gr * gr).astype(np.float32)
    m1[mask] = 0.0
    m2[mask] = 0.0
    step, lr = 5, 1e-3
    th_o, m1_o, m2_o = oc.adam(vec32.astype(np.float64), g, m1.astype(np.float64),
                               m2.astype(np.float64), step, lr, frozen=mask)
    # GPU
    act0 = torch.zeros((n**3, 16), dtype=torch.int16, device="cuda")
    P.net_prep(n, torch.as_tensor(r32).cuda().reshape(-1), torch.as_tensor(phi32).cuda().reshape(-1),
               float(s_r), float(s_phi), float(kap), act0)
    th_t = torch.as_tensor(vec32).cuda()
    m1_t, m2_t = torch.as_tensor(m1).cuda(), torch.as_tensor(m2).cuda()
    scratch = torch.zeros(P.net_scratch_bytes(n), dtype=torch.uint8, device="cuda")
    loss_t = torch.zeros(1, dtype=torch.float32, device="cuda")
    P.net_train_step(n, th_t, m1_t, m2_t, step, lr, act0, torch.as_tensor(tgt32).cuda().reshape(-1),
                     float(ts), scratch, loss_t)
    th_g, m1_g, m2_g = (t.cpu().numpy().astype(np.float64) for t in (th_t, m1_t, m2_t))
    loss_g = float(loss_t.item())
    live = ~mask
    g_from_m1 = (m1_g - 0.9 * m1) / 0.1
    log(f"  loss gpu {loss_g:.6e} oracle {loss_o:.6e}; gradient rel rms "
        f"{rel_rms(g_from_m1[live], g[live]):.2e}; update rel rms "
        f"{rel_rms((th_g - vec32)[live], (th_o - vec32)[live]):.2e}")
    # the two sides round the same FP32 sums to BF16; they differ only where a
    # sum falls within FP32 accumulation error of a rounding boundary
    assert abs(loss_g - loss_o) <= 1e-4 * loss_o
    assert rel_rms(g_from_m1[live], g[live]) < 1e-4
    assert rel_rms(m2_g[live], m2_o[live]) < 1e-4
    assert rel_rms((th_g - vec32)[live], (th_o - vec32)[live]) < 1e-4
    assert np.all(th_g[mask] == 0.0)
