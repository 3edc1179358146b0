"""Oracle for the learned warm start's 3D convolution net (FP64 NumPy).

TEST INFRASTRUCTURE ONLY.  The net is not from the paper: it is the learned
initial guess for the multigrid solve of the implicit gravity step (the solve
itself is Sec. 2.1 Eq. 4 read as in pm.py).  Five 3x3x3 convolution layers,
16 channels, ReLU between layers, periodic padding on an n^3 mesh, inputs
and weights rounded to BF16 where the GPU stores them in BF16.

Layout (shared convention with the C ABI, not code): activations are
(n, n, n, C) arrays indexed [k, j, i, c]; a layer's weights are W[t, ci, co]
with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) reading the input at
(i+dx, j+dy, k+dz); y[v, co] = b[co] + sum_t sum_ci x[v + off_t, ci] W[t, ci, co].

Pinned by tests/test_oracle_conv.py: a per-voxel brute-force sum, the adjoint
identity <conv(x), g> = <x, dgrad(g)>,
and central finite differences of the loss for every gradient.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
C = 16
N_LAYERS = 5
N_INPUTS = 3      # channels of the net input: residual, previous potential, kappa h^2


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shifted(x: np.ndarray, dx: int, dy: int, dz: int) -> np.ndarray:
    """s[k, j, i] = x[k + dz, j + dy, i + dx] with periodic wrap."""
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(0, 1, 2))


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """y[v, co] = b[co] + sum_t sum_ci x[v + off_t, ci] w[t, ci, co]."""
    n = x.shape[0]
    y = np.zeros((n, n, n, w.shape[2]))
    for t, (dx, dy, dz) in enumerate(TAPS):
        y += shifted(x, dx, dy, dz) @ w[t]
    if b is not None:
        y += b
    return y


def conv_wgrad(x: np.ndarray, g: np.ndarray):
    """Gradients of sum(y * g) for y = conv(x, w, b): dW[t] = sum_v
    x[v + off_t]^T g[v], db = sum_v g[v]."""
    dw = np.zeros((27, x.shape[3], g.shape[3]))
    xs = x.reshape(-1, x.shape[3])
    gs = g.reshape(-1, g.shape[3])
    for t, (dx, dy, dz) in enumerate(TAPS):
        dw[t] = shifted(x, dx, dy, dz).reshape(-1, x.shape[3]).T @ gs
    return dw, gs.sum(axis=0), xs


def conv_dgrad(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of sum(y * g) with respect to x: dx[u, ci] =
    sum_t sum_co g[u - off_t, co] w[t, ci, co]."""
    n = g.shape[0]
    dx_ = np.zeros((n, n, n, w.shape[1]))
    for t, (dx, dy, dz) in enumerate(TAPS):
        dx_ += shifted(g, -dx, -dy, -dz) @ w[t].T
    return dx_


def forward(x0: np.ndarray, params: list, round_bf16: bool = True):
    """Net forward.  params = [(W_l, b_l)] * 5 with W_l (27, 16, 16).  Returns
    the list of activations [a0, a1, ..., a4] (post-ReLU, BF16-rounded when
    round_bf16) and the FP64 output (n, n, n) of channel 0 of layer 5."""
    acts = [bf16_round(x0) if round_bf16 else x0]
    for l, (w, b) in enumerate(params):
        wq = bf16_round(w) if round_bf16 else w
        y = conv(acts[-1], wq, b)
        if l < N_LAYERS - 1:
            y = np.maximum(y, 0.0)
            acts.append(bf16_round(y) if round_bf16 else y)
        else:
            return acts, y[..., 0]
    raise AssertionError


def backward(acts: list, params: list, g_out: np.ndarray, round_bf16: bool = False):
    """Gradients of sum(out * g_out) with respect to every W_l, b_l, through
    the ReLUs (dy/dx = 1 where the activation is positive)."""
    n = g_out.shape[0]
    g = np.zeros((n, n, n, C))
    g[..., 0] = g_out
    grads = [None] * N_LAYERS
    for l in range(N_LAYERS - 1, -1, -1):
        w = params[l][0]
        wq = bf16_round(w) if round_bf16 else w
        gq = bf16_round(g) if round_bf16 else g
        dw, db, _ = conv_wgrad(acts[l], gq)
        grads[l] = (dw, db)
        if l > 0:
            g = conv_dgrad(gq, wq) * (acts[l] > 0)
    return grads


def init_params(seed: int, scale: float = 1.0):
    """He-style random initial weights (FP64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for l in range(N_LAYERS):
        fan_in = 27 * (N_INPUTS if l == 0 else C)
        w = rng.normal(0.0, scale * np.sqrt(2.0 / fan_in), size=(27, C, C))
        if l == 0:
            w[:, N_INPUTS:, :] = 0.0
        if l == N_LAYERS - 1:
            w[:, :, 1:] = 0.0
        b = np.zeros(C)
        params.append((w, b))
    return params


def frozen_mask() -> np.ndarray:
    """Parameters the training keeps at zero, in flat order: input channels
    >= N_INPUTS of layer 0 and output channels >= 1 (weights and bias) of the
    last layer."""
    out = []
    for l in range(N_LAYERS):
        w = np.zeros((27, C, C), dtype=bool)
        b = np.zeros(C, dtype=bool)
        if l == 0:
            w[:, N_INPUTS:, :] = True
        if l == N_LAYERS - 1:
            w[:, :, 1:] = True
            b[1:] = True
        out.append(np.concatenate([w.ravel(), b]))
    return np.concatenate(out)


def adam(theta, grad, m1, m2, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8, frozen=None):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) on flat FP64 vectors:
    biased first and second moment estimates, bias correction by 1 - b^t,
    theta -= lr m_hat / (sqrt(v_hat) + eps).  Frozen entries are set to zero
    and keep their moments.  Returns (theta, m1, m2)."""
    m1n = b1 * m1 + (1.0 - b1) * grad
    m2n = b2 * m2 + (1.0 - b2) * grad * grad
    mh = m1n / (1.0 - b1 ** step)
    vh = m2n / (1.0 - b2 ** step)
    th = theta - lr * mh / (np.sqrt(vh) + eps)
    if frozen is not None:
        th = np.where(frozen, 0.0, th)
        m1n = np.where(frozen, m1, m1n)
        m2n = np.where(frozen, m2, m2n)
    return th, m1n, m2n


def train_step_grads(x0: np.ndarray, params: list, target: np.ndarray, target_scale: float):
    """Loss mean((out - target_scale target)^2) of the net on input x0 and
    its gradients as the GPU forms them: BF16 activations and weights, the
    output gradient 2 (out - t) / V rounded to BF16 and every back-propagated
    gradient rounded to BF16.  Returns (loss, flat FP64 gradient)."""
    acts, out = forward(x0, params, round_bf16=True)
    d = out - target * target_scale
    g_out = bf16_round(2.0 * d / d.size)
    grads = backward(acts, params, g_out, round_bf16=True)
    flat = np.concatenate([np.concatenate([dw.ravel(), db]) for dw, db in grads])
    return float(np.mean(d * d)), flat


def flatten(params: list) -> np.ndarray:
    """FP32 parameter vector in the C ABI order: per layer W (27,16,16) then b (16)."""
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in params]).astype(np.float32)


def unflatten(vec: np.ndarray) -> list:
    out = []
    per = 27 * C * C + C
    for l in range(N_LAYERS):
        seg = np.asarray(vec[l * per:(l + 1) * per], dtype=np.float64)
        out.append((seg[:27 * C * C].reshape(27, C, C), seg[27 * C * C:].copy()))
    return out
