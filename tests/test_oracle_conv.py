"""Pins for the oracle's conv net (CPU only): brute-force per-voxel sums,
BF16 rounding, and central finite differences of every gradient."""
import numpy as np
import pytest

from oracle import conv as oc


def test_bf16_round_known_values():
    x = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7 + 2**-9, 3.14159265, -2.5e-3, 0.0,
                  1.0 + 2**-7 + 2**-8 + 2**-10, 1.0 + 3 * 2**-8])
    got = oc.bf16_round(x)
    # BF16 keeps 8 significant bits (spacing 2^-7 above 1):
    assert got[0] == 1.0 and got[1] == 1.0        # tie -> even
    assert got[2] == 1.0 + 2**-7                  # below the midpoint -> down
    assert got[6] == 1.0 + 2**-6                  # above the midpoint -> up
    assert got[7] == 1.0 + 2**-6                  # tie between odd 1+2^-7 and even 1+2^-6
    assert abs(got[3] - 3.140625) < 1e-12
    assert abs(got[4] / -2.5e-3 - 1) < 2**-8
    assert got[5] == 0.0


def test_conv_matches_brute_force():
    rng = np.random.Generator(np.random.PCG64(1))
    n = 5
    x = rng.normal(size=(n, n, n, 3))
    w = rng.normal(size=(27, 3, 4))
    b = rng.normal(size=4)
    y = oc.conv(x, w, b)
    for (k, j, i) in [(0, 0, 0), (4, 2, 1), (2, 4, 4)]:
        ref = b.copy()
        for t, (dx, dy, dz) in enumerate(oc.TAPS):
            ref += x[(k + dz) % n, (j + dy) % n, (i + dx) % n] @ w[t]
        assert np.allclose(y[k, j, i], ref, rtol=1e-12, atol=1e-12)


def test_dgrad_is_adjoint_of_conv():
    rng = np.random.Generator(np.random.PCG64(2))
    n = 4
    x = rng.normal(size=(n, n, n, 3))
    g = rng.normal(size=(n, n, n, 5))
    w = rng.normal(size=(27, 3, 5))
    lhs = np.sum(oc.conv(x, w) * g)
    rhs = np.sum(x * oc.conv_dgrad(g, w))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_net_gradients_central_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    n = 4
    params = oc.init_params(7)
    x0 = np.zeros((n, n, n, oc.C))
    x0[..., :2] = rng.normal(size=(n, n, n, 2))
    g_out = rng.normal(size=(n, n, n))

    def loss(ps):
        _, out = oc.forward(x0, ps, round_bf16=False)
        return np.sum(out * g_out)

    acts, _ = oc.forward(x0, params, round_bf16=False)
    grads = oc.backward(acts, params, g_out)
    eps = 1e-6
    for l in range(oc.N_LAYERS):
        for (t, ci, co) in [(13, 0, 0), (0, 1, 0), (26, 0, 0)] if l == 0 else \
                [(13, 3, 0), (4, 0, 0), (22, 15, 0)] if l == 4 else [(13, 2, 5), (1, 7, 9)]:
            pp = [(w.copy(), b.copy()) for w, b in params]
            pm_ = [(w.copy(), b.copy()) for w, b in params]
            pp[l][0][t, ci, co] += eps
            pm_[l][0][t, ci, co] -= eps
            fd = (loss(pp) - loss(pm_)) / (2 * eps)
            assert grads[l][0][t, ci, co] == pytest.approx(fd, rel=1e-5, abs=1e-8), (l, t, ci, co)
        co = 0 if l == 4 else 3
        pp = [(w.copy(), b.copy()) for w, b in params]
        pm_ = [(w.copy(), b.copy()) for w, b in params]
        pp[l][1][co] += eps
        pm_[l][1][co] -= eps
        fd = (loss(pp) - loss(pm_)) / (2 * eps)
        assert grads[l][1][co] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_flatten_roundtrip():
    params = oc.init_params(1)
    vec = oc.flatten(params)
    assert vec.size == 5 * (27 * 256 + 16)
    back = oc.unflatten(vec)
    for (w, b), (w2, b2) in zip(params, back):
        assert np.allclose(w.astype(np.float32), w2) and np.allclose(b, b2)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2, so every step moves theta by lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m1, m2 = np.zeros(4), np.zeros(4), np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        th, m1, m2 = oc.adam(th, g, m1, m2, t, lr, eps=eps)
        assert np.allclose(th, -t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_keeps_frozen_parameters_zero():
    mask = oc.frozen_mask()
    assert mask.size == 5 * (27 * 256 + 16)
    per = 27 * 256 + 16
    w0 = mask[:27 * 256].reshape(27, 16, 16)
    assert w0[:, 3:, :].all() and not w0[:, :3, :].any()
    w4 = mask[4 * per:4 * per + 27 * 256].reshape(27, 16, 16)
    assert w4[:, :, 1:].all() and not w4[:, :, 0].any()
    rng = np.random.Generator(np.random.PCG64(0))
    th = rng.normal(size=mask.size)
    m1, m2 = rng.normal(size=mask.size), rng.uniform(size=mask.size)
    th2, m1b, m2b = oc.adam(th, rng.normal(size=mask.size), m1, m2, 3, 1e-3, frozen=mask)
    assert np.all(th2[mask] == 0.0) and np.array_equal(m1b[mask], m1[mask])
    assert np.array_equal(m2b[mask], m2[mask])
