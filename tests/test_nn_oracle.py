"""Pins of the surrogate-network oracle (oracle/nn_oracle.py) against
library routines, adjoint identities, finite differences and closed forms."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn_oracle as N


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_round_bf16_matches_torch_and_ties_to_even():
    import torch
    r = rng(0)
    x = np.concatenate([r.standard_normal(5000) * 10.0 ** r.uniform(-6, 6, 5000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.round_bf16(x), ref)
    assert N.round_bf16(1.0 + 2 ** -8) == 1.0
    assert N.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_conv3x3_is_zero_padded_correlation():
    r = rng(1)
    x = r.standard_normal((2, 7, 9, 3))
    w = r.standard_normal((4, 9, 3))
    b = r.standard_normal(4)
    y = N.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = np.full((7, 9), b[o])
            for c in range(3):
                ref += correlate2d(x[n, :, :, c], w[o, :, c].reshape(3, 3), mode="same",
                                   boundary="fill", fillvalue=0.0)
            assert np.allclose(y[n, :, :, o], ref, rtol=0, atol=1e-12)


def test_conv3x3_gradients_are_adjoints():
    r = rng(2)
    x = r.standard_normal((2, 6, 5, 4))
    w = r.standard_normal((3, 9, 4))
    dy = r.standard_normal((2, 6, 5, 3))
    lhs = np.sum(N.conv3x3(x, w) * dy)
    assert np.isclose(lhs, np.sum(x * N.conv3x3_grad_input(dy, w)), rtol=1e-12)
    dw, db = N.conv3x3_grad_weight(dy, x)
    assert np.isclose(lhs, np.sum(w * dw), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_pool_and_upsample_gradients_are_adjoints():
    r = rng(3)
    x = r.standard_normal((2, 8, 6, 3))
    y = r.standard_normal((2, 4, 3, 3))
    assert np.isclose(np.sum(N.pool2(x) * y), np.sum(x * N.pool2_grad(y)), rtol=1e-12)
    z = r.standard_normal((2, 16, 12, 3))
    assert np.isclose(np.sum(N.up2(x) * z), np.sum(x * N.up2_grad(z)), rtol=1e-12)
    # averaging a constant gives the constant; upsampling replicates
    assert np.allclose(N.pool2(np.full((1, 4, 4, 1), 2.5)), 2.5)
    assert N.up2(x)[0, 5, 3, 1] == x[0, 2, 1, 1]


def test_leaky_grad_and_mse_by_finite_differences():
    r = rng(4)
    z = r.standard_normal(50)
    h = 1e-6
    dy = r.standard_normal(50)
    fd = (N.leaky(z + h, 0.1) - N.leaky(z - h, 0.1)) / (2 * h) * dy
    assert np.allclose(N.leaky_grad(dy, N.leaky(z, 0.1), 0.1), fd, atol=1e-8)
    out, tgt = r.standard_normal((3, 4)), r.standard_normal((3, 4))
    loss, g = N.mse(out, tgt)
    e = np.zeros_like(out)
    e[1, 2] = h
    fd = (N.mse(out + e, tgt)[0] - N.mse(out - e, tgt)[0]) / (2 * h)
    assert abs(g[1, 2] - fd) < 1e-9


def test_adamw_closed_forms():
    r = rng(5)
    p0, g = r.standard_normal(20), r.standard_normal(20)
    lr, eps = 1e-3, 1e-8
    m = v = np.zeros(20)
    # a constant gradient: bias-corrected moments equal g and g^2 at every
    # step, so each step moves by lr g / (|g| + eps)
    p = p0
    for t in range(1, 6):
        p, m, v = N.adamw_step(p, g, m, v, t, lr, eps=eps)
        assert np.allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
    # zero gradient: pure decoupled decay, p_t = p_0 (1 - lr wd)^t
    p, m, v = p0, np.zeros(20), np.zeros(20)
    for t in range(1, 4):
        p, m, v = N.adamw_step(p, np.zeros(20), m, v, t, lr, wd=0.01)
    assert np.allclose(p, p0 * (1 - lr * 0.01) ** 3, rtol=1e-14)


def test_unet_shapes_and_parameter_count():
    sh = N.unet_shapes()
    assert sh[0] == (16, 9, 16) and sh[9] == (256, 9, 256) and sh[10] == (128, 9, 384)
    assert sh[-1] == (16, 9, 16)
    assert sum(o * t * c for o, t, c in sh) == 1965312


def small_net(seed, levels=3, base=4, cin=4, cout=4):
    r = rng(seed)
    shapes = N.unet_shapes(cin=cin, base=base, levels=levels, cout=cout)
    return [(r.standard_normal(s) / np.sqrt(9 * s[2]), 0.1 * r.standard_normal(s[0]))
            for s in shapes]


def test_unet_gradients_by_finite_differences():
    """Reverse pass of the whole encoder-decoder in FP64 (no bf16 rounding)
    against central differences of the loss."""
    params = small_net(6)
    r = rng(7)
    x = r.standard_normal((2, 8, 8, 4))
    tgt = r.standard_normal((2, 8, 8, 3))
    loss, grads = N.unet_loss_grads(params, x, tgt, levels=3, base=4, bf16=False)
    h = 1e-6
    for k in (0, 3, 5, len(params) - 1):
        w, b = params[k]
        for idx in [tuple(r.integers(0, s) for s in w.shape) for _ in range(3)]:
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            pp = list(params)
            pp[k] = (wp, b)
            lp = N.unet_loss_grads(pp, x, tgt, levels=3, base=4, bf16=False)[0]
            pp[k] = (wm, b)
            lm = N.unet_loss_grads(pp, x, tgt, levels=3, base=4, bf16=False)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(grads[k][0][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, idx)
        bp, bm = b.copy(), b.copy()
        bp[0] += h
        bm[0] -= h
        pp = list(params)
        pp[k] = (w, bp)
        lp = N.unet_loss_grads(pp, x, tgt, levels=3, base=4, bf16=False)[0]
        pp[k] = (w, bm)
        lm = N.unet_loss_grads(pp, x, tgt, levels=3, base=4, bf16=False)[0]
        assert abs(grads[k][1][0] - (lp - lm) / (2 * h)) <= 1e-6


def test_unet_bf16_rounding_changes_little():
    params = small_net(8)
    r = rng(9)
    x = r.standard_normal((1, 8, 8, 4))
    a = N.unet_forward(params, x, levels=3, base=4, bf16=False)
    b = N.unet_forward(params, x, levels=3, base=4, bf16=True)
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 1e-4 < rel < 3e-2
